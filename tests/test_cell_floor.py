"""The two FP32 forms of the hash-grid cell index used by the GPU encoders,
emulated bit for bit on the host, against the exact floor of u N.

The cell of a coordinate u in [0, 1] at resolution N is floor(u N) of the
exact product, clamped to N - 1, with the fractional position w = u N - cell
(the encoder H of Sec. 3.2, multi-level tables as in InstantNGP, whose level
vertices are the integer points of the coordinate scaled by N). The GPU forms
it from FP32 operations only, in two ways (a floor of an fma residual; the
product's error and a compare), whose agreement with the exact floor rests on
a rounding argument. FP32 arithmetic is reproduced exactly here: the product
of two FP32 numbers is exact in FP64, so rounding it to FP32 gives fl(u N);
u N - x for an integer-valued FP32 x is exact in FP64 (at most 49 significant
bits), so rounding it to FP32 gives the fma fl(u N - x). Every u next to every
cell boundary of several resolutions must give the exact cell and the
once-rounded fractional position."""
import numpy as np
import pytest

F32 = np.float32


def cell_floor_fma(u, n):
    """fl = floor(fl(u N)); fl += floor(fl(u N - fl)); clamp; w = fl(u N - fl)."""
    un = u.astype(np.float64) * n                 # exact
    p = un.astype(F32)
    fl = np.floor(p).astype(np.float64)
    fl = fl + np.floor((un - fl).astype(F32)).astype(np.float64)
    fl = np.minimum(fl, n - 1)
    return fl.astype(np.int64), (un - fl).astype(F32)


def cell_floor_sel(u, n):
    """e = fl(u N - p); fl = floor(p) - [fl == p and e < 0]; clamp; w = (p - fl) + e."""
    un = u.astype(np.float64) * n
    p = un.astype(F32)
    e = (un - p.astype(np.float64)).astype(F32)
    fl = np.floor(p)
    fl = np.where((fl == p) & (e < 0), fl - F32(1), fl)
    fl = np.minimum(fl, F32(n - 1))
    w = ((p - fl).astype(F32) + e).astype(F32)
    return fl.astype(np.int64), w


def boundary_coordinates(n, rng, per_side=4, n_k=400):
    k = np.unique(np.concatenate([[0, 1, n - 1, n], rng.integers(0, n + 1, n_k)]))
    base = (k.astype(np.float64) / n).astype(F32)
    out = [base]
    lo, hi = base.copy(), base.copy()
    for _ in range(per_side):
        lo = np.nextafter(lo, F32(-1))
        hi = np.nextafter(hi, F32(2))
        out += [lo, hi]
    u = np.concatenate(out + [rng.random(4000).astype(F32)])
    return np.clip(u, F32(0), F32(1))


@pytest.mark.parametrize("n", [16, 22, 30, 128, 2047, 2048, 131072, (1 << 24) - 1])
def test_both_forms_give_the_exact_cell_and_weight(n):
    rng = np.random.default_rng(n)
    u = boundary_coordinates(n, rng)
    un = u.astype(np.float64) * n
    cell = np.minimum(np.floor(un), n - 1).astype(np.int64)
    w_exact = (un - cell).astype(F32)               # once-rounded fractional position
    for form in (cell_floor_fma, cell_floor_sel):
        c, w = form(u, n)
        bad = np.flatnonzero(c != cell)
        assert bad.size == 0, (form.__name__, u[bad[:5]], c[bad[:5]], cell[bad[:5]])
        assert np.array_equal(w, w_exact), form.__name__


def test_the_rounding_case_occurs():
    # the case the forms exist for: fl(u N) is an integer while u N is below it
    rng = np.random.default_rng(1)
    hits = 0
    for n in (22, 30, 2047, 131072):
        u = boundary_coordinates(n, rng)
        un = u.astype(np.float64) * n
        p = un.astype(F32).astype(np.float64)
        hits += int(np.sum((p == np.floor(p)) & (un < p)))
    assert hits > 0
