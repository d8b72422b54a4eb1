"""Pins of the oracle's specular BRDF factors and of the denoiser's
edge-stopping weights, each against a value computed another way.

* GGX D: its projected-area normalisation, integrated by quadrature, and the
  textbook form of Walter et al. 2007 written in tan(theta_h).
* Smith visibility: the height-correlated masking-shadowing function
  G2 = 1 / (1 + Lambda(v) + Lambda(l)) of Heitz (JCGT 2014), with Lambda
  integrated numerically from the GGX slope distribution (not from its closed
  form), at oblique and grazing pairs where it differs from the separable
  product G1(v) G1(l).
* Schlick Fresnel at chosen half-angles, through the full BRDF.
* SVGF (Sec. 4.1; the depth gradient by finite differences, supplementary
  rendering details): the depth weight on a planar depth ramp, where the
  finite-difference gradient is exact and every tap's weight is known in
  closed form; the variance-guided luminance weight on a two-level step image,
  computed by hand; the variance carried through the iterations with squared
  weights.
None needs a GPU.
"""
import math

import numpy as np
import pytest
from scipy import integrate, ndimage

from oracle import oracle as O


def _lambda_by_quadrature(mu, alpha):
    """Smith Lambda of the isotropic GGX distribution for a direction at
    cos(theta) = mu, integrated from the marginal slope density
    P2(x) = 1 / (2 alpha (1 + x^2/alpha^2)^(3/2)):
    Lambda = (1/c) int_c^inf (x - c) P2(x) dx, c = cot(theta)."""
    c = mu / math.sqrt(1.0 - mu * mu)

    def p2(x):
        return 1.0 / (2.0 * alpha * (1.0 + (x / alpha) ** 2) ** 1.5)

    val, err = integrate.quad(lambda x: (x - c) * p2(x), c, np.inf, epsabs=1e-15, epsrel=1e-13,
                              limit=400)
    return val / c


def _ggx_walter(cos_h, alpha):
    """GGX distribution as written by Walter et al. 2007:
    alpha^2 / (pi cos^4 (alpha^2 + tan^2)^2)."""
    t2 = (1.0 - cos_h * cos_h) / (cos_h * cos_h)
    return alpha ** 2 / (math.pi * cos_h ** 4 * (alpha ** 2 + t2) ** 2)


def _pair(mu_v, mu_l, phi):
    n = np.array([0.0, 0.0, 1.0])
    sv, sl = math.sqrt(1 - mu_v ** 2), math.sqrt(1 - mu_l ** 2)
    v = np.array([sv, 0.0, mu_v])
    l = np.array([sl * math.cos(phi), sl * math.sin(phi), mu_l])
    return n, v, l


def pin_lambda_quadrature_matches_closed_form():
    for alpha in (0.09, 0.36, 0.81):
        for mu in (0.05, 0.3, 0.8):
            lq = _lambda_by_quadrature(mu, alpha)
            t2 = (1 - mu * mu) / (mu * mu)
            assert abs(lq - (math.sqrt(1 + alpha ** 2 * t2) - 1) / 2) < 1e-10


def pin_smith_visibility_is_height_correlated():
    """Vis * 4 (n.l)(n.v) = 1 / (1 + Lambda(v) + Lambda(l)) at oblique and
    grazing pairs; the separable product 1 / ((1 + Lambda(v))(1 + Lambda(l)))
    differs there by more than 1e-3 relative in at least one case."""
    worst_sep = 0.0
    for r in (0.3, 0.6, 0.9):
        alpha = r * r
        for mu_v, mu_l, phi in ((0.3, 0.8, 0.7), (0.1, 0.5, 2.0), (0.05, 0.9, 3.0), (0.2, 0.2, 1.0),
                                (0.6, 0.7, 0.3)):
            n, v, l = _pair(mu_v, mu_l, phi)
            D, Vis, P = O.brdf_terms(n[None], v[None], l[None], np.array([r]))
            lv, ll = _lambda_by_quadrature(mu_v, alpha), _lambda_by_quadrature(mu_l, alpha)
            g2 = 1.0 / (1.0 + lv + ll)
            got = Vis[0] * 4.0 * mu_l * mu_v
            assert abs(got - g2) <= 1e-10 * g2, (r, mu_v, mu_l, got, g2)
            sep = 1.0 / ((1.0 + lv) * (1.0 + ll))
            worst_sep = max(worst_sep, abs(sep - g2) / g2)
    assert worst_sep > 1e-3


def pin_ggx_distribution_normalised_and_textbook():
    """int D(h) (n.h) dw_h = 1 over the hemisphere, and D matches Walter's
    tan-form at sampled half-vector angles."""
    n = np.array([[0.0, 0.0, 1.0]])
    for r in (0.3, 0.6, 1.0):
        alpha = r * r

        def d_of(th):
            h = np.array([[math.sin(th), 0.0, math.cos(th)]])
            D, _, _ = O.brdf_terms(n, h, h, np.array([r]))  # v = l = h gives half vector h
            return D[0]

        # substitute theta = atan(alpha s): the lobe width scales with alpha
        def integrand(s):
            th = math.atan(alpha * s)
            dth = alpha / (1.0 + (alpha * s) ** 2)
            return d_of(th) * math.cos(th) * math.sin(th) * dth

        val, _ = integrate.quad(integrand, 0.0, np.inf, epsabs=1e-13, epsrel=1e-11, limit=400)
        assert abs(2.0 * math.pi * val - 1.0) < 1e-8, (r, 2 * math.pi * val)
        for th in (0.0, 0.2, 0.7, 1.2, 1.5):
            ref = _ggx_walter(math.cos(th), alpha)
            assert abs(d_of(th) - ref) <= 1e-12 * ref


def _reflect_pair(h, c, tang):
    """v and l with normalize(v + l) = h and v.h = c (tang: unit, orthogonal to h)."""
    v = c * h + math.sqrt(1 - c * c) * tang
    l = 2 * c * h - v
    return v, l


def pin_schlick_fresnel_through_the_brdf():
    """With metallic m and albedo a, F0 = 0.04 (1 - m) + a m and
    f - (1 - m) a / pi = D F Vis with F = F0 + (1 - F0)(1 - v.h)^5.  At
    v.h = 1/2 and F0 = 0.04 this is 0.04 + 0.96/32 = 0.07; as v.h -> 0, F -> 1.
    D and Vis come from Walter's form and the quadrature Lambda."""
    n = np.array([0.0, 0.0, 1.0])
    cases = []
    # symmetric about the normal (h = n), v.h = 1/2
    cases.append((n.copy(), 0.5, np.array([1.0, 0.0, 0.0])))
    # tilted half vectors
    for th_h, c in ((0.3, 0.5), (0.25, 0.2), (0.1, 0.05), (0.4, 0.8)):
        h = np.array([math.sin(th_h), 0.0, math.cos(th_h)])
        tang = np.array([0.0, 1.0, 0.0])
        cases.append((h, c, tang))
    for h, c, tang in cases:
        v, l = _reflect_pair(h, c, tang)
        assert v @ n > 0 and l @ n > 0
        for r in (0.3, 0.7):
            alpha = r * r
            for m, a in ((0.0, 0.5), (1.0, 0.25), (0.3, 0.8)):
                av = np.full((1, 3), a)
                f, *_ = O.brdf(n[None], v[None], l[None], av, np.array([r]), np.array([m]))
                spec = f[0, 0] - (1 - m) * a / math.pi
                F0 = 0.04 * (1 - m) + a * m
                F = F0 + (1 - F0) * (1 - c) ** 5
                mu_v, mu_l = float(v @ n), float(l @ n)
                g2 = 1.0 / (1.0 + _lambda_by_quadrature(mu_v, alpha) + _lambda_by_quadrature(mu_l, alpha))
                ref = _ggx_walter(float(h @ n), alpha) * F * g2 / (4 * mu_v * mu_l)
                assert abs(spec - ref) <= 1e-9 * ref, (c, r, m, spec, ref)
    # the half-angle value itself
    v, l = _reflect_pair(n, 0.5, np.array([1.0, 0.0, 0.0]))
    _, _, P = O.brdf_terms(n[None], v[None], l[None], np.array([0.5]))
    assert abs(0.04 + 0.96 * P[0] - 0.07) < 1e-15
    # grazing v.h -> 0: P -> 1
    v, l = _reflect_pair(np.array([0.0, 0.0, 1.0]), 1e-6, np.array([1.0, 0.0, 0.0]))
    _, _, P = O.brdf_terms(n[None], v[None], l[None], np.array([0.5]))
    assert abs(P[0] - 1.0) < 1e-5


# ---------------------------------------------------------------- denoiser --
H3 = np.array([1 / 16, 1 / 4, 3 / 8, 1 / 4, 1 / 16])


def pin_denoise_depth_weight_on_a_ramp():
    """Depth z = a x + b y (a = 1, b = 1/8, exact in FP32): forward
    differences give the gradient (a, b) exactly at every pixel, so for the
    tap (i, j) at step s the depth weight is
    exp(-|s(a i + b j)| / (sigma_z |s(a i + b j)| + 1e-6)) everywhere.  With
    constant normals and a colour pattern of constant luminance (two colours
    whose luminance differs by zero in exact arithmetic) the filter is the
    a-trous cascade with that kernel, taps outside dropped and renormalised,
    computed here with scipy's correlate."""
    Hh, Ww = 29, 37
    yy, xx = np.mgrid[0:Hh, 0:Ww]
    a, b = 1.0, 0.125
    depth = (a * xx + b * yy).astype(np.float32)
    assert np.array_equal(depth.astype(np.float64), a * xx + b * yy)
    nrm = np.zeros((Hh, Ww, 3), np.float32)
    nrm[..., 1] = 1.0
    # luminance 0.2126 R + 0.7152 G + 0.0722 B: dR = 3576/4096, dG = -1063/4096
    # change it by 0.2126*3576 - 0.7152*1063 = 0 (exactly, in decimal)
    base = np.array([0.5, 1.0, 0.75])
    alt = base + np.array([3576.0, -1063.0, 0.0]) / 4096.0
    rng = np.random.default_rng(4)
    pick = rng.integers(0, 2, (Hh, Ww))
    img = np.where(pick[..., None] == 1, alt, base).astype(np.float32)
    assert np.array_equal(img.astype(np.float64), np.where(pick[..., None] == 1, alt, base))
    for sz in (1.0, 0.5):
        out = O.denoise(img, depth, nrm, iters=4, sigma_z=sz, sigma_n=128.0, sigma_l=4.0)
        ref = img.astype(np.float64)
        ones = np.ones((Hh, Ww))
        for it in range(4):
            s = 1 << it
            K = np.zeros((4 * s + 1, 4 * s + 1))
            for j in range(-2, 3):
                for i in range(-2, 3):
                    dz = abs(s * (a * i + b * j))
                    K[(j + 2) * s, (i + 2) * s] = H3[i + 2] * H3[j + 2] * math.exp(-dz / (sz * dz + 1e-6))
            norm = ndimage.correlate(ones, K, mode="constant", cval=0.0)
            ref = np.stack([ndimage.correlate(ref[..., c], K, mode="constant", cval=0.0) / norm
                            for c in range(3)], -1)
        assert np.max(np.abs(out - ref)) < 1e-6, np.max(np.abs(out - ref))


def pin_denoise_luminance_weight_on_a_step():
    """Grey image, value A in columns 0..5 and B from column 6, constant depth
    and normals.  At pixel (8, 5) the 7x7 windows of columns 4, 5 and 6 hold
    5/2, 4/3 and 3/4 columns of A/B, so their luminance variances are
    10/49, 12/49 and 12/49 of (A - B)^2, and the 3x3 blur gives
    (10/4 + 12/2 + 12/4)/49 = 11.5/49 of it.  One iteration weights the B taps
    by exp(-|A - B| / (sigma_l sqrt(11.5/49) |A - B|)) and the A taps by 1."""
    Hh, Ww = 16, 12
    A, B = 1.0, 3.0
    img = np.full((Hh, Ww, 3), A, np.float32)
    img[:, 6:] = B
    depth = np.full((Hh, Ww), 2.0, np.float32)
    nrm = np.zeros((Hh, Ww, 3), np.float32)
    nrm[..., 2] = 1.0
    for sl in (4.0, 1.5):
        out = O.denoise(img, depth, nrm, iters=1, sigma_z=1.0, sigma_n=128.0, sigma_l=sl)
        wB = math.exp(-1.0 / (sl * math.sqrt(11.5 / 49.0)))
        hA = 1 / 16 + 1 / 4 + 3 / 8     # taps at columns 3, 4, 5
        hB = 1 / 4 + 1 / 16             # taps at columns 6, 7
        ref = (hA * A + hB * wB * B) / (hA + hB * wB)
        # 1e-9: the 1e-10 guard in the weight's denominator and the rounding
        # of the luminance coefficients, which sum to one only in decimal
        assert np.allclose(out[8, 5], ref, rtol=1e-9, atol=0), (out[8, 5] - ref)


def pin_denoise_variance_propagates_with_squared_weights():
    """With every edge-stopping weight at one (huge sigma_z and sigma_l,
    sigma_n = 0) the luminance variance leaving iteration k is
    sum_q w_q^2 var_q / (sum_q w_q)^2 with the B3 weights of that step, the
    initial variance being the population variance of the luminance over the
    7x7 window's taps inside the image."""
    rng = np.random.default_rng(9)
    Hh, Ww = 21, 26
    img = np.exp(rng.standard_normal((Hh, Ww, 3))).astype(np.float32)
    depth = rng.uniform(1, 3, (Hh, Ww)).astype(np.float32)
    nrm = np.zeros((Hh, Ww, 3), np.float32)
    nrm[..., 0] = 1.0
    c = img.astype(np.float64)
    lum = 0.2126 * c[..., 0] + 0.7152 * c[..., 1] + 0.0722 * c[..., 2]
    ones = np.ones((Hh, Ww))
    box = np.ones((7, 7))
    cnt = ndimage.correlate(ones, box, mode="constant", cval=0.0)
    m1 = ndimage.correlate(lum, box, mode="constant", cval=0.0) / cnt
    m2 = ndimage.correlate(lum * lum, box, mode="constant", cval=0.0) / cnt
    var = np.maximum(m2 - m1 * m1, 0.0)
    for iters in (1, 2, 3):
        _, got = O.denoise(img, depth, nrm, iters=iters, sigma_z=1e30, sigma_n=0.0, sigma_l=1e30,
                           return_var=True)
        v = var.copy()
        for it in range(iters):
            s = 1 << it
            k1 = np.zeros(4 * s + 1)
            k1[::s] = H3
            K = np.outer(k1, k1)
            v = ndimage.correlate(v, K * K, mode="constant", cval=0.0) / \
                ndimage.correlate(ones, K, mode="constant", cval=0.0) ** 2
        assert np.max(np.abs(got - v)) <= 1e-12 * np.max(v), iters


PINS = [pin_lambda_quadrature_matches_closed_form, pin_smith_visibility_is_height_correlated,
        pin_ggx_distribution_normalised_and_textbook, pin_schlick_fresnel_through_the_brdf,
        pin_denoise_depth_weight_on_a_ramp, pin_denoise_luminance_weight_on_a_step,
        pin_denoise_variance_propagates_with_squared_weights]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__[4:] for p in PINS])
def test_pin(pin):
    pin()


def test_render_and_backward_reject_missing_pointers():
    """The Python guard rejects shade mode without normals or view vectors,
    and the C entry points themselves return -1 (writing nothing) for the
    NULL pointers the guard would have caught."""
    import ctypes as C
    import hg_inputs as H
    rng = np.random.Generator(np.random.PCG64(3))
    L, log2T = 2, 10
    model = dict(table=(rng.standard_normal((L, 1 << log2T, 2)) * 0.1).astype(np.float32),
                 brdf=H.make_mlp(2 * L, 64, 5, rng), irt=H.make_mlp(2 * L + 3, 64, 2, rng),
                 res=[4, 8])
    om = O.OracleModel(model, H.BOX_LO, H.BOX_EXTENT)
    oe = O.OracleEnv(np.ones((4, 8, 3), np.float32))
    pos = np.zeros((3, 3), np.float32)
    nrm = np.tile(np.float32([0, 1, 0]), (3, 1))
    with pytest.raises(ValueError):
        O.render(om, oe, O.sampling(4), pos, nrm, None)
    with pytest.raises(ValueError):
        O.render(om, oe, O.sampling(4), pos, None, nrm)
    # straight to C, past the Python guard
    P, keep = O._points(pos, nrm, None, None)
    rgb = np.full((3, 3), 7.0)
    rc = O.lib().or_render(C.byref(om.c), C.byref(oe.c), C.byref(O.sampling(4)), C.byref(P),
                           C.c_int32(1), O._p(rgb), None, None)
    assert rc == -1 and np.all(rgb == 7.0)
    P, keep = O._points(pos, None, None, None)
    g = np.zeros(3, np.float32)
    gt = np.zeros(om.table.shape)
    gb, gi = np.zeros(om.n_brdf_params()), np.zeros(om.n_irt_params())
    rc = O.lib().or_backward(C.byref(om.c), C.byref(oe.c), C.byref(O.sampling(4)), C.byref(P),
                             C.c_int32(1), O._p(np.zeros((3, 3), np.float32)), O._p(g), O._p(g),
                             O._p(gt), O._p(gb), O._p(gi), None)
    assert rc == -1 and not gt.any()
