"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, invariants, special cases that reduce to
a textbook routine, or finite differences.  None needs a GPU.
"""
import math
import os

import numpy as np
import pytest

import hg_inputs as H
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LO, EXT = H.BOX_LO, H.BOX_EXTENT


def small_model(L=4, log2T=10, res=None, seed=11, hidden=64):
    res = res or H.level_resolutions(L, 4, 32)
    rng = np.random.Generator(np.random.PCG64(seed))
    table = (rng.standard_normal((L, 1 << log2T, 2)) * 0.1).astype(np.float32)
    nf = 2 * L
    return dict(table=table, brdf=H.make_mlp(nf, hidden, 5, rng), irt=H.make_mlp(nf + 3, hidden, 2, rng),
                res=res)


def const_mlp(n_in, n_out, bias, hidden=64):
    """MLP whose output is the constant `bias` (zero weights)."""
    return [np.zeros((hidden, n_in), np.float32), np.zeros(hidden, np.float32),
            np.zeros((hidden, hidden), np.float32), np.zeros(hidden, np.float32),
            np.zeros((n_out, hidden), np.float32), np.asarray(bias, np.float32)]


def logit(p):
    return math.log(p / (1 - p))


# ---------------------------------------------------------------- Philox ---
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        assert O.philox(w[0:4], w[4:6]) == w[6:10]


def test_uniforms_are_bin_centres():
    pid = np.arange(4096, dtype=np.uint32)
    u = O.uniforms(7, pid, np.zeros_like(pid), pid % 8, 1)
    k = u * 65536 - 0.5
    assert np.all(k == np.round(k)) and u.min() > 0 and u.max() < 1
    # roughly uniform
    assert abs(u.mean() - 0.5) < 0.02


# ---------------------------------------------------------------- sampler --
def rand_normals(n, seed=3):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("N", [2, 8, 32, 128, 512])
def test_sampler_unit_hemisphere_strata(N):
    n = rand_normals(64)
    nn = np.repeat(n, N, axis=0)
    pid = np.repeat(np.arange(64), N)
    k = np.tile(np.arange(N), 64)
    w = O.sample_dirs(7, nn, pid, 5, k, 1, N)
    assert np.allclose(np.linalg.norm(w, axis=1), 1, atol=1e-14)
    cos = np.sum(w * nn, axis=1)
    assert cos.min() > 0
    # stratum of s1 = 1 - cos^2 (frame independent): a = k // n_b
    na = 1 << (int(math.log2(N)) // 2)
    nb = N // na
    u = O.uniforms(7, pid, np.full_like(pid, 5), k, 1)
    s1 = (k // nb + u[:, 0]) / na
    assert np.allclose(cos, np.sqrt(1 - s1), atol=1e-13)
    # azimuth differences are frame independent: tangential parts of two
    # samples of one point subtend 2*pi*(s2_i - s2_j)
    s2 = (k % nb + u[:, 1]) / nb
    wt = w - cos[:, None] * nn
    wt /= np.linalg.norm(wt, axis=1, keepdims=True)
    wt = wt.reshape(64, N, 3)
    s2 = s2.reshape(64, N)
    c = np.einsum("pi,pi->p", wt[:, 0], wt[:, -1])
    assert np.allclose(c, np.cos(2 * np.pi * (s2[:, 0] - s2[:, -1])), atol=1e-10)
    # orientation: the frame is right-handed, so the cross product of the
    # tangential parts points along +n with the sign of sin(2 pi ds2)
    cr = np.einsum("pi,pi->p", np.cross(wt[:, 0], wt[:, -1]), n)
    assert np.allclose(cr, np.sin(2 * np.pi * (s2[:, -1] - s2[:, 0])), atol=1e-10)


def test_sampler_cosine_moment_and_determinism():
    n = np.tile(np.array([[0.0, 1.0, 0.0]]), (1, 1))
    N = 1024
    nn = np.repeat(rand_normals(32), N, axis=0)
    k = np.tile(np.arange(N), 32)
    pid = np.repeat(np.arange(32), N)
    w = O.sample_dirs(7, nn, pid, 0, k, 0, N)
    cos = np.sum(w * nn, axis=1)
    # cosine-weighted hemisphere: E[cos] = 2/3, E[cos^2] = 1/2
    assert abs(cos.mean() - 2 / 3) < 1e-3
    assert abs((cos ** 2).mean() - 0.5) < 1e-3
    w2 = O.sample_dirs(7, nn, pid, 0, k, 0, N)
    assert np.array_equal(w, w2)
    w3 = O.sample_dirs(8, nn, pid, 0, k, 0, N)
    assert not np.allclose(w, w3)
    del n


# ---------------------------------------------------------------- encoder --
def test_hash_index_structure():
    """Spatial hash of Mueller et al. 2022 Eq. 4: xor of coordinate*prime with
    primes (1, 2654435761, 805459861), mod 2^32, masked to T."""
    m = small_model(L=1, log2T=10, res=[64])  # (65)^3 > 2^10: hashed
    om = O.OracleModel(m, LO, EXT)
    T = 1 << 10
    N = 64

    def vertex_pos(v):
        return np.array([LO + EXT * v[0] / N, LO + EXT * v[1] / N, LO + EXT * v[2] / N], np.float32)

    def idx_of(v):
        i, w = O.encode_index(om, vertex_pos(v)[None])
        assert np.all(w[0, 0] == 0)
        return int(i[0, 0, 0])

    assert idx_of((0, 0, 0)) == 0
    assert idx_of((5, 0, 0)) == 5
    assert idx_of((0, 1, 0)) == 2654435761 % T
    assert idx_of((0, 0, 1)) == 805459861 % T
    assert idx_of((0, 3, 0)) == (3 * 2654435761 % 2 ** 32) % T
    for v in [(3, 5, 7), (13, 40, 2), (63, 63, 63)]:
        assert idx_of(v) == idx_of((v[0], 0, 0)) ^ idx_of((0, v[1], 0)) ^ idx_of((0, 0, v[2]))


def test_dense_index_is_bijection_and_hashed_in_range():
    m = small_model(L=3, log2T=12, res=[8, 12, 40])   # 729, 2197 dense; 68921 hashed
    om = O.OracleModel(m, LO, EXT)
    res = m["res"]
    for l, N in enumerate(res[:2]):
        # sample every cell at its centre; corner bit b of the cell c is the
        # vertex c + (b&1, b>>1&1, b>>2&1)
        c = np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3)
        pos = (LO + EXT * (c + 0.5) / N).astype(np.float32)
        idx, w = O.encode_index(om, pos)
        assert np.all(np.abs(w[:, l] - 0.5) < 1e-6)
        seen = {}
        for b in range(8):
            dv = np.array([b & 1, (b >> 1) & 1, (b >> 2) & 1])
            v = c + dv
            key = v[:, 0] + 1000 * (v[:, 1] + 1000 * v[:, 2])
            for kk, ii in zip(key, idx[:, l, b]):
                assert seen.setdefault(int(kk), int(ii)) == int(ii)
        vals = np.array(list(seen.values()))
        assert len(seen) == (N + 1) ** 3 and len(np.unique(vals)) == (N + 1) ** 3
        assert vals.max() < (N + 1) ** 3
    rng = np.random.default_rng(0)
    pos = rng.uniform(-9, 9, (20000, 3)).astype(np.float32)
    idx, w = O.encode_index(om, pos)
    assert idx.max() < (1 << 12)
    assert w.min() >= 0 and w.max() <= 1


def test_vertex_reproduction_and_partition_of_unity():
    m = small_model(L=3, log2T=14, res=[16, 32, 64])
    om = O.OracleModel(m, LO, EXT)
    rng = np.random.default_rng(1)
    # positions exactly on vertices of level 2 (N=64) are vertices of no
    # coarser level in general, but on level 2 exactly one corner has weight 1
    v = rng.integers(0, 65, (500, 3))
    pos = (LO + EXT * v / 64).astype(np.float32)
    f = O.encode(om, pos)
    idx, w = O.encode_index(om, pos)
    corner = (w[:, 2, 0] == 1) * 1 + (w[:, 2, 1] == 1) * 2 + (w[:, 2, 2] == 1) * 4
    e = m["table"][2][idx[np.arange(500), 2, corner]]
    assert np.array_equal(f[:, 4:6], e.astype(np.float64))
    # all-ones table: every level's interpolated feature is exactly 1
    m1 = dict(m)
    m1["table"] = np.ones_like(m["table"])
    om1 = O.OracleModel(m1, LO, EXT)
    pos = rng.uniform(-10, 10, (5000, 3)).astype(np.float32)
    assert np.max(np.abs(O.encode(om1, pos) - 1)) < 1e-15


def test_trilinear_reproduces_affine_fields():
    """Dense levels filled with an affine function of the vertex coordinate:
    trilinear interpolation reproduces it exactly, per axis and per level."""
    res = [6, 9]
    L, log2T = 2, 10
    m = small_model(L=L, log2T=log2T, res=res)
    A = np.array([[0.3, -0.7, 1.1], [-0.2, 0.5, 0.9]])
    c = np.array([0.25, -1.5])
    tab = np.zeros((L, 1 << log2T, 2), np.float32)
    for l, N in enumerate(res):
        g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        dense = g[:, 0] + (N + 1) * (g[:, 1] + (N + 1) * g[:, 2])
        for k in range(2):
            tab[l, dense, k] = (g @ A[k] + c[k]) / N
    m["table"] = tab
    om = O.OracleModel(m, LO, EXT)
    rng = np.random.default_rng(2)
    pos = rng.uniform(LO, LO + EXT, (4000, 3)).astype(np.float32)
    f = O.encode(om, pos)
    u = (pos.astype(np.float32) - np.float32(LO)).astype(np.float64) / EXT
    for l, N in enumerate(res):
        p = u * N
        for k in range(2):
            # stored values are FP32 roundings of the affine field
            ref = (p @ A[k] + c[k]) / N
            assert np.max(np.abs(f[:, 2 * l + k] - ref)) < 1e-6
    # with an exactly representable field the reproduction is exact
    A2 = np.array([[1.0, 2.0, 4.0], [0.5, -1.0, 0.25]])
    tab2 = np.zeros_like(tab)
    for l, N in enumerate(res):
        g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        dense = g[:, 0] + (N + 1) * (g[:, 1] + (N + 1) * g[:, 2])
        for k in range(2):
            tab2[l, dense, k] = g @ A2[k]
    m["table"] = tab2
    om = O.OracleModel(m, LO, EXT)
    f = O.encode(om, pos)
    for l, N in enumerate(res):
        for k in range(2):
            assert np.max(np.abs(f[:, 2 * l + k] - (u * N) @ A2[k])) < 1e-12


def test_encode_clamps_outside_box():
    m = small_model(L=2, log2T=10, res=[4, 8])
    om = O.OracleModel(m, LO, EXT)
    inside = np.array([[LO, 0.0, LO + EXT]], np.float32)
    outside = np.array([[LO - 3.0, 0.0, LO + EXT + 5.0]], np.float32)
    assert np.array_equal(O.encode(om, inside), O.encode(om, outside))


# -------------------------------------------------------------------- MLP --
def test_mlp_matches_numpy_matmul():
    m = small_model(L=16, log2T=10, res=list(range(4, 20)))
    om = O.OracleModel(m, LO, EXT)
    rng = np.random.default_rng(4)
    for which, ws in (("brdf", m["brdf"]), ("irt", m["irt"])):
        x = rng.standard_normal((257, ws[0].shape[1]))
        W = [w.astype(np.float64) for w in ws]
        h = np.maximum(x @ W[0].T + W[1], 0)
        h = np.maximum(h @ W[2].T + W[3], 0)
        ref = h @ W[4].T + W[5]
        assert np.max(np.abs(O.mlp_forward(om, which, x) - ref)) < 1e-13


# -------------------------------------------------------------------- env --
def texel_dir(i, j, H_, W_):
    th = (j + 0.5) / H_ * np.pi
    ph = (i + 0.5) / W_ * 2 * np.pi - np.pi
    return np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], -1)


def test_env_lookup_texel_centres_and_seam():
    env = H.make_env(8, 16, seed=9)
    oe = O.OracleEnv(env)
    jj, ii = np.meshgrid(np.arange(8), np.arange(16), indexing="ij")
    d = texel_dir(ii.ravel(), jj.ravel(), 8, 16)
    out = O.env_lookup(oe, d)
    assert np.max(np.abs(out - env.reshape(-1, 3))) < 1e-12
    # constant map
    oe1 = O.OracleEnv(np.full((8, 16, 3), 2.5, np.float32))
    rng = np.random.default_rng(5)
    v = rng.standard_normal((1000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    assert np.max(np.abs(O.env_lookup(oe1, v) - 2.5)) < 1e-13
    # midpoint between two horizontally adjacent centres -> average; across
    # the azimuth seam (column W-1 to column 0) as well
    for (i0, i1) in ((3, 4), (15, 0)):
        th = (2 + 0.5) / 8 * np.pi
        ph0 = (i0 + 0.5) / 16 * 2 * np.pi - np.pi
        ph = ph0 + 0.5 / 16 * 2 * np.pi
        dd = np.array([[np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)]])
        assert np.allclose(O.env_lookup(oe, dd)[0], 0.5 * (env[2, i0] + env[2, i1]), atol=1e-12)
    # continuity across phi = +-pi
    eps = 1e-9
    a = np.array([[-np.cos(eps), 0.3, np.sin(eps)], [-np.cos(eps), 0.3, -np.sin(eps)]])
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    o = O.env_lookup(oe, a)
    assert np.allclose(o[0], o[1], atol=1e-6)


# ------------------------------------------------------------------- BRDF --
def test_brdf_closed_forms_and_reciprocity():
    rng = np.random.default_rng(6)
    n = np.array([[0.0, 0.0, 1.0]])
    # normal incidence v = l = n: h = n, D = 1/(pi alpha^2), Vis = 1/4, F = F0
    for r in (0.09, 0.3, 0.7, 1.0):
        a = np.array([[0.2, 0.5, 0.9]])
        for mm in (0.0, 0.4):
            f, *_ = O.brdf(n, n, n, a, [r], [mm])
            al2 = r ** 4
            F0 = 0.04 * (1 - mm) + a * mm
            ref = (1 - mm) * a / np.pi + F0 / (np.pi * al2) * 0.25
            assert np.allclose(f, ref, rtol=1e-13)
    # reciprocity
    v = rng.standard_normal((200, 3)); v[:, 2] = np.abs(v[:, 2]) + 0.05
    l = rng.standard_normal((200, 3)); l[:, 2] = np.abs(l[:, 2]) + 0.05
    v /= np.linalg.norm(v, axis=1, keepdims=True); l /= np.linalg.norm(l, axis=1, keepdims=True)
    nn = np.repeat(n, 200, 0)
    a = rng.uniform(0, 1, (200, 3)); r = rng.uniform(0.09, 1, 200); m = rng.uniform(0, 1, 200)
    f1, *_ = O.brdf(nn, v, l, a, r, m)
    f2, *_ = O.brdf(nn, l, v, a, r, m)
    assert np.allclose(f1, f2, rtol=1e-12)
    # below the horizon: zero
    lb = l.copy(); lb[:, 2] *= -1
    f3, *_ = O.brdf(nn, v, lb, a, r, m)
    assert np.all(f3 == 0)
    # diffuse-only flag
    f4, *_ = O.brdf(nn, v, l, a, r, m, diffuse_only=True)
    assert np.allclose(f4, a / np.pi, rtol=1e-15)


def test_brdf_derivatives_match_finite_differences():
    rng = np.random.default_rng(7)
    cnt = 100
    n = rand_normals(cnt, 11)
    def hemi(seed):
        x = rand_normals(cnt, seed)
        s = np.sign(np.sum(x * n, 1))[:, None]
        return x * s
    v, l = hemi(12), hemi(13)
    a = rng.uniform(0.05, 0.95, (cnt, 3)); r = rng.uniform(0.1, 0.99, cnt); m = rng.uniform(0.05, 0.95, cnt)
    f, dfa, dfr, dfm = O.brdf(n, v, l, a, r, m)
    h = 1e-6
    for c in range(3):
        ap, am = a.copy(), a.copy(); ap[:, c] += h; am[:, c] -= h
        fd = (O.brdf(n, v, l, ap, r, m)[0][:, c] - O.brdf(n, v, l, am, r, m)[0][:, c]) / (2 * h)
        assert np.allclose(fd, dfa[:, c], rtol=1e-6, atol=1e-8)
    fd = (O.brdf(n, v, l, a, r + h, m)[0] - O.brdf(n, v, l, a, r - h, m)[0]) / (2 * h)
    assert np.allclose(fd, dfr, rtol=1e-5, atol=1e-7)
    fd = (O.brdf(n, v, l, a, r, m + h)[0] - O.brdf(n, v, l, a, r, m - h)[0]) / (2 * h)
    assert np.allclose(fd, dfm, rtol=1e-6, atol=1e-8)


def test_specular_energy_bound():
    """Directional albedo of the specular lobe with F = 1 (m = 1, a = 1) is at
    most 1 and approaches 1 for a near-mirror (microfacet energy balance)."""
    nth, nph = 2000, 256
    th = (np.arange(nth) + 0.5) / nth * (np.pi / 2)
    ph = (np.arange(nph) + 0.5) / nph * 2 * np.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    l = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1).reshape(-1, 3)
    dw = (np.pi / 2 / nth) * (2 * np.pi / nph) * np.sin(TH).ravel()
    cnt = l.shape[0]
    n = np.tile([0.0, 0.0, 1.0], (cnt, 1))
    alb = []
    for r in (0.3, 0.6, 1.0):
        for vth in (0.0, 0.8):
            v = np.tile([np.sin(vth), 0.0, np.cos(vth)], (cnt, 1))
            f, *_ = O.brdf(n, v, l, np.ones((cnt, 3)), np.full(cnt, r), np.ones(cnt))
            e = np.sum(f[:, 0] * l[:, 2] * dw)
            assert e <= 1.0 + 2e-3
            alb.append((r, vth, e))
    # smoother -> closer to 1
    assert alb[0][2] > 0.97 and alb[0][2] > alb[2][2] > alb[4][2]


# ----------------------------------------------------------------- render --
def furnace_model(L=4, log2T=10, v_logit=40.0, albedo=(0.3, 0.6, 0.9), d_raw=0.0):
    m = small_model(L=L, log2T=log2T)
    nf = 2 * L
    m["brdf"] = const_mlp(nf, 5, [logit(albedo[0]), logit(albedo[1]), logit(albedo[2]), 0.0, -40.0])
    m["irt"] = const_mlp(nf + 3, 2, [v_logit, d_raw])
    return m


def scene_points(n=64, seed=1):
    pos, nrm, wo = H.make_scene(8, n // 8, seed=seed)
    return pos, nrm, wo


@pytest.mark.parametrize("indirect", [False, True])
def test_white_furnace(indirect):
    """Constant environment L, full visibility, Lambertian albedo a:
    Eq. (1) returns a*L exactly for every pixel and every sample count."""
    m = furnace_model()
    om = O.OracleModel(m, LO, EXT)
    L_ = 1.7
    oe = O.OracleEnv(np.full((8, 16, 3), L_, np.float32))
    pos, nrm, wo = scene_points()
    # the decoder outputs sigmoid of the FP32 bias; the map holds FP32(L)
    a = 1 / (1 + np.exp(-np.array([np.float32(logit(x)) for x in (0.3, 0.6, 0.9)], np.float64)))
    Lf = float(np.float32(L_))
    for N in (4, 32):
        s = O.sampling(N, 8, 7, O.DIFFUSE_ONLY)
        rgb, vis, dep = O.render(om, oe, s, pos, nrm, wo, indirect=indirect)
        assert np.max(np.abs(rgb / (a * Lf) - 1)) < 1e-13
        assert np.all(vis > 1 - 1e-15)
        assert np.allclose(dep, math.log(2), atol=1e-15)


def test_two_bounce_closed_form():
    """Constant visibility c everywhere, constant albedo a, diffuse, constant
    environment L: L'_o = a c L, L_in = c L + (1-c) a c L and
    L_o = a c L (1 + (1-c) a) (Eq. 1 with Eq. 2)."""
    c = 0.35
    alb = (0.3, 0.6, 0.9)
    m = furnace_model(v_logit=logit(c), albedo=alb)
    om = O.OracleModel(m, LO, EXT)
    L_ = 2.0
    oe = O.OracleEnv(np.full((8, 16, 3), L_, np.float32))
    pos, nrm, wo = scene_points()
    s = O.sampling(16, 8, 7, O.DIFFUSE_ONLY)
    a = np.array(alb, np.float32).astype(np.float64)
    # the sigmoid of the FP32 bias is what the network outputs
    cc = 1 / (1 + math.exp(-float(np.float32(logit(c)))))
    aa = 1 / (1 + np.exp(-np.array([np.float32(logit(x)) for x in alb], np.float64)))
    rgb, _, _ = O.render(om, oe, s, pos, nrm, wo, indirect=True)
    ref = aa * cc * L_ * (1 + (1 - cc) * aa)
    assert np.max(np.abs(rgb / ref - 1)) < 1e-13
    rgbd, _, _ = O.render(om, oe, s, pos, nrm, wo, indirect=False)
    assert np.max(np.abs(rgbd / (aa * cc * L_) - 1)) < 1e-13
    # query mode: L_in itself
    dirs = rand_normals(64, 21)
    q, v, d = O.render(om, oe, s, pos, dirs=dirs, indirect=True)
    assert np.max(np.abs(q / (cc * L_ + (1 - cc) * aa * cc * L_) - 1)) < 1e-13
    del a


def test_bounce_point_and_depth_mapping():
    """The secondary albedo is sigmoid(f_0(x')) with f_0 affine in position on
    dense levels, so L_in pins x' = x + t w with t = near + (far-near) d,
    d = min(softplus(o_1), 1)."""
    L, log2T, res = 2, 10, [4, 8]
    m = small_model(L=L, log2T=log2T, res=res)
    tab = np.zeros((L, 1 << log2T, 2), np.float32)
    # level 0 feature 0 = g . v / N  (affine in position)
    gvec = np.array([0.5, -0.25, 0.125])
    N = res[0]
    grid = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    dense = grid[:, 0] + (N + 1) * (grid[:, 1] + (N + 1) * grid[:, 2])
    tab[0, dense, 0] = grid @ gvec
    m["table"] = tab
    nf, hid = 2 * L, 64
    W0 = np.zeros((hid, nf), np.float32); W0[0, 0] = 1.0
    b0 = np.full(hid, 10.0, np.float32)
    W1 = np.eye(hid, dtype=np.float32); b1 = np.zeros(hid, np.float32)
    W2 = np.zeros((5, hid), np.float32); W2[0:3, 0] = 1.0
    b2 = np.array([-10.0, -10.0, -10.0, 0.0, -40.0], np.float32)
    m["brdf"] = [W0, b0, W1, b1, W2, b2]
    for d_raw, c in ((-1.0, 0.4), (0.3, 0.7), (5.0, 0.2)):
        m["irt"] = const_mlp(nf + 3, 2, [logit(c), d_raw])
        om = O.OracleModel(m, LO, EXT)
        oe = O.OracleEnv(np.full((4, 8, 3), 1.0, np.float32))
        rng = np.random.default_rng(8)
        x = rng.uniform(-2, 2, (50, 3)).astype(np.float32)
        w = rand_normals(50, 9).astype(np.float32)
        s = O.sampling(1, 8, 7, O.DIFFUSE_ONLY)
        rgb, vis, dep = O.render(om, oe, s, x, dirs=w, indirect=True)
        cc = 1 / (1 + math.exp(-float(np.float32(logit(c)))))
        sp = math.log1p(math.exp(float(np.float32(d_raw))))
        d = min(sp, 1.0)
        assert np.allclose(dep, d, rtol=1e-15)
        t = 0.05 + 1.45 * d
        xb = x.astype(np.float64) + t * w.astype(np.float64)
        u = (xb - LO) / EXT
        ab = 1 / (1 + np.exp(-(u * N) @ gvec))
        ref = cc + (1 - cc) * ab * cc
        assert np.max(np.abs(rgb[:, 0] / ref - 1)) < 1e-12


def test_mc_estimate_converges_to_irradiance():
    """V = 1, Lambertian: the estimator of Eq. (1) converges to
    a/pi * integral of L(w) cos(theta) over the hemisphere, computed here by
    quadrature of the bilinearly interpolated map."""
    Hh, Ww = 8, 16
    env = H.make_env(Hh, Ww, seed=10)
    oe = O.OracleEnv(env)
    m = furnace_model(albedo=(0.5, 0.5, 0.5))
    om = O.OracleModel(m, LO, EXT)
    normals = np.array([[0, 1, 0], [0.6, 0.8, 0], [0, 0.6, -0.8], [0.48, -0.6, 0.64]], np.float32)
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    pos = np.zeros((4, 3), np.float32)
    reps = []
    for seed in range(8):
        s = O.sampling(16384, 8, 100 + seed, O.DIFFUSE_ONLY)
        reps.append(O.render(om, oe, s, pos, normals, normals, indirect=False, want_vis=False)[0])
    reps = np.array(reps)
    mean, sem = reps.mean(0), reps.std(0, ddof=1) / math.sqrt(len(reps))
    # quadrature
    nt, npp = 800, 1600
    th = (np.arange(nt) + 0.5) / nt * np.pi
    ph = (np.arange(npp) + 0.5) / npp * 2 * np.pi - np.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.cos(TH), np.sin(TH) * np.sin(PH)], -1).reshape(-1, 3)
    dw = (np.pi / nt) * (2 * np.pi / npp) * np.sin(TH).ravel()
    Ld = O.env_lookup(oe, d)
    a = 1 / (1 + math.exp(-float(np.float32(0.0))))
    for p in range(4):
        cos = np.maximum(d @ normals[p].astype(np.float64), 0)
        E = (Ld * (cos * dw)[:, None]).sum(0)
        ref = a / np.pi * E
        # within 4 standard errors of independent replicas (+ quadrature)
        assert np.all(np.abs(mean[p] - ref) <= 4 * sem[p] + 2e-4 * ref), (p, mean[p], sem[p], ref)
        assert np.all(sem[p] < 5e-3 * ref)


# ------------------------------------------------------------- gradients --
def _loss_fd_setup(seed=0, n=48, L=4, log2T=10):
    m = small_model(L=L, log2T=log2T, res=[4, 8, 16, 32], seed=seed)
    # move the tracer's depth head away from the softplus clamp
    m["irt"][5] = np.array([0.2, -0.5], np.float32)
    env = H.make_env(8, 16, seed=4)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    w = rand_normals(n, seed + 50).astype(np.float32)
    g_rgb = rng.standard_normal((n, 3)).astype(np.float32)
    g_vis = rng.standard_normal(n).astype(np.float32)
    g_dep = rng.standard_normal(n).astype(np.float32)
    return m, env, x, w, g_rgb, g_vis, g_dep


def _objective(m, env, x, w, g_rgb, g_vis, g_dep, samp):
    om = O.OracleModel(m, LO, EXT)
    oe = O.OracleEnv(env)
    rgb, vis, dep = O.render(om, oe, samp, x, dirs=w, indirect=True)
    return float(np.sum(rgb * g_rgb) + np.sum(vis * g_vis) + np.sum(dep * g_dep))


def _fd(m, key, index, env, x, w, g_rgb, g_vis, g_dep, samp, h):
    def arr(mm):
        if key == "table":
            return mm["table"]
        k, i = key
        return mm[k][i]
    vals = []
    for s in (+1, -1):
        mm = {k: (v.copy() if isinstance(v, np.ndarray) else
                  [a.copy() for a in v] if k in ("brdf", "irt") else v)
              for k, v in m.items()}
        a = arr(mm)
        a[index] = np.float32(a[index] + s * h)
        vals.append((_objective(mm, env, x, w, g_rgb, g_vis, g_dep, samp), float(a[index])))
    return (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])


def test_gradients_match_central_differences():
    """Analytic query-mode backward vs FP64 central differences on sampled
    parameters of all kinds (tables on every level, every layer of both
    MLPs).  Parameters whose +-h evaluations straddle a kink (ReLU mask, cell
    boundary, clamp) are detected by disagreement between two step sizes
    and resampled."""
    m, env, x, w, g_rgb, g_vis, g_dep = _loss_fd_setup()
    samp = O.sampling(1, 8, 7, 0)
    om = O.OracleModel(m, LO, EXT)
    oe = O.OracleEnv(env)
    G = O.backward(om, oe, samp, x, w, g_rgb, g_vis, g_dep, indirect=True)
    rng = np.random.default_rng(123)
    checked = 0
    cand = []
    nz = np.argwhere(np.abs(G["table"]) > 1e-6)
    for l in range(m["table"].shape[0]):
        rows = nz[nz[:, 0] == l]
        for r in rows[rng.permutation(len(rows))[:8]]:
            cand.append(("table", tuple(r)))
    for k in ("brdf", "irt"):
        for i in range(6):
            a = m[k][i]
            gi = G[k][i]
            flat = np.argwhere(np.abs(gi) > 1e-7)
            for r in flat[rng.permutation(len(flat))[:3]]:
                cand.append(((k, i), tuple(r)))
    for key, index in cand:
        ana = G["table"][index] if key == "table" else G[key[0]][key[1]][index]
        fd1 = _fd(m, key, index, env, x, w, g_rgb, g_vis, g_dep, samp, 1e-4)
        fd2 = _fd(m, key, index, env, x, w, g_rgb, g_vis, g_dep, samp, 2.5e-5)
        scale = max(abs(fd1), abs(fd2), 1e-3)
        if abs(fd1 - fd2) > 1e-6 * scale:
            continue  # kink between the two evaluations
        assert abs(ana - fd1) <= 2e-6 * scale, (key, index, ana, fd1, fd2)
        checked += 1
    assert checked >= 40, checked


def test_position_gradient_matches_finite_differences():
    m, env, x, w, g_rgb, g_vis, g_dep = _loss_fd_setup(seed=3, n=16)
    x = (np.round(x.astype(np.float64) * 2 ** 20) / 2 ** 20).astype(np.float32)
    samp = O.sampling(1, 8, 7, 0)
    om = O.OracleModel(m, LO, EXT)
    oe = O.OracleEnv(env)
    G = O.backward(om, oe, samp, x, w, g_rgb, g_vis, g_dep, indirect=True, want_pos=True)
    ok = 0
    for p in range(16):
        for d in range(3):
            # positions and steps on the 2^-20 lattice keep x - lo exact in FP32
            def f(h):
                xx = x.copy(); xx[p, d] = np.float32(x[p, d] + h)
                return _objective(m, env, xx, w, g_rgb, g_vis, g_dep, samp), float(xx[p, d])
            (a, xa), (b, xb) = f(128 * 2.0 ** -20), f(-128 * 2.0 ** -20)
            (c, xc), (e, xe) = f(32 * 2.0 ** -20), f(-32 * 2.0 ** -20)
            fd1, fd2 = (a - b) / (xa - xb), (c - e) / (xc - xe)
            sc = max(abs(fd1), 1e-2)
            if abs(fd1 - fd2) > 1e-5 * sc:
                continue
            assert abs(G["pos"][p, d] - fd1) < 1e-5 * sc
            ok += 1
    assert ok >= 30


# ------------------------------------------------------------- loss/Adam --
def test_l2_loss_values():
    n = 10
    tgt = H.make_targets(n)
    rgb = tgt[:, :3].copy(); vis = tgt[:, 3].copy(); dep = tgt[:, 4].copy()
    loss, gr, gv, gd = O.l2_loss(rgb, vis, dep, tgt)
    assert loss == 0 and np.all(gr == 0)
    loss, gr, gv, gd = O.l2_loss(rgb + 1, vis + 1, dep + 1, tgt)
    assert abs(loss - 5.0) < 1e-6   # five unit residuals per sample
    assert np.allclose(gr, 2.0 / n, atol=1e-6) and np.allclose(gv, 2.0 / n, atol=1e-6)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(9)
    p = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    z = np.zeros(1000)
    lr, eps = 2e-3, 1e-8
    p1, m1, v1 = O.adam(p, g, z, z, 1, lr=lr, eps=eps)
    # with zero moments, bias-corrected m = g and v = g^2 after one step
    assert np.allclose(p1 - p, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    wd = 1e-2
    p1, _, _ = O.adam(p, g, z, z, 1, lr=lr, eps=eps, wd=wd)
    ge = g + wd * p
    assert np.allclose(p1 - p, -lr * ge / (np.abs(ge) + eps), rtol=1e-12, atol=1e-15)
    # second step with constant gradient keeps the unit-size update
    p2, _, _ = O.adam(p1, g, m1, v1, 2, lr=lr, eps=eps)
    # (bias-corrected moments are again g and g^2)
    assert np.allclose(p2 - p1, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)


# ------------------------------------------------------- hard visibility --
def test_hard_visibility_gates_the_bounce():
    """Hard visibility (Sec. 3.2 "Overview"): v = [o0 > 0]; a visible ray
    takes the environment radiance, a shadow ray takes L'_o built from the
    visible secondary rays only.  The tracer here outputs o0 = w_y, so
    v = [w_y > 0] at the primary and at the bounce point."""
    L, log2T = 4, 10
    m = small_model(L=L, log2T=log2T)
    nf, hid = 2 * L, 64
    W0 = np.zeros((hid, nf + 3), np.float32); W0[0, nf + 1] = 1.0     # h1[0] = w_y + 10
    b0 = np.full(hid, 10.0, np.float32)
    W1 = np.eye(hid, dtype=np.float32); b1 = np.zeros(hid, np.float32)
    W2 = np.zeros((2, hid), np.float32); W2[0, 0] = 1.0
    b2 = np.array([-10.0, 0.3], np.float32)                          # o0 = w_y
    m["irt"] = [W0, b0, W1, b1, W2, b2]
    alb = (0.3, 0.6, 0.9)
    m["brdf"] = const_mlp(nf, 5, [logit(a) for a in alb] + [0.0, -40.0])
    om = O.OracleModel(m, LO, EXT)
    L_ = 1.5
    oe = O.OracleEnv(np.full((8, 16, 3), L_, np.float32))
    n = 200
    x = np.random.default_rng(4).uniform(-1, 1, (n, 3)).astype(np.float32)
    w = rand_normals(n, 33).astype(np.float32)
    s = O.sampling(1, 8, 7, O.DIFFUSE_ONLY | O.HARD_VIS)
    rgb, vis, dep = O.render(om, oe, s, x, dirs=w, indirect=True)
    aa = 1 / (1 + np.exp(-np.array([np.float32(logit(a)) for a in alb], np.float64)))
    Lf = float(np.float32(L_))
    wd = w.astype(np.float64)
    assert np.array_equal(vis, (wd[:, 1] > 0).astype(np.float64))
    for p in range(n):
        if wd[p, 1] > 0:
            ref = np.full(3, Lf)
        else:
            nb = np.repeat(-wd[p:p + 1], 8, 0)
            wj = O.sample_dirs(7, nb, p, 0, np.arange(8), 1, 8)
            ref = aa * Lf * np.mean(wj[:, 1] > 0)
        assert np.allclose(rgb[p], ref, rtol=1e-12, atol=1e-15), (p, rgb[p], ref)
    # direct-only: L_in = v L
    rgbd, _, _ = O.render(om, oe, s, x, dirs=w, indirect=False)
    assert np.allclose(rgbd, (wd[:, 1:2] > 0) * Lf, rtol=1e-15)
    # soft visibility on the same model differs (sigmoid of w_y, bounce always on)
    rgbs, viss, _ = O.render(om, oe, O.sampling(1, 8, 7, O.DIFFUSE_ONLY), x, dirs=w, indirect=True)
    assert np.allclose(viss, 1 / (1 + np.exp(-wd[:, 1])), rtol=1e-7)


# ---------------------------------------------------------------- denoiser --
def _atrous_reference(img, iters):
    """Plain a-trous B3-spline cascade (taps outside the image dropped and the
    remaining weights renormalised) via scipy's correlate: the SVGF filter
    with every edge-stopping weight equal to one."""
    from scipy import ndimage
    h = np.array([1 / 16, 1 / 4, 3 / 8, 1 / 4, 1 / 16])
    out = img.astype(np.float64)
    ones = np.ones(img.shape[:2])
    for it in range(iters):
        step = 1 << it
        k1 = np.zeros(4 * step + 1)
        k1[::step] = h
        K = np.outer(k1, k1)
        norm = ndimage.correlate(ones, K, mode="constant", cval=0.0)
        out = np.stack([ndimage.correlate(out[..., c], K, mode="constant", cval=0.0) / norm for c in range(3)], -1)
    return out


def test_denoise_constant_image_is_fixed():
    rng = np.random.default_rng(0)
    H, W = 37, 53
    img = np.full((H, W, 3), [0.7, 1.3, 2.0], np.float32)
    depth = rng.uniform(1, 5, (H, W)).astype(np.float32)
    nrm = rand_normals(H * W, 2).reshape(H, W, 3).astype(np.float32)
    out = O.denoise(img, depth, nrm)
    assert np.max(np.abs(out - img)) < 1e-12


def test_denoise_without_edge_stopping_is_atrous():
    rng = np.random.default_rng(1)
    H, W = 40, 47
    img = rng.uniform(0, 3, (H, W, 3)).astype(np.float32)
    depth = rng.uniform(1, 5, (H, W)).astype(np.float32)
    nrm = rand_normals(H * W, 3).reshape(H, W, 3).astype(np.float32)
    for iters in (1, 3, 5):
        out = O.denoise(img, depth, nrm, iters=iters, sigma_z=1e30, sigma_n=0.0, sigma_l=1e30)
        assert np.max(np.abs(out - _atrous_reference(img, iters))) < 1e-12


def test_denoise_stops_at_normal_edges():
    """Normals (0,0,1) on the left and (1,0,0) on the right: n_p . n_q = 0
    across the edge, so each half keeps its own constant colour exactly."""
    H, W = 32, 48
    img = np.zeros((H, W, 3), np.float32)
    img[:, : W // 2] = [1.0, 0.5, 0.25]
    img[:, W // 2:] = [4.0, 3.0, 2.0]
    nrm = np.zeros((H, W, 3), np.float32)
    nrm[:, : W // 2, 2] = 1
    nrm[:, W // 2:, 0] = 1
    depth = np.full((H, W), 2.0, np.float32)
    out = O.denoise(img, depth, nrm)
    assert np.max(np.abs(out - img)) < 1e-12


@pytest.mark.parametrize("h,w", [(9, 13), (1, 7), (7, 1)])
def test_denoise_commutes_with_transpose(h, w):
    """The B3 footprint, the 3x3 variance blur and the depth-gradient
    contraction are symmetric in x and y, so filtering the transposed image
    gives the transposed result (a swapped index or stride breaks this)."""
    rng = np.random.default_rng(h * 100 + w)
    img = np.exp(rng.standard_normal((h, w, 3))).astype(np.float32)
    depth = rng.uniform(1, 3, (h, w)).astype(np.float32)
    nrm = rand_normals(h * w, 5).reshape(h, w, 3).astype(np.float32)
    a = O.denoise(img, depth, nrm)
    b = O.denoise(img.transpose(1, 0, 2), depth.T, nrm.transpose(1, 0, 2))
    assert np.max(np.abs(a - b.transpose(1, 0, 2))) <= 1e-12 * np.max(np.abs(a))


def test_denoise_single_pixel_is_identity():
    """A 1x1 image has only its own tap (all edge-stopping weights 1)."""
    img = np.array([[[0.3, 2.0, 7.5]]], np.float32)
    out = O.denoise(img, np.array([[2.5]], np.float32), np.array([[[0.0, 0.6, 0.8]]], np.float32))
    assert np.array_equal(out, img.astype(np.float64))


# --------------------------------------------------- multiple importance sampling --
def _sphere_grid(nt, npp):
    th = (np.arange(nt) + 0.5) / nt * np.pi
    ph = (np.arange(npp) + 0.5) / npp * 2 * np.pi - np.pi
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.cos(TH), np.sin(TH) * np.sin(PH)], -1).reshape(-1, 3)
    dw = (np.pi / nt) * (2 * np.pi / npp) * np.sin(TH).ravel()
    return d, dw


def _grid_uniforms(k):
    u = (np.arange(k) + 0.5) / k
    U1, U2 = np.meshgrid(u, u, indexing="ij")
    return np.stack([U1.ravel(), U2.ravel()], 1)


def test_env_sampling_of_a_constant_map_is_the_uniform_sphere():
    """Equal texels: every texel's probability is its solid angle, so the
    CDF inversion is linear in cos(theta) and phi: w_y = 1 - 2 s1 and
    phi = -pi + 2 pi s2 exactly, with density 1/(4 pi)."""
    oe = O.OracleEnv(np.full((8, 16, 3), 2.5, np.float32))
    s = np.random.default_rng(0).uniform(0, 1, (2000, 2))
    w, pdf = O.env_sample(oe, s)
    assert np.allclose(w[:, 1], 1 - 2 * s[:, 0], rtol=0, atol=1e-12)
    assert np.allclose(np.arctan2(w[:, 2], w[:, 0]), -np.pi + 2 * np.pi * s[:, 1], rtol=0, atol=1e-11)
    assert np.allclose(np.linalg.norm(w, axis=1), 1, atol=1e-14)
    assert np.allclose(pdf, 1 / (4 * np.pi), rtol=1e-12)
    # an all-black map falls back to the same uniform distribution
    w0, pdf0 = O.env_sample(O.OracleEnv(np.zeros((8, 16, 3), np.float32)), s)
    assert np.allclose(w0, w, atol=1e-12) and np.allclose(pdf0, pdf, rtol=1e-12)


def test_env_density_is_normalised_and_matches_the_sampler():
    """Density of a random map (sun lobe included) integrates to 1 over the
    sphere (fine quadrature); a regular grid of uniforms lands in every
    texel in proportion to that texel's probability, and the density the
    sampler returns equals the density looked up at the direction."""
    Hh, Ww = 8, 16
    oe = O.OracleEnv(H.make_env(Hh, Ww, seed=12))
    d, dw = _sphere_grid(1600, 3200)
    assert abs(np.sum(O.env_density(oe, d) * dw) - 1) < 2e-3
    s = _grid_uniforms(1024)
    w, pdf = O.env_sample(oe, s)
    ct, marg, cond, dens = O.env_dist(oe)
    th = np.arccos(np.clip(w[:, 1], -1, 1))
    phi = np.arctan2(w[:, 2], w[:, 0])
    y = np.clip(np.floor(th / np.pi * Hh).astype(int), 0, Hh - 1)
    x = np.clip(np.floor((phi + np.pi) / (2 * np.pi) * Ww).astype(int), 0, Ww - 1)
    freq = np.bincount(y * Ww + x, minlength=Hh * Ww) / len(s)
    omega = (2 * np.pi / Ww) * (ct[:-1] - ct[1:])
    prob = (dens * omega[:, None]).ravel()
    assert abs(prob.sum() - 1) < 1e-12
    assert np.max(np.abs(freq - prob)) < 4 / 1024
    inside = (np.abs(th / np.pi * Hh - np.round(th / np.pi * Hh)) > 1e-6) & \
             (np.abs((phi + np.pi) / (2 * np.pi) * Ww - np.round((phi + np.pi) / (2 * np.pi) * Ww)) > 1e-6)
    assert np.allclose(pdf[inside], O.env_density(oe, w[inside]), rtol=1e-12)


def test_vndf_at_normal_incidence_with_alpha_one_is_uniform():
    """alpha = 1 and v = n: the visible normals are cosine distributed and
    their reflections cover the sphere uniformly: l_z = 1 - 2 s1, azimuth
    2 pi s2 (in the normal's frame), density 1/(4 pi) everywhere."""
    k = 500
    s = np.random.default_rng(1).uniform(0, 1, (k, 2))
    n = np.tile([0.0, 0.0, 1.0], (k, 1))
    l = O.ggx_sample(n, n, np.ones(k), s)
    assert np.allclose(l[:, 2], 1 - 2 * s[:, 0], atol=1e-12)
    az = np.mod(np.arctan2(l[:, 1], l[:, 0]), 2 * np.pi)
    assert np.allclose(np.cos(az - 2 * np.pi * s[:, 1]), 1, atol=1e-10)
    d, _ = _sphere_grid(40, 80)
    nn = np.tile([0.0, 0.0, 1.0], (len(d), 1))
    assert np.allclose(O.ggx_density(nn, nn, np.ones(len(d)), d), 1 / (4 * np.pi), rtol=1e-12)


@pytest.mark.parametrize("r,vdeg", [(0.5, 0.0), (0.7, 50.0), (0.9, 80.0), (1.0, 30.0)])
def test_vndf_density_is_normalised_and_matches_the_sampler(r, vdeg):
    """The reflected-direction density integrates to one over the sphere,
    and the expectations of test functions under the sampler (regular grid
    of uniforms) equal their integrals against the density."""
    nrm = np.array([0.0, 0.6, 0.8])
    t = np.array([1.0, 0.0, 0.0])
    a = math.radians(vdeg)
    v = math.cos(a) * nrm + math.sin(a) * t
    d, dw = _sphere_grid(1600, 3200)
    cnt = len(d)
    pdf = O.ggx_density(np.tile(nrm, (cnt, 1)), np.tile(v, (cnt, 1)), np.full(cnt, r), d)
    assert abs(np.sum(pdf * dw) - 1) < 2e-3
    s = _grid_uniforms(512)
    k = len(s)
    l = O.ggx_sample(np.tile(nrm, (k, 1)), np.tile(v, (k, 1)), np.full(k, r), s)
    assert np.allclose(np.linalg.norm(l, axis=1), 1, atol=1e-12)
    for g in (lambda q: q @ nrm, lambda q: (q @ t) ** 2, lambda q: (q @ v > 0.9).astype(float)):
        assert abs(np.mean(g(l)) - np.sum(g(d) * pdf * dw)) < 3e-3


def test_mis_estimate_converges_to_the_rendering_integral():
    """V = 1, specular metallic BRDF under the sun-lobe environment: the
    balance-heuristic estimator (light + GGX rays) converges to the
    quadrature of f_r L cos over the hemisphere (8 replicas, within 4
    standard errors).  A sampler that disagreed with its own density would
    bias it."""
    Hh, Ww = 16, 32
    env = H.make_env(Hh, Ww, seed=10)
    oe = O.OracleEnv(env)
    rr_logit, mm_logit = logit((0.45 - 0.09) / 0.91), logit(0.6)
    m = small_model()
    m["brdf"] = const_mlp(8, 5, [logit(0.3), logit(0.6), logit(0.9), rr_logit, mm_logit])
    m["irt"] = const_mlp(11, 2, [40.0, 0.0])
    om = O.OracleModel(m, LO, EXT)
    normals = np.array([[0, 1, 0], [0.6, 0.8, 0], [0.48, 0.6, 0.64]], np.float64)
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    views = np.array([[0.3, 0.9, 0.3], [0.0, 1.0, 0.0], [-0.2, 0.5, 0.84]], np.float64)
    views /= np.linalg.norm(views, axis=1, keepdims=True)
    pos = np.zeros((3, 3), np.float32)
    reps = []
    for seed in range(8):
        s = O.sampling(2 * 4096, 8, 200 + seed, O.MIS)
        reps.append(O.render(om, oe, s, pos, normals.astype(np.float32), views.astype(np.float32),
                             indirect=False, want_vis=False)[0])
    reps = np.array(reps)
    mean, sem = reps.mean(0), reps.std(0, ddof=1) / math.sqrt(len(reps))
    d, dw = _sphere_grid(1600, 3200)
    Ld = O.env_lookup(oe, d)
    sig = lambda z: 1 / (1 + math.exp(-float(np.float32(z))))
    alb = np.array([sig(logit(0.3)), sig(logit(0.6)), sig(logit(0.9))])
    rough, metal = 0.09 + 0.91 * sig(rr_logit), sig(mm_logit)
    for p in range(3):
        n32, v32 = normals[p].astype(np.float32).astype(np.float64), views[p].astype(np.float32).astype(np.float64)
        cnt = len(d)
        f = O.brdf(np.tile(n32, (cnt, 1)), np.tile(v32, (cnt, 1)), d, np.tile(alb, (cnt, 1)),
                   np.full(cnt, rough), np.full(cnt, metal))
        f = f[0] if isinstance(f, tuple) else f
        cos = np.maximum(d @ n32, 0)
        ref = (f * Ld * (cos * dw)[:, None]).sum(0)
        assert np.all(np.abs(mean[p] - ref) <= 4 * sem[p] + 2e-3 * ref), (p, mean[p], sem[p], ref)
        assert np.all(sem[p] < 2e-2 * ref)


# ------------------------------------------------------ decoder normal head --
@pytest.mark.parametrize("n_raw", [(0.0, 2.5, 0.0), (0.0, -0.7, 0.0), (3.0, 0.0, 3.0), (0.0, 0.0, 0.0)])
def test_decoder_normal_head_orients_the_bounce(n_raw):
    """8-output decoder (the paper's model shape): the secondary normal is
    o[5..7] normalised (the facing normal -w when that vector is zero).
    Hard visibility with a tracer whose visibility logit is w_y, a constant
    environment L and a diffuse decoder: a shadow ray (w_y < 0) returns
    a L times the fraction of its 8 secondary rays, sampled about n', with
    w_y > 0; with n' = +y that is all of them, with n' = -y none."""
    L = 4
    m = small_model(L=L, log2T=10)
    nf, hid = 2 * L, 64
    W0 = np.zeros((hid, nf + 3), np.float32); W0[0, nf + 1] = 1.0
    b0 = np.full(hid, 10.0, np.float32)
    W1 = np.eye(hid, dtype=np.float32); b1 = np.zeros(hid, np.float32)
    W2 = np.zeros((2, hid), np.float32); W2[0, 0] = 1.0
    m["irt"] = [W0, b0, W1, b1, W2, np.array([-10.0, 0.3], np.float32)]
    alb = (0.3, 0.6, 0.9)
    m["brdf"] = const_mlp(nf, 8, [logit(a) for a in alb] + [0.0, -40.0] + list(n_raw))
    om = O.OracleModel(m, LO, EXT)
    Lc = 1.5
    oe = O.OracleEnv(np.full((8, 16, 3), Lc, np.float32))
    n = 64
    x = np.random.default_rng(5).uniform(-1, 1, (n, 3)).astype(np.float32)
    w = rand_normals(n, 44)
    w[:, 1] = -np.abs(w[:, 1]) - 0.05
    w = (w / np.linalg.norm(w, axis=1, keepdims=True)).astype(np.float32)
    rgb, vis, _ = O.render(om, oe, O.sampling(1, 8, 7, O.DIFFUSE_ONLY | O.HARD_VIS), x, dirs=w, indirect=True)
    assert np.all(vis == 0)
    aa = 1 / (1 + np.exp(-np.array([np.float32(logit(a)) for a in alb], np.float64)))
    nr = np.array([np.float32(v) for v in n_raw], np.float64)
    for p in range(n):
        wd = w[p].astype(np.float64)
        nb = nr / np.linalg.norm(nr) if np.linalg.norm(nr) > 0 else -wd
        wj = O.sample_dirs(7, np.repeat(nb[None], 8, 0), p, 0, np.arange(8), 1, 8)
        frac = np.mean(wj[:, 1] > 0)
        if n_raw[1] > 0 and n_raw[0] == 0:
            assert frac == 1.0
        if n_raw[1] < 0:
            assert frac == 0.0
        assert np.allclose(rgb[p], aa * float(np.float32(Lc)) * frac, rtol=1e-12, atol=1e-15), (p, rgb[p])


def test_paper_level_layout():
    """The paper's encoder (Sec. 4.1): 14 levels from 16 to 131072 give the
    growth factor 2 exactly, so N_l = 16 * 2^l; with T = 2^17 exactly the
    first two levels are dense.  At the finest level a vertex position is
    reproduced exactly (weights 0/1), and the hash of a vertex on an axis is
    the coordinate times its prime, masked to T."""
    res = H.level_resolutions(14, 16, 131072)
    assert res == [16 << l for l in range(14)]
    T = 1 << 17
    assert [(N + 1) ** 3 <= T for N in res] == [True, True] + [False] * 12
    m = small_model(L=14, log2T=17, res=res)
    om = O.OracleModel(m, LO, EXT)
    N = res[-1]
    k = np.random.default_rng(6).integers(0, N + 1, (300, 3))
    pos = (LO + EXT * k / N).astype(np.float32)
    assert np.array_equal(pos.astype(np.float64), LO + EXT * k / N)   # exact in FP32
    idx, w = O.encode_index(om, pos)
    assert np.all(np.isin(w[:, 13], [0.0, 1.0]))
    f = O.encode(om, pos)
    corner = (w[:, 13, 0] == 1) * 1 + (w[:, 13, 1] == 1) * 2 + (w[:, 13, 2] == 1) * 4
    assert np.array_equal(f[:, 26:28], m["table"][13][idx[np.arange(300), 13, corner]].astype(np.float64))
    one = np.array([[LO + EXT * 7 / N, LO, LO], [LO, LO + EXT * 5 / N, LO]], np.float32)
    i1, w1 = O.encode_index(om, one)
    assert int(i1[0, 13, 0]) == 7 % T and int(i1[1, 13, 0]) == (5 * 2654435761 % 2 ** 32) % T
