"""Host-only checks of the C ABI: the library loads, exports every symbol
declared in include/hg.h, and rejects malformed arguments on the host before
any device work (these calls never reach the GPU)."""
import ctypes as C
import os
import re

import pytest

import paper_2409_10327_amd as hg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "hg.h")).read()
    return sorted(set(re.findall(r"^(?:hg_status|const char \*|size_t)\s*(hg_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    syms = header_symbols()
    assert len(syms) == 17, syms
    L = hg.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(hg.EXPORTS)


FAKE = 0x7f0000000000  # 16-byte aligned non-null placeholder (never dereferenced)


def fake_model(**over):
    m = hg.Model()
    g = m.grid
    g.L, g.F, g.log2_T = 16, 2, 14
    for i, r in enumerate([16, 20, 25, 32, 40, 50, 64, 80, 101, 128, 161, 203, 256, 322, 406, 512]):
        g.res[i] = r
    g.box_lo, g.box_extent, g.dtype, g.table = -8.0, 16.0, hg.HG_F32, FAKE
    for mm, nin, nout in ((m.brdf, 32, 5), (m.irt, 35, 2)):
        mm.n_in, mm.n_hidden, mm.n_out, mm.dtype = nin, 64, nout, hg.HG_F32
        for k in range(3):
            mm.W[k] = FAKE
            mm.b[k] = FAKE
    m.t_near, m.t_far, m.f0 = 0.05, 1.5, 0.04
    for k, v in over.items():
        obj, attr = k.split(".") if "." in k else (None, k)
        setattr(getattr(m, obj) if obj else m, attr, v)
    return m


def call_render(m=None, env=None, samp=None, pts=None, rgb=FAKE):
    m = m or fake_model()
    if env is None:
        env = hg.Env(); env.H, env.W, env.rgb = 16, 32, FAKE
    samp = samp or hg.sampling_struct(32, 8, 7, 0)
    if pts is None:
        pts = hg.Points(); pts.n, pts.pos, pts.nrm, pts.wo, pts.dir = 10, FAKE, FAKE, FAKE, None
    return hg.lib().hg_render_indirect(C.byref(m), C.byref(env), C.byref(samp), C.byref(pts), C.c_void_p(rgb),
                                       None, None, None)


@pytest.mark.parametrize("field,value,status", [
    ("grid.F", 3, hg.HG_E_UNSUPPORTED),
    ("grid.L", 17, hg.HG_E_UNSUPPORTED),
    ("grid.L", 0, hg.HG_E_UNSUPPORTED),
    ("grid.log2_T", 9, hg.HG_E_INVALID),
    ("grid.log2_T", 25, hg.HG_E_INVALID),
    ("grid.box_extent", 12.0, hg.HG_E_INVALID),
    ("grid.table", 0, hg.HG_E_INVALID),
    ("grid.table", FAKE + 4, hg.HG_E_INVALID),
    ("grid.dtype", 7, hg.HG_E_INVALID),
    ("t_far", 0.01, hg.HG_E_INVALID),
])
def test_model_validation(field, value, status):
    assert call_render(fake_model(**{field: value})) == status
    assert hg.lib().hg_last_error().decode() != ""


def test_brdf_outputs_and_normal_head():
    m = fake_model()
    m.brdf.n_out = 6
    assert call_render(m) == hg.HG_E_UNSUPPORTED
    m = fake_model()
    m.brdf.n_out = 8
    env = hg.Env(); env.H, env.W, env.rgb = 16, 32, FAKE
    s = hg.sampling_struct(1, 8, 7, 0)
    q = hg.Points(); q.n, q.pos, q.nrm, q.wo, q.dir = 10, FAKE, None, None, FAKE
    gb = (C.c_void_p * 6)(*[FAKE] * 6)
    f = C.c_void_p(FAKE)
    # the normal head is forward only
    assert hg.lib().hg_backward(C.byref(m), C.byref(env), C.byref(s), C.byref(q), 1, f, f, f, f, gb, gb, None,
                                None, 0, None) == hg.HG_E_UNSUPPORTED


def test_mlp_shape_and_dtype_pairs():
    m = fake_model()
    m.brdf.n_hidden = 32
    assert call_render(m) == hg.HG_E_UNSUPPORTED
    m = fake_model()
    m.irt.n_in = 34
    assert call_render(m) == hg.HG_E_UNSUPPORTED
    m = fake_model()
    m.brdf.dtype = hg.HG_BF16
    assert call_render(m) == hg.HG_E_INVALID  # brdf and irt dtypes differ
    m = fake_model()
    m.grid.dtype = hg.HG_F16   # F16 table + F32 MLPs: backward only
    assert call_render(m) == hg.HG_E_UNSUPPORTED


def test_res_must_increase():
    m = fake_model()
    m.grid.res[5] = m.grid.res[4]
    assert call_render(m) == hg.HG_E_INVALID


@pytest.mark.parametrize("n_dirs,n_dirs2", [(0, 8), (3, 8), (2048, 8), (32, 0), (32, 6), (32, 128)])
def test_sampling_validation(n_dirs, n_dirs2):
    assert call_render(samp=hg.sampling_struct(n_dirs, n_dirs2, 7, 0)) == hg.HG_E_INVALID


def test_unknown_flags_rejected():
    assert call_render(samp=hg.sampling_struct(32, 8, 7, 8)) == hg.HG_E_INVALID


def test_mis_validation():
    L = hg.lib()
    env = hg.Env(); env.H, env.W, env.rgb, env.dist = 16, 32, FAKE, None
    mis = hg.sampling_struct(32, 8, 7, hg.HG_MIS)
    assert call_render(env=env, samp=mis) == hg.HG_E_INVALID               # no distribution
    env.dist = FAKE + 4
    assert call_render(env=env, samp=mis) == hg.HG_E_INVALID               # misaligned distribution
    env.dist = FAKE
    assert call_render(env=env, samp=hg.sampling_struct(1, 8, 7, hg.HG_MIS)) == hg.HG_E_INVALID  # n_dirs = 1
    q = hg.Points(); q.n, q.pos, q.nrm, q.wo, q.dir = 10, FAKE, None, None, FAKE
    assert call_render(env=env, samp=mis, pts=q) == hg.HG_E_UNSUPPORTED  # query mode
    # distribution size: H float4 rows, (H+1) + H (W+1) float2 CDF pairs, H W floats
    assert L.hg_env_sampling_size(16, 32) == 16 * 16 + (17 + 16 * 33) * 8 + 16 * 32 * 4
    assert L.hg_env_sampling_size(0, 32) == 0 and L.hg_env_sampling_size(16, 9000) == 0
    need = L.hg_env_sampling_size(16, 32)
    host = (C.c_float * (16 * 32 * 3))()
    assert L.hg_env_build_sampling(host, 16, 32, None, need, None) == hg.HG_E_INVALID
    assert L.hg_env_build_sampling(None, 16, 32, C.c_void_p(FAKE), need, None) == hg.HG_E_INVALID
    assert L.hg_env_build_sampling(host, 16, 32, C.c_void_p(FAKE), need - 1, None) == hg.HG_E_INVALID
    assert L.hg_env_build_sampling(host, 16, 32, C.c_void_p(FAKE + 8), need, None) == hg.HG_E_INVALID
    assert L.hg_env_build_sampling(host, 9000, 16, C.c_void_p(FAKE), 1 << 30, None) == hg.HG_E_INVALID
    assert L.hg_env_build_sampling(host, 16, 0, C.c_void_p(FAKE), 1 << 30, None) == hg.HG_E_INVALID


def test_points_validation():
    p = hg.Points(); p.n, p.pos, p.nrm, p.wo, p.dir = 10, FAKE, None, FAKE, None
    assert call_render(pts=p) == hg.HG_E_INVALID            # shade mode needs normals
    p = hg.Points(); p.n, p.pos, p.nrm, p.wo, p.dir = -1, FAKE, FAKE, FAKE, None
    assert call_render(pts=p) == hg.HG_E_INVALID
    p = hg.Points(); p.n, p.pos, p.nrm, p.wo, p.dir = 0, None, None, None, None
    assert call_render(pts=p, rgb=0) == hg.HG_OK            # n == 0 is a no-op
    assert call_render(rgb=0) == hg.HG_E_INVALID


def test_denoise_noalloc_validation():
    L = hg.lib()
    f = FAKE
    prm = hg.DenoiseParams(5, 1.0, 128.0, 4.0)
    assert hg.DENOISE_NOALLOC_MAX_PIXELS == 1 << 20
    # beyond the static workspace, or malformed: rejected before any device call
    assert L.hg_denoise_noalloc(f, f, f, 1024, 1025, C.byref(prm), f, None) == hg.HG_E_INVALID
    assert "static workspace" in L.hg_last_error().decode()
    assert L.hg_denoise_noalloc(f, f, f, 0, 8, C.byref(prm), f, None) == hg.HG_E_INVALID
    assert L.hg_denoise_noalloc(None, f, f, 8, 8, C.byref(prm), f, None) == hg.HG_E_INVALID
    assert L.hg_denoise_noalloc(f, f, f, 8, 8, C.byref(prm), f + 4, None) == hg.HG_E_INVALID
    bad = hg.DenoiseParams(11, 1.0, 128.0, 4.0)
    assert L.hg_denoise_noalloc(f, f, f, 8, 8, C.byref(bad), f, None) == hg.HG_E_INVALID


def test_denoise_validation():
    L = hg.lib()
    prm = hg.DenoiseParams(5, 1.0, 128.0, 4.0)
    assert L.hg_denoise_workspace_size(800, 800) == 800 * 800 * 12 * 4
    f = C.c_void_p(FAKE)
    need = L.hg_denoise_workspace_size(8, 8)
    assert L.hg_denoise(f, f, f, 8, 8, C.byref(prm), f, f, need - 4, None) == hg.HG_E_INVALID
    assert L.hg_denoise(f, f, f, 0, 8, C.byref(prm), f, f, need, None) == hg.HG_E_INVALID
    bad = hg.DenoiseParams(11, 1.0, 128.0, 4.0)
    assert L.hg_denoise(f, f, f, 8, 8, C.byref(bad), f, f, need, None) == hg.HG_E_INVALID
    bad = hg.DenoiseParams(5, -1.0, 128.0, 4.0)
    assert L.hg_denoise(f, f, f, 8, 8, C.byref(bad), f, f, need, None) == hg.HG_E_INVALID


def test_other_entry_points_validate():
    L = hg.lib()
    g = fake_model().grid
    assert L.hg_encode(C.byref(g), C.c_void_p(FAKE), 10, None, None) == hg.HG_E_INVALID
    assert L.hg_encode(C.byref(g), None, 0, None, None) == hg.HG_OK
    assert L.hg_encode_index(C.byref(g), C.c_void_p(FAKE), 10, None, None, None) == hg.HG_E_INVALID
    assert L.hg_l2_loss(None, None, None, None, 5, C.c_void_p(FAKE), None, None, None, None) == hg.HG_E_INVALID
    T = hg.AdamTensor * 2
    good = hg.AdamTensor(FAKE, FAKE, FAKE, FAKE, 10, 0.0, 0, None)
    assert L.hg_adam_step_multi(None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_OK
    assert L.hg_adam_step_multi(None, 2, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    assert L.hg_adam_step_multi(T(good, good), -1, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    assert L.hg_adam_step_multi(T(good, good), 17, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    assert L.hg_adam_step_multi(T(good, good), 2, 0, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    assert L.hg_adam_step_multi(T(good, good), 2, 1, 1e-3, 0.9, 0.999, 1e-8, 2, None) == hg.HG_E_INVALID
    assert L.hg_adam_step_multi(T(good, good), 2, 1, 1e-3, 1.0, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    nul = hg.AdamTensor(None, FAKE, FAKE, FAKE, 10, 0.0, 0, None)
    assert L.hg_adam_step_multi(T(good, nul), 2, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    badsh = hg.AdamTensor(FAKE, FAKE, FAKE, FAKE, 10, 0.0, hg.HG_F32, FAKE)
    assert L.hg_adam_step_multi(T(good, badsh), 2, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    neg = hg.AdamTensor(FAKE, FAKE, FAKE, FAKE, -1, 0.0, 0, None)
    assert L.hg_adam_step_multi(T(good, neg), 2, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    nanwd = hg.AdamTensor(FAKE, FAKE, FAKE, FAKE, 10, float("nan"), 0, None)
    assert L.hg_adam_step_multi(T(good, nanwd), 2, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == hg.HG_E_INVALID
    need = L.hg_morton_order_workspace_size(10)
    assert need > 0 and L.hg_morton_order_workspace_size(0) == 0 and L.hg_morton_order_workspace_size(-1) == 0
    assert L.hg_morton_order_workspace_size(1 << 31) == 0
    f = C.c_void_p(FAKE)
    assert L.hg_morton_order(None, 0, -8.0, 16.0, None, None, 0, None) == hg.HG_OK
    assert L.hg_morton_order(f, -1, -8.0, 16.0, f, f, need, None) == hg.HG_E_INVALID
    assert L.hg_morton_order(f, 10, -8.0, 12.0, f, f, need, None) == hg.HG_E_INVALID  # extent not 2^k
    assert L.hg_morton_order(f, 10, float("nan"), 16.0, f, f, need, None) == hg.HG_E_INVALID
    assert L.hg_morton_order(None, 10, -8.0, 16.0, f, f, need, None) == hg.HG_E_INVALID
    assert L.hg_morton_order(f, 10, -8.0, 16.0, None, f, need, None) == hg.HG_E_INVALID
    assert L.hg_morton_order(f, 10, -8.0, 16.0, f, C.c_void_p(FAKE + 16), need, None) == hg.HG_E_INVALID
    assert L.hg_morton_order(f, 10, -8.0, 16.0, f, f, need - 1, None) == hg.HG_E_INVALID
    assert L.hg_adam_step(C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), 10, 0,
                          1e-3, 0.9, 0.999, 1e-8, 0.0, None, 0, None) == hg.HG_E_INVALID
    assert L.hg_adam_step(C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), 10, 1,
                          1e-3, 1.0, 0.999, 1e-8, 0.0, None, 0, None) == hg.HG_E_INVALID
    m = fake_model()
    env = hg.Env(); env.H, env.W, env.rgb = 16, 32, FAKE
    s = hg.sampling_struct(1, 8, 7, 0)
    p = hg.Points(); p.n, p.pos, p.nrm, p.wo, p.dir = 10, FAKE, FAKE, FAKE, None
    gb = (C.c_void_p * 6)(*[FAKE] * 6)
    # backward needs query-mode points
    assert L.hg_backward(C.byref(m), C.byref(env), C.byref(s), C.byref(p), 1, C.c_void_p(FAKE), C.c_void_p(FAKE),
                         C.c_void_p(FAKE), C.c_void_p(FAKE), gb, gb, None, None, 0, None) == hg.HG_E_INVALID
    p.dir = FAKE
    sh = hg.sampling_struct(1, 8, 7, hg.HG_HARD_VIS)   # hard visibility is forward-only
    assert L.hg_backward(C.byref(m), C.byref(env), C.byref(sh), C.byref(p), 1, C.c_void_p(FAKE), C.c_void_p(FAKE),
                         C.c_void_p(FAKE), C.c_void_p(FAKE), gb, gb, None, None, 0, None) == hg.HG_E_UNSUPPORTED
    # BF16 MLPs with FP16 tables (the mixed backward) pass the dtype checks:
    # without a workspace the call then stops at the workspace check
    m.brdf.dtype = m.irt.dtype = hg.HG_BF16
    m.grid.dtype = hg.HG_F16
    assert L.hg_backward(C.byref(m), C.byref(env), C.byref(s), C.byref(p), 1, C.c_void_p(FAKE), C.c_void_p(FAKE),
                         C.c_void_p(FAKE), C.c_void_p(FAKE), gb, gb, None, None, 0, None) == hg.HG_E_INVALID
    assert "ws" in L.hg_last_error().decode()
    # BF16 MLPs with an FP32 table are no supported pair
    m.grid.dtype = hg.HG_F32
    assert L.hg_backward(C.byref(m), C.byref(env), C.byref(s), C.byref(p), 1, C.c_void_p(FAKE), C.c_void_p(FAKE),
                         C.c_void_p(FAKE), C.c_void_p(FAKE), gb, gb, None, None, 0, None) != hg.HG_OK


def test_backward_workspace():
    """The backward needs a workspace of at least the queried size, 256-byte
    aligned (two records per query with the bounce, one without)."""
    L = hg.lib()
    assert L.hg_backward_workspace_size(1, 0) == 0 and L.hg_backward_workspace_size(1, -3) == 0
    assert L.hg_backward_workspace_size(1, 1 << 30) == 0 and L.hg_backward_workspace_size(2, 1000) == 0
    n = 1000
    need = L.hg_backward_workspace_size(1, n)
    assert need >= 2 * n * (16 + 128 + 16) and L.hg_backward_workspace_size(0, n) >= n * (16 + 128 + 16)
    m = fake_model()
    env = hg.Env(); env.H, env.W, env.rgb = 16, 32, FAKE
    s = hg.sampling_struct(1, 8, 7, 0)
    p = hg.Points(); p.n, p.pos, p.nrm, p.wo, p.dir = n, FAKE, None, None, FAKE
    gb = (C.c_void_p * 6)(*[FAKE] * 6)
    f = C.c_void_p(FAKE)
    call = lambda ws, nb: L.hg_backward(C.byref(m), C.byref(env), C.byref(s), C.byref(p), 1, f, f, f, f, gb, gb,
                                        None, ws, nb, None)
    assert call(None, need) == hg.HG_E_INVALID                 # missing
    assert call(C.c_void_p(FAKE + 16), need) == hg.HG_E_INVALID  # not 256-byte aligned
    assert call(f, need - 1) == hg.HG_E_INVALID                 # too small
    assert "ws" in L.hg_last_error().decode()


def test_membench_exports_and_validation():
    """libhg_membench.so exports every call of include/hg_membench.h and
    rejects malformed arguments before any launch."""
    from paper_2409_10327_amd import membench as MB
    src = open(os.path.join(ROOT, "include", "hg_membench.h")).read()
    syms = sorted(set(re.findall(r"^int\s+(hgmb_\w+)\s*\(", src, re.M)))
    assert syms == sorted(MB.EXPORTS), syms
    L = MB.lib()
    for s_ in syms:
        assert hasattr(L, s_)
    f = C.c_void_p(FAKE)
    assert L.hgmb_gather(f, 20, 12, 1, 1, 0, f, None) == 1           # item size
    assert L.hgmb_gather(C.c_void_p(FAKE + 4), 20, 8, 1, 1, 0, f, None) == 1  # alignment
    assert L.hgmb_gather(f, 29, 8, 1, 1, 0, f, None) == 1            # table beyond 2^31 bytes
    assert L.hgmb_gather(f, 20, 8, 0, 1, 0, f, None) == 1            # no blocks
    assert L.hgmb_gather_indexed(f, 8, C.c_void_p(FAKE + 4), 16, 1, f, None) == 1  # index alignment
    assert L.hgmb_gather_indexed(f, 8, f, 16, 0, f, None) == 1       # no blocks
    assert L.hgmb_gather_indexed(f, 8, None, 0, 1, f, None) == 0     # empty stream: nothing launched
    assert L.hgmb_atomic(f, 20, 1, 1, 3, 0, None) == 1               # lanes per address not a power of two
    assert L.hgmb_atomic(f, 20, 1, 1, 128, 0, None) == 1
    assert L.hgmb_atomic_lines(f, 20, 1, 1, 32, 0, None) == 1        # a group beyond one line
    assert L.hgmb_atomic_lines(f, 20, 1, 1, 6, 0, None) == 1         # not a power of two
    assert L.hgmb_atomic_lines(C.c_void_p(FAKE + 4), 20, 1, 1, 2, 0, None) == 1  # alignment
    assert L.hgmb_mfma(2, 1, 1, 1, f, None) == 1                     # kind
    assert L.hgmb_mfma(0, 1, 1, 3, f, None) == 1                     # chains
