// hg_api.hip -- the C ABI (include/hg.h): host-side validation and dispatch.
//
// Every entry point validates its arguments on the host before enqueuing
// anything; a failure returns an error code and leaves a message for
// hg_last_error().  No entry point allocates device memory.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hg.h"
#include "hg_launch.h"
#include "hg_order.h"
#include "hg_train.h"

namespace {

thread_local std::string g_err;

hg_status fail(hg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hg_status hip_status(hipError_t e, const char *where) {
    if (e == hipSuccess) return HG_OK;
    return fail(HG_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= v) ++l;
    return l;
}

#define REQUIRE(cond, ...)                                   \
    do {                                                     \
        if (!(cond)) return fail(HG_E_INVALID, __VA_ARGS__); \
    } while (0)
#define SUPPORT(cond, ...)                                       \
    do {                                                         \
        if (!(cond)) return fail(HG_E_UNSUPPORTED, __VA_ARGS__); \
    } while (0)
#define CHECK(expr)                                \
    do {                                           \
        hg_status st_ = (expr);                    \
        if (st_ != HG_OK) return st_;              \
    } while (0)

// the backward's radix sort counts records (two per query) in int
constexpr int64_t kMaxBackwardN = (int64_t(1) << 30) - 1;

hg_status check_ptr(const void *p, const char *name, size_t align = 16) {
    REQUIRE(p != nullptr, "%s is NULL", name);
    REQUIRE(aligned(p, align), "%s is not %zu-byte aligned", name, align);
    return HG_OK;
}

hg_status check_grid(const hg_grid *g, hg::GridK &k) {
    REQUIRE(g != nullptr, "grid is NULL");
    SUPPORT(g->F == hg::kF, "F = %d (only F = 2 is built)", g->F);
    SUPPORT(g->L >= 1 && g->L <= hg::kL, "L = %d outside [1, 16]", g->L);
    REQUIRE(g->log2_T >= 10 && g->log2_T <= 24, "log2_T = %d outside [10, 24]", g->log2_T);
    REQUIRE(std::isfinite(g->box_lo), "box_lo is not finite");
    int ex = 0;
    const float mant = std::frexp(g->box_extent, &ex);
    REQUIRE(g->box_extent > 0.0f && mant == 0.5f, "box_extent %g is not a power of two", (double)g->box_extent);
    REQUIRE(g->dtype == HG_F32 || g->dtype == HG_F16, "table dtype must be HG_F32 or HG_F16");
    CHECK(check_ptr(g->table, "grid.table"));
    const uint64_t T = uint64_t(1) << g->log2_T;
    k.table = g->table;
    k.L = (uint32_t)g->L;
    k.log2T = (uint32_t)g->log2_T;
    k.Tmask = (uint32_t)(T - 1);
    k.lo = g->box_lo;
    k.inv_ext = 1.0f / g->box_extent;
    k.dense_mask = 0;
    for (int l = 0; l < g->L; ++l) {
        const int32_t N = g->res[l];
        REQUIRE(N >= 2 && N <= (1 << 20), "res[%d] = %d outside [2, 2^20]", l, N);
        REQUIRE(l == 0 || N > g->res[l - 1], "res is not strictly increasing at level %d", l);
        k.resf[l] = (float)N;
        k.nm1f[l] = (float)(N - 1);
        k.dscale[l] = (float)N / g->box_extent;
        k.stride[l] = (uint32_t)(N + 1);
        const uint64_t s = (uint64_t)N + 1;
        if (s * s * s <= T) k.dense_mask |= 1u << l;
    }
    for (int l = g->L; l < hg::kL; ++l) {  // unused slots
        k.resf[l] = 2.0f;
        k.nm1f[l] = 1.0f;
        k.dscale[l] = 0.0f;
        k.stride[l] = 3;
    }
    return HG_OK;
}

hg_status check_mlp(const hg_mlp *m, const char *name, int n_in, int n_out, hg::MlpK &k) {
    SUPPORT(m->n_in == n_in && m->n_hidden == hg::kH && m->n_out == n_out,
            "%s shape %d->%d->%d->%d (expected %d->64->64->%d)", name, m->n_in, m->n_hidden, m->n_hidden,
            m->n_out, n_in, n_out);
    REQUIRE(m->dtype == HG_F32 || m->dtype == HG_BF16, "%s dtype must be HG_F32 or HG_BF16", name);
    for (int i = 0; i < 3; ++i) {
        char nm[64];
        snprintf(nm, sizeof nm, "%s.W[%d]", name, i);
        CHECK(check_ptr(m->W[i], nm));
        snprintf(nm, sizeof nm, "%s.b[%d]", name, i);
        CHECK(check_ptr(m->b[i], nm));
    }
    k.W0 = m->W[0]; k.b0 = m->b[0];
    k.W1 = m->W[1]; k.b1 = m->b[1];
    k.W2 = m->W[2]; k.b2 = m->b[2];
    return HG_OK;
}

enum class Prec { F32, Mixed, F16TableF32Mlp };

hg_status check_model(const hg_model *m, hg::RenderK &k, Prec &prec) {
    REQUIRE(m != nullptr, "model is NULL");
    CHECK(check_grid(&m->grid, k.g));
    SUPPORT(m->brdf.n_out == 5 || m->brdf.n_out == 8, "brdf n_out = %d (5, or 8 with the normal head)",
            m->brdf.n_out);
    CHECK(check_mlp(&m->brdf, "brdf", hg::kNF, m->brdf.n_out, k.brdf));
    k.brdf_out = m->brdf.n_out;
    CHECK(check_mlp(&m->irt, "irt", hg::kNI, 2, k.irt));
    REQUIRE(m->brdf.dtype == m->irt.dtype, "brdf and irt must share a dtype");
    if (m->grid.dtype == HG_F32 && m->brdf.dtype == HG_F32) prec = Prec::F32;
    else if (m->grid.dtype == HG_F16 && m->brdf.dtype == HG_BF16) prec = Prec::Mixed;
    else if (m->grid.dtype == HG_F16 && m->brdf.dtype == HG_F32) prec = Prec::F16TableF32Mlp;
    else return fail(HG_E_UNSUPPORTED, "unsupported precision pair (table %d, mlp %d)", m->grid.dtype, m->brdf.dtype);
    REQUIRE(std::isfinite(m->t_near) && std::isfinite(m->t_far) && m->t_far > m->t_near,
            "t_near/t_far must be finite with t_far > t_near");
    REQUIRE(std::isfinite(m->f0) && m->f0 >= 0.0f && m->f0 <= 1.0f, "f0 must lie in [0, 1]");
    k.t_near = m->t_near;
    k.t_span = m->t_far - m->t_near;
    k.f0 = m->f0;
    return HG_OK;
}

hg_status check_env(const hg_env *e, hg::EnvK &k) {
    REQUIRE(e != nullptr, "env is NULL");
    REQUIRE(e->H >= 1 && e->W >= 1 && (int64_t)e->H * e->W <= (int64_t(1) << 26), "env size %dx%d invalid", e->H,
            e->W);
    CHECK(check_ptr(e->rgb, "env.rgb"));
    k.rgb = e->rgb;
    k.H = e->H;
    k.W = e->W;
    k.Hf = (float)e->H;
    k.Wf = (float)e->W;
    k.rows = nullptr;
    k.marg = k.cond = nullptr;
    k.dens = nullptr;
    if (e->dist) {
        REQUIRE(aligned(e->dist, 16), "env.dist is not 16-byte aligned");
        k.rows = static_cast<const float4 *>(e->dist);
        k.marg = reinterpret_cast<const float2 *>(k.rows + e->H);
        k.cond = k.marg + (e->H + 1);
        k.dens = reinterpret_cast<const float *>(k.cond + (size_t)e->H * (e->W + 1));
    }
    return HG_OK;
}

size_t env_sampling_bytes(int32_t H, int32_t W) { return hg::env_dist_bytes(H, W); }

hg_status check_sampling(const hg_sampling *s, bool need_primary, hg::SampK &k) {
    REQUIRE(s != nullptr, "sampling is NULL");
    if (need_primary)
        REQUIRE(pow2(s->n_dirs) && s->n_dirs <= 1024, "n_dirs = %d is not a power of two in [1, 1024]", s->n_dirs);
    REQUIRE(pow2(s->n_dirs2) && s->n_dirs2 <= 64, "n_dirs2 = %d is not a power of two in [1, 64]", s->n_dirs2);
    REQUIRE((s->flags & ~(HG_DIFFUSE_ONLY | HG_HARD_VIS | HG_MIS)) == 0, "unknown sampling flags 0x%x", s->flags);
    const bool mis = (s->flags & HG_MIS) != 0;
    if (mis) {
        SUPPORT(need_primary, "HG_MIS applies to shade mode only");
        REQUIRE(s->n_dirs >= 2, "HG_MIS needs n_dirs = 2M >= 2");
    }
    const int N = need_primary ? s->n_dirs : 1;
    const int na = 1 << (ilog2(N) / 2), nb = N / na;
    const int N2 = s->n_dirs2;
    const int na2 = 1 << (ilog2(N2) / 2), nb2 = N2 / na2;
    k.n_dirs = (uint32_t)N;
    k.n_dirs2 = (uint32_t)N2;
    k.key0 = (uint32_t)(s->seed & 0xffffffffu);
    k.key1 = (uint32_t)(s->seed >> 32);
    k.flags = s->flags;
    k.nb_shift = (uint32_t)ilog2(nb);
    k.nb2_shift = (uint32_t)ilog2(nb2);
    k.inv_na = 1.0f / (float)na;
    k.inv_nb = 1.0f / (float)nb;
    k.inv_na2 = 1.0f / (float)na2;
    k.inv_nb2 = 1.0f / (float)nb2;
    k.g_shift = (uint32_t)ilog2(N < 64 ? N : 64);
    // strata of the M samples of each MIS strategy
    const int M = mis ? N / 2 : 1;
    const int nam = 1 << (ilog2(M) / 2), nbm = M / nam;
    k.m_half = (uint32_t)M;
    k.nbm_shift = (uint32_t)ilog2(nbm);
    k.inv_nam = 1.0f / (float)nam;
    k.inv_nbm = 1.0f / (float)nbm;
    return HG_OK;
}

hg_status check_points(const hg_points *p, bool &query) {
    REQUIRE(p != nullptr, "points is NULL");
    REQUIRE(p->n >= 0 && p->n < (int64_t(1) << 31), "n = %lld outside [0, 2^31)", (long long)p->n);
    query = p->dir != nullptr;
    if (p->n == 0) return HG_OK;
    CHECK(check_ptr(p->pos, "points.pos"));
    if (query) {
        CHECK(check_ptr(p->dir, "points.dir"));
    } else {
        CHECK(check_ptr(p->nrm, "points.nrm"));
        CHECK(check_ptr(p->wo, "points.wo"));
    }
    return HG_OK;
}

hg_status render(const hg_model *model, const hg_env *env, const hg_sampling *samp, const hg_points *pts,
                 float *rgb, float *vis, float *depth, hipStream_t stream, bool indirect) {
    g_err.clear();
    hg::RenderK k{};
    Prec prec;
    bool query = false;
    CHECK(check_model(model, k, prec));
    CHECK(check_env(env, k.env));
    CHECK(check_points(pts, query));
    CHECK(check_sampling(samp, !query, k.s));
    SUPPORT(prec != Prec::F16TableF32Mlp, "rendering needs (F32 table, F32 MLP) or (F16 table, BF16 MLP)");
    REQUIRE((samp->flags & HG_MIS) == 0 || env->dist != nullptr,
            "HG_MIS needs env.dist (hg_env_build_sampling)");
    if (pts->n == 0) return HG_OK;
    CHECK(check_ptr(rgb, "rgb"));
    if (query) {
        REQUIRE((vis == nullptr) == (depth == nullptr), "vis and depth must both be set or both be NULL");
    } else {
        REQUIRE((vis == nullptr) == (depth == nullptr), "vis and depth must both be set or both be NULL");
    }
    if (vis) {
        CHECK(check_ptr(vis, "vis"));
        CHECK(check_ptr(depth, "depth"));
    }
    k.pos = pts->pos;
    k.nrm = pts->nrm;
    k.wo = pts->wo;
    k.dir = pts->dir;
    k.rgb = rgb;
    k.vis = vis;
    k.depth = depth;
    k.n = pts->n;
    // the matrix-core kernel in every mode (shade mode with fewer than 16
    // directions per point: per-lane features, up to 64 points per wave)
    const hipError_t e = prec == Prec::Mixed ? hg::launch_render_mixed(k, indirect, query, stream)
                                             : hg::launch_render_f32_mma(k, indirect, query, stream);
    return hip_status(e, indirect ? "hg_render_indirect" : "hg_render_direct");
}

}  // namespace

extern "C" {

const char *hg_last_error(void) { return g_err.c_str(); }

hg_status hg_encode(const hg_grid *grid, const float *pos, int64_t n, float *feat, hipStream_t stream) {
    g_err.clear();
    hg::GridK k{};
    CHECK(check_grid(grid, k));
    REQUIRE(n >= 0, "n = %lld is negative", (long long)n);
    if (n == 0) return HG_OK;
    CHECK(check_ptr(pos, "pos"));
    CHECK(check_ptr(feat, "feat"));
    return hip_status(hg::launch_encode(k, grid->dtype == HG_F16, pos, n, feat, stream), "hg_encode");
}

hg_status hg_encode_index(const hg_grid *grid, const float *pos, int64_t n, uint32_t *idx, float *w,
                          hipStream_t stream) {
    g_err.clear();
    hg::GridK k{};
    CHECK(check_grid(grid, k));
    REQUIRE(n >= 0, "n = %lld is negative", (long long)n);
    if (n == 0) return HG_OK;
    CHECK(check_ptr(pos, "pos"));
    CHECK(check_ptr(idx, "idx"));
    if (w) CHECK(check_ptr(w, "w"));
    return hip_status(hg::launch_encode_index(k, pos, n, idx, w, stream), "hg_encode_index");
}

hg_status hg_render_direct(const hg_model *model, const hg_env *env, const hg_sampling *samp, const hg_points *pts,
                           float *rgb, float *vis, float *depth, hipStream_t stream) {
    return render(model, env, samp, pts, rgb, vis, depth, stream, false);
}

hg_status hg_render_indirect(const hg_model *model, const hg_env *env, const hg_sampling *samp,
                             const hg_points *pts, float *rgb, float *vis, float *depth, hipStream_t stream) {
    return render(model, env, samp, pts, rgb, vis, depth, stream, true);
}

// Bound on the radix sort's temporary storage that hg_backward_workspace_size
// reserves for `records` keys (the exact need is queried at call time and
// checked against it).
static size_t sort_bound(int64_t records) { return (size_t(2) << 20) + (size_t)records * 8; }

size_t hg_backward_workspace_size(int32_t indirect, int64_t n) {
    if ((indirect != 0 && indirect != 1) || n <= 0 || n > kMaxBackwardN) return 0;
    const int R = indirect ? 2 : 1;
    return hg::backward_ws_layout(n, R, sort_bound(R * n), nullptr, nullptr);
}

hg_status hg_backward(const hg_model *model, const hg_env *env, const hg_sampling *samp, const hg_points *pts,
                      int32_t indirect, const float *g_rgb, const float *g_vis, const float *g_depth, float *g_table,
                      float *const g_brdf[6], float *const g_irt[6], float *g_pos, void *ws, size_t ws_bytes,
                      hipStream_t stream) {
    g_err.clear();
    hg::BwdK k{};
    Prec prec;
    bool query = false;
    CHECK(check_model(model, k.r, prec));
    CHECK(check_env(env, k.r.env));
    CHECK(check_points(pts, query));
    REQUIRE(query || pts->n == 0, "hg_backward needs query-mode points (dir != NULL)");
    CHECK(check_sampling(samp, false, k.r.s));
    SUPPORT((samp->flags & (HG_HARD_VIS | HG_MIS)) == 0, "hard visibility and MIS are forward-only modes");
    SUPPORT(model->brdf.n_out == 5, "the decoder's normal head is forward-only (hg_backward needs n_out = 5)");
    REQUIRE(indirect == 0 || indirect == 1, "indirect must be 0 or 1");
    if (pts->n == 0) return HG_OK;
    CHECK(check_ptr(g_rgb, "g_rgb"));
    CHECK(check_ptr(g_vis, "g_vis"));
    CHECK(check_ptr(g_depth, "g_depth"));
    CHECK(check_ptr(g_table, "g_table"));
    REQUIRE(g_brdf != nullptr && g_irt != nullptr, "g_brdf / g_irt arrays are NULL");
    for (int i = 0; i < 6; ++i) {
        char nm[32];
        snprintf(nm, sizeof nm, "g_brdf[%d]", i);
        CHECK(check_ptr(g_brdf[i], nm));
        snprintf(nm, sizeof nm, "g_irt[%d]", i);
        CHECK(check_ptr(g_irt[i], nm));
        k.gb[i] = g_brdf[i];
        k.gi[i] = g_irt[i];
    }
    if (g_pos) CHECK(check_ptr(g_pos, "g_pos"));
    k.r.pos = pts->pos;
    k.r.dir = pts->dir;
    k.r.n = pts->n;
    k.g_rgb = g_rgb;
    k.g_vis = g_vis;
    k.g_dep = g_depth;
    k.g_table = g_table;
    k.g_pos = g_pos;
    {
        const int R = indirect ? 2 : 1;
        REQUIRE(pts->n <= kMaxBackwardN, "n = %lld above %lld", (long long)pts->n, (long long)kMaxBackwardN);
        CHECK(check_ptr(ws, "ws", 256));
        REQUIRE(ws_bytes >= hg_backward_workspace_size(indirect, pts->n),
                "ws_bytes %zu < hg_backward_workspace_size %zu", ws_bytes,
                hg_backward_workspace_size(indirect, pts->n));
        const int64_t rec = R * pts->n;
        size_t tmp = 0;
        CHECK(hip_status(hg::backward_sort_bytes(rec, tmp), "hg_backward: sort size"));
        if (tmp > sort_bound(rec))
            return fail(HG_E_WORKSPACE, "sort needs %zu bytes, above the reserved %zu", tmp, sort_bound(rec));
        hg::backward_ws_layout(pts->n, R, sort_bound(rec), ws, &k.ws);
    }
    return hip_status(hg::launch_backward(k, model->grid.dtype == HG_F16, prec == Prec::Mixed, indirect != 0, stream),
                      "hg_backward");
}

// Bound on the radix sort's temporary storage that
// hg_morton_order_workspace_size reserves (checked at call time).
static size_t morton_sort_bound(int64_t n) { return (size_t(2) << 20) + (size_t)n * 16; }

size_t hg_morton_order_workspace_size(int64_t n) {
    if (n <= 0 || n > INT32_MAX) return 0;
    return hg::morton_ws_layout(n, morton_sort_bound(n));
}

hg_status hg_morton_order(const float *pos, int64_t n, float box_lo, float box_extent, int32_t *perm, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
    g_err.clear();
    REQUIRE(n >= 0 && n <= INT32_MAX, "n = %lld outside [0, 2^31 - 1]", (long long)n);
    REQUIRE(std::isfinite(box_lo), "box_lo is not finite");
    int ex = 0;
    const float mant = std::frexp(box_extent, &ex);
    REQUIRE(box_extent > 0.0f && mant == 0.5f, "box_extent %g is not a power of two", (double)box_extent);
    if (n == 0) return HG_OK;
    CHECK(check_ptr(pos, "pos", 4));
    CHECK(check_ptr(perm, "perm", 4));
    CHECK(check_ptr(ws, "ws", 256));
    REQUIRE(ws_bytes >= hg_morton_order_workspace_size(n), "ws_bytes %zu < hg_morton_order_workspace_size %zu",
            ws_bytes, hg_morton_order_workspace_size(n));
    size_t tmp = 0;
    CHECK(hip_status(hg::morton_sort_bytes(n, tmp), "hg_morton_order: sort size"));
    if (tmp > morton_sort_bound(n))
        return fail(HG_E_WORKSPACE, "sort needs %zu bytes, above the reserved %zu", tmp, morton_sort_bound(n));
    return hip_status(hg::launch_morton_order(pos, n, box_lo, box_extent, perm, ws, morton_sort_bound(n), stream),
                      "hg_morton_order");
}

hg_status hg_l2_loss(const float *rgb, const float *vis, const float *depth, const float *tgt, int64_t n,
                     float *loss, float *g_rgb, float *g_vis, float *g_depth, hipStream_t stream) {
    g_err.clear();
    REQUIRE(n >= 0, "n = %lld is negative", (long long)n);
    CHECK(check_ptr(loss, "loss", 4));
    if (n > 0) {
        CHECK(check_ptr(rgb, "rgb"));
        CHECK(check_ptr(vis, "vis"));
        CHECK(check_ptr(depth, "depth"));
        CHECK(check_ptr(tgt, "tgt"));
        CHECK(check_ptr(g_rgb, "g_rgb"));
        CHECK(check_ptr(g_vis, "g_vis"));
        CHECK(check_ptr(g_depth, "g_depth"));
    }
    return hip_status(hg::launch_l2_loss(rgb, vis, depth, tgt, n, loss, g_rgb, g_vis, g_depth, stream),
                      "hg_l2_loss");
}

hg_status hg_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int32_t step, float lr,
                       float beta1, float beta2, float eps, float weight_decay, void *shadow, hg_dtype shadow_dtype,
                       hipStream_t stream) {
    g_err.clear();
    REQUIRE(n >= 0, "n = %lld is negative", (long long)n);
    REQUIRE(step >= 1, "step = %d must be >= 1", step);
    REQUIRE(std::isfinite(lr) && std::isfinite(eps) && std::isfinite(weight_decay), "non-finite hyper-parameter");
    REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f, "betas must lie in [0, 1)");
    int kind = 0;
    if (shadow) {
        REQUIRE(shadow_dtype == HG_F16 || shadow_dtype == HG_BF16, "shadow dtype must be HG_F16 or HG_BF16");
        kind = shadow_dtype == HG_F16 ? 1 : 2;
    }
    if (n == 0) return HG_OK;
    CHECK(check_ptr(param, "param"));
    CHECK(check_ptr(grad, "grad"));
    CHECK(check_ptr(m, "m"));
    CHECK(check_ptr(v, "v"));
    if (shadow) CHECK(check_ptr(shadow, "shadow", 8));
    const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
    REQUIRE(bc1 > 0.0 && bc2 > 0.0, "bias correction vanishes (beta = 0 and step too large?)");
    return hip_status(hg::launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, weight_decay, (float)bc1,
                                      (float)bc2, shadow, kind, stream),
                      "hg_adam_step");
}

static_assert(HG_ADAM_MAX_TENSORS == hg::kAdamMax, "tensor count per launch");

hg_status hg_adam_step_multi(const hg_adam_tensor *tensors, int32_t count, int32_t step, float lr, float beta1,
                             float beta2, float eps, int32_t zero_grad, hipStream_t stream) {
    g_err.clear();
    REQUIRE(count >= 0 && count <= HG_ADAM_MAX_TENSORS, "count = %d outside [0, %d]", count, HG_ADAM_MAX_TENSORS);
    REQUIRE(zero_grad == 0 || zero_grad == 1, "zero_grad must be 0 or 1");
    REQUIRE(step >= 1, "step = %d must be >= 1", step);
    REQUIRE(std::isfinite(lr) && std::isfinite(eps), "non-finite hyper-parameter");
    REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f, "betas must lie in [0, 1)");
    if (count == 0) return HG_OK;
    REQUIRE(tensors != nullptr, "tensors is NULL");
    hg::AdamMultiK k{};
    for (int t = 0; t < count; ++t) {
        const hg_adam_tensor &x = tensors[t];
        REQUIRE(x.n >= 0 && x.n <= (int64_t(1) << 36), "tensors[%d].n = %lld outside [0, 2^36]", t, (long long)x.n);
        REQUIRE(std::isfinite(x.weight_decay), "tensors[%d].weight_decay is not finite", t);
        int kind = 0;
        if (x.shadow) {
            REQUIRE(x.shadow_dtype == HG_F16 || x.shadow_dtype == HG_BF16,
                    "tensors[%d]: shadow dtype must be HG_F16 or HG_BF16", t);
            kind = x.shadow_dtype == HG_F16 ? 1 : 2;
        }
        if (x.n > 0) {
            CHECK(check_ptr(x.param, "param"));
            CHECK(check_ptr(x.grad, "grad"));
            CHECK(check_ptr(x.m, "m"));
            CHECK(check_ptr(x.v, "v"));
            if (x.shadow) CHECK(check_ptr(x.shadow, "shadow", 8));
        }
        k.param[t] = x.param;
        k.grad[t] = x.grad;
        k.m[t] = x.m;
        k.v[t] = x.v;
        k.shadow[t] = x.shadow;
        k.n[t] = x.n;
        k.wd[t] = x.weight_decay;
        k.kind[t] = kind;
    }
    const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
    REQUIRE(bc1 > 0.0 && bc2 > 0.0, "bias correction vanishes (beta = 0 and step too large?)");
    k.count = count;
    k.zero_grad = zero_grad;
    k.lr = lr;
    k.b1 = beta1;
    k.b2 = beta2;
    k.eps = eps;
    // the same reciprocals launch_adam forms, so both entry points compute alike
    k.inv_bc1 = 1.0f / (float)bc1;
    k.inv_sqrt_bc2 = 1.0f / sqrtf((float)bc2);
    return hip_status(hg::launch_adam_multi(k, stream), "hg_adam_step_multi");
}

size_t hg_env_sampling_size(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0 || H > 8192 || W > 8192) return 0;
    return env_sampling_bytes(H, W);
}

hg_status hg_env_build_sampling(const float *rgb_host, int32_t H, int32_t W, void *dist, size_t bytes,
                                hipStream_t stream) {
    g_err.clear();
    REQUIRE(rgb_host != nullptr, "rgb_host is NULL");
    REQUIRE(H >= 1 && W >= 1 && H <= 8192 && W <= 8192, "env size %dx%d outside [1, 8192]^2", H, W);
    CHECK(check_ptr(dist, "dist"));
    REQUIRE(bytes >= env_sampling_bytes(H, W), "bytes %zu < %zu", bytes, env_sampling_bytes(H, W));
    std::vector<unsigned char> host(env_sampling_bytes(H, W));
    hg::build_env_dist_host(rgb_host, H, W, host.data());
    CHECK(hip_status(hipMemcpyAsync(dist, host.data(), host.size(), hipMemcpyHostToDevice, stream),
                     "hg_env_build_sampling: copy"));
    // the staging buffer is freed on return
    return hip_status(hipStreamSynchronize(stream), "hg_env_build_sampling: synchronise");
}

size_t hg_denoise_workspace_size(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0) return 0;
    return hg::denoise_workspace_floats(H, W) * sizeof(float);
}

}  // extern "C"

namespace {

hg_status check_denoise(const float *rgb, const float *depth, const float *nrm, int32_t H, int32_t W,
                        const hg_denoise_params *params, const float *out) {
    REQUIRE(params != nullptr, "params is NULL");
    REQUIRE(H >= 1 && W >= 1 && (int64_t)H * W < (int64_t(1) << 28) && H <= 65535 * 16,
            "image size %dx%d invalid", H, W);
    REQUIRE(params->iterations >= 0 && params->iterations <= 10, "iterations = %d outside [0, 10]",
            params->iterations);
    REQUIRE(std::isfinite(params->sigma_z) && std::isfinite(params->sigma_n) && std::isfinite(params->sigma_l) &&
                params->sigma_z >= 0.0f && params->sigma_n >= 0.0f && params->sigma_l >= 0.0f,
            "sigmas must be finite and non-negative");
    CHECK(check_ptr(rgb, "rgb"));
    CHECK(check_ptr(depth, "depth"));
    CHECK(check_ptr(nrm, "nrm"));
    CHECK(check_ptr(out, "out"));
    return HG_OK;
}

}  // namespace

extern "C" {

hg_status hg_denoise(const float *rgb, const float *depth, const float *nrm, int32_t H, int32_t W,
                     const hg_denoise_params *params, float *out, void *work, size_t work_bytes,
                     hipStream_t stream) {
    g_err.clear();
    CHECK(check_denoise(rgb, depth, nrm, H, W, params, out));
    CHECK(check_ptr(work, "work"));
    REQUIRE(work_bytes >= hg_denoise_workspace_size(H, W), "work_bytes %zu < %zu", work_bytes,
            hg_denoise_workspace_size(H, W));
    return hip_status(hg::launch_denoise(rgb, depth, nrm, H, W, params->iterations, params->sigma_z,
                                         params->sigma_n, params->sigma_l, out, static_cast<float *>(work), stream),
                      "hg_denoise");
}

hg_status hg_denoise_noalloc(const float *rgb, const float *depth, const float *nrm, int32_t H, int32_t W,
                             const hg_denoise_params *params, float *out, hipStream_t stream) {
    g_err.clear();
    CHECK(check_denoise(rgb, depth, nrm, H, W, params, out));
    REQUIRE((int64_t)H * W <= HG_DENOISE_NOALLOC_MAX_PIXELS,
            "image %dx%d exceeds the static workspace of %d pixels (use hg_denoise with a caller workspace)", H, W,
            HG_DENOISE_NOALLOC_MAX_PIXELS);
    float *ws = nullptr;
    size_t ws_floats = 0;
    CHECK(hip_status(hg::denoise_scratch(stream, &ws, &ws_floats), "hg_denoise_noalloc: device scratch lookup"));
    REQUIRE(hg::denoise_workspace_floats(H, W) <= ws_floats, "static workspace too small");
    return hip_status(hg::launch_denoise(rgb, depth, nrm, H, W, params->iterations, params->sigma_z,
                                         params->sigma_n, params->sigma_l, out, ws, stream),
                      "hg_denoise_noalloc");
}

}  // extern "C"
