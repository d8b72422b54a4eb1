/*
 * oracle.c -- plain FP64 CPU reference of the hash-grid secondary-ray renderer.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table
 * or constant generator with the HIP path; both receive the same seeded
 * inputs (FP32 masters) and each implements the counter-based generator
 * Philox4x32-10 from its published definition.
 *
 * What is computed (paper: "Baking Relightable NeRF for Real-time
 * Direct/Indirect Illumination Rendering", arXiv 2409.10327):
 *   - hash-grid encoder f = H(x), multi-level tables as InstantNGP
 *     (Sec. 3.2 "Indirect Illumination Renderer", Sec. 4.1 settings);
 *   - BRDF decoder B(f) -> albedo, roughness (0.09 + 0.91 sigmoid), metallic
 *     (Sec. 3.2; output mapping in Sec. 3.3);
 *   - implicit ray tracer I(f, w) -> visibility (sigmoid) and depth
 *     min-max normalised to [near, far] with outputs clamped to 1
 *     (Sec. 3.2 items 1-2; near/far from the supplementary training details);
 *   - one recursive bounce at x' = x + t w with 8 secondary rays
 *     (Sec. 3.1, Sec. 3.2 "Overview", supplementary "Rendering Details");
 *   - incoming radiance of Eq. (2) and the Monte Carlo rendering equation
 *     Eq. (1) over environment-map light (Sec. 2.2);
 *   - microfacet BRDF: Lambert diffuse + GGX (alpha = r^2), Schlick Fresnel,
 *     height-correlated Smith visibility (Sec. 4.1, Sec. 4.2, supplementary
 *     roughness-remapping ablation);
 *   - L2 distillation loss, its analytic gradient and Adam.
 * Readings where the paper is silent are stated next to each function.
 *
 * Everything is evaluated in double precision from FP32 inputs, in the
 * plainest order, with OpenMP only over independent points.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_MAXF 64      /* max L*F */
#define OR_MAXIN 67     /* max L*F + 3 */
#define OR_MAXH 64      /* hidden width */
#define OR_MAXOUT 8
#define OR_MAXL 32
#define OR_MAXN2 64     /* max secondary directions */

#define OR_DIFFUSE_ONLY 1u
#define OR_HARD_VIS 2u     /* binary visibility, bounce only on shadow rays */
#define OR_MIS 4u          /* primary directions: light + GGX-VNDF rays, balance heuristic */

typedef struct {
    int32_t L, F, log2_T;
    int32_t res[OR_MAXL];
    double lo, extent;
    const float *table; /* [L][T][F] */
} or_grid;

typedef struct {
    int32_t n_in, n_hidden, n_out;
    const float *W0, *b0, *W1, *b1, *W2, *b2; /* W[k]: [out][in] */
} or_mlp;

typedef struct {
    or_grid grid;
    or_mlp brdf, irt;
    double t_near, t_far, f0;
} or_model;

typedef struct {
    int32_t H, W;
    const float *rgb; /* [H][W][3] */
} or_env;

typedef struct {
    int32_t n_dirs, n_dirs2;
    uint64_t seed;
    uint32_t flags;
} or_sampling;

typedef struct {
    int64_t n;
    const float *pos, *nrm, *wo, *dir; /* [n][3]; dir != NULL selects query mode */
    const uint32_t *pid;               /* [n] point ids for the sampler, NULL: 0..n-1 */
} or_points;

static uint32_t point_id(const or_points *P, int64_t p) { return P->pid ? P->pid[p] : (uint32_t)p; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies counter     */
/* words 0 and 2 by the round multipliers, mixes the high halves with the   */
/* other two words and the key, and the key is bumped by the Weyl constants */
/* between rounds.                                                          */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Stratified cosine-weighted direction about a unit normal n.              */
/* Reading: the paper samples light directions with stratified sampling     */
/* (supplementary training and rendering details) and evaluates Eq. (1)     */
/* with the sampling pdf.  Directions are drawn from a cosine-weighted      */
/* hemisphere (pdf = cos/pi) with N = n_a x n_b strata, n_a = 2^floor(log2  */
/* N / 2).  Sample k lies in stratum (k / n_b, k % n_b).                     */
/* The uniforms come from Philox4x32-10 with key = seed and counter         */
/* (pid, q, k >> 2, tag); word k & 3 is split into two 16-bit halves and    */
/* each is mapped to the centre of its 2^-16 bin.                           */
/* Disk-to-hemisphere mapping (Malley's method); orthonormal basis of       */
/* Duff et al., "Building an Orthonormal Basis, Revisited", JCGT 2017.      */
/* ------------------------------------------------------------------------ */
static void onb(const double n[3], double t[3], double b[3])
{
    double sgn = copysign(1.0, n[2]);
    double a = -1.0 / (sgn + n[2]);
    double bb = n[0] * n[1] * a;
    t[0] = 1.0 + sgn * n[0] * n[0] * a;
    t[1] = sgn * bb;
    t[2] = -sgn * n[0];
    b[0] = bb;
    b[1] = sgn + n[1] * n[1] * a;
    b[2] = -n[1];
}

static int ilog2(int n)
{
    int l = 0;
    while ((1 << (l + 1)) <= n) ++l;
    return l;
}

static void uniforms(uint64_t seed, uint32_t pid, uint32_t q, uint32_t k, uint32_t tag,
                     double *u1, double *u2)
{
    uint32_t ctr[4] = {pid, q, k >> 2, tag};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    uint32_t w = o[k & 3u];
    *u1 = ((double)(w & 0xffffu) + 0.5) / 65536.0;
    *u2 = ((double)(w >> 16) + 0.5) / 65536.0;
}

static void sample_dir(uint64_t seed, uint32_t pid, uint32_t q, uint32_t k, uint32_t tag,
                       int nstrata, const double n[3], double w[3])
{
    double u1, u2;
    uniforms(seed, pid, q, k, tag, &u1, &u2);
    int na = 1 << (ilog2(nstrata) / 2);
    int nb = nstrata / na;
    int a = (int)k / nb, b = (int)k % nb;
    double s1 = (a + u1) / na;
    double s2 = (b + u2) / nb;
    double r = sqrt(s1), ph = 2.0 * M_PI * s2;
    double lx = r * cos(ph), ly = r * sin(ph), lz = sqrt(1.0 - s1);
    double t[3], bt[3];
    onb(n, t, bt);
    for (int d = 0; d < 3; ++d) w[d] = lx * t[d] + ly * bt[d] + lz * n[d];
}

void or_sample_dirs(uint64_t seed, const double *nrm, const uint32_t *pid, const uint32_t *q,
                    const uint32_t *k, uint32_t tag, int32_t nstrata, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        sample_dir(seed, pid[i], q[i], k[i], tag, nstrata, nrm + 3 * i, out + 3 * i);
}

void or_uniforms(uint64_t seed, const uint32_t *pid, const uint32_t *q, const uint32_t *k,
                 uint32_t tag, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) uniforms(seed, pid[i], q[i], k[i], tag, out + 2 * i, out + 2 * i + 1);
}

/* ------------------------------------------------------------------------ */
/* Hash-grid encoder H (InstantNGP multi-resolution tables, Sec. 3.2).      */
/* Reading: positions in the cube [lo, lo+extent]^3 map to u in [0,1]^3,    */
/* clamped.  For FP32 positions the subtraction x - lo is rounded to FP32   */
/* (the extent is a power of two, so the division is exact); positions     */
/* computed here in FP64 (bounce points) use u in FP64.  At level l with    */
/* resolution N_l: p = u N_l, cell c = min(floor(p), N_l - 1), w = p - c.   */
/* Vertex index: dense row-major when (N_l+1)^3 <= T, otherwise the spatial */
/* hash of Mueller et al. 2022 (Eq. 4): xor of coordinates times primes     */
/* (1, 2654435761, 805459861) modulo 2^32, masked to T.  Trilinear blend;   */
/* features concatenated level-major.                                       */
/* ------------------------------------------------------------------------ */
static uint32_t vertex_index(int N, uint32_t T, uint32_t vx, uint32_t vy, uint32_t vz)
{
    uint64_t s = (uint64_t)(N + 1);
    if (s * s * s <= (uint64_t)T)
        return (uint32_t)(vx + s * (vy + s * vz));
    uint32_t h = (vx * 1u) ^ (vy * 2654435761u) ^ (vz * 805459861u);
    return h & (T - 1u);
}

typedef struct {
    uint32_t idx[OR_MAXL][8];
    double w[OR_MAXL][3];     /* fractional position inside the cell */
    int inside[3];            /* 1 if u was not clamped (gradient passes) */
} enc_rec;

static void encode_u(const or_grid *g, const double u_raw[3], double *f, enc_rec *rec)
{
    const uint32_t T = 1u << g->log2_T;
    double u[3];
    for (int d = 0; d < 3; ++d) {
        u[d] = u_raw[d] < 0.0 ? 0.0 : (u_raw[d] > 1.0 ? 1.0 : u_raw[d]);
        if (rec) rec->inside[d] = (u_raw[d] > 0.0 && u_raw[d] < 1.0);
    }
    for (int l = 0; l < g->L; ++l) {
        int N = g->res[l];
        uint32_t c[3];
        double w[3];
        for (int d = 0; d < 3; ++d) {
            double p = u[d] * N;
            double cf = floor(p);
            if (cf > N - 1) cf = N - 1;
            c[d] = (uint32_t)cf;
            w[d] = p - cf;
        }
        for (int k = 0; k < g->F; ++k) f[l * g->F + k] = 0.0;
        for (int corner = 0; corner < 8; ++corner) {
            int dx = corner & 1, dy = (corner >> 1) & 1, dz = (corner >> 2) & 1;
            uint32_t idx = vertex_index(N, T, c[0] + dx, c[1] + dy, c[2] + dz);
            double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
            const float *e = g->table + ((size_t)l * T + idx) * g->F;
            for (int k = 0; k < g->F; ++k) f[l * g->F + k] += wt * (double)e[k];
            if (rec) rec->idx[l][corner] = idx;
        }
        if (rec)
            for (int d = 0; d < 3; ++d) rec->w[l][d] = w[d];
    }
}

static void pos_to_u_f32(const or_grid *g, const float x[3], double u[3])
{
    float lo = (float)g->lo;
    for (int d = 0; d < 3; ++d) {
        float s = x[d] - lo; /* rounded to FP32 */
        u[d] = (double)s / g->extent;
    }
}

static void pos_to_u_f64(const or_grid *g, const double x[3], double u[3])
{
    for (int d = 0; d < 3; ++d) u[d] = (x[d] - g->lo) / g->extent;
}

void or_encode(const or_grid *g, const float *pos, int64_t n, double *feat)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u[3];
        pos_to_u_f32(g, pos + 3 * i, u);
        encode_u(g, u, feat + (size_t)i * g->L * g->F, NULL);
    }
}

/* Encode at FP64 positions (used to pin bounce-point encodes). */
void or_encode_f64(const or_grid *g, const double *pos, int64_t n, double *feat)
{
    for (int64_t i = 0; i < n; ++i) {
        double u[3];
        pos_to_u_f64(g, pos + 3 * i, u);
        encode_u(g, u, feat + (size_t)i * g->L * g->F, NULL);
    }
}

/* Vertex indices [n][L][8] (corner bit 0 = +x, bit 1 = +y, bit 2 = +z) and
 * in-cell weights [n][L][3] for FP32 positions. */
void or_encode_index(const or_grid *g, const float *pos, int64_t n, uint32_t *idx, double *wts)
{
    double f[OR_MAXF];
#pragma omp parallel for schedule(static) private(f)
    for (int64_t i = 0; i < n; ++i) {
        double u[3];
        enc_rec rec;
        pos_to_u_f32(g, pos + 3 * i, u);
        encode_u(g, u, f, &rec);
        for (int l = 0; l < g->L; ++l) {
            for (int c = 0; c < 8; ++c) idx[((size_t)i * g->L + l) * 8 + c] = rec.idx[l][c];
            if (wts)
                for (int d = 0; d < 3; ++d) wts[((size_t)i * g->L + l) * 3 + d] = rec.w[l][d];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Three-layer MLP with ReLU hidden activations (Sec. 4.1: 3 layers, width  */
/* 64).  W[k] is stored [out][in].                                          */
/* ------------------------------------------------------------------------ */
static void linear(const float *W, const float *b, int n_out, int n_in, const double *x, double *y)
{
    for (int o = 0; o < n_out; ++o) {
        double acc = (double)b[o];
        for (int i = 0; i < n_in; ++i) acc += (double)W[(size_t)o * n_in + i] * x[i];
        y[o] = acc;
    }
}

static void mlp_fwd(const or_mlp *m, const double *in, double *h1, double *h2, double *out)
{
    linear(m->W0, m->b0, m->n_hidden, m->n_in, in, h1);
    for (int k = 0; k < m->n_hidden; ++k) h1[k] = h1[k] > 0.0 ? h1[k] : 0.0;
    linear(m->W1, m->b1, m->n_hidden, m->n_hidden, h1, h2);
    for (int k = 0; k < m->n_hidden; ++k) h2[k] = h2[k] > 0.0 ? h2[k] : 0.0;
    linear(m->W2, m->b2, m->n_out, m->n_hidden, h2, out);
}

void or_mlp_forward(const or_mlp *m, const double *in, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double h1[OR_MAXH], h2[OR_MAXH];
        mlp_fwd(m, in + (size_t)i * m->n_in, h1, h2, out + (size_t)i * m->n_out);
    }
}

/* Gradient of one MLP evaluation: accumulates parameter gradients into
 * g (packed W0,b0,W1,b1,W2,b2) and returns d/d(input) in gin. */
static void mlp_bwd(const or_mlp *m, const double *in, const double *h1, const double *h2,
                    const double *gout, double *g, double *gin)
{
    const int ni = m->n_in, nh = m->n_hidden, no = m->n_out;
    double *gW0 = g, *gb0 = gW0 + nh * ni, *gW1 = gb0 + nh, *gb1 = gW1 + nh * nh;
    double *gW2 = gb1 + nh, *gb2 = gW2 + no * nh;
    double gp2[OR_MAXH], gp1[OR_MAXH];
    for (int o = 0; o < no; ++o) {
        gb2[o] += gout[o];
        for (int k = 0; k < nh; ++k) gW2[o * nh + k] += gout[o] * h2[k];
    }
    for (int k = 0; k < nh; ++k) {
        double s = 0.0;
        for (int o = 0; o < no; ++o) s += (double)m->W2[o * nh + k] * gout[o];
        gp2[k] = h2[k] > 0.0 ? s : 0.0;
    }
    for (int k = 0; k < nh; ++k) {
        gb1[k] += gp2[k];
        for (int j = 0; j < nh; ++j) gW1[k * nh + j] += gp2[k] * h1[j];
    }
    for (int j = 0; j < nh; ++j) {
        double s = 0.0;
        for (int k = 0; k < nh; ++k) s += (double)m->W1[k * nh + j] * gp2[k];
        gp1[j] = h1[j] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < nh; ++j) {
        gb0[j] += gp1[j];
        for (int i = 0; i < ni; ++i) gW0[j * ni + i] += gp1[j] * in[i];
    }
    for (int i = 0; i < ni; ++i) {
        double s = 0.0;
        for (int j = 0; j < nh; ++j) s += (double)m->W0[j * ni + i] * gp1[j];
        gin[i] = s;
    }
}

static int64_t mlp_nparams(const or_mlp *m)
{
    return (int64_t)m->n_hidden * m->n_in + m->n_hidden + (int64_t)m->n_hidden * m->n_hidden +
           m->n_hidden + (int64_t)m->n_out * m->n_hidden + m->n_out;
}

/* ------------------------------------------------------------------------ */
/* Output heads.                                                            */
/* B: albedo = sigmoid, roughness = 0.09 + 0.91 sigmoid (Sec. 3.3),         */
/*    metallic = sigmoid.                                                   */
/* I: V = sigmoid(o0) (Sec. 3.3: sigmoid maps visibility to [0,1]);         */
/*    depth d = min(softplus(o1), 1) -- min-max normalised depth clamped to */
/*    1 = far (Sec. 3.2 item 2); t = near + (far - near) d.                 */
/* ------------------------------------------------------------------------ */
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }
static double softplus(double z) { return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z))); }

/* ------------------------------------------------------------------------ */
/* Environment lookup (image-based lighting, Sec. 2.2: the incoming        */
/* radiance is interpolated from the equirectangular map).  Reading: y is   */
/* up; azimuth phi = atan2(w_z, w_x), polar angle theta from +y computed as */
/* atan2(sqrt(w_x^2 + w_z^2), w_y); texel centres at +1/2; bilinear,        */
/* columns wrap, rows clamp.                                                */
/* ------------------------------------------------------------------------ */
static void env_lookup(const or_env *e, const double w[3], double out[3])
{
    const int H = e->H, W = e->W;
    double phi = atan2(w[2], w[0]);
    double th = atan2(sqrt(w[0] * w[0] + w[2] * w[2]), w[1]);
    double s = (phi + M_PI) / (2.0 * M_PI) * W - 0.5;
    double q = th / M_PI * H - 0.5;
    double xf = floor(s), yf = floor(q);
    double fx = s - xf, fy = q - yf;
    long x0 = (long)xf;
    x0 = ((x0 % W) + W) % W;
    long x1 = (x0 + 1) % W;
    long y0 = (long)yf, y1 = y0 + 1;
    if (y0 < 0) y0 = 0;
    if (y0 > H - 1) y0 = H - 1;
    if (y1 < 0) y1 = 0;
    if (y1 > H - 1) y1 = H - 1;
    for (int c = 0; c < 3; ++c) {
        double e00 = e->rgb[(y0 * W + x0) * 3 + c], e01 = e->rgb[(y0 * W + x1) * 3 + c];
        double e10 = e->rgb[(y1 * W + x0) * 3 + c], e11 = e->rgb[(y1 * W + x1) * 3 + c];
        out[c] = (1.0 - fy) * ((1.0 - fx) * e00 + fx * e01) + fy * ((1.0 - fx) * e10 + fx * e11);
    }
}

void or_env_lookup(const or_env *e, const double *dirs, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) env_lookup(e, dirs + 3 * i, out + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Microfacet BRDF f_r(n, v, l; a, r, m).                                   */
/* Diffuse: Lambert (1-m) a / pi ("simplified Disney" albedo term).         */
/* Specular: GGX D with alpha = r^2, Schlick Fresnel with F0 = mix(f0, a,   */
/* m) (f0 = 0.04, Sec. 5), height-correlated Smith visibility (Sec. 4.2 and */
/* the supplementary roughness-remapping ablation).  NdotL <= 0 returns 0;  */
/* NdotV is clamped below at 1e-4.  With the diffuse-only flag the value is */
/* a / pi.  Also returns d f / d a (per channel), d f / d r, d f / d m.      */
/* ------------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* The three factors of the specular lobe for n.l > 0: the GGX normal
 * distribution D(h) with alpha = r^2, the Schlick weight P = (1 - v.h)^5
 * (F = F0 + (1 - F0) P), and the visibility term Vis = G2 / (4 n.l n.v) of
 * the height-correlated Smith masking-shadowing function
 * G2 = 1 / (1 + Lambda(v) + Lambda(l)) (Heitz, "Understanding the
 * Masking-Shadowing Function in Microfacet-Based BRDFs", JCGT 2014), written
 * with Lambda(w) = (sqrt(1 + alpha^2 tan^2) - 1) / 2 cleared of fractions. */
typedef struct {
    double NdotL, NdotV, NdotH, VdotH, a2, Q, D, sv, sl, A, B, Vis, P;
} spec_terms;

static void spec_eval(const double n[3], const double v[3], const double l[3], double r,
                      spec_terms *t)
{
    t->NdotL = dot3(n, l);
    double NdotV = dot3(n, v);
    if (NdotV < 1e-4) NdotV = 1e-4;
    t->NdotV = NdotV;
    double h[3] = {l[0] + v[0], l[1] + v[1], l[2] + v[2]};
    double hn = sqrt(dot3(h, h));
    if (hn > 0.0) {
        for (int d = 0; d < 3; ++d) h[d] /= hn;
    } else {
        for (int d = 0; d < 3; ++d) h[d] = n[d];
    }
    double NdotH = dot3(n, h);
    t->NdotH = NdotH < 0.0 ? 0.0 : NdotH;
    double VdotH = dot3(v, h);
    t->VdotH = VdotH < 0.0 ? 0.0 : VdotH;
    double alpha = r * r;
    t->a2 = alpha * alpha;
    t->Q = t->NdotH * t->NdotH * (t->a2 - 1.0) + 1.0;
    t->D = t->a2 / (M_PI * t->Q * t->Q);
    t->sv = sqrt(NdotV * NdotV * (1.0 - t->a2) + t->a2);
    t->sl = sqrt(t->NdotL * t->NdotL * (1.0 - t->a2) + t->a2);
    t->A = t->NdotL * t->sv;
    t->B = NdotV * t->sl;
    t->Vis = 0.5 / (t->A + t->B);
    t->P = pow(1.0 - t->VdotH, 5.0);
}

/* Specular factors for pinning: D, Vis and P per sample (0 where n.l <= 0). */
void or_brdf_terms(const double *n, const double *v, const double *l, const double *r, int64_t cnt,
                   double *D, double *Vis, double *P)
{
    for (int64_t i = 0; i < cnt; ++i) {
        spec_terms t;
        spec_eval(n + 3 * i, v + 3 * i, l + 3 * i, r[i], &t);
        int lit = t.NdotL > 0.0;
        D[i] = lit ? t.D : 0.0;
        Vis[i] = lit ? t.Vis : 0.0;
        P[i] = lit ? t.P : 0.0;
    }
}

static void brdf_eval(const double n[3], const double v[3], const double l[3], const double a[3],
                      double r, double m, double f0, int diffuse_only, double f[3],
                      double dfa[3], double dfr[3], double dfm[3])
{
    double NdotL = dot3(n, l);
    if (NdotL <= 0.0) {
        for (int c = 0; c < 3; ++c) f[c] = dfa[c] = dfr[c] = dfm[c] = 0.0;
        return;
    }
    if (diffuse_only) {
        for (int c = 0; c < 3; ++c) {
            f[c] = a[c] / M_PI;
            dfa[c] = 1.0 / M_PI;
            dfr[c] = dfm[c] = 0.0;
        }
        return;
    }
    spec_terms t;
    spec_eval(n, v, l, r, &t);
    const double NdotV = t.NdotV, NdotH = t.NdotH, a2 = t.a2, Q = t.Q, D = t.D;
    const double sv = t.sv, sl = t.sl, A = t.A, B = t.B, Vis = t.Vis, P = t.P;
    /* derivatives with respect to a2 = r^4 */
    double dD_da2 = (Q - 2.0 * a2 * NdotH * NdotH) / (M_PI * Q * Q * Q);
    double dA_da2 = NdotL * (1.0 - NdotV * NdotV) / (2.0 * sv);
    double dB_da2 = NdotV * (1.0 - NdotL * NdotL) / (2.0 * sl);
    double dVis_da2 = -0.5 * (dA_da2 + dB_da2) / ((A + B) * (A + B));
    double da2_dr = 4.0 * r * r * r;
    for (int c = 0; c < 3; ++c) {
        double F0 = f0 * (1.0 - m) + a[c] * m;
        double F = F0 + (1.0 - F0) * P;
        f[c] = (1.0 - m) * a[c] / M_PI + D * F * Vis;
        dfa[c] = (1.0 - m) / M_PI + D * Vis * (1.0 - P) * m;
        dfm[c] = -a[c] / M_PI + D * Vis * (1.0 - P) * (a[c] - f0);
        dfr[c] = F * (dD_da2 * Vis + D * dVis_da2) * da2_dr;
    }
}

void or_brdf(const double *n, const double *v, const double *l, const double *a, const double *r,
             const double *m, double f0, int32_t diffuse_only, int64_t cnt, double *f, double *dfa,
             double *dfr, double *dfm)
{
    for (int64_t i = 0; i < cnt; ++i) {
        double t1[3], t2[3], t3[3];
        brdf_eval(n + 3 * i, v + 3 * i, l + 3 * i, a + 3 * i, r[i], m[i], f0, diffuse_only,
                  f + 3 * i, dfa ? dfa + 3 * i : t1, dfr ? dfr + 3 * i : t2, dfm ? dfm + 3 * i : t3);
    }
}

/* ------------------------------------------------------------------------ */
/* Multiple importance sampling of the primary directions (Sec. 4.1: one    */
/* light-importance ray and one GGX ray drawn from the distribution of      */
/* visible normals per primary point, combined with Veach's balance         */
/* heuristic).  With n_dirs = 2M, directions k = 0..M-1 are light samples    */
/* and k = M..2M-1 GGX samples; each strategy stratifies its M samples like  */
/* the cosine sampler.  Sample i carries the weight                          */
/*   c_i = 2 f_r(w_i) (n.w_i) / (p_env(w_i) + p_ggx(w_i))                    */
/* so that L_o = 1/N sum_i c_i L_in(w_i) is the balance-heuristic estimator  */
/* with M samples per strategy.                                              */
/*                                                                          */
/* Light distribution (reading): piecewise constant in solid angle over the */
/* equirectangular texels.  Texel (y, x) spans theta in [pi y/H, pi(y+1)/H] */
/* and phi in [-pi + 2 pi x/W, -pi + 2 pi (x+1)/W] (the lookup's texel       */
/* centres); its probability is proportional to its luminance times its     */
/* solid angle (2 pi/W)(cos theta_y - cos theta_{y+1}); inside the texel the */
/* direction is uniform in solid angle.  The density is therefore           */
/* lum(texel) / sum_texels lum * solid angle.  An all-black map falls back  */
/* to the uniform sphere; a black row samples its columns uniformly (it is  */
/* never chosen).  Rows and columns are found by inverting the marginal and */
/* conditional CDFs with the two uniforms of the sample (continuous         */
/* inversion: the offset inside the chosen interval places the direction    */
/* inside the texel).  Uniforms: Philox counter (pid, 0, k >> 2, tag) with   */
/* tag 2 for light and 3 for GGX samples, 16-bit halves at bin centres.     */
/*                                                                          */
/* GGX visible-normal sampling: Heitz, "Sampling the GGX Distribution of    */
/* Visible Normals", JCGT 2018, with alpha = r^2 (the BRDF's alpha).  The    */
/* view is taken in the normal's frame with its normal component clamped to */
/* 1e-4 and renormalised (v_s); the reflected direction has the density     */
/*   p_ggx(l) = G1(v_s) D(h) / (4 n.v_s),  h = normalize(v_s + l),           */
/* for v_s.h > 0 and n.h > 0 (0 otherwise),                                */
/* G1(v) = 2 n.v / (n.v + sqrt(a2 + (1 - a2)(n.v)^2)).                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int H, W;
    double *ct;   /* [H+1] cos(pi y / H) */
    double *marg; /* [H+1] marginal CDF over rows */
    double *cond; /* [H][W+1] conditional CDF over the columns of each row */
    double *dens; /* [H][W] solid-angle density of each texel */
} env_dist;

static void env_dist_build(const or_env *E, env_dist *D)
{
    const int H = E->H, W = E->W;
    D->H = H;
    D->W = W;
    D->ct = (double *)malloc((size_t)(H + 1) * sizeof(double));
    D->marg = (double *)malloc((size_t)(H + 1) * sizeof(double));
    D->cond = (double *)malloc((size_t)H * (W + 1) * sizeof(double));
    D->dens = (double *)malloc((size_t)H * W * sizeof(double));
    double *wt = (double *)malloc((size_t)H * W * sizeof(double));
    double *row = (double *)malloc((size_t)H * sizeof(double));
    for (int y = 0; y <= H; ++y) D->ct[y] = cos(M_PI * y / H);
    double total = 0.0;
    for (int y = 0; y < H; ++y) {
        const double omega = 2.0 * M_PI / W * (D->ct[y] - D->ct[y + 1]);
        for (int x = 0; x < W; ++x) {
            const float *t = E->rgb + ((size_t)y * W + x) * 3;
            wt[y * W + x] = (0.2126 * t[0] + 0.7152 * t[1] + 0.0722 * t[2]) * omega;
        }
    }
    for (int i = 0; i < H * W; ++i) total += wt[i];
    const int uniform = !(total > 0.0);
    if (uniform) {
        total = 0.0;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) wt[y * W + x] = 2.0 * M_PI / W * (D->ct[y] - D->ct[y + 1]);
        for (int i = 0; i < H * W; ++i) total += wt[i];
    }
    for (int y = 0; y < H; ++y) {
        double *c = D->cond + (size_t)y * (W + 1);
        double r = 0.0;
        for (int x = 0; x < W; ++x) r += wt[y * W + x];
        row[y] = r;
        c[0] = 0.0;
        double acc = 0.0;
        for (int x = 0; x < W; ++x) {
            acc += wt[y * W + x];
            c[x + 1] = r > 0.0 ? acc / r : (double)(x + 1) / W;
        }
        c[W] = 1.0;
        const double omega = 2.0 * M_PI / W * (D->ct[y] - D->ct[y + 1]);
        for (int x = 0; x < W; ++x) D->dens[y * W + x] = wt[y * W + x] / total / omega;
    }
    D->marg[0] = 0.0;
    double acc = 0.0;
    for (int y = 0; y < H; ++y) {
        acc += row[y];
        D->marg[y + 1] = acc / total;
    }
    D->marg[H] = 1.0;
    free(wt);
    free(row);
}

static void env_dist_free(env_dist *D)
{
    free(D->ct);
    free(D->marg);
    free(D->cond);
    free(D->dens);
}

/* largest i in [0, n-1] with c[i] <= u, for a nondecreasing c[0..n] */
static int cdf_find(const double *c, int n, double u)
{
    int i = 0;
    for (int k = 1; k < n; ++k)
        if (c[k] <= u) i = k;
    return i;
}

static double env_density(const env_dist *D, const double w[3])
{
    double phi = atan2(w[2], w[0]);
    double th = atan2(sqrt(w[0] * w[0] + w[2] * w[2]), w[1]);
    int x = (int)floor((phi + M_PI) / (2.0 * M_PI) * D->W);
    int y = (int)floor(th / M_PI * D->H);
    x = x < 0 ? 0 : (x >= D->W ? D->W - 1 : x);
    y = y < 0 ? 0 : (y >= D->H ? D->H - 1 : y);
    return D->dens[y * D->W + x];
}

/* light sample from the stratified uniforms (s1, s2); returns its density */
static double env_sample(const env_dist *D, double s1, double s2, double w[3])
{
    const int H = D->H, W = D->W;
    int y = cdf_find(D->marg, H, s1);
    double fv = (s1 - D->marg[y]) / (D->marg[y + 1] - D->marg[y]);
    const double *c = D->cond + (size_t)y * (W + 1);
    int x = cdf_find(c, W, s2);
    double fu = (s2 - c[x]) / (c[x + 1] - c[x]);
    double cth = D->ct[y] - fv * (D->ct[y] - D->ct[y + 1]);
    double sth = sqrt((1.0 - cth) * (1.0 + cth));
    double phi = -M_PI + 2.0 * M_PI * (x + fu) / W;
    w[0] = sth * cos(phi);
    w[1] = cth;
    w[2] = sth * sin(phi);
    return D->dens[y * W + x];
}

static double ggx_g1(double nv, double a2) { return 2.0 * nv / (nv + sqrt(a2 + (1.0 - a2) * nv * nv)); }

/* view in the normal's frame (t, b, n), normal component clamped, unit */
static void ggx_view(const double n[3], const double v[3], double vl[3], double t[3], double b[3])
{
    onb(n, t, b);
    vl[0] = dot3(v, t);
    vl[1] = dot3(v, b);
    vl[2] = dot3(v, n);
    if (vl[2] < 1e-4) vl[2] = 1e-4;
    double s = sqrt(dot3(vl, vl));
    for (int d = 0; d < 3; ++d) vl[d] /= s;
}

static double ggx_density(const double n[3], const double v[3], double r, const double l[3])
{
    double vl[3], t[3], b[3];
    ggx_view(n, v, vl, t, b);
    double ll[3] = {dot3(l, t), dot3(l, b), dot3(l, n)};
    double h[3] = {vl[0] + ll[0], vl[1] + ll[1], vl[2] + ll[2]};
    double hn = sqrt(dot3(h, h));
    if (!(hn > 0.0)) return 0.0;
    for (int d = 0; d < 3; ++d) h[d] /= hn;
    double vh = dot3(vl, h);
    if (!(vh > 0.0)) return 0.0;
    double nh = h[2];
    if (!(nh > 0.0)) return 0.0; /* microfacet normals lie above the surface */
    double alpha = r * r, a2 = alpha * alpha;
    double Q = nh * nh * (a2 - 1.0) + 1.0;
    double Dh = a2 / (M_PI * Q * Q);
    return ggx_g1(vl[2], a2) * Dh / (4.0 * vl[2]);
}

static void ggx_sample(const double n[3], const double v[3], double r, double s1, double s2, double l[3])
{
    double vl[3], t[3], b[3];
    ggx_view(n, v, vl, t, b);
    const double alpha = r * r;
    double vh[3] = {alpha * vl[0], alpha * vl[1], vl[2]};
    double s = sqrt(dot3(vh, vh));
    for (int d = 0; d < 3; ++d) vh[d] /= s;
    double lensq = vh[0] * vh[0] + vh[1] * vh[1];
    double T1[3], T2[3];
    if (lensq > 0.0) {
        double il = 1.0 / sqrt(lensq);
        T1[0] = -vh[1] * il; T1[1] = vh[0] * il; T1[2] = 0.0;
    } else {
        T1[0] = 1.0; T1[1] = 0.0; T1[2] = 0.0;
    }
    T2[0] = vh[1] * T1[2] - vh[2] * T1[1];
    T2[1] = vh[2] * T1[0] - vh[0] * T1[2];
    T2[2] = vh[0] * T1[1] - vh[1] * T1[0];
    double rr = sqrt(s1), ph = 2.0 * M_PI * s2;
    double t1 = rr * cos(ph), t2 = rr * sin(ph);
    double sv = 0.5 * (1.0 + vh[2]);
    t2 = (1.0 - sv) * sqrt(1.0 - t1 * t1) + sv * t2;
    double tz = 1.0 - t1 * t1 - t2 * t2;
    tz = tz > 0.0 ? sqrt(tz) : 0.0;
    double nh[3];
    for (int d = 0; d < 3; ++d) nh[d] = t1 * T1[d] + t2 * T2[d] + tz * vh[d];
    double ne[3] = {alpha * nh[0], alpha * nh[1], nh[2] > 0.0 ? nh[2] : 0.0};
    double en = sqrt(dot3(ne, ne));
    for (int d = 0; d < 3; ++d) ne[d] /= en;
    double vn = dot3(vl, ne);
    double ll[3];
    for (int d = 0; d < 3; ++d) ll[d] = 2.0 * vn * ne[d] - vl[d];
    for (int d = 0; d < 3; ++d) l[d] = ll[0] * t[d] + ll[1] * b[d] + ll[2] * n[d];
}

/* stratified uniforms of sample k out of M (same strata as the cosine sampler) */
static void strat_uniforms(uint64_t seed, uint32_t pid, uint32_t k, uint32_t tag, int M, double *s1, double *s2)
{
    double u1, u2;
    uniforms(seed, pid, 0u, k, tag, &u1, &u2);
    int na = 1 << (ilog2(M) / 2);
    int nb = M / na;
    *s1 = ((int)k / nb + u1) / na;
    *s2 = ((int)k % nb + u2) / nb;
}

/* direction i of a primary point under MIS: returns w and the scalar
   2 (n.w) / (p_env + p_ggx) that multiplies f_r (0 below the horizon, and 0
   in the measure-zero case where both densities vanish) */
static double mis_direction(const env_dist *D, const or_sampling *S, uint32_t pid, int i, const double n[3],
                            const double v[3], double r, double w[3])
{
    const int M = S->n_dirs / 2;
    double s1, s2;
    if (i < M) {
        strat_uniforms(S->seed, pid, (uint32_t)i, 2u, M, &s1, &s2);
        double pe = env_sample(D, s1, s2, w);
        double nl = dot3(n, w), den = pe + ggx_density(n, v, r, w);
        return (nl > 0.0 && den > 0.0) ? 2.0 * nl / den : 0.0;
    }
    strat_uniforms(S->seed, pid, (uint32_t)(i - M), 3u, M, &s1, &s2);
    ggx_sample(n, v, r, s1, s2, w);
    double nl = dot3(n, w), den = env_density(D, w) + ggx_density(n, v, r, w);
    return (nl > 0.0 && den > 0.0) ? 2.0 * nl / den : 0.0;
}

void or_env_dist(const or_env *E, double *ct, double *marg, double *cond, double *dens)
{
    env_dist D;
    env_dist_build(E, &D);
    const int H = E->H, W = E->W;
    memcpy(ct, D.ct, (size_t)(H + 1) * sizeof(double));
    memcpy(marg, D.marg, (size_t)(H + 1) * sizeof(double));
    memcpy(cond, D.cond, (size_t)H * (W + 1) * sizeof(double));
    memcpy(dens, D.dens, (size_t)H * W * sizeof(double));
    env_dist_free(&D);
}

void or_env_sample(const or_env *E, const double *s, int64_t n, double *w, double *pdf)
{
    env_dist D;
    env_dist_build(E, &D);
    for (int64_t i = 0; i < n; ++i) pdf[i] = env_sample(&D, s[2 * i], s[2 * i + 1], w + 3 * i);
    env_dist_free(&D);
}

void or_env_density(const or_env *E, const double *w, int64_t n, double *pdf)
{
    env_dist D;
    env_dist_build(E, &D);
    for (int64_t i = 0; i < n; ++i) pdf[i] = env_density(&D, w + 3 * i);
    env_dist_free(&D);
}

void or_ggx_sample(const double *n, const double *v, const double *r, const double *s, int64_t cnt, double *l)
{
    for (int64_t i = 0; i < cnt; ++i) ggx_sample(n + 3 * i, v + 3 * i, r[i], s[2 * i], s[2 * i + 1], l + 3 * i);
}

void or_ggx_density(const double *n, const double *v, const double *r, const double *l, int64_t cnt, double *pdf)
{
    for (int64_t i = 0; i < cnt; ++i) pdf[i] = ggx_density(n + 3 * i, v + 3 * i, r[i], l + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Incoming radiance along (x, w): Eq. (2).                                 */
/*   V, d from I(f(x), w); x' = x + t w (Sec. 3.1).                          */
/*   Bounce (Sec. 3.2 "Overview"): f' = H(x'), (a', r', m') = B(f'), N'     */
/*   new directions about n' with visibility V'_j = sigmoid(I(f', w'_j)_0); */
/*   L'_o = 1/N' sum_j pi f_r(n', v', w'_j) V'_j L_env(w'_j).               */
/*   Reading: a 5-output decoder has no normal head, so the secondary       */
/*   surface faces the tracer, n' = v' = -w; an 8-output decoder (the       */
/*   paper's model shape, Sec. 3.2) gives n' = o[5..7]/|o[5..7]| (the       */
/*   facing normal if that vector is zero) with view v' = -w.  Visibility   */
/*   is used soft (sigmoid) in Eq. (2) and the bounce is evaluated for every */
/*   direction, weighted by (1 - V).                                        */
/*   L_in = V L_env(w) + (1 - V) L'_o; direct-only: L_in = V L_env(w).       */
/* ------------------------------------------------------------------------ */
static void incoming(const or_model *M, const or_env *E, const or_sampling *S, int indirect,
                     const double *f, const float *x, const double w[3], uint32_t pid, uint32_t q,
                     double Lin[3], double *V, double *dep)
{
    const or_grid *g = &M->grid;
    const int nf = g->L * g->F;
    double z[OR_MAXIN], h1[OR_MAXH], h2[OR_MAXH], o[OR_MAXOUT];
    for (int i = 0; i < nf; ++i) z[i] = f[i];
    z[nf] = w[0]; z[nf + 1] = w[1]; z[nf + 2] = w[2];
    mlp_fwd(&M->irt, z, h1, h2, o);
    const int hard = (S->flags & OR_HARD_VIS) != 0;
    /* hard visibility (Sec. 3.2 "Overview"): v = 1 when sigmoid(o0) > 1/2 */
    double vis = hard ? (o[0] > 0.0 ? 1.0 : 0.0) : sigmoid(o[0]);
    double sp = softplus(o[1]);
    double d = sp < 1.0 ? sp : 1.0;
    double t = M->t_near + (M->t_far - M->t_near) * d;
    double Le[3];
    env_lookup(E, w, Le);
    *V = vis;
    *dep = d;
    if (!indirect || (hard && vis == 1.0)) {
        /* direct only, or a visible ray under hard visibility: no bounce */
        for (int c = 0; c < 3; ++c) Lin[c] = vis * Le[c];
        return;
    }
    double xb[3], u[3], fb[OR_MAXF], ob[OR_MAXOUT];
    for (int k = 0; k < 3; ++k) xb[k] = (double)x[k] + t * w[k];
    pos_to_u_f64(g, xb, u);
    encode_u(g, u, fb, NULL);
    mlp_fwd(&M->brdf, fb, h1, h2, ob);
    double ab[3] = {sigmoid(ob[0]), sigmoid(ob[1]), sigmoid(ob[2])};
    double rb = 0.09 + 0.91 * sigmoid(ob[3]);
    double mb = sigmoid(ob[4]);
    /* secondary view -w; normal: the decoder's normal head n/|n| when it has
       one (outputs 5..7), else the facing normal -w (reading, see above) */
    double vb[3] = {-w[0], -w[1], -w[2]};
    double nb[3] = {-w[0], -w[1], -w[2]};
    if (M->brdf.n_out >= 8) {
        double nn = sqrt(ob[5] * ob[5] + ob[6] * ob[6] + ob[7] * ob[7]);
        if (nn > 0.0)
            for (int k = 0; k < 3; ++k) nb[k] = ob[5 + k] / nn;
    }
    double Lo[3] = {0, 0, 0};
    const int N2 = S->n_dirs2;
    for (int j = 0; j < N2; ++j) {
        double wj[3], Ej[3], fr[3], t1[3], t2[3], t3[3];
        sample_dir(S->seed, pid, q, (uint32_t)j, 1u, N2, nb, wj);
        for (int i = 0; i < nf; ++i) z[i] = fb[i];
        z[nf] = wj[0]; z[nf + 1] = wj[1]; z[nf + 2] = wj[2];
        mlp_fwd(&M->irt, z, h1, h2, o);
        /* hard visibility: only visible secondary rays contribute */
        double vj = hard ? (o[0] > 0.0 ? 1.0 : 0.0) : sigmoid(o[0]);
        env_lookup(E, wj, Ej);
        brdf_eval(nb, vb, wj, ab, rb, mb, M->f0, (S->flags & OR_DIFFUSE_ONLY) != 0, fr, t1, t2, t3);
        for (int c = 0; c < 3; ++c) Lo[c] += M_PI * fr[c] * vj * Ej[c];
    }
    for (int c = 0; c < 3; ++c) {
        Lo[c] /= N2;
        Lin[c] = vis * Le[c] + (1.0 - vis) * Lo[c];
    }
}

/* ------------------------------------------------------------------------ */
/* Rendering.                                                               */
/* Shade mode (P->dir == NULL): Eq. (1) at each primary point with N        */
/* cosine-distributed directions; with pdf = cos/pi every sample carries    */
/* the weight pi f_r.  (a, r, m) = B(H(x)), normal and view from the input. */
/* With OR_MIS the N directions and their weights come from mis_direction. */
/*   rgb[p] = 1/N sum_i pi f_r(n, w_o, w_i) L_in(x, w_i);                    */
/*   vis/depth (optional) [p][N] hold V and d of each direction.            */
/* Query mode (P->dir != NULL): rgb[p] = L_in(x_p, dir_p), vis[p] = V,       */
/*   depth[p] = d (the distillation outputs, Sec. 3.3).                      */
/* ------------------------------------------------------------------------ */
/* Returns 0, or -1 without touching the outputs when a required pointer is
 * NULL (shade mode needs nrm and wo). */
int32_t or_render(const or_model *M, const or_env *E, const or_sampling *S, const or_points *P,
                  int32_t indirect, double *rgb, double *vis, double *depth)
{
    if (!M || !E || !S || !P || !rgb || (P->n > 0 && !P->pos)) return -1;
    if (P->n > 0 && !P->dir && (!P->nrm || !P->wo)) return -1;
    if (!M->grid.table || !E->rgb) return -1;
    const or_grid *g = &M->grid;
    const int nf = g->L * g->F;
    const int query = P->dir != NULL;
    const int mis = !query && (S->flags & OR_MIS) != 0;
    env_dist D;
    if (mis) env_dist_build(E, &D);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < P->n; ++p) {
        double f[OR_MAXF], u[3];
        const float *x = P->pos + 3 * p;
        pos_to_u_f32(g, x, u);
        encode_u(g, u, f, NULL);
        if (query) {
            double w[3] = {P->dir[3 * p], P->dir[3 * p + 1], P->dir[3 * p + 2]};
            double Lin[3], V, d;
            incoming(M, E, S, indirect, f, x, w, point_id(P, p), 0u, Lin, &V, &d);
            for (int c = 0; c < 3; ++c) rgb[3 * p + c] = Lin[c];
            if (vis) vis[p] = V;
            if (depth) depth[p] = d;
            continue;
        }
        double h1[OR_MAXH], h2[OR_MAXH], ob[OR_MAXOUT];
        mlp_fwd(&M->brdf, f, h1, h2, ob);
        double a[3] = {sigmoid(ob[0]), sigmoid(ob[1]), sigmoid(ob[2])};
        double r = 0.09 + 0.91 * sigmoid(ob[3]);
        double m = sigmoid(ob[4]);
        double n[3] = {P->nrm[3 * p], P->nrm[3 * p + 1], P->nrm[3 * p + 2]};
        double v[3] = {P->wo[3 * p], P->wo[3 * p + 1], P->wo[3 * p + 2]};
        double Lo[3] = {0, 0, 0};
        const int N = S->n_dirs;
        for (int i = 0; i < N; ++i) {
            double w[3], Lin[3], V, d, fr[3], t1[3], t2[3], t3[3];
            double wt = M_PI; /* cosine sampling: pi f_r per sample */
            if (mis)
                wt = mis_direction(&D, S, point_id(P, p), i, n, v, r, w);
            else
                sample_dir(S->seed, point_id(P, p), 0u, (uint32_t)i, 0u, N, n, w);
            incoming(M, E, S, indirect, f, x, w, point_id(P, p), (uint32_t)i, Lin, &V, &d);
            brdf_eval(n, v, w, a, r, m, M->f0, (S->flags & OR_DIFFUSE_ONLY) != 0, fr, t1, t2, t3);
            for (int c = 0; c < 3; ++c) Lo[c] += wt * fr[c] * Lin[c];
            if (vis) vis[p * N + i] = V;
            if (depth) depth[p * N + i] = d;
        }
        for (int c = 0; c < 3; ++c) rgb[3 * p + c] = Lo[c] / N;
    }
    if (mis) env_dist_free(&D);
    (void)nf;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* L2 distillation loss (reading of Sec. 3.3 with squared errors):          */
/*   loss = 1/n sum_p [ sum_c (rgb - t_c)^2 + (vis - t_3)^2 + (d - t_4)^2 ]  */
/* Returns the loss; writes its gradient with respect to each prediction.   */
/* ------------------------------------------------------------------------ */
double or_l2_loss(const float *rgb, const float *vis, const float *dep, const float *tgt, int64_t n,
                  double *g_rgb, double *g_vis, double *g_dep)
{
    double loss = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        for (int c = 0; c < 3; ++c) {
            double e = (double)rgb[3 * p + c] - tgt[5 * p + c];
            loss += e * e;
            if (g_rgb) g_rgb[3 * p + c] = 2.0 * e / n;
        }
        double ev = (double)vis[p] - tgt[5 * p + 3];
        double ed = (double)dep[p] - tgt[5 * p + 4];
        loss += ev * ev + ed * ed;
        if (g_vis) g_vis[p] = 2.0 * ev / n;
        if (g_dep) g_dep[p] = 2.0 * ed / n;
    }
    return loss / n;
}

/* ------------------------------------------------------------------------ */
/* Analytic backward of query mode (the distillation forward).              */
/* Given upstream gradients of rgb (L_in), vis (V) and depth (d), adds the  */
/* gradients with respect to the tables g_table [L][T][F], the decoder      */
/* g_brdf and the tracer g_irt (each packed W0,b0,W1,b1,W2,b2) and,          */
/* optionally, writes d/dx into g_pos [n][3].                               */
/* Chain: L_in = V Le + (1-V) L'_o; L'_o depends on (a',r',m') = B(H(x')),   */
/* on V'_j = sigmoid(I(H(x'), w'_j)_0) and, through x' = x + t w with       */
/* t = near + (far-near) min(softplus(o1), 1), on o1 of I(H(x), w).          */
/* The clamps pass no gradient where active (softplus >= 1, u outside       */
/* (0,1)); the bounce directions depend only on w, which is an input.       */
/* ------------------------------------------------------------------------ */
static void scatter_table(const or_grid *g, const enc_rec *rec, const double *gf, double *g_table)
{
    const uint32_t T = 1u << g->log2_T;
    for (int l = 0; l < g->L; ++l) {
        const double *w = rec->w[l];
        for (int corner = 0; corner < 8; ++corner) {
            int dx = corner & 1, dy = (corner >> 1) & 1, dz = (corner >> 2) & 1;
            double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
            size_t base = ((size_t)l * T + rec->idx[l][corner]) * g->F;
            for (int k = 0; k < g->F; ++k) {
                double v = wt * gf[l * g->F + k];
#pragma omp atomic
                g_table[base + k] += v;
            }
        }
    }
}

/* d/dx of the encoding contracted with gf (position gradient). */
static void encode_dx(const or_grid *g, const enc_rec *rec, const double *gf, double gx[3])
{
    const uint32_t T = 1u << g->log2_T;
    gx[0] = gx[1] = gx[2] = 0.0;
    for (int l = 0; l < g->L; ++l) {
        const double *w = rec->w[l];
        double scale = g->res[l] / g->extent;
        for (int corner = 0; corner < 8; ++corner) {
            int dl[3] = {corner & 1, (corner >> 1) & 1, (corner >> 2) & 1};
            double fac[3], dfac[3];
            for (int d = 0; d < 3; ++d) {
                fac[d] = dl[d] ? w[d] : 1.0 - w[d];
                dfac[d] = dl[d] ? 1.0 : -1.0;
            }
            const float *e = g->table + ((size_t)l * T + rec->idx[l][corner]) * g->F;
            double ge = 0.0;
            for (int k = 0; k < g->F; ++k) ge += gf[l * g->F + k] * (double)e[k];
            gx[0] += ge * dfac[0] * fac[1] * fac[2] * scale;
            gx[1] += ge * fac[0] * dfac[1] * fac[2] * scale;
            gx[2] += ge * fac[0] * fac[1] * dfac[2] * scale;
        }
    }
    for (int d = 0; d < 3; ++d)
        if (!rec->inside[d]) gx[d] = 0.0;
}

/* Query mode only.  Returns 0, or -1 without touching the outputs when a
 * required pointer is NULL (g_pos may be NULL). */
int32_t or_backward(const or_model *M, const or_env *E, const or_sampling *S, const or_points *P,
                    int32_t indirect, const float *g_rgb, const float *g_vis, const float *g_dep,
                    double *g_table, double *g_brdf, double *g_irt, double *g_pos)
{
    if (!M || !E || !S || !P || !g_rgb || !g_vis || !g_dep || !g_table || !g_brdf || !g_irt) return -1;
    if (P->n > 0 && (!P->pos || !P->dir)) return -1;
    if (!M->grid.table || !E->rgb) return -1;
    const or_grid *g = &M->grid;
    const int nf = g->L * g->F;
    const int64_t nb_par = mlp_nparams(&M->brdf), ni_par = mlp_nparams(&M->irt);
    const double span = M->t_far - M->t_near;
    const int diffuse = (S->flags & OR_DIFFUSE_ONLY) != 0;
#pragma omp parallel
    {
        double *lb = (double *)calloc((size_t)nb_par, sizeof(double));
        double *li = (double *)calloc((size_t)ni_par, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < P->n; ++p) {
            const float *x = P->pos + 3 * p;
            double w[3] = {P->dir[3 * p], P->dir[3 * p + 1], P->dir[3 * p + 2]};
            double u[3], f[OR_MAXF], z[OR_MAXIN], h1[OR_MAXH], h2[OR_MAXH], o[OR_MAXOUT];
            enc_rec rx, rb;
            pos_to_u_f32(g, x, u);
            encode_u(g, u, f, &rx);
            for (int i = 0; i < nf; ++i) z[i] = f[i];
            z[nf] = w[0]; z[nf + 1] = w[1]; z[nf + 2] = w[2];
            mlp_fwd(&M->irt, z, h1, h2, o);
            double V = sigmoid(o[0]);
            double sp = softplus(o[1]);
            double d = sp < 1.0 ? sp : 1.0;
            double t = M->t_near + span * d;
            double Le[3];
            env_lookup(E, w, Le);
            double G[3] = {g_rgb[3 * p], g_rgb[3 * p + 1], g_rgb[3 * p + 2]};
            double gV = g_vis[p], gd = g_dep[p];
            double gxb[3] = {0, 0, 0};
            if (indirect) {
                double xb[3], ub[3], fb[OR_MAXF], hb1[OR_MAXH], hb2[OR_MAXH], ob[OR_MAXOUT];
                for (int k = 0; k < 3; ++k) xb[k] = (double)x[k] + t * w[k];
                pos_to_u_f64(g, xb, ub);
                encode_u(g, ub, fb, &rb);
                mlp_fwd(&M->brdf, fb, hb1, hb2, ob);
                double ab[3] = {sigmoid(ob[0]), sigmoid(ob[1]), sigmoid(ob[2])};
                double s3 = sigmoid(ob[3]);
                double rr = 0.09 + 0.91 * s3;
                double mb = sigmoid(ob[4]);
                double nbv[3] = {-w[0], -w[1], -w[2]};
                const int N2 = S->n_dirs2;
                double wj[OR_MAXN2][3], Ej[OR_MAXN2][3], cj[OR_MAXN2][3], Vj[OR_MAXN2];
                double dca[OR_MAXN2][3], dcr[OR_MAXN2][3], dcm[OR_MAXN2][3];
                double Lo[3] = {0, 0, 0};
                for (int j = 0; j < N2; ++j) {
                    sample_dir(S->seed, point_id(P, p), 0u, (uint32_t)j, 1u, N2, nbv, wj[j]);
                    for (int i = 0; i < nf; ++i) z[i] = fb[i];
                    z[nf] = wj[j][0]; z[nf + 1] = wj[j][1]; z[nf + 2] = wj[j][2];
                    mlp_fwd(&M->irt, z, h1, h2, o);
                    Vj[j] = sigmoid(o[0]);
                    env_lookup(E, wj[j], Ej[j]);
                    double fr[3];
                    brdf_eval(nbv, nbv, wj[j], ab, rr, mb, M->f0, diffuse, fr, dca[j], dcr[j], dcm[j]);
                    for (int c = 0; c < 3; ++c) {
                        cj[j][c] = M_PI * fr[c];
                        dca[j][c] *= M_PI;
                        dcr[j][c] *= M_PI;
                        dcm[j][c] *= M_PI;
                        Lo[c] += cj[j][c] * Vj[j] * Ej[j][c];
                    }
                }
                for (int c = 0; c < 3; ++c) Lo[c] /= N2;
                for (int c = 0; c < 3; ++c) gV += G[c] * (Le[c] - Lo[c]);
                double gLo[3] = {(1.0 - V) * G[0], (1.0 - V) * G[1], (1.0 - V) * G[2]};
                double gfb[OR_MAXF], gz[OR_MAXIN];
                for (int i = 0; i < nf; ++i) gfb[i] = 0.0;
                double ga[3] = {0, 0, 0}, gr = 0.0, gm = 0.0;
                for (int j = 0; j < N2; ++j) {
                    double gvj = 0.0;
                    for (int c = 0; c < 3; ++c) gvj += gLo[c] * cj[j][c] * Ej[j][c];
                    gvj /= N2;
                    double go[OR_MAXOUT] = {0};
                    go[0] = gvj * Vj[j] * (1.0 - Vj[j]);
                    /* recompute the tracer activations at (f', w'_j) */
                    for (int i = 0; i < nf; ++i) z[i] = fb[i];
                    z[nf] = wj[j][0]; z[nf + 1] = wj[j][1]; z[nf + 2] = wj[j][2];
                    mlp_fwd(&M->irt, z, h1, h2, o);
                    mlp_bwd(&M->irt, z, h1, h2, go, li, gz);
                    for (int i = 0; i < nf; ++i) gfb[i] += gz[i];
                    for (int c = 0; c < 3; ++c) {
                        double gc = gLo[c] * Vj[j] * Ej[j][c] / N2;
                        ga[c] += gc * dca[j][c];
                        gr += gc * dcr[j][c];
                        gm += gc * dcm[j][c];
                    }
                }
                double gob[OR_MAXOUT] = {0};
                for (int c = 0; c < 3; ++c) gob[c] = ga[c] * ab[c] * (1.0 - ab[c]);
                gob[3] = gr * 0.91 * s3 * (1.0 - s3);
                gob[4] = gm * mb * (1.0 - mb);
                mlp_bwd(&M->brdf, fb, hb1, hb2, gob, lb, gz);
                for (int i = 0; i < nf; ++i) gfb[i] += gz[i];
                scatter_table(g, &rb, gfb, g_table);
                encode_dx(g, &rb, gfb, gxb);
                double gt = gxb[0] * w[0] + gxb[1] * w[1] + gxb[2] * w[2];
                gd += span * gt;
            } else {
                for (int c = 0; c < 3; ++c) gV += G[c] * Le[c];
            }
            /* tracer at (f(x), w) */
            for (int i = 0; i < nf; ++i) z[i] = f[i];
            z[nf] = w[0]; z[nf + 1] = w[1]; z[nf + 2] = w[2];
            mlp_fwd(&M->irt, z, h1, h2, o);
            double go[OR_MAXOUT] = {0};
            go[0] = gV * V * (1.0 - V);
            go[1] = sp < 1.0 ? gd * sigmoid(o[1]) : 0.0;
            double gz[OR_MAXIN];
            mlp_bwd(&M->irt, z, h1, h2, go, li, gz);
            scatter_table(g, &rx, gz, g_table);
            if (g_pos) {
                double gx[3];
                encode_dx(g, &rx, gz, gx);
                for (int k = 0; k < 3; ++k) g_pos[3 * p + k] = gx[k] + gxb[k];
            }
        }
#pragma omp critical
        {
            for (int64_t i = 0; i < nb_par; ++i) g_brdf[i] += lb[i];
            for (int64_t i = 0; i < ni_par; ++i) g_irt[i] += li[i];
        }
        free(lb);
        free(li);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adam (Kingma & Ba 2015) with bias correction; weight decay added to the  */
/* gradient (L2 form).  One step t >= 1 over n parameters, in FP64.         */
/* ------------------------------------------------------------------------ */
void or_adam(double *param, const double *grad, double *m, double *v, int64_t n, int32_t step,
             double lr, double b1, double b2, double eps, double wd)
{
    double bc1 = 1.0 - pow(b1, step), bc2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        double gi = grad[i] + wd * param[i];
        m[i] = b1 * m[i] + (1.0 - b1) * gi;
        v[i] = b2 * v[i] + (1.0 - b2) * gi * gi;
        double mh = m[i] / bc1, vh = v[i] / bc2;
        param[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Spatial variance-guided a-trous filter (SVGF, Schied et al. 2017) without */
/* its temporal parts, as the paper applies it to the MC result (Sec. 4.1);  */
/* the clip-space depth gradient is a finite difference of the depth map    */
/* (supplementary "Rendering Details").  Readings:                          */
/*  - luminance l = 0.2126 R + 0.7152 G + 0.0722 B;                          */
/*  - initial variance: unweighted 7x7 moments, var = E[l^2] - E[l]^2,       */
/*    over the taps inside the image;                                       */
/*  - depth gradient: forward differences z(x+1,y)-z(x,y), z(x,y+1)-z(x,y)   */
/*    (backward at the last column/row, zero along an axis one pixel long); */
/*  - iteration k (k = 0..iters-1) uses step 2^k and the 5x5 B3-spline taps  */
/*    h = (1/16, 1/4, 3/8, 1/4, 1/16); taps outside the image are skipped;  */
/*  - weights w = h h * exp(-|z_p - z_q| / (sz |grad z_p . (p-q)| + 1e-6))   */
/*              * max(0, n_p . n_q)^sn                                       */
/*              * exp(-|l_p - l_q| / (sl sqrt(g3(var)_p) + 1e-10)),          */
/*    g3 = 3x3 binomial blur (1,2,1)/4 x (1,2,1)/4 of the variance (edges    */
/*    clamped);                                                             */
/*  - colour c' = sum w c / sum w, variance var' = sum w^2 var / (sum w)^2.  */
/* Inputs rgb [H][W][3], depth [H][W], nrm [H][W][3]; output [H][W][3].      */
/* ------------------------------------------------------------------------ */
static double lum(const double *c) { return 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]; }

void or_denoise(const float *rgb, const float *depth, const float *nrm, int32_t H, int32_t W, int32_t iters,
                double sz, double sn, double sl, double *out, double *var_out)
{
    const size_t P = (size_t)H * W;
    double *c = (double *)malloc(P * 3 * sizeof(double));
    double *c2 = (double *)malloc(P * 3 * sizeof(double));
    double *var = (double *)malloc(P * sizeof(double));
    double *var2 = (double *)malloc(P * sizeof(double));
    double *gx = (double *)malloc(P * sizeof(double));
    double *gy = (double *)malloc(P * sizeof(double));
    double *g3 = (double *)malloc(P * sizeof(double));
    for (size_t i = 0; i < 3 * P; ++i) c[i] = rgb[i];
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            gx[p] = x + 1 < W ? (double)depth[p + 1] - depth[p] : (x > 0 ? (double)depth[p] - depth[p - 1] : 0.0);
            gy[p] = y + 1 < H ? (double)depth[p + W] - depth[p] : (y > 0 ? (double)depth[p] - depth[p - W] : 0.0);
            double s1 = 0, s2 = 0;
            int cnt = 0;
            for (int dy = -3; dy <= 3; ++dy)
                for (int dx = -3; dx <= 3; ++dx) {
                    int xx = x + dx, yy = y + dy;
                    if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                    double l = lum(c + 3 * ((size_t)yy * W + xx));
                    s1 += l;
                    s2 += l * l;
                    ++cnt;
                }
            double m = s1 / cnt, v = s2 / cnt - m * m;
            var[p] = v > 0 ? v : 0;
        }
    static const double h[5] = {1.0 / 16, 1.0 / 4, 3.0 / 8, 1.0 / 4, 1.0 / 16};
    for (int it = 0; it < iters; ++it) {
        const int step = 1 << it;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double s = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int xx = x + dx < 0 ? 0 : (x + dx >= W ? W - 1 : x + dx);
                        int yy = y + dy < 0 ? 0 : (y + dy >= H ? H - 1 : y + dy);
                        s += (dx ? 0.25 : 0.5) * (dy ? 0.25 : 0.5) * var[(size_t)yy * W + xx];
                    }
                g3[(size_t)y * W + x] = s;
            }
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t p = (size_t)y * W + x;
                double lp = lum(c + 3 * p), zp = depth[p];
                const float *np = nrm + 3 * p;
                double ws = 0, acc[3] = {0, 0, 0}, vacc = 0;
                double lden = sl * sqrt(g3[p] > 0 ? g3[p] : 0) + 1e-10;
                for (int j = -2; j <= 2; ++j)
                    for (int i = -2; i <= 2; ++i) {
                        int xx = x + i * step, yy = y + j * step;
                        if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                        size_t q = (size_t)yy * W + xx;
                        double zq = depth[q];
                        double wz = exp(-fabs(zp - zq) / (sz * fabs(gx[p] * i * step + gy[p] * j * step) + 1e-6));
                        double nd = (double)np[0] * nrm[3 * q] + (double)np[1] * nrm[3 * q + 1] +
                                    (double)np[2] * nrm[3 * q + 2];
                        double wn = pow(nd > 0 ? nd : 0, sn);
                        double wl = exp(-fabs(lp - lum(c + 3 * q)) / lden);
                        double w = h[i + 2] * h[j + 2] * wz * wn * wl;
                        ws += w;
                        for (int k = 0; k < 3; ++k) acc[k] += w * c[3 * q + k];
                        vacc += w * w * var[q];
                    }
                for (int k = 0; k < 3; ++k) c2[3 * p + k] = acc[k] / ws;
                var2[p] = vacc / (ws * ws);
            }
        double *t = c; c = c2; c2 = t;
        t = var; var = var2; var2 = t;
    }
    for (size_t i = 0; i < 3 * P; ++i) out[i] = c[i];
    if (var_out)
        for (size_t i = 0; i < P; ++i) var_out[i] = var[i];
    free(c); free(c2); free(var); free(var2); free(gx); free(gy); free(g3);
}
