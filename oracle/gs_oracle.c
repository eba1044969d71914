/*
 * CPU oracle for the underwater Gaussian rasterizer -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the HIP renderer: it is a plain, slow,
 * brute-force evaluation of what the renderer computes, in FP64, with no tiles.
 *
 * What it computes (paper sections cited by name):
 *   - Preliminaries / 3DGS: a scene is N anisotropic Gaussians (mean, covariance
 *     factored as rotation x scale, SH colour, opacity); a pixel's colour is
 *     the front-to-back alpha composite of eq. (3dgs_orig) over the Gaussians
 *     sorted by increasing depth, with alpha from eq. (opacity_impact) evaluated
 *     on the 2D affine (EWA) projection of the covariance.
 *   - Direct Rendering for Underwater Scenes, eq. (3dgs_uw): the composite is
 *     attenuated by exp(-B_d z) and backscatter B_inf (1 - exp(-B_b z)) is added,
 *     per colour channel.
 *   - Estimating Dense Depth Maps, eq. (Depth): z is the alpha-weighted mean
 *     depth of the contributors; Implementation section: optional logistic map
 *     z = 2/(1+exp(-0.1 zhat)) - 1, either inside the medium term or only on the
 *     depth image shown for visualisation.
 *   - eq. (scattering_approx): the clean image J is the in-air composite C_air
 *     before attenuation; it is an output with its own upstream gradient.
 *   - Appendix "Partial Derivatives": gradients of the medium terms.  The
 *     oracle's backward is the exact derivative of its own forward (the printed
 *     appendix omits the factor z in dL/dB_d and dL/dB_b and the dependence of
 *     z on alpha); it is pinned against FP64 central differences.
 *
 * Discrete rules the paper inherits from 3DGS without stating them (readings):
 *   alpha = min(alpha_max, o exp(-q/2)); a Gaussian with alpha < alpha_min is
 *   skipped; the walk stops before blending a Gaussian that would bring the
 *   transmittance below t_min; EWA dilation eps on the diagonal of the 2D
 *   covariance; Gaussians with view depth <= near are culled; pixel centres at
 *   (u + 1/2, v + 1/2); ties in depth order broken by Gaussian index; colour =
 *   max(0, 1/2 + sum_lm Y_lm(dir) k_lm); empty pixels (no contributor) sit at
 *   infinite range (backscatter B_inf where B_b > 0, else 0; z := 1 in
 *   logistic mode).
 *
 * Depth order and culling use the FP32 view depth produced by the key path
 * (orc_key_path), an exact FP32 sequence with no fused multiply-adds that the
 * renderer reproduces bit for bit; everything else is FP64.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];   /* world -> camera rotation, row-major */
    float t[3];   /* world -> camera translation */
    float near_z;
} orc_cam;

typedef struct {
    int32_t tile_w, tile_h;
    int32_t depth_mode;   /* 0: metric zhat; 1: logistic 2/(1+e^{-0.1 zhat}) - 1 */
    int32_t sh_degree;
    float kappa_f32;      /* extent factor used by the FP32 key path */
    float dilation_f32;   /* EWA dilation as the FP32 key path sees it */
    double alpha_min, alpha_max, t_min, dilation;
    double band;          /* relative margin under which a decision is "ambiguous" */
    int32_t depth_output; /* depth image: 0 = the z the medium uses; 1 = logistic map of zhat */
} orc_opts;

/* ------------------------------------------------------------------------ */
/* FP32 key path: view depth, culling and tile rectangle.                    */
/* The exact operation order is part of the specification: every product and */
/* sum is a separately rounded FP32 op (no FMA), divisions and square roots   */
/* are IEEE correctly rounded.                                               */
/* ------------------------------------------------------------------------ */
static int finitef_(float v) { return isfinite(v) ? 1 : 0; }

void orc_key_path(int64_t n, const double* means, const double* scales, const double* quats,
                  const orc_cam* cam, const orc_opts* o,
                  uint32_t* depth_bits, int32_t* rect, uint8_t* culled)
{
    const float* Rv = cam->R;
    const float* tv = cam->t;
    const int tiles_x = (cam->width + o->tile_w - 1) / o->tile_w;
    const int tiles_y = (cam->height + o->tile_h - 1) / o->tile_h;
    const float inv_tw = 1.0f / (float)o->tile_w;
    const float inv_th = 1.0f / (float)o->tile_h;
    for (int64_t i = 0; i < n; ++i) {
        float mx = (float)means[3 * i + 0], my = (float)means[3 * i + 1], mz = (float)means[3 * i + 2];
        float s0 = (float)scales[3 * i + 0], s1 = (float)scales[3 * i + 1], s2 = (float)scales[3 * i + 2];
        float qw = (float)quats[4 * i + 0], qx = (float)quats[4 * i + 1];
        float qy = (float)quats[4 * i + 2], qz = (float)quats[4 * i + 3];
        rect[4 * i + 0] = 0; rect[4 * i + 1] = 0; rect[4 * i + 2] = -1; rect[4 * i + 3] = -1;
        depth_bits[i] = 0xFFFFFFFFu;
        culled[i] = 1;

        float tx = ((Rv[0] * mx + Rv[1] * my) + Rv[2] * mz) + tv[0];
        float ty = ((Rv[3] * mx + Rv[4] * my) + Rv[5] * mz) + tv[1];
        float tz = ((Rv[6] * mx + Rv[7] * my) + Rv[8] * mz) + tv[2];
        float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
        if (!(tz > cam->near_z) || !(n2 > 0.0f) || !finitef_(tx) || !finitef_(ty) ||
            !finitef_(s0) || !finitef_(s1) || !finitef_(s2) || !finitef_(n2))
            continue;
        float nrm = sqrtf(n2);
        float w = qw / nrm, x = qx / nrm, y = qy / nrm, z = qz / nrm;
        float xx = x * x, yy = y * y, zz = z * z;
        float xy = x * y, xz = x * z, yz = y * z;
        float wx = w * x, wy = w * y, wz = w * z;
        float Q[9];
        Q[0] = 1.0f - 2.0f * (yy + zz); Q[1] = 2.0f * (xy - wz);        Q[2] = 2.0f * (xz + wy);
        Q[3] = 2.0f * (xy + wz);        Q[4] = 1.0f - 2.0f * (xx + zz); Q[5] = 2.0f * (yz - wx);
        Q[6] = 2.0f * (xz - wy);        Q[7] = 2.0f * (yz + wx);        Q[8] = 1.0f - 2.0f * (xx + yy);
        float M[9];
        for (int r = 0; r < 3; ++r) {
            M[3 * r + 0] = Q[3 * r + 0] * s0;
            M[3 * r + 1] = Q[3 * r + 1] * s1;
            M[3 * r + 2] = Q[3 * r + 2] * s2;
        }
        float V[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                V[3 * r + c] = (Rv[3 * r + 0] * M[c] + Rv[3 * r + 1] * M[3 + c]) + Rv[3 * r + 2] * M[6 + c];
        float u = tx / tz, v = ty / tz;
        float a = cam->fx / tz, b = cam->fy / tz;
        float T0[3], T1[3];
        for (int c = 0; c < 3; ++c) {
            T0[c] = a * (V[c] - u * V[6 + c]);
            T1[c] = b * (V[3 + c] - v * V[6 + c]);
        }
        float sxx = ((T0[0] * T0[0] + T0[1] * T0[1]) + T0[2] * T0[2]) + o->dilation_f32;
        float syy = ((T1[0] * T1[0] + T1[1] * T1[1]) + T1[2] * T1[2]) + o->dilation_f32;
        float px = cam->fx * u + cam->cx;
        float py = cam->fy * v + cam->cy;
        float ex = sqrtf(o->kappa_f32 * sxx);
        float ey = sqrtf(o->kappa_f32 * syy);
        if (!finitef_(px) || !finitef_(py) || !finitef_(ex) || !finitef_(ey))
            continue;
        float lx = floorf((px - ex) * inv_tw), hx = floorf((px + ex) * inv_tw);
        float ly = floorf((py - ey) * inv_th), hy = floorf((py + ey) * inv_th);
        float x0 = lx > 0.0f ? lx : 0.0f;
        float y0 = ly > 0.0f ? ly : 0.0f;
        float x1 = hx < (float)(tiles_x - 1) ? hx : (float)(tiles_x - 1);
        float y1 = hy < (float)(tiles_y - 1) ? hy : (float)(tiles_y - 1);
        culled[i] = 0;
        uint32_t bits;
        memcpy(&bits, &tz, 4);
        depth_bits[i] = bits;
        if (x0 <= x1 && y0 <= y1) {
            rect[4 * i + 0] = (int32_t)x0; rect[4 * i + 1] = (int32_t)y0;
            rect[4 * i + 2] = (int32_t)x1; rect[4 * i + 3] = (int32_t)y1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3, orthonormal on the unit sphere,     */
/* Condon-Shortley phase, index k = l^2 + l + m.  Written from the textbook   */
/* definition Y_lm = N_lm P_l^|m|(cos th) {cos m phi | sin |m| phi} as        */
/* polynomials in the unit direction (x, y, z).                               */
/* ------------------------------------------------------------------------ */
static void sh_basis(int deg, double x, double y, double z, double* Y, double* dY /* [16][3] or NULL */)
{
    const double pi = M_PI;
    const double c0 = 0.5 * sqrt(1.0 / pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = sqrt(15.0 / (4.0 * pi));
    const double c20 = sqrt(5.0 / (16.0 * pi));
    const double c22 = sqrt(15.0 / (16.0 * pi));
    const double c33 = sqrt(35.0 / (32.0 * pi));
    const double c32 = sqrt(105.0 / (4.0 * pi));
    const double c31 = sqrt(21.0 / (32.0 * pi));
    const double c30 = sqrt(7.0 / (16.0 * pi));
    const double c322 = sqrt(105.0 / (16.0 * pi));
    double d[16][3];
    memset(d, 0, sizeof(d));
    Y[0] = c0;
    if (deg >= 1) {
        Y[1] = -c1 * y; d[1][1] = -c1;
        Y[2] = c1 * z;  d[2][2] = c1;
        Y[3] = -c1 * x; d[3][0] = -c1;
    }
    if (deg >= 2) {
        Y[4] = c2a * x * y;           d[4][0] = c2a * y; d[4][1] = c2a * x;
        Y[5] = -c2a * y * z;          d[5][1] = -c2a * z; d[5][2] = -c2a * y;
        Y[6] = c20 * (3.0 * z * z - 1.0); d[6][2] = c20 * 6.0 * z;
        Y[7] = -c2a * x * z;          d[7][0] = -c2a * z; d[7][2] = -c2a * x;
        Y[8] = c22 * (x * x - y * y); d[8][0] = 2.0 * c22 * x; d[8][1] = -2.0 * c22 * y;
    }
    if (deg >= 3) {
        Y[9] = -c33 * y * (3.0 * x * x - y * y);
        d[9][0] = -c33 * 6.0 * x * y; d[9][1] = -c33 * (3.0 * x * x - 3.0 * y * y);
        Y[10] = c32 * x * y * z;
        d[10][0] = c32 * y * z; d[10][1] = c32 * x * z; d[10][2] = c32 * x * y;
        Y[11] = -c31 * y * (5.0 * z * z - 1.0);
        d[11][1] = -c31 * (5.0 * z * z - 1.0); d[11][2] = -c31 * 10.0 * y * z;
        Y[12] = c30 * (5.0 * z * z * z - 3.0 * z);
        d[12][2] = c30 * (15.0 * z * z - 3.0);
        Y[13] = -c31 * x * (5.0 * z * z - 1.0);
        d[13][0] = -c31 * (5.0 * z * z - 1.0); d[13][2] = -c31 * 10.0 * x * z;
        Y[14] = c322 * z * (x * x - y * y);
        d[14][0] = c322 * 2.0 * x * z; d[14][1] = -c322 * 2.0 * y * z; d[14][2] = c322 * (x * x - y * y);
        Y[15] = -c33 * x * (x * x - 3.0 * y * y);
        d[15][0] = -c33 * (3.0 * x * x - 3.0 * y * y); d[15][1] = c33 * 6.0 * x * y;
    }
    if (dY) memcpy(dY, d, sizeof(d));
}

void orc_sh_basis(int deg, int64_t n, const double* dirs, double* Y /* [n][16] */)
{
    for (int64_t i = 0; i < n; ++i) {
        double tmp[16] = {0};
        sh_basis(deg, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], tmp, NULL);
        memcpy(Y + 16 * i, tmp, sizeof(tmp));
    }
}

/* ------------------------------------------------------------------------ */
/* FP64 projection of one Gaussian into one view (Preliminaries: EWA).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double Rq[9], M[9], V[9], t[3];
    double a, b, c;        /* 2D covariance incl. dilation: [[a,b],[b,c]] */
    double det;
    double Q[3];           /* conic: Qxx, Qxy, Qyy */
    double m[2], d;
    double qhat[4], qnorm;
    double dir[3], vnorm;
    double Y[16];
    double color[3];
    int clamp[3];
} proj64;

static void quat_rot(const double* qh, double* R)
{
    double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void project_one(const double* mu, const double* s, const double* q, const double* sh, int deg,
                        int64_t stride_sh, const orc_cam* cam, const orc_opts* o, proj64* P)
{
    double Rv[9], tv[3];
    for (int k = 0; k < 9; ++k) Rv[k] = cam->R[k];
    for (int k = 0; k < 3; ++k) tv[k] = cam->t[k];
    P->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) P->qhat[k] = q[k] / P->qnorm;
    quat_rot(P->qhat, P->Rq);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) P->M[3 * r + c] = P->Rq[3 * r + c] * s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            P->V[3 * r + c] = Rv[3 * r] * P->M[c] + Rv[3 * r + 1] * P->M[3 + c] + Rv[3 * r + 2] * P->M[6 + c];
    for (int r = 0; r < 3; ++r)
        P->t[r] = Rv[3 * r] * mu[0] + Rv[3 * r + 1] * mu[1] + Rv[3 * r + 2] * mu[2] + tv[r];
    double tx = P->t[0], ty = P->t[1], tz = P->t[2];
    double fx = cam->fx, fy = cam->fy;
    /* Jacobian of pi(t) = (fx tx/tz + cx, fy ty/tz + cy) */
    double J00 = fx / tz, J02 = -fx * tx / (tz * tz);
    double J11 = fy / tz, J12 = -fy * ty / (tz * tz);
    double T0[3], T1[3];
    for (int c = 0; c < 3; ++c) {
        T0[c] = J00 * P->V[c] + J02 * P->V[6 + c];
        T1[c] = J11 * P->V[3 + c] + J12 * P->V[6 + c];
    }
    P->a = T0[0] * T0[0] + T0[1] * T0[1] + T0[2] * T0[2] + o->dilation;
    P->b = T0[0] * T1[0] + T0[1] * T1[1] + T0[2] * T1[2];
    P->c = T1[0] * T1[0] + T1[1] * T1[1] + T1[2] * T1[2] + o->dilation;
    P->det = P->a * P->c - P->b * P->b;
    P->Q[0] = P->c / P->det;
    P->Q[1] = -P->b / P->det;
    P->Q[2] = P->a / P->det;
    P->m[0] = fx * tx / tz + cam->cx;
    P->m[1] = fy * ty / tz + cam->cy;
    P->d = tz;
    /* camera centre = -Rv^T tv; viewing direction from camera to mean */
    double cc[3];
    for (int k = 0; k < 3; ++k) cc[k] = -(Rv[k] * tv[0] + Rv[3 + k] * tv[1] + Rv[6 + k] * tv[2]);
    double vv[3] = {mu[0] - cc[0], mu[1] - cc[1], mu[2] - cc[2]};
    P->vnorm = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
    for (int k = 0; k < 3; ++k) P->dir[k] = vv[k] / P->vnorm;
    memset(P->Y, 0, sizeof(P->Y));
    sh_basis(deg, P->dir[0], P->dir[1], P->dir[2], P->Y, NULL);
    int ncoef = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < ncoef; ++k) acc += P->Y[k] * sh[(3 * k + ch) * stride_sh];
        P->clamp[ch] = acc < 0.0;
        P->color[ch] = acc < 0.0 ? 0.0 : acc;
    }
}

/* Scene arrays: means[n][3], scales[n][3], quats[n][4], opacity[n],
 * sh[n][(deg+1)^2 * 3] with element (k, ch) at k*3 + ch. */
typedef struct {
    int64_t n;
    const double *means, *scales, *quats, *opacity, *sh;
} orc_scene;

static void project_all(const orc_scene* S, const orc_cam* cam, const orc_opts* o, proj64* P)
{
    int ncoef = (o->sh_degree + 1) * (o->sh_degree + 1);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i)
        project_one(S->means + 3 * i, S->scales + 3 * i, S->quats + 4 * i, S->sh + (int64_t)ncoef * 3 * i,
                    o->sh_degree, 1, cam, o, &P[i]);
}

/* Exported FP64 projection: mean2d[n][2], conic[n][3], cov[n][3], color[n][3], depth[n]. */
void orc_project(const orc_scene* S, const orc_cam* cam, const orc_opts* o,
                 double* mean2d, double* conic, double* cov, double* color, double* depth, uint8_t* color_clamp)
{
    proj64* P = (proj64*)malloc(sizeof(proj64) * (size_t)(S->n > 0 ? S->n : 1));
    project_all(S, cam, o, P);
    for (int64_t i = 0; i < S->n; ++i) {
        mean2d[2 * i] = P[i].m[0]; mean2d[2 * i + 1] = P[i].m[1];
        conic[3 * i] = P[i].Q[0]; conic[3 * i + 1] = P[i].Q[1]; conic[3 * i + 2] = P[i].Q[2];
        cov[3 * i] = P[i].a; cov[3 * i + 1] = P[i].b; cov[3 * i + 2] = P[i].c;
        for (int k = 0; k < 3; ++k) { color[3 * i + k] = P[i].color[k]; color_clamp[3 * i + k] = (uint8_t)P[i].clamp[k]; }
        depth[i] = P[i].d;
    }
    free(P);
}

/* ------------------------------------------------------------------------ */
/* Depth order: non-culled Gaussians sorted by (FP32 depth bits, index).     */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key; int64_t idx; } kv_t;
static int kv_cmp(const void* A, const void* B)
{
    const kv_t* a = (const kv_t*)A;
    const kv_t* b = (const kv_t*)B;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int64_t depth_order(int64_t n, const uint32_t* dbits, const uint8_t* culled, int64_t* order)
{
    kv_t* kv = (kv_t*)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (!culled[i]) { kv[m].key = dbits[i]; kv[m].idx = i; ++m; }
    qsort(kv, (size_t)m, sizeof(kv_t), kv_cmp);
    for (int64_t k = 0; k < m; ++k) order[k] = kv[k].idx;
    free(kv);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel front-to-back walk (eq. 3dgs_orig, eq. opacity_impact, Depth). */
/* ------------------------------------------------------------------------ */
#define MAX_FLIPS 4
typedef struct { int64_t pos; int type; } decision_t; /* type 0: skip test, 1: termination test */

typedef struct {
    double C[3], D, W, T;
    int64_t n;
    uint64_t hash;
    int n_amb;
    decision_t amb[MAX_FLIPS];
} walk_out;

typedef struct {
    const proj64* P;
    const double* opacity;
    const int64_t* order;
    int64_t m;
    const orc_opts* o;
} walk_ctx;

static int is_flipped(const decision_t* flips, int nf, int64_t pos, int type)
{
    for (int k = 0; k < nf; ++k)
        if (flips[k].pos == pos && flips[k].type == type) return 1;
    return 0;
}

static uint64_t mix64(uint64_t h, uint64_t v)
{
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

/* Optional per-contributor record for the backward. */
typedef struct { int64_t g; double alpha, e, T; int clamped; double dx, dy; } contrib_t;

static void walk_pixel(const walk_ctx* ctx, double px, double py, const decision_t* flips, int nf,
                       walk_out* out, contrib_t* list, int64_t list_cap)
{
    const orc_opts* o = ctx->o;
    double T = 1.0, C[3] = {0, 0, 0}, D = 0, W = 0;
    int64_t n = 0;
    uint64_t h = 0x12345678ull;
    out->n_amb = 0;
    for (int64_t k = 0; k < ctx->m; ++k) {
        int64_t g = ctx->order[k];
        const proj64* P = &ctx->P[g];
        double dx = px - P->m[0], dy = py - P->m[1];
        double q = P->Q[0] * dx * dx + 2.0 * P->Q[1] * dx * dy + P->Q[2] * dy * dy;
        double e = exp(-0.5 * q);
        double araw = ctx->opacity[g] * e;
        int clamped = araw > o->alpha_max;
        double alpha = clamped ? o->alpha_max : araw;
        int skip = alpha < o->alpha_min;
        if (fabs(alpha - o->alpha_min) <= o->band * o->alpha_min && out->n_amb < MAX_FLIPS) {
            out->amb[out->n_amb].pos = k; out->amb[out->n_amb].type = 0; out->n_amb++;
        }
        if (is_flipped(flips, nf, k, 0)) skip = !skip;
        if (skip) continue;
        double Tn = T * (1.0 - alpha);
        int stop = Tn < o->t_min;
        if (fabs(Tn - o->t_min) <= o->band * o->t_min && out->n_amb < MAX_FLIPS) {
            out->amb[out->n_amb].pos = k; out->amb[out->n_amb].type = 1; out->n_amb++;
        }
        if (is_flipped(flips, nf, k, 1)) stop = !stop;
        if (stop) break;
        double w = alpha * T;
        for (int c = 0; c < 3; ++c) C[c] += w * P->color[c];
        D += w * P->d;
        W += w;
        if (list && n < list_cap) {
            list[n].g = g; list[n].alpha = alpha; list[n].e = e; list[n].T = T;
            list[n].clamped = clamped; list[n].dx = dx; list[n].dy = dy;
        }
        T = Tn;
        ++n;
        h = mix64(h, (uint64_t)g * 2u + (uint64_t)clamped);
    }
    for (int c = 0; c < 3; ++c) out->C[c] = C[c];
    out->D = D; out->W = W; out->T = T; out->n = n; out->hash = mix64(h, (uint64_t)n);
}

/* Logistic map of the Implementation section: 2/(1 + e^{-0.1 zhat}) - 1. */
static double logistic_depth(double zh) { return 2.0 / (1.0 + exp(-0.1 * zh)) - 1.0; }

/* Medium epilogue (eq. 3dgs_uw with eq. Depth).  Writes rgb[3], depth, alpha.  The depth
 * image is the z the medium uses, or (depth_output 1) the logistic map of zhat that the
 * Implementation section applies for visualisation. */
static void medium_epilogue(const walk_out* w, const double* med, const orc_opts* o, double* rgb, double* depth, double* alpha)
{
    const double *Bd = med, *Bb = med + 3, *Binf = med + 6;
    if (w->W > 0.0) {
        double zh = w->D / w->W;
        double z = o->depth_mode == 1 ? logistic_depth(zh) : zh;
        for (int c = 0; c < 3; ++c)
            rgb[c] = w->C[c] * exp(-Bd[c] * z) + Binf[c] * (1.0 - exp(-Bb[c] * z));
        *depth = o->depth_output == 1 ? logistic_depth(zh) : z;
    } else {
        for (int c = 0; c < 3; ++c) {
            if (o->depth_mode == 1) rgb[c] = Binf[c] * (1.0 - exp(-Bb[c]));
            else rgb[c] = Bb[c] > 0.0 ? Binf[c] : 0.0;
        }
        *depth = 0.0;
    }
    *alpha = w->W;
}

static void setup_ctx(const orc_scene* S, const orc_cam* cam, const orc_opts* o, walk_ctx* ctx,
                      proj64** Pout, int64_t** order_out)
{
    int64_t n = S->n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    proj64* P = (proj64*)malloc(sizeof(proj64) * nn);
    project_all(S, cam, o, P);
    uint32_t* dbits = (uint32_t*)malloc(4 * nn);
    int32_t* rect = (int32_t*)malloc(16 * nn);
    uint8_t* culled = (uint8_t*)malloc(nn);
    orc_key_path(n, S->means, S->scales, S->quats, cam, o, dbits, rect, culled);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * nn);
    int64_t m = depth_order(n, dbits, culled, order);
    free(dbits); free(rect); free(culled);
    ctx->P = P; ctx->opacity = S->opacity; ctx->order = order; ctx->m = m; ctx->o = o;
    *Pout = P; *order_out = order;
}

/*
 * Render npix pixels (pix[k] = (u, v) integer pixel coordinates).
 * Outputs per pixel: rgb[3], depth, alpha, cair[3], tfinal, ncontrib, hash.
 * If max_var > 0, ambiguous threshold decisions (relative margin <= band) of the
 * main walk are flipped in every non-empty combination (at most 2^3 - 1) and
 * the resulting (rgb[3], depth, alpha) are written to var[k][j][5]; nvar[k]
 * counts them.
 */
void orc_render(const orc_scene* S, const orc_cam* cam, const double* medium, const orc_opts* o,
                int64_t npix, const int32_t* pix,
                double* rgb, double* depth, double* alpha, double* cair, double* tfinal,
                int64_t* ncontrib, uint64_t* hash, int32_t max_var, int32_t* nvar, double* var)
{
    walk_ctx ctx;
    proj64* P;
    int64_t* order;
    setup_ctx(S, cam, o, &ctx, &P, &order);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; ++k) {
        double px = pix[2 * k] + 0.5, py = pix[2 * k + 1] + 0.5;
        walk_out w;
        walk_pixel(&ctx, px, py, NULL, 0, &w, NULL, 0);
        medium_epilogue(&w, medium, o, rgb + 3 * k, depth + k, alpha + k);
        for (int c = 0; c < 3; ++c) cair[3 * k + c] = w.C[c];
        tfinal[k] = w.T;
        ncontrib[k] = w.n;
        hash[k] = w.hash;
        if (max_var > 0) {
            int na = w.n_amb < 3 ? w.n_amb : 3;
            int cnt = 0;
            for (int mask = 1; mask < (1 << na) && cnt < max_var; ++mask) {
                decision_t fl[3];
                int nf = 0;
                for (int b = 0; b < na; ++b)
                    if (mask & (1 << b)) fl[nf++] = w.amb[b];
                walk_out wv;
                walk_pixel(&ctx, px, py, fl, nf, &wv, NULL, 0);
                double* dst = var + ((size_t)k * max_var + cnt) * 5;
                medium_epilogue(&wv, medium, o, dst, dst + 3, dst + 4);
                ++cnt;
            }
            nvar[k] = cnt;
        }
    }
    free(P);
    free(order);
}

/* ------------------------------------------------------------------------ */
/* Backward, pixel part: exact derivative of the per-pixel forward.           */
/* Produces per-Gaussian 2D gradients g2d[n][10] =                            */
/*   (m_x, m_y, Q_xx, Q_xy, Q_yy, opacity, r, g, b, depth)                    */
/* where Q_xy is the single off-diagonal conic entry (q = Qxx dx^2 +          */
/* 2 Qxy dx dy + Qyy dy^2), and the medium gradient gmed[9] =                 */
/* (dB_d[3], dB_b[3], dB_inf[3]).  Both are ACCUMULATED (+=).                 */
/* Upstream gradients: of the attenuated colour C_uw, of the depth image and  */
/* (grad_cair) of the in-air composite C_air, the clean image J of            */
/* eq. (scattering_approx) that the medium attenuates.                        */
/* ------------------------------------------------------------------------ */
void orc_backward_pixels(const orc_scene* S, const orc_cam* cam, const double* medium, const orc_opts* o,
                         int64_t npix, const int32_t* pix, const double* grad_rgb /*[npix][3]*/,
                         const double* grad_depth /*[npix] or NULL*/, const double* grad_cair /*[npix][3] or NULL*/,
                         double* g2d, double* gmed)
{
    walk_ctx ctx;
    proj64* P;
    int64_t* order;
    setup_ctx(S, cam, o, &ctx, &P, &order);
    const double *Bd = medium, *Bb = medium + 3, *Binf = medium + 6;
    int64_t cap = ctx.m > 0 ? ctx.m : 1;
    /* Per-pixel contribution lists, accumulated serially afterwards so the
     * result does not depend on thread scheduling. */
    typedef struct { int64_t g; double v[10]; } gitem;
    gitem** items = (gitem**)calloc((size_t)(npix > 0 ? npix : 1), sizeof(gitem*));
    int64_t* nitems = (int64_t*)calloc((size_t)(npix > 0 ? npix : 1), sizeof(int64_t));
    double* pmed = (double*)calloc((size_t)(npix > 0 ? npix : 1) * 9, sizeof(double));
    #pragma omp parallel
    {
        contrib_t* list = (contrib_t*)malloc(sizeof(contrib_t) * (size_t)cap);
        double* sfx = (double*)malloc(sizeof(double) * (size_t)(cap + 1));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < npix; ++k) {
            double px = pix[2 * k] + 0.5, py = pix[2 * k + 1] + 0.5;
            walk_out w;
            walk_pixel(&ctx, px, py, NULL, 0, &w, list, cap);
            const double* G = grad_rgb + 3 * k;
            double Gz = grad_depth ? grad_depth[k] : 0.0;
            double* pm = pmed + 9 * k;
            if (!(w.W > 0.0)) {
                for (int c = 0; c < 3; ++c) {
                    if (o->depth_mode == 1) {
                        double Sx = exp(-Bb[c]);
                        pm[6 + c] = G[c] * (1.0 - Sx);
                        pm[3 + c] = G[c] * Binf[c] * Sx;
                    } else {
                        pm[6 + c] = Bb[c] > 0.0 ? G[c] : 0.0;
                    }
                }
                continue;
            }
            double zh = w.D / w.W;
            double z = o->depth_mode == 1 ? logistic_depth(zh) : zh;
            double A[3], Sx[3], dz = 0.0;
            for (int c = 0; c < 3; ++c) {
                A[c] = exp(-Bd[c] * z);
                Sx[c] = exp(-Bb[c] * z);
                pm[c] = -G[c] * w.C[c] * z * A[c];
                pm[3 + c] = G[c] * Binf[c] * z * Sx[c];
                pm[6 + c] = G[c] * (1.0 - Sx[c]);
                dz += G[c] * (-Bd[c] * w.C[c] * A[c] + Binf[c] * Bb[c] * Sx[c]);
            }
            /* d(logistic)/d(zhat) = 0.05 (1 - y^2) for y = tanh(0.05 zhat) */
            double dzh = o->depth_mode == 1 ? dz * 0.05 * (1.0 - z * z) : dz;
            if (o->depth_output == 1) {
                double y = logistic_depth(zh);
                dzh += Gz * 0.05 * (1.0 - y * y);
            } else {
                dzh += o->depth_mode == 1 ? Gz * 0.05 * (1.0 - z * z) : Gz;
            }
            /* upstream gradient of the accumulators (C_air[3], D, W) */
            const double* GJ = grad_cair ? grad_cair + 3 * k : NULL;
            double gC[3];
            for (int c = 0; c < 3; ++c) gC[c] = G[c] * A[c] + (GJ ? GJ[c] : 0.0);
            double gD = dzh / w.W;
            double gW = -dzh * zh / w.W;
            int64_t n = w.n;
            /* sfx[i] = sum_{j > i} (g . f_j) w_j */
            sfx[n] = 0.0;
            for (int64_t i = n - 1; i >= 0; --i) {
                const proj64* Pj = &P[list[i].g];
                double gf = gC[0] * Pj->color[0] + gC[1] * Pj->color[1] + gC[2] * Pj->color[2] + gD * Pj->d + gW;
                double wj = list[i].alpha * list[i].T;
                sfx[i] = (i + 1 <= n ? sfx[i + 1] : 0.0) + gf * wj;
            }
            gitem* it = (gitem*)malloc(sizeof(gitem) * (size_t)(n > 0 ? n : 1));
            for (int64_t i = 0; i < n; ++i) {
                const contrib_t* L = &list[i];
                const proj64* Pi = &P[L->g];
                double gf = gC[0] * Pi->color[0] + gC[1] * Pi->color[1] + gC[2] * Pi->color[2] + gD * Pi->d + gW;
                double wi = L->alpha * L->T;
                double dalpha = L->T * gf - sfx[i + 1] / (1.0 - L->alpha);
                gitem* g = &it[i];
                memset(g, 0, sizeof(*g));
                g->g = L->g;
                for (int c = 0; c < 3; ++c) g->v[6 + c] = gC[c] * wi;
                g->v[9] = gD * wi;
                if (!L->clamped) {
                    double op = ctx.opacity[L->g];
                    g->v[5] = dalpha * L->e;
                    double dq = -0.5 * op * L->e * dalpha;   /* alpha = o exp(-q/2) */
                    double dx = L->dx, dy = L->dy;
                    g->v[2] = dq * dx * dx;
                    g->v[3] = dq * 2.0 * dx * dy;
                    g->v[4] = dq * dy * dy;
                    /* dx = px - m_x, so dq/dm_x = -2 (Qxx dx + Qxy dy) */
                    g->v[0] = dq * -2.0 * (Pi->Q[0] * dx + Pi->Q[1] * dy);
                    g->v[1] = dq * -2.0 * (Pi->Q[1] * dx + Pi->Q[2] * dy);
                }
            }
            items[k] = it;
            nitems[k] = n;
        }
        free(list);
        free(sfx);
    }
    for (int64_t k = 0; k < npix; ++k) {
        for (int64_t i = 0; i < nitems[k]; ++i)
            for (int c = 0; c < 10; ++c) g2d[10 * items[k][i].g + c] += items[k][i].v[c];
        for (int c = 0; c < 9; ++c) gmed[c] += pmed[9 * k + c];
        free(items[k]);
    }
    free(items); free(nitems); free(pmed);
    free(P); free(order);
}

/* ------------------------------------------------------------------------ */
/* Backward, projection part: chain the 2D gradients back to the 3D params.   */
/* Gradients are ACCUMULATED into dmeans[n][3], dscales[n][3], dquats[n][4],  */
/* dopacity[n], dsh[n][ncoef*3] (so views can be summed).                     */
/* ------------------------------------------------------------------------ */
void orc_backward_project(const orc_scene* S, const orc_cam* cam, const orc_opts* o, const double* g2d,
                          double* dmeans, double* dscales, double* dquats, double* dopacity, double* dsh)
{
    int deg = o->sh_degree;
    int ncoef = (deg + 1) * (deg + 1);
    double Rv[9], tv[3];
    for (int k = 0; k < 9; ++k) Rv[k] = cam->R[k];
    for (int k = 0; k < 3; ++k) tv[k] = cam->t[k];
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->n; ++i) {
        const double* gg = g2d + 10 * i;
        int any = 0;
        for (int c = 0; c < 10; ++c) any |= gg[c] != 0.0;
        if (!any) continue;
        proj64 P;
        const double* mu = S->means + 3 * i;
        const double* s = S->scales + 3 * i;
        const double* sh = S->sh + (int64_t)ncoef * 3 * i;
        project_one(mu, s, S->quats + 4 * i, sh, deg, 1, cam, o, &P);
        double tx = P.t[0], ty = P.t[1], tz = P.t[2];
        double fx = cam->fx, fy = cam->fy;
        double J00 = fx / tz, J02 = -fx * tx / (tz * tz);
        double J11 = fy / tz, J12 = -fy * ty / (tz * tz);
        /* conic -> covariance: Q = inv([[a,b],[b,c]]) */
        double a = P.a, b = P.b, c = P.c, det2 = P.det * P.det;
        double gQxx = gg[2], gQxy = gg[3], gQyy = gg[4];
        double ga = (-gQxx * c * c + gQxy * b * c - gQyy * b * b) / det2;
        double gb = (2.0 * gQxx * b * c - gQxy * (a * c + b * b) + 2.0 * gQyy * a * b) / det2;
        double gc = (-gQxx * b * b + gQxy * a * b - gQyy * a * a) / det2;
        /* covariance = T2 T2^T + eps I */
        double T0[3], T1[3], gT0[3], gT1[3];
        for (int k = 0; k < 3; ++k) {
            T0[k] = J00 * P.V[k] + J02 * P.V[6 + k];
            T1[k] = J11 * P.V[3 + k] + J12 * P.V[6 + k];
        }
        for (int k = 0; k < 3; ++k) {
            gT0[k] = 2.0 * ga * T0[k] + gb * T1[k];
            gT1[k] = 2.0 * gc * T1[k] + gb * T0[k];
        }
        /* T2 = J V */
        double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0, gV[9];
        for (int k = 0; k < 3; ++k) {
            gJ00 += gT0[k] * P.V[k];
            gJ02 += gT0[k] * P.V[6 + k];
            gJ11 += gT1[k] * P.V[3 + k];
            gJ12 += gT1[k] * P.V[6 + k];
            gV[k] = gT0[k] * J00;
            gV[3 + k] = gT1[k] * J11;
            gV[6 + k] = gT0[k] * J02 + gT1[k] * J12;
        }
        /* V = Rv M */
        double gM[9];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                gM[3 * r + k] = Rv[r] * gV[k] + Rv[3 + r] * gV[3 + k] + Rv[6 + r] * gV[6 + k];
        /* M = Rq diag(s) */
        double gRq[9];
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int r = 0; r < 3; ++r) {
                acc += gM[3 * r + k] * P.Rq[3 * r + k];
                gRq[3 * r + k] = gM[3 * r + k] * s[k];
            }
            dscales[3 * i + k] += acc;
        }
        /* Rq(qhat) */
        double w = P.qhat[0], x = P.qhat[1], y = P.qhat[2], z = P.qhat[3];
        const double* G = gRq;
        double gw = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
        double gx = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] + z * G[6] + w * G[7] - 2.0 * x * G[8]);
        double gy = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - 2.0 * y * G[8]);
        double gz = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0 * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
        double gqh[4] = {gw, gx, gy, gz};
        double dotq = gqh[0] * P.qhat[0] + gqh[1] * P.qhat[1] + gqh[2] * P.qhat[2] + gqh[3] * P.qhat[3];
        for (int k = 0; k < 4; ++k) dquats[4 * i + k] += (gqh[k] - P.qhat[k] * dotq) / P.qnorm;
        /* t: through J, the mean and the depth */
        double gtx = gJ02 * (-fx / (tz * tz)) + gg[0] * fx / tz;
        double gty = gJ12 * (-fy / (tz * tz)) + gg[1] * fy / tz;
        double gtz = gJ00 * (-fx / (tz * tz)) + gJ02 * (2.0 * fx * tx / (tz * tz * tz))
                   + gJ11 * (-fy / (tz * tz)) + gJ12 * (2.0 * fy * ty / (tz * tz * tz))
                   - gg[0] * fx * tx / (tz * tz) - gg[1] * fy * ty / (tz * tz) + gg[9];
        double gmu[3];
        for (int k = 0; k < 3; ++k) gmu[k] = Rv[k] * gtx + Rv[3 + k] * gty + Rv[6 + k] * gtz;
        /* SH colour */
        double Y[16], dY[16][3];
        memset(Y, 0, sizeof(Y));
        sh_basis(deg, P.dir[0], P.dir[1], P.dir[2], Y, &dY[0][0]);
        double gdir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
            if (P.clamp[ch]) continue;
            double gcol = gg[6 + ch];
            for (int k = 0; k < ncoef; ++k) {
                dsh[(int64_t)ncoef * 3 * i + 3 * k + ch] += Y[k] * gcol;
                double shv = sh[3 * k + ch];
                for (int j = 0; j < 3; ++j) gdir[j] += gcol * shv * dY[k][j];
            }
        }
        double dd = gdir[0] * P.dir[0] + gdir[1] * P.dir[1] + gdir[2] * P.dir[2];
        for (int k = 0; k < 3; ++k) gmu[k] += (gdir[k] - P.dir[k] * dd) / P.vnorm;
        for (int k = 0; k < 3; ++k) dmeans[3 * i + k] += gmu[k];
        dopacity[i] += gg[5];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
