// Projection of 3D Gaussians into the views (Preliminaries, 3DGS: covariance
// from rotation and scale; EWA affine projection of the covariance; SH colour)
// and its adjoint.  One thread per Gaussian loops over the views, so the
// structure-of-arrays parameters are read once per launch with coalesced loads.
// The SH part of the adjoint runs in its own kernel from factors the adjoint
// stores (k_adam_sh for one view, k_sh_views for several), which reads each SH
// coefficient once and spreads a Gaussian's coefficients over four waves.
//
// The key path (view depth, 2D mean, diagonal of the 2D covariance, tile
// rectangle) is a fixed sequence of separately rounded FP32 operations: this
// file is compiled with -ffp-contract=off and uses no fused multiply-adds on
// that path, with IEEE division and square root, so the sort keys are
// reproducible bit for bit.
#include <string.h>

#include "internal.h"

namespace gs {

namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kConicScale = -0.5f * kLog2e;   // A = kConicScale * Qxx, etc.

// Real orthonormal SH, Condon-Shortley phase, k = l^2 + l + m.
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.4886025119029199f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY20 = 0.31539156525252005f;
constexpr float kY22 = 0.5462742152960396f;
constexpr float kY33 = 0.5900435899266435f;
constexpr float kY32 = 2.890611442640554f;
constexpr float kY31 = 0.4570457994644658f;
constexpr float kY30 = 0.3731763325901154f;
constexpr float kY322 = 1.445305721320277f;

// Real SH basis function k (0 <= k < (DEG+1)^2) at the unit direction (x, y, z); k is a
// compile-time constant wherever the callers' loops are unrolled.
__device__ __forceinline__ float sh_basis(int k, float x, float y, float z) {
    const float xx = x * x, yy = y * y, zz = z * z;
    switch (k) {
        case 0: return kY0;
        case 1: return -kY1 * y;
        case 2: return kY1 * z;
        case 3: return -kY1 * x;
        case 4: return kY2a * x * y;
        case 5: return -kY2a * y * z;
        case 6: return kY20 * (2.0f * zz - xx - yy);
        case 7: return -kY2a * x * z;
        case 8: return kY22 * (xx - yy);
        case 9: return -kY33 * y * (3.0f * xx - yy);
        case 10: return kY32 * x * y * z;
        case 11: return -kY31 * y * (4.0f * zz - xx - yy);
        case 12: return kY30 * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
        case 13: return -kY31 * x * (4.0f * zz - xx - yy);
        case 14: return kY322 * z * (xx - yy);
        default: return -kY33 * x * (xx - 3.0f * yy);
    }
}

template <int DEG>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* Y) {
#pragma unroll
    for (int k = 0; k < (DEG + 1) * (DEG + 1); ++k) Y[k] = sh_basis(k, x, y, z);
}

// Adds w * grad Y_k(x, y, z) (of the polynomial forms above) to (gx, gy, gz).
__device__ __forceinline__ void sh_grad_add(int k, float x, float y, float z, float w, float& gx, float& gy,
                                            float& gz) {
    const float xx = x * x, yy = y * y, zz = z * z;
    switch (k) {
        case 1: gy += -kY1 * w; break;
        case 2: gz += kY1 * w; break;
        case 3: gx += -kY1 * w; break;
        case 4: gx += kY2a * y * w; gy += kY2a * x * w; break;
        case 5: gy += -kY2a * z * w; gz += -kY2a * y * w; break;
        case 6: gx += -2.f * kY20 * x * w; gy += -2.f * kY20 * y * w; gz += 4.f * kY20 * z * w; break;
        case 7: gx += -kY2a * z * w; gz += -kY2a * x * w; break;
        case 8: gx += 2.f * kY22 * x * w; gy += -2.f * kY22 * y * w; break;
        case 9: gx += -kY33 * 6.f * x * y * w; gy += -kY33 * (3.f * xx - 3.f * yy) * w; break;
        case 10: gx += kY32 * y * z * w; gy += kY32 * x * z * w; gz += kY32 * x * y * w; break;
        case 11:
            gx += kY31 * 2.f * x * y * w;
            gy += -kY31 * (4.f * zz - xx - 3.f * yy) * w;
            gz += -kY31 * 8.f * y * z * w;
            break;
        case 12:
            gx += -kY30 * 6.f * x * z * w;
            gy += -kY30 * 6.f * y * z * w;
            gz += kY30 * (6.f * zz - 3.f * xx - 3.f * yy) * w;
            break;
        case 13:
            gx += -kY31 * (4.f * zz - 3.f * xx - yy) * w;
            gy += kY31 * 2.f * x * y * w;
            gz += -kY31 * 8.f * x * z * w;
            break;
        case 14: gx += kY322 * 2.f * x * z * w; gy += -kY322 * 2.f * y * z * w; gz += kY322 * (xx - yy) * w; break;
        case 15: gx += -kY33 * (3.f * xx - 3.f * yy) * w; gy += kY33 * 6.f * x * y * w; break;
        default: break;   // Y_0 is constant
    }
}

// Gradient of sum_k w_k Y_k(x, y, z) w.r.t. (x, y, z).  Summed in four interleaved partial sums
// (k = s, s + 4, ... for s = 0..3, each in increasing k) combined as ((P0 + P1) + P2) + P3: the
// order in which k_adam_sh forms it with four threads per group of Gaussians.
template <int DEG>
__device__ __forceinline__ void sh_grad(float x, float y, float z, const float* w, float* g) {
    float P[4][3];
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
        P[sub][0] = P[sub][1] = P[sub][2] = 0.f;
#pragma unroll
        for (int k = sub; k < (DEG + 1) * (DEG + 1); k += 4) sh_grad_add(k, x, y, z, w[k], P[sub][0], P[sub][1], P[sub][2]);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) g[q] = ((P[0][q] + P[1][q]) + P[2][q]) + P[3][q];
}

struct Cam {
    float R[9], t[3], fx, fy, cx, cy, near_z;
    int W, H;
};

__device__ __forceinline__ Cam load_cam(const gs_camera* c) {
    Cam k;
#pragma unroll
    for (int i = 0; i < 9; ++i) k.R[i] = c->R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) k.t[i] = c->t[i];
    k.fx = c->fx; k.fy = c->fy; k.cx = c->cx; k.cy = c->cy; k.near_z = c->near_z;
    k.W = c->width; k.H = c->height;
    return k;
}

// Quantities of the FP32 key path (and what the rest of the projection reuses).
struct Proj {
    float t[3];          // camera-space mean
    float qh[4];         // normalised quaternion
    float Rq[9];         // rotation of the Gaussian
    float V[9];          // Rv * Rq * diag(s)
    float u, v, a, b;    // tx/tz, ty/tz, fx/tz, fy/tz
    float T0[3], T1[3];  // 2x3 factor of the 2D covariance
    float sxx, syy, px, py;
    bool valid;
};

// Exact FP32 sequence shared with the key specification.  Returns valid=false
// for culled / non-finite Gaussians.
__device__ __forceinline__ void key_path(const Cam& c, float mx, float my, float mz, float s0, float s1,
                                         float s2, float qw, float qx, float qy, float qz, float dil,
                                         Proj& P) {
    P.t[0] = ((c.R[0] * mx + c.R[1] * my) + c.R[2] * mz) + c.t[0];
    P.t[1] = ((c.R[3] * mx + c.R[4] * my) + c.R[5] * mz) + c.t[1];
    P.t[2] = ((c.R[6] * mx + c.R[7] * my) + c.R[8] * mz) + c.t[2];
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    P.valid = (P.t[2] > c.near_z) && (n2 > 0.0f) && isfinite(P.t[0]) && isfinite(P.t[1]) && isfinite(s0) &&
              isfinite(s1) && isfinite(s2) && isfinite(n2);
    float nrm = __builtin_sqrtf(n2);
    float w = qw / nrm, x = qx / nrm, y = qy / nrm, z = qz / nrm;
    P.qh[0] = w; P.qh[1] = x; P.qh[2] = y; P.qh[3] = z;
    float xx = x * x, yy = y * y, zz = z * z;
    float xy = x * y, xz = x * z, yz = y * z;
    float wx = w * x, wy = w * y, wz = w * z;
    float* Q = P.Rq;
    Q[0] = 1.0f - 2.0f * (yy + zz); Q[1] = 2.0f * (xy - wz);        Q[2] = 2.0f * (xz + wy);
    Q[3] = 2.0f * (xy + wz);        Q[4] = 1.0f - 2.0f * (xx + zz); Q[5] = 2.0f * (yz - wx);
    Q[6] = 2.0f * (xz - wy);        Q[7] = 2.0f * (yz + wx);        Q[8] = 1.0f - 2.0f * (xx + yy);
    float M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = Q[3 * r + 0] * s0;
        M[3 * r + 1] = Q[3 * r + 1] * s1;
        M[3 * r + 2] = Q[3 * r + 2] * s2;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            P.V[3 * r + k] = (c.R[3 * r + 0] * M[k] + c.R[3 * r + 1] * M[3 + k]) + c.R[3 * r + 2] * M[6 + k];
    float tz = P.t[2];
    P.u = P.t[0] / tz;
    P.v = P.t[1] / tz;
    P.a = c.fx / tz;
    P.b = c.fy / tz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.T0[k] = P.a * (P.V[k] - P.u * P.V[6 + k]);
        P.T1[k] = P.b * (P.V[3 + k] - P.v * P.V[6 + k]);
    }
    P.sxx = ((P.T0[0] * P.T0[0] + P.T0[1] * P.T0[1]) + P.T0[2] * P.T0[2]) + dil;
    P.syy = ((P.T1[0] * P.T1[0] + P.T1[1] * P.T1[1]) + P.T1[2] * P.T1[2]) + dil;
    P.px = c.fx * P.u + c.cx;
    P.py = c.fy * P.v + c.cy;
}

__device__ __forceinline__ void camera_centre(const Cam& c, float* cc) {
#pragma unroll
    for (int k = 0; k < 3; ++k) cc[k] = -(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]);
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_fwd(gs_gaussians g, int32_t views, const gs_camera* cams,
                                                       const ViewInfo* vt, int tile_w, int tile_h, float kappa,
                                                       float dil, Record* rec, uint32_t* counts, uint2* rects,
                                                       uint32_t* depth_keys, uint32_t* dkeys_sort,
                                                       uint32_t* dvals_sort, SavedHeader* hdr) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float mx = g.means[i], my = g.means[n + i], mz = g.means[2 * n + i];
    const float s0 = g.scales[i], s1 = g.scales[n + i], s2 = g.scales[2 * n + i];
    const float qw = g.quats[i], qx = g.quats[n + i], qy = g.quats[2 * n + i], qz = g.quats[3 * n + i];
    const float op = g.opacity[i];
    float sh[NC * 3];
    bool finite = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(s0) && isfinite(s1) &&
                  isfinite(s2) && isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz) && isfinite(op);
#pragma unroll
    for (int k = 0; k < NC * 3; ++k) {
        sh[k] = g.sh[(int64_t)k * n + i];
        finite = finite && isfinite(sh[k]);
    }
    if (!finite) atomicOr(&hdr->status, GS_STATUS_NONFINITE_INPUT);
    const float inv_tw = 1.0f / (float)tile_w;   // exact: tile sizes are powers of two
    const float inv_th = 1.0f / (float)tile_h;
    for (int v = 0; v < views; ++v) {
        const int64_t e = (int64_t)v * n + i;
        const Cam c = load_cam(cams + v);
        const ViewInfo vi = vt[v];
        Proj P;
        key_path(c, mx, my, mz, s0, s1, s2, qw, qx, qy, qz, dil, P);
        const float ex = __builtin_sqrtf(kappa * P.sxx);
        const float ey = __builtin_sqrtf(kappa * P.syy);
        const bool ok = finite && P.valid && isfinite(P.px) && isfinite(P.py) && isfinite(ex) && isfinite(ey);
        uint32_t cnt = 0;
        uint32_t dkey = 0xFFFFFFFFu;
        uint2 rc = make_uint2(0xFFFFu, 0u);   // empty rectangle (x0 > x1)
        if (ok) {
            dkey = __float_as_uint(P.t[2]);
            const float lx = __builtin_floorf((P.px - ex) * inv_tw);
            const float hx = __builtin_floorf((P.px + ex) * inv_tw);
            const float ly = __builtin_floorf((P.py - ey) * inv_th);
            const float hy = __builtin_floorf((P.py + ey) * inv_th);
            const float x0 = lx > 0.0f ? lx : 0.0f;
            const float y0 = ly > 0.0f ? ly : 0.0f;
            const float x1 = hx < (float)(vi.tiles_x - 1) ? hx : (float)(vi.tiles_x - 1);
            const float y1 = hy < (float)(vi.tiles_y - 1) ? hy : (float)(vi.tiles_y - 1);
            if (x0 <= x1 && y0 <= y1) {
                const uint32_t ix0 = (uint32_t)x0, iy0 = (uint32_t)y0, ix1 = (uint32_t)x1, iy1 = (uint32_t)y1;
                rc = make_uint2(ix0 | (iy0 << 16), ix1 | (iy1 << 16));
                cnt = (ix1 - ix0 + 1) * (iy1 - iy0 + 1);
            }
            // Conic of the dilated 2D covariance, pre-scaled for exp2.
            const float sxy = (P.T0[0] * P.T1[0] + P.T0[1] * P.T1[1]) + P.T0[2] * P.T1[2];
            const float det = P.sxx * P.syy - sxy * sxy;
            const float id = 1.0f / det;
            const float A = kConicScale * (P.syy * id);
            const float B = 2.0f * kConicScale * (-sxy * id);
            const float C = kConicScale * (P.sxx * id);
            // View-dependent colour.
            float cc[3];
            camera_centre(c, cc);
            float dx = mx - cc[0], dy = my - cc[1], dz = mz - cc[2];
            const float il = 1.0f / __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
            dx *= il; dy *= il; dz *= il;
            float Y[16];
            sh_eval<DEG>(dx, dy, dz, Y);
            float col[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.5f;
#pragma unroll
                for (int k = 0; k < NC; ++k) acc = fmaf(Y[k], sh[3 * k + ch], acc);
                // clamped channels (acc < 0, or not a number) store -0: blends as 0, and tells the
                // adjoint that the channel passes no gradient to the SH coefficients
                col[ch] = acc > 0.0f ? acc : (acc == 0.0f ? 0.0f : -0.0f);
            }
            Record r;
            r.a = make_float4(P.px, P.py, A, B);
            const bool pos = op > 0.0f;
            r.b = make_float4(C, pos ? log2f(op) : -INFINITY, col[0], col[1]);
            r.c = make_float4(col[2], P.t[2], pos ? 1.0f / op : 0.0f, 0.0f);
            rec[e] = r;
        }
        counts[e] = cnt;
        rects[e] = rc;
        depth_keys[e] = dkey;
        // entries that touch no tile sort after every visible one (they emit nothing)
        dkeys_sort[e] = cnt ? dkey : 0xFFFFFFFFu;
        dvals_sort[e] = (uint32_t)e;
    }
}

// Adjoint of k_project_fwd.  grad2d[e][10] = d/d(m_x, m_y, A, B, C, opacity, r, g, b, depth)
// of the record of entry e = v * n + i.  Gradients of all views are summed in registers, then
// either written once (overwrite) or, when `fused`, used for one Adam step of the raw
// parameters (log-scales and opacity logits through the activations' derivatives) that also
// stores the activated scales and opacities the next forward reads.
//
// The SH gradient of one view is the outer product Y(dir) x (colour gradient of the
// unclamped channels).  With one view (ONE) the kernel keeps those 16 + 3 factors instead of
// 48 accumulators, which bounds its register use; the clamp of each channel is read from the
// forward's record (a clamped channel holds -0).  With several views the SH part runs in
// k_sh_views: this kernel stores, in adam.shf, the means' gradient without its SH term and each
// view's colour gradient of the unclamped channels (zero for a view the Gaussian misses).
template <int DEG, bool FUSED, bool ONE, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_project_bwd(gs_gaussians g, int32_t views, const gs_camera* cams,
                                                       float dil, const float* __restrict__ grad2d,
                                                       const Record* __restrict__ rec, gs_gaussian_grads out,
                                                       AdamFused adam) {
    static_assert(ONE || SPLIT, "several views: the SH part runs in k_sh_views");
    static_assert(!(ONE && SPLIT) || FUSED, "one view: the split is the fused Adam path");
    constexpr int NC = (DEG + 1) * (DEG + 1);
    constexpr bool MULTI = !ONE;
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (FUSED && guard_set(adam.guard)) return;   // skipped training step: nothing changes
    const float mx = g.means[i], my = g.means[n + i], mz = g.means[2 * n + i];
    const float s[3] = {g.scales[i], g.scales[n + i], g.scales[2 * n + i]};
    const float qw = g.quats[i], qx = g.quats[n + i], qy = g.quats[2 * n + i], qz = g.quats[3 * n + i];
    float gmu[3] = {0.f, 0.f, 0.f}, gsc[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, gop = 0.f;
    float Y1[16], gc1[3], dir1[3], il1 = 0.f;  // one view: the factors of its SH gradient
#pragma unroll
    for (int k = 0; k < 16; ++k) Y1[k] = 0.f;
    gc1[0] = gc1[1] = gc1[2] = 0.f;
    dir1[0] = dir1[1] = dir1[2] = 0.f;
    for (int v = 0; v < views; ++v) {
        const float* gg = grad2d + ((int64_t)v * n + i) * kGrad2D;
        float G[kGrad2D];
        bool any = false;
#pragma unroll
        for (int k = 0; k < kGrad2D; ++k) {
            G[k] = gg[k];
            any = any || (G[k] != 0.0f);
        }
        if (!any) {
            if (MULTI) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) adam.shf[(int64_t)(3 + 3 * v + ch) * n + i] = 0.0f;
            }
            continue;
        }
        const Cam c = load_cam(cams + v);
        Proj P;
        key_path(c, mx, my, mz, s[0], s[1], s[2], qw, qx, qy, qz, dil, P);
        const float tx = P.t[0], ty = P.t[1], tz = P.t[2];
        gop += G[5];
        // pre-scaled conic (A, B, C) -> conic Q = inverse covariance
        const float gQxx = kConicScale * G[2];
        const float gQxy = 2.0f * kConicScale * G[3];
        const float gQyy = kConicScale * G[4];
        const float a = P.sxx, c2 = P.syy;
        const float b = (P.T0[0] * P.T1[0] + P.T0[1] * P.T1[1]) + P.T0[2] * P.T1[2];
        const float det = a * c2 - b * b;
        const float id2 = 1.0f / (det * det);
        const float ga = (-gQxx * c2 * c2 + gQxy * b * c2 - gQyy * b * b) * id2;
        const float gb = (2.0f * gQxx * b * c2 - gQxy * (a * c2 + b * b) + 2.0f * gQyy * a * b) * id2;
        const float gc = (-gQxx * b * b + gQxy * a * b - gQyy * a * a) * id2;
        // covariance = T T^T + dil I, T = J V with J = [[a_, 0, -a_ u], [0, b_, -b_ v]]
        const float J00 = P.a, J02 = -P.a * P.u, J11 = P.b, J12 = -P.b * P.v;
        float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f, gV[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float gT0 = 2.0f * ga * P.T0[k] + gb * P.T1[k];
            const float gT1 = 2.0f * gc * P.T1[k] + gb * P.T0[k];
            gJ00 += gT0 * P.V[k];
            gJ02 += gT0 * P.V[6 + k];
            gJ11 += gT1 * P.V[3 + k];
            gJ12 += gT1 * P.V[6 + k];
            gV[k] = gT0 * J00;
            gV[3 + k] = gT1 * J11;
            gV[6 + k] = gT0 * J02 + gT1 * J12;
        }
        // V = Rv M, M = Rq diag(s)
        float gRq[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float gM = c.R[r] * gV[k] + c.R[3 + r] * gV[3 + k] + c.R[6 + r] * gV[6 + k];
                acc += gM * P.Rq[3 * r + k];
                gRq[3 * r + k] = gM * s[k];
            }
            gsc[k] += acc;
        }
        {
            const float w = P.qh[0], x = P.qh[1], y = P.qh[2], z = P.qh[3];
            const float* R = gRq;
            const float gw = 2.f * (-z * R[1] + y * R[2] + z * R[3] - x * R[5] - y * R[6] + x * R[7]);
            const float gx = 2.f * (y * R[1] + z * R[2] + y * R[3] - 2.f * x * R[4] - w * R[5] + z * R[6] +
                                    w * R[7] - 2.f * x * R[8]);
            const float gy = 2.f * (-2.f * y * R[0] + x * R[1] + w * R[2] + x * R[3] + z * R[5] - w * R[6] +
                                    z * R[7] - 2.f * y * R[8]);
            const float gz = 2.f * (-2.f * z * R[0] - w * R[1] + x * R[2] + w * R[3] - 2.f * z * R[4] +
                                    y * R[5] + x * R[6] + y * R[7]);
            const float dot = gw * w + gx * x + gy * y + gz * z;
            const float in = 1.0f / __builtin_sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
            gq[0] += (gw - w * dot) * in;
            gq[1] += (gx - x * dot) * in;
            gq[2] += (gy - y * dot) * in;
            gq[3] += (gz - z * dot) * in;
        }
        // camera-space mean: through J, the 2D mean and the depth
        const float itz = 1.0f / tz, itz2 = itz * itz, itz3 = itz2 * itz;
        const float gtx = -gJ02 * c.fx * itz2 + G[0] * c.fx * itz;
        const float gty = -gJ12 * c.fy * itz2 + G[1] * c.fy * itz;
        const float gtz = -gJ00 * c.fx * itz2 + gJ02 * 2.f * c.fx * tx * itz3 - gJ11 * c.fy * itz2 +
                          gJ12 * 2.f * c.fy * ty * itz3 - G[0] * c.fx * tx * itz2 - G[1] * c.fy * ty * itz2 +
                          G[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) gmu[k] += c.R[k] * gtx + c.R[3 + k] * gty + c.R[6 + k] * gtz;
        // SH colour: colour = max(0, 1/2 + sum_k Y_k(dir) sh_k); no gradient through a clamped channel
        const Record& r = rec[(int64_t)v * n + i];
        const float col[3] = {r.b.z, r.b.w, r.c.x};
        float gce[3];
        bool live = false;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            gce[ch] = signbit(col[ch]) ? 0.0f : G[6 + ch];
            live = live || gce[ch] != 0.0f;
        }
        if (MULTI) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) adam.shf[(int64_t)(3 + 3 * v + ch) * n + i] = gce[ch];
            continue;
        }
        if (!live) continue;
        float cc[3];
        camera_centre(c, cc);
        float d0 = mx - cc[0], d1 = my - cc[1], d2 = mz - cc[2];
        const float il = 1.0f / __builtin_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
        d0 *= il; d1 *= il; d2 *= il;
        float Y[16];
        sh_eval<DEG>(d0, d1, d2, Y);
#pragma unroll
        for (int k = 0; k < 16; ++k) Y1[k] = Y[k];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gc1[ch] = gce[ch];
        dir1[0] = d0;
        dir1[1] = d1;
        dir1[2] = d2;
        il1 = il;
        if (DEG > 0 && !SPLIT) {   // split: k_adam_sh adds this term, reading the SH coefficients once
            float wk[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) wk[k] = 0.f;
            // streamed in groups of four coefficients: hoisting all 48 loads would hold 48 registers
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                if (k % 4 == 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) wk[k] += gce[ch] * g.sh[(int64_t)(3 * k + ch) * n + i];
            }
            __builtin_amdgcn_sched_barrier(0);
            float gd[3];
            sh_grad<DEG>(d0, d1, d2, wk, gd);
            const float dd = gd[0] * d0 + gd[1] * d1 + gd[2] * d2;
            gmu[0] += (gd[0] - d0 * dd) * il;
            gmu[1] += (gd[1] - d1 * dd) * il;
            gmu[2] += (gd[2] - d2 * dd) * il;
        }
    }
    // regularisers on the activated opacity and scales (once per Gaussian, whatever its views)
    gop += adam.reg_o;
#pragma unroll
    for (int k = 0; k < 3; ++k) gsc[k] += adam.reg_s;
    // SH gradient element j = 3 k + channel (one view)
    auto shg = [&](int j) { return Y1[j / 3] * gc1[j % 3]; };
    if (MULTI) {   // k_sh_views adds the SH term
#pragma unroll
        for (int k = 0; k < 3; ++k) adam.shf[(int64_t)k * n + i] = gmu[k];
    }
    if (!FUSED) {
        if (!MULTI) {
            out.means[i] = gmu[0]; out.means[n + i] = gmu[1]; out.means[2 * n + i] = gmu[2];
        }
        out.scales[i] = gsc[0]; out.scales[n + i] = gsc[1]; out.scales[2 * n + i] = gsc[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) out.quats[(int64_t)k * n + i] = gq[k];
        out.opacity[i] = gop;
        if (!MULTI) {
#pragma unroll
            for (int k = 0; k < NC * 3; ++k) out.sh[(int64_t)k * n + i] = shg(k);
        }
        return;
    }
    const float ibc1 = adam.bc[0], ibc2 = adam.bc[1];
    // parameters, moments and activated copies are streamed (non-temporal), as in the flat Adam kernel
    auto step = [&](const gs_adam_group& G, int64_t j, float grad) {
        float m = __builtin_nontemporal_load(G.m + j), v = __builtin_nontemporal_load(G.v + j);
        const float np = adam_update(__builtin_nontemporal_load(G.param + j), grad, m, v, G.lr, adam.b1, adam.b2,
                                     adam.eps, ibc1, ibc2);
        __builtin_nontemporal_store(np, G.param + j);
        __builtin_nontemporal_store(m, G.m + j);
        __builtin_nontemporal_store(v, G.v + j);
        return np;
    };
    // The updates below are fenced for the scheduler in groups (16 SH coefficients = 48 loads
    // in flight): hoisting every parameter's and moment's load ahead of the arithmetic would
    // need several hundred registers.
    if (!SPLIT) {
#pragma unroll
        for (int k = 0; k < 3; ++k) step(adam.g[0], (int64_t)k * n + i, gmu[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {   // d exp(l)/dl = exp(l) = the activated scale
        const float nl = step(adam.g[1], (int64_t)k * n + i, gsc[k] * s[k]);
        __builtin_nontemporal_store(expf(nl), adam.g[1].activated + (int64_t)k * n + i);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) step(adam.g[2], (int64_t)k * n + i, gq[k]);
    __builtin_amdgcn_sched_barrier(0);
    {   // d sigmoid(x)/dx = o (1 - o)
        const float o = g.opacity[i];
        const float nx = step(adam.g[3], i, gop * (o * (1.0f - o)));
        __builtin_nontemporal_store(1.0f / (1.0f + expf(-nx)), adam.g[3].activated + i);
    }
    if (MULTI) return;   // the means' and the SH coefficients' steps run in k_sh_views
    if (SPLIT) {   // the means' and the SH coefficients' steps run in k_adam_sh from these
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            adam.shf[(int64_t)k * n + i] = dir1[k];
            adam.shf[(int64_t)(3 + k) * n + i] = gc1[k];
            adam.shf[(int64_t)(7 + k) * n + i] = gmu[k];
        }
        adam.shf[(int64_t)6 * n + i] = il1;
        return;
    }
#pragma unroll
    for (int k = 0; k < NC * 3; ++k) {
        if (k % 16 == 0) __builtin_amdgcn_sched_barrier(0);
        step(adam.g[4], (int64_t)k * n + i, shg(k));
    }
}

// One wave's share of k_adam_sh: SH coefficients k = SUB, SUB + 4, ... of its lane's W Gaussians
// stepped, and that partial sum of the means' SH term accumulated into P.
template <int DEG, int W, int SUB>
__device__ __forceinline__ void adam_sh_sweep(const AdamFused& adam, int64_t n, int64_t i0,
                                              const float (&dir)[3][W], const float (&gc)[3][W],
                                              const bool (&live)[W], float (&P)[W][3]) {
    using VW = float __attribute__((ext_vector_type(W)));
    constexpr int NC = (DEG + 1) * (DEG + 1);
    const float ibc1 = adam.bc[0], ibc2 = adam.bc[1];
    const gs_adam_group& G = adam.g[4];
#pragma unroll
    for (int k = SUB; k < NC; k += 4) {
        __builtin_amdgcn_sched_barrier(0);
        float Yk[W], wk[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            Yk[w] = live[w] ? sh_basis(k, dir[0][w], dir[1][w], dir[2][w]) : 0.f;
            wk[w] = 0.f;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t j = (int64_t)(3 * k + c) * n + i0;
            VW p = __builtin_nontemporal_load(reinterpret_cast<const VW*>(G.param + j));
            VW m = __builtin_nontemporal_load(reinterpret_cast<const VW*>(G.m + j));
            VW v = __builtin_nontemporal_load(reinterpret_cast<const VW*>(G.v + j));
#pragma unroll
            for (int w = 0; w < W; ++w) {
                wk[w] += gc[c][w] * p[w];   // the coefficient before its update
                float mw = m[w], vw = v[w];
                p[w] = adam_update(p[w], Yk[w] * gc[c][w], mw, vw, G.lr, adam.b1, adam.b2, adam.eps, ibc1, ibc2);
                m[w] = mw;
                v[w] = vw;
            }
            __builtin_nontemporal_store(p, reinterpret_cast<VW*>(G.param + j));
            __builtin_nontemporal_store(m, reinterpret_cast<VW*>(G.m + j));
            __builtin_nontemporal_store(v, reinterpret_cast<VW*>(G.v + j));
        }
#pragma unroll
        for (int w = 0; w < W; ++w) sh_grad_add(k, dir[0][w], dir[1][w], dir[2][w], wk[w], P[w][0], P[w][1], P[w][2]);
    }
}

// Adam steps of the means and the SH coefficients, one view, from what the split adjoint
// stored (kShf planes: view direction, colour gradient of the unclamped channels, inverse
// distance to the camera centre, the means' gradient without its SH term).  The gradient of SH
// coefficient k, channel c is Y_k(dir) gc_c, as the adjoint forms it.  The means' SH term,
// sum_k (sum_c gc_c sh_kc) grad Y_k, is formed from the coefficients read here before their
// update, so the 48 gradient planes are never written and the coefficients are read once.
// A workgroup's four waves share 64 groups of W Gaussians (W = 4: 16-byte accesses, which
// needs n % 4 == 0): wave s steps coefficients s, s + 4, ... and keeps that partial sum of the
// means' term; the partial sums meet in LDS and are combined in sh_grad's order, and wave
// q < 3 steps coordinate q of the means.
template <int DEG, int W>
__global__ __launch_bounds__(kBlock) void k_adam_sh(int64_t n, AdamFused adam) {
    using VW = float __attribute__((ext_vector_type(W)));
    static_assert(kBlock == 256, "four waves per workgroup");
    if (guard_set(adam.guard)) return;   // skipped training step (the whole workgroup leaves)
    __shared__ float sP[4][3][W][64];
    const int sub = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i0 = ((int64_t)blockIdx.x * 64 + lane) * W;
    const bool active = i0 < n;   // lanes past the end still meet the barrier
    const float* f = adam.shf;
    auto plane = [&](int q) { return *reinterpret_cast<const VW*>(f + (int64_t)q * n + i0); };
    float dir[3][W], gc[3][W], P[W][3];
    bool live[W];
    if (active) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const VW d = plane(q), c = plane(3 + q);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                dir[q][w] = d[w];
                gc[q][w] = c[w];
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            live[w] = gc[0][w] != 0.0f || gc[1][w] != 0.0f || gc[2][w] != 0.0f;
            P[w][0] = P[w][1] = P[w][2] = 0.f;
        }
        switch (sub) {   // wave-uniform
            case 0: adam_sh_sweep<DEG, W, 0>(adam, n, i0, dir, gc, live, P); break;
            case 1: adam_sh_sweep<DEG, W, 1>(adam, n, i0, dir, gc, live, P); break;
            case 2: adam_sh_sweep<DEG, W, 2>(adam, n, i0, dir, gc, live, P); break;
            default: adam_sh_sweep<DEG, W, 3>(adam, n, i0, dir, gc, live, P); break;
        }
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
            for (int q = 0; q < 3; ++q) sP[sub][q][w][lane] = P[w][q];
    }
    __syncthreads();
    if (!active || sub == 3) return;
    // coordinate q = sub of the means: the SH colour's term (partial sums in sh_grad's order)
    // added to the adjoint's part, then the step
    const int q = sub;
    const VW il = plane(6), gpart = plane(7 + q);
    const gs_adam_group& M = adam.g[0];
    const float ibc1 = adam.bc[0], ibc2 = adam.bc[1];
    const int64_t j = (int64_t)q * n + i0;
    VW p = __builtin_nontemporal_load(reinterpret_cast<const VW*>(M.param + j));
    VW m = __builtin_nontemporal_load(reinterpret_cast<const VW*>(M.m + j));
    VW v = __builtin_nontemporal_load(reinterpret_cast<const VW*>(M.v + j));
#pragma unroll
    for (int w = 0; w < W; ++w) {
        float g = gpart[w];
        if (DEG > 0 && live[w]) {
            float gd[3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                gd[r] = ((sP[0][r][w][lane] + sP[1][r][w][lane]) + sP[2][r][w][lane]) + sP[3][r][w][lane];
            const float dd = gd[0] * dir[0][w] + gd[1] * dir[1][w] + gd[2] * dir[2][w];
            g += (gd[q] - dir[q][w] * dd) * il[w];
        }
        float mw = m[w], vw = v[w];
        p[w] = adam_update(p[w], g, mw, vw, M.lr, adam.b1, adam.b2, adam.eps, ibc1, ibc2);
        m[w] = mw;
        v[w] = vw;
    }
    __builtin_nontemporal_store(p, reinterpret_cast<VW*>(M.param + j));
    __builtin_nontemporal_store(m, reinterpret_cast<VW*>(M.m + j));
    __builtin_nontemporal_store(v, reinterpret_cast<VW*>(M.v + j));
}

// Several views: the SH part of the adjoint and, when fused, the Adam steps of the SH
// coefficients and the means, from what k_project_bwd stored in adam.shf (the means' gradient
// without its SH term, then per view the colour gradient of the unclamped channels).  View v's
// direction is formed again from the mean and the camera centre, as the adjoint forms it.  The
// gradient of SH coefficient k, channel c is the sum over the views, in order, of Y_k(dir) gc_c;
// the means' SH term is, per view, sum_k (sum_c gc_c sh_kc) grad Y_k(dir) projected on the plane
// normal to dir and scaled by the inverse distance, with the coefficients before their update.
// A workgroup's four waves share 64 groups of W Gaussians: wave s handles coefficients s, s + 4,
// ... and that part of the means' term; the parts meet in LDS, ((0 + 1) + 2) + 3, and wave q < 3
// finishes coordinate q of the means.  Without FUSED the gradients are written instead.
template <int DEG, int W, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_sh_views(gs_gaussians g, int32_t views, const gs_camera* cams,
                                                    gs_gaussian_grads out, AdamFused adam) {
    using VW = float __attribute__((ext_vector_type(W)));
    static_assert(kBlock == 256, "four waves per workgroup");
    if (FUSED && guard_set(adam.guard)) return;   // skipped training step (the whole workgroup leaves)
    constexpr int NC = (DEG + 1) * (DEG + 1);
    constexpr int KS = (NC + 3) / 4;   // coefficients per wave, at most
    __shared__ float sP[4][3][W][64];
    const int64_t n = g.n;
    const int sub = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i0 = ((int64_t)blockIdx.x * 64 + lane) * W;
    const bool active = i0 < n;   // lanes past the end still meet the barrier
    const float* f = adam.shf;
    auto vload = [&](const float* base, int64_t q) { return *reinterpret_cast<const VW*>(base + q * n + i0); };
    if (active) {
        float mu[3][W], co[KS][3][W], gs[KS][3][W], R[W][3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const VW x = vload(g.means, q);
#pragma unroll
            for (int w = 0; w < W; ++w) mu[q][w] = x[w];
        }
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int k = sub + 4 * j;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                VW x = {};
                if (k < NC) x = vload(g.sh, 3 * k + c);
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    co[j][c][w] = x[w];
                    gs[j][c][w] = 0.f;
                }
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) R[w][0] = R[w][1] = R[w][2] = 0.f;
        for (int v = 0; v < views; ++v) {
            const Cam cam = load_cam(cams + v);
            float cc[3];
            camera_centre(cam, cc);
            const VW c0 = vload(f, 3 + 3 * v), c1 = vload(f, 4 + 3 * v), c2 = vload(f, 5 + 3 * v);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const float gce[3] = {c0[w], c1[w], c2[w]};
                if (gce[0] == 0.0f && gce[1] == 0.0f && gce[2] == 0.0f) continue;
                float d0 = mu[0][w] - cc[0], d1 = mu[1][w] - cc[1], d2 = mu[2][w] - cc[2];
                const float il = 1.0f / __builtin_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
                d0 *= il; d1 *= il; d2 *= il;
                float Q[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int j = 0; j < KS; ++j) {
                    const int k = sub + 4 * j;
                    if (k >= NC) break;
                    const float Yk = sh_basis(k, d0, d1, d2);
#pragma unroll
                    for (int c = 0; c < 3; ++c) gs[j][c][w] += Yk * gce[c];
                    if (DEG > 0) {
                        const float wk = (gce[0] * co[j][0][w] + gce[1] * co[j][1][w]) + gce[2] * co[j][2][w];
                        sh_grad_add(k, d0, d1, d2, wk, Q[0], Q[1], Q[2]);
                    }
                }
                if (DEG > 0) {
                    const float dd = Q[0] * d0 + Q[1] * d1 + Q[2] * d2;
                    R[w][0] += (Q[0] - d0 * dd) * il;
                    R[w][1] += (Q[1] - d1 * dd) * il;
                    R[w][2] += (Q[2] - d2 * dd) * il;
                }
            }
        }
        const float ibc1 = FUSED ? adam.bc[0] : 0.f, ibc2 = FUSED ? adam.bc[1] : 0.f;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int k = sub + 4 * j;
            if (k >= NC) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t idx = (int64_t)(3 * k + c) * n + i0;
                VW r;
                if (FUSED) {
                    const gs_adam_group& G = adam.g[4];
                    VW m = __builtin_nontemporal_load(reinterpret_cast<const VW*>(G.m + idx));
                    VW v = __builtin_nontemporal_load(reinterpret_cast<const VW*>(G.v + idx));
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        float mw = m[w], vw = v[w];
                        r[w] = adam_update(co[j][c][w], gs[j][c][w], mw, vw, G.lr, adam.b1, adam.b2, adam.eps,
                                           ibc1, ibc2);
                        m[w] = mw;
                        v[w] = vw;
                    }
                    __builtin_nontemporal_store(r, reinterpret_cast<VW*>(G.param + idx));
                    __builtin_nontemporal_store(m, reinterpret_cast<VW*>(G.m + idx));
                    __builtin_nontemporal_store(v, reinterpret_cast<VW*>(G.v + idx));
                } else {
#pragma unroll
                    for (int w = 0; w < W; ++w) r[w] = gs[j][c][w];
                    *reinterpret_cast<VW*>(out.sh + idx) = r;
                }
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
            for (int q = 0; q < 3; ++q) sP[sub][q][w][lane] = R[w][q];
    }
    __syncthreads();
    if (!active || sub == 3) return;
    const int q = sub;
    const VW gpart = vload(f, q);
    VW r;
#pragma unroll
    for (int w = 0; w < W; ++w)
        r[w] = gpart[w] + (((sP[0][q][w][lane] + sP[1][q][w][lane]) + sP[2][q][w][lane]) + sP[3][q][w][lane]);
    const int64_t j = (int64_t)q * n + i0;
    if (FUSED) {
        const gs_adam_group& M = adam.g[0];
        const float ibc1 = adam.bc[0], ibc2 = adam.bc[1];
        VW p = __builtin_nontemporal_load(reinterpret_cast<const VW*>(M.param + j));
        VW m = __builtin_nontemporal_load(reinterpret_cast<const VW*>(M.m + j));
        VW v = __builtin_nontemporal_load(reinterpret_cast<const VW*>(M.v + j));
#pragma unroll
        for (int w = 0; w < W; ++w) {
            float mw = m[w], vw = v[w];
            p[w] = adam_update(p[w], r[w], mw, vw, M.lr, adam.b1, adam.b2, adam.eps, ibc1, ibc2);
            m[w] = mw;
            v[w] = vw;
        }
        __builtin_nontemporal_store(p, reinterpret_cast<VW*>(M.param + j));
        __builtin_nontemporal_store(m, reinterpret_cast<VW*>(M.m + j));
        __builtin_nontemporal_store(v, reinterpret_cast<VW*>(M.v + j));
    } else {
        *reinterpret_cast<VW*>(out.means + j) = r;
    }
}

}  // namespace

hipError_t launch_adam_sh(int64_t n, int sh_degree, const AdamFused& adam, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (!adam.shf) return hipErrorInvalidValue;
    // 16-byte accesses need every plane (offset k n) and the base pointers 16-byte aligned
    const uintptr_t bases = (uintptr_t)adam.shf | (uintptr_t)adam.g[4].param | (uintptr_t)adam.g[4].m |
                            (uintptr_t)adam.g[4].v | (uintptr_t)adam.g[0].param | (uintptr_t)adam.g[0].m |
                            (uintptr_t)adam.g[0].v;
    const bool v4 = n % 4 == 0 && bases % 16 == 0;
    const int64_t per = v4 ? 4 : 1;
    const unsigned grid = (unsigned)(((n + per - 1) / per + 63) / 64);   // 64 groups of `per` per workgroup
#define GS_ASH(D)                                                                                    \
    if (v4)                                                                                          \
        hipLaunchKernelGGL((k_adam_sh<D, 4>), dim3(grid), dim3(kBlock), 0, s, n, adam);              \
    else                                                                                             \
        hipLaunchKernelGGL((k_adam_sh<D, 1>), dim3(grid), dim3(kBlock), 0, s, n, adam)
    switch (sh_degree) {
        case 0: GS_ASH(0); break;
        case 1: GS_ASH(1); break;
        case 2: GS_ASH(2); break;
        default: GS_ASH(3); break;
    }
#undef GS_ASH
    return hipGetLastError();
}

hipError_t launch_sh_views(const gs_gaussians& g, int32_t views, const gs_camera* cams,
                           const gs_gaussian_grads& grads, const AdamFused& adam, int fused, hipStream_t s) {
    const int64_t n = g.n;
    if (n == 0) return hipSuccess;
    if (!adam.shf || views < 2) return hipErrorInvalidValue;
    uintptr_t bases = (uintptr_t)adam.shf | (uintptr_t)g.means | (uintptr_t)g.sh;
    if (fused)
        bases |= (uintptr_t)adam.g[4].param | (uintptr_t)adam.g[4].m | (uintptr_t)adam.g[4].v |
                 (uintptr_t)adam.g[0].param | (uintptr_t)adam.g[0].m | (uintptr_t)adam.g[0].v;
    else
        bases |= (uintptr_t)grads.sh | (uintptr_t)grads.means;
    const int per = (n % kShViewsW == 0 && bases % (4 * kShViewsW) == 0) ? kShViewsW : 1;
    const unsigned grid = (unsigned)(((n + per - 1) / per + 63) / 64);   // 64 groups of `per` per workgroup
#define GS_SHV(D, WW)                                                                                          \
    if (fused)                                                                                                 \
        hipLaunchKernelGGL((k_sh_views<D, WW, true>), dim3(grid), dim3(kBlock), 0, s, g, views, cams, grads, adam); \
    else                                                                                                       \
        hipLaunchKernelGGL((k_sh_views<D, WW, false>), dim3(grid), dim3(kBlock), 0, s, g, views, cams, grads, adam)
#define GS_SHVD(D)            \
    if (per == kShViewsW) {   \
        GS_SHV(D, kShViewsW); \
    } else {                  \
        GS_SHV(D, 1);         \
    }
    switch (g.sh_degree) {
        case 0: GS_SHVD(0); break;
        case 1: GS_SHVD(1); break;
        case 2: GS_SHVD(2); break;
        default: GS_SHVD(3); break;
    }
#undef GS_SHVD
#undef GS_SHV
    return hipGetLastError();
}

hipError_t launch_project_fwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const ViewInfo* vt,
                              const gs_options& o, Record* rec, uint32_t* counts, uint2* rects,
                              uint32_t* depth_keys, uint32_t* dkeys_sort, uint32_t* dvals_sort,
                              SavedHeader* hdr, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    const unsigned grid = (unsigned)((g.n + kBlock - 1) / kBlock);
#define GS_PF(D)                                                                                            \
    hipLaunchKernelGGL(k_project_fwd<D>, dim3(grid), dim3(kBlock), 0, s, g, views, cams, vt, o.tile_w,      \
                       o.tile_h, o.kappa, o.dilation, rec, counts, rects, depth_keys, dkeys_sort, dvals_sort, hdr)
    switch (g.sh_degree) {
        case 0: GS_PF(0); break;
        case 1: GS_PF(1); break;
        case 2: GS_PF(2); break;
        default: GS_PF(3); break;
    }
#undef GS_PF
    return hipGetLastError();
}

namespace {

template <int D, bool F>
void project_bwd_launch(const gs_gaussians& g, int32_t views, const gs_camera* cams, float dil, const float* grad2d,
                        const Record* rec, const gs_gaussian_grads& grads, const AdamFused& adam, unsigned grid,
                        hipStream_t s) {
    if (views == 1 && F && adam.shf)
        hipLaunchKernelGGL((k_project_bwd<D, true, true, true>), dim3(grid), dim3(kBlock), 0, s, g, views, cams, dil,
                           grad2d, rec, grads, adam);
    else if (views == 1)
        hipLaunchKernelGGL((k_project_bwd<D, F, true, false>), dim3(grid), dim3(kBlock), 0, s, g, views, cams, dil,
                           grad2d, rec, grads, adam);
    else
        hipLaunchKernelGGL((k_project_bwd<D, F, false, true>), dim3(grid), dim3(kBlock), 0, s, g, views, cams, dil,
                           grad2d, rec, grads, adam);
}

hipError_t project_bwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const gs_options& o,
                       const float* grad2d, const Record* rec, const gs_gaussian_grads& grads, const AdamFused& adam_in,
                       int fused, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    AdamFused adam = adam_in;
    // lambda_o mean(o) and lambda_s mean(s) over n and 3 n entries (FP64 quotient rounded once)
    adam.reg_o = (float)((double)o.reg_opacity / (double)g.n);
    adam.reg_s = (float)((double)o.reg_scale / (3.0 * (double)g.n));
    const unsigned grid = (unsigned)((g.n + kBlock - 1) / kBlock);
#define GS_PB(D)                                                                                     \
    if (fused)                                                                                       \
        project_bwd_launch<D, true>(g, views, cams, o.dilation, grad2d, rec, grads, adam, grid, s);  \
    else                                                                                             \
        project_bwd_launch<D, false>(g, views, cams, o.dilation, grad2d, rec, grads, adam, grid, s)
    switch (g.sh_degree) {
        case 0: GS_PB(0); break;
        case 1: GS_PB(1); break;
        case 2: GS_PB(2); break;
        default: GS_PB(3); break;
    }
#undef GS_PB
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project_bwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const gs_options& o,
                              const float* grad2d, const Record* rec, gs_gaussian_grads grads, float* planes,
                              hipStream_t s) {
    AdamFused none;
    memset(&none, 0, sizeof(none));
    none.shf = planes;
    if (views > 1 && !planes) return hipErrorInvalidValue;
    return project_bwd(g, views, cams, o, grad2d, rec, grads, none, 0, s);
}

hipError_t launch_project_bwd_adam(const gs_gaussians& g, int32_t views, const gs_camera* cams, const gs_options& o,
                                   const float* grad2d, const Record* rec, const AdamFused& adam, hipStream_t s) {
    gs_gaussian_grads none;
    memset(&none, 0, sizeof(none));
    return project_bwd(g, views, cams, o, grad2d, rec, none, adam, 1, s);
}

}  // namespace gs
