// Image loss of eq. (3DGSoriginalLoss) / (OurFinalLoss): (1 - lambda) L1 + lambda D-SSIM per
// view, summed over the views, and its gradient w.r.t. the rendered image, in one pass.
//
// D-SSIM = 1 - mean SSIM (per colour channel, 11x11 Gaussian window of standard deviation 1.5,
// zero padding, C1 = 0.01^2, C2 = 0.03^2).  SSIM depends on the rendered channel x only
// through three windowed sums at every pixel p, m1 = w*x, m2 = w*x^2 and m12 = w*(x y), so
//     dL/dx(q) = sum_p w(q - p) [a(p) + 2 x(q) b(p) + y(q) c(p)],
// with (a, b, c) = dL/dS(p) * (dS/dm1, dS/dm2, dS/dm12)(p).  One workgroup owns a 32x16 tile of
// one channel: it stages x and y with a 10-pixel halo in LDS, forms the five windowed sums on
// the tile with a 5-pixel halo (a horizontal then a vertical 11-tap pass, the window being
// separable), the SSIM value and (a, b, c) there, and the three windowed sums of (a, b, c) on
// the tile (the adjoint of a zero-padded symmetric window sum is the same window sum over the
// image), so no intermediate map reaches HBM: the pass reads x and y and writes the gradient.
// Each workgroup writes its tile's sums of |x - y| and of SSIM to a partial buffer, which one
// workgroup adds in a fixed order into the per-view losses (deterministic).
#include <math.h>
#include <string.h>

#include <mutex>

#include "internal.h"

namespace gs {
namespace {

constexpr int kTW = 32, kTH = 16;             // output tile of one workgroup (one channel)
constexpr int kR = 5;                         // window radius
constexpr int kTaps = 2 * kR + 1;
constexpr int kIW = kTW + 4 * kR, kIH = kTH + 4 * kR;   // staged input (two halos)
constexpr int kMW = kTW + 2 * kR, kMH = kTH + 2 * kR;   // windowed sums and SSIM terms (one halo)
constexpr int kLossThreads = 256;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct LossView {
    int32_t width, height, tiles_x, tiles_y;
    int64_t pix_base;       // first pixel of the view (images are 3 planes per view)
    int32_t block_base;     // first workgroup of the view
    int32_t pad;
};

struct LossArgs {
    LossView v[GS_MAX_VIEWS];
    int32_t views;
    int32_t blocks;
    float g[kTaps];         // normalised 1D Gaussian, the window's separable factor
    float lambda;
    const float* pred;
    const float* target;
    float* grad;            // nullable
    float* partial;         // [blocks][2]: sum |x - y|, sum SSIM over the tile's pixels
};

__global__ __launch_bounds__(kLossThreads) void k_l1_dssim(LossArgs a) {
    // x and y staged; after the first window pass the same memory holds (a, b, c) on the tile with
    // one halo (three workgroups fit per CU)
    __shared__ float stage[2 * kIH * kIW];
    __shared__ float hm[5][kIH][kMW];          // horizontal sums; reused for the adjoint's horizontal pass
    static_assert(3 * kMH * kMW <= 2 * kIH * kIW, "(a, b, c) fit in the staging memory");
    float(*sx)[kIW] = reinterpret_cast<float(*)[kIW]>(stage);
    float(*sy)[kIW] = reinterpret_cast<float(*)[kIW]>(stage + kIH * kIW);
    float(*sd)[kMH][kMW] = reinterpret_cast<float(*)[kMH][kMW]>(stage);
    __shared__ float red[2][kLossThreads / 64];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    int v = 0;
    while (v + 1 < a.views && blk >= a.v[v + 1].block_base) ++v;
    const LossView vw = a.v[v];
    const int local = blk - vw.block_base;
    const int ntiles = vw.tiles_x * vw.tiles_y;
    const int ch = local / ntiles;
    const int t = local - ch * ntiles;
    const int x0 = (t % vw.tiles_x) * kTW, y0 = (t / vw.tiles_x) * kTH;
    const int W = vw.width, H = vw.height;
    const int64_t plane = (int64_t)W * H;
    const int64_t base = 3 * vw.pix_base + (int64_t)ch * plane;
    const float* X = a.pred + base;
    const float* Y = a.target + base;

    // ---- stage x and y with a 2R halo (zero outside the image)
    for (int i = tid; i < kIH * kIW; i += kLossThreads) {
        const int r = i / kIW, c = i - r * kIW;
        const int gy = y0 - 2 * kR + r, gx = x0 - 2 * kR + c;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        sx[r][c] = in ? X[(int64_t)gy * W + gx] : 0.0f;
        sy[r][c] = in ? Y[(int64_t)gy * W + gx] : 0.0f;
    }
    __syncthreads();
    // The four window passes are register-blocked: a thread reads a run of LDS values once and
    // forms several consecutive outputs from registers, each with the taps in order (the same
    // FMA chain per output as a one-output-per-thread pass).
    // ---- horizontal window sums of x, y, x^2, y^2, x y on every staged row, one-halo columns:
    //      thread (row, run) forms kH1 consecutive columns
    constexpr int kH1 = 6, kH1Runs = kMW / kH1;
    static_assert(kH1Runs * kH1 == kMW && kIH * kH1Runs <= kLossThreads, "one pass");
    if (tid < kIH * kH1Runs) {
        const int r = tid / kH1Runs, c0 = (tid - r * kH1Runs) * kH1;
        float xv[kH1 + kTaps - 1], yv[kH1 + kTaps - 1];
#pragma unroll
        for (int j = 0; j < kH1 + kTaps - 1; ++j) {
            xv[j] = sx[r][c0 + j];
            yv[j] = sy[r][c0 + j];
        }
#pragma unroll
        for (int o = 0; o < kH1; ++o) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
            for (int k = 0; k < kTaps; ++k) {
                const float x = xv[o + k], y = yv[o + k], w = a.g[k];
                s0 = fmaf(w, x, s0);
                s1 = fmaf(w, y, s1);
                s2 = fmaf(w, x * x, s2);
                s3 = fmaf(w, y * y, s3);
                s4 = fmaf(w, x * y, s4);
            }
            hm[0][r][c0 + o] = s0;
            hm[1][r][c0 + o] = s1;
            hm[2][r][c0 + o] = s2;
            hm[3][r][c0 + o] = s3;
            hm[4][r][c0 + o] = s4;
        }
    }
    __syncthreads();
    // ---- vertical sums, SSIM and its derivatives w.r.t. (m1, m2, m12) on the one-halo region:
    //      thread (column, run) forms kV1 consecutive rows
    const float dscale = -a.lambda / (3.0f * (float)plane);   // dL/dS: L holds lambda (1 - mean S)
    float s_sum = 0.0f;
    constexpr int kV1 = 5, kV1Runs = (kMH + kV1 - 1) / kV1;
    static_assert(kMW * kV1Runs <= kLossThreads, "one pass");
    if (tid < kMW * kV1Runs) {
        const int c = tid % kMW, r0 = (tid / kMW) * kV1;
        float m[5][kV1];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            float col[kV1 + kTaps - 1];
#pragma unroll
            for (int j = 0; j < kV1 + kTaps - 1; ++j) col[j] = r0 + j < kIH ? hm[q][r0 + j][c] : 0.0f;
#pragma unroll
            for (int o = 0; o < kV1; ++o) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < kTaps; ++k) acc = fmaf(a.g[k], col[o + k], acc);
                m[q][o] = acc;
            }
        }
#pragma unroll
        for (int o = 0; o < kV1; ++o) {
            const int r = r0 + o;
            if (r >= kMH) break;
            const int gy = y0 - kR + r, gx = x0 - kR + c;
            float da = 0.f, db = 0.f, dc = 0.f;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const float mx = m[0][o], my = m[1][o];
                const float sxx = m[2][o] - mx * mx, syy = m[3][o] - my * my, sxy = m[4][o] - mx * my;
                const float A1 = fmaf(2.0f * mx, my, kC1), A2 = fmaf(2.0f, sxy, kC2);
                const float B1 = fmaf(mx, mx, fmaf(my, my, kC1)), B2 = sxx + syy + kC2;
                const float iden = 1.0f / (B1 * B2);
                const float S = A1 * A2 * iden;
                // 1/B1 = B2 iden and 1/B2 = B1 iden: one division per pixel
                const float di = dscale * iden;
                da = 2.0f * di * (my * (A2 - A1) - S * mx * (B2 - B1));
                db = -di * S * B1;
                dc = 2.0f * di * A1;
                if (r >= kR && r < kR + kTH && c >= kR && c < kR + kTW) s_sum += S;
            }
            sd[0][r][c] = da;
            sd[1][r][c] = db;
            sd[2][r][c] = dc;
        }
    }
    __syncthreads();
    // ---- adjoint: horizontal sums of (a, b, c) on the one-halo rows, tile columns: thread (row,
    //      run) forms kH2 consecutive columns
    constexpr int kH2 = 4, kH2Runs = kTW / kH2;
    static_assert(kH2Runs * kH2 == kTW && kMH * kH2Runs <= kLossThreads, "one pass");
    if (tid < kMH * kH2Runs) {
        const int r = tid / kH2Runs, c0 = (tid - r * kH2Runs) * kH2;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float row[kH2 + kTaps - 1];
#pragma unroll
            for (int j = 0; j < kH2 + kTaps - 1; ++j) row[j] = sd[q][r][c0 + j];
#pragma unroll
            for (int o = 0; o < kH2; ++o) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < kTaps; ++k) acc = fmaf(a.g[k], row[o + k], acc);
                hm[q][r][c0 + o] = acc;
            }
        }
    }
    __syncthreads();
    // ---- vertical sums, the gradient and the tile's L1 sum: thread (column, run) forms kV2
    //      consecutive rows
    const float l1g = (1.0f - a.lambda) / (3.0f * (float)plane);
    float l_sum = 0.0f;
    constexpr int kV2 = 2, kV2Runs = kTH / kV2;
    static_assert(kV2Runs * kV2 == kTH && kTW * kV2Runs <= kLossThreads, "one pass");
    if (tid < kTW * kV2Runs) {
        const int c = tid % kTW, r0 = (tid / kTW) * kV2;
        float g3[3][kV2];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float col[kV2 + kTaps - 1];
#pragma unroll
            for (int j = 0; j < kV2 + kTaps - 1; ++j) col[j] = hm[q][r0 + j][c];
#pragma unroll
            for (int o = 0; o < kV2; ++o) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < kTaps; ++k) acc = fmaf(a.g[k], col[o + k], acc);
                g3[q][o] = acc;
            }
        }
#pragma unroll
        for (int o = 0; o < kV2; ++o) {
            const int r = r0 + o;
            const int gy = y0 + r, gx = x0 + c;
            if (gx >= W || gy >= H) continue;
            const float xv = X[(int64_t)gy * W + gx], yv = Y[(int64_t)gy * W + gx];
            const float d = xv - yv;
            l_sum += fabsf(d);
            if (a.grad) {
                const float sg = d > 0.0f ? l1g : (d < 0.0f ? -l1g : 0.0f);
                a.grad[base + (int64_t)gy * W + gx] = sg + fmaf(2.0f * xv, g3[1][o], fmaf(yv, g3[2][o], g3[0][o]));
            }
        }
    }
    // ---- the tile's sums, reduced over the workgroup in a fixed order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s_sum += __shfl_xor(s_sum, off);
        l_sum += __shfl_xor(l_sum, off);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = l_sum;
        red[1][tid >> 6] = s_sum;
    }
    __syncthreads();
    if (tid == 0) {
        float l = 0.f, s = 0.f;
#pragma unroll
        for (int w = 0; w < kLossThreads / 64; ++w) {
            l += red[0][w];
            s += red[1][w];
        }
        a.partial[2 * (int64_t)blk] = l;
        a.partial[2 * (int64_t)blk + 1] = s;
    }
}

// One workgroup: for each view, the sum of its tiles' partials (fixed strides and tree), then
// loss[v] = (1 - lambda) sum|x - y| / n + lambda (1 - sum S / n), n = 3 W H, and loss[views] = the
// sum over the views.
__global__ __launch_bounds__(kLossThreads) void k_loss_reduce(LossArgs a, float* loss) {
    __shared__ float red[2][kLossThreads];
    const int tid = threadIdx.x;
    float total = 0.0f;
    for (int v = 0; v < a.views; ++v) {
        const LossView vw = a.v[v];
        const int b0 = vw.block_base;
        const int b1 = v + 1 < a.views ? a.v[v + 1].block_base : a.blocks;
        float l = 0.f, s = 0.f;
        for (int b = b0 + tid; b < b1; b += kLossThreads) {
            l += a.partial[2 * (int64_t)b];
            s += a.partial[2 * (int64_t)b + 1];
        }
        red[0][tid] = l;
        red[1][tid] = s;
        __syncthreads();
        for (int off = kLossThreads / 2; off > 0; off >>= 1) {
            if (tid < off) {
                red[0][tid] += red[0][tid + off];
                red[1][tid] += red[1][tid + off];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const float n = 3.0f * (float)vw.width * (float)vw.height;
            const float lv = (1.0f - a.lambda) * (red[0][0] / n) + a.lambda * (1.0f - red[1][0] / n);
            loss[v] = lv;
            total += lv;
        }
        __syncthreads();
    }
    if (tid == 0) loss[a.views] = total;
}

// Host: the per-view tile table, the number of workgroups and the window's 1D factor.
int loss_layout(int32_t n_views, const gs_camera* cams, float lambda, LossArgs* a) {
    if (!cams || n_views < 1 || n_views > GS_MAX_VIEWS || !(lambda >= 0.0f && lambda <= 1.0f))
        return GS_ERR_INVALID_ARGUMENT;
    memset(a, 0, sizeof(*a));
    int64_t blocks = 0, pixels = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_camera& c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 32768 || c.height > 32768) return GS_ERR_INVALID_ARGUMENT;
        LossView& lv = a->v[v];
        lv.width = c.width;
        lv.height = c.height;
        lv.tiles_x = (c.width + kTW - 1) / kTW;
        lv.tiles_y = (c.height + kTH - 1) / kTH;
        lv.pix_base = pixels;
        lv.block_base = (int32_t)blocks;
        blocks += 3LL * lv.tiles_x * lv.tiles_y;
        pixels += (int64_t)c.width * c.height;
        if (blocks >= (1LL << 30)) return GS_ERR_INVALID_ARGUMENT;
    }
    a->views = n_views;
    a->blocks = (int32_t)blocks;
    double g[kTaps], sum = 0.0;
    for (int k = 0; k < kTaps; ++k) {
        const double r = (double)(k - kR);
        g[k] = exp(-r * r / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < kTaps; ++k) a->g[k] = (float)(g[k] / sum);
    a->lambda = lambda;
    return GS_OK;
}

}  // namespace

int loss_partial_bytes(int32_t n_views, const gs_camera* cams, size_t* bytes) {
    LossArgs a;
    const int rc = loss_layout(n_views, cams, 0.0f, &a);
    if (rc != GS_OK) return rc;
    *bytes = (size_t)a.blocks * 2 * sizeof(float);
    return GS_OK;
}

int launch_l1_dssim(int32_t n_views, const gs_camera* cams, const float* pred, const float* target, float lambda,
                    float* loss, float* grad, float* partial, size_t partial_bytes, hipStream_t s) {
    LossArgs a;
    const int rc = loss_layout(n_views, cams, lambda, &a);
    if (rc != GS_OK) return rc;
    if (!pred || !target || !partial || (!loss && !grad)) return GS_ERR_INVALID_ARGUMENT;
    if (partial_bytes < (size_t)a.blocks * 2 * sizeof(float)) return GS_ERR_WORKSPACE_TOO_SMALL;
    a.pred = pred;
    a.target = target;
    a.grad = grad;
    a.partial = partial;
    hipLaunchKernelGGL(k_l1_dssim, dim3((unsigned)a.blocks), dim3(kLossThreads), 0, s, a);
    if (loss) hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(kLossThreads), 0, s, a, loss);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

// Scratch of gs_l1_dssim_loss_noalloc: the per-workgroup partial sums live in a file-scope
// device array (each device holds its own copy until the process ends), so that entry point
// allocates nothing.  2^20 workgroups (8 MiB) cover 64 views of 1920 x 1080 (783,360).
constexpr int64_t kNoAllocMaxBlocks = 1LL << 20;
static __device__ __align__(256) float scratch[2 * kNoAllocMaxBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, found once

// The device address of `scratch` on the current device.  In host code the array's name is a
// host-side stand-in, so its address must come from hipGetSymbolAddress (once per device, with
// that device current); every later use goes through the returned pointer.
int scratch_address(float** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GS_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return GS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS_ERR_HIP;
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

int gs_l1_dssim_loss_noalloc(int32_t n_views, const gs_camera* host_cams, const float* pred, const float* target,
                             float lambda, float* loss, float* grad, gs_stream_t stream) {
    size_t need = 0;
    int rc = loss_partial_bytes(n_views, host_cams, &need);
    if (rc != GS_OK) return rc;
    if (need > (size_t)kNoAllocMaxBlocks * 2 * sizeof(float)) return GS_ERR_WORKSPACE_TOO_SMALL;
    float* partial = nullptr;
    rc = scratch_address(&partial);
    if (rc != GS_OK) return rc;
    return launch_l1_dssim(n_views, host_cams, pred, target, lambda, loss, grad, partial,
                           (size_t)kNoAllocMaxBlocks * 2 * sizeof(float), static_cast<hipStream_t>(stream));
}

int gs_loss_workspace_query(int32_t n_views, const gs_camera* host_cams, size_t* workspace_bytes) {
    if (!workspace_bytes) return GS_ERR_INVALID_ARGUMENT;
    return loss_partial_bytes(n_views, host_cams, workspace_bytes);
}

int gs_l1_dssim_loss(int32_t n_views, const gs_camera* host_cams, const float* pred, const float* target,
                     float lambda, float* loss, float* grad, void* workspace, size_t workspace_bytes,
                     gs_stream_t stream) {
    return launch_l1_dssim(n_views, host_cams, pred, target, lambda, loss, grad, static_cast<float*>(workspace),
                           workspace_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
