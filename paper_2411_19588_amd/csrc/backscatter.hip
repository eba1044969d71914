// Backscatter estimation (Sec. Optimization; appendix "Backscatter Estimation", Alg. 1 and
// Alg. 2) and the L_best prior of eq. (OurFinalLoss), for packed views.
//
// Per view, from an observed image I (CHW) and a rendered depth z (eq. Depth; 0 where no
// Gaussian contributes):
//   1. I and z are resized bilinearly to `resize_height` rows and negative values set to 0
//      (Alg. 1, first steps);
//   2. the pixels with a depth are cut into `edges - 1` evenly spaced depth clusters between the
//      smallest and the largest depth; in each cluster of n pixels, the ceil(p_dark n) pixels of
//      smallest squared RGB norm (ties: lower pixel index) are the dark pixels (Alg. 2);
//   3. the dark pixels' depth range is cut into `intervals - 1` evenly spaced intervals; per
//      channel and interval, the smallest dark value (ties: lower pixel index) and its depth are
//      one point (Alg. 1);
//   4. per channel, the bounded nonlinear least-squares fit of Binf (1 - exp(-Bb z)) to the
//      points, Binf in [0, 1], Bb in [0, 5] (Sec. Optimization).
//
// Every quantity that decides a cluster, a rank or an interval is FP32, computed by a fixed
// sequence of separately rounded operations (the library is built without contraction):
//   resize axis   s = (i + 1/2) (n_in / n_out) - 1/2, clamped at 0; i0 = floor(s),
//                 i1 = min(i0 + 1, n_in - 1), w = s - i0;
//                 out = (1 - wy) ((1 - wx) a00 + wx a01) + wy ((1 - wx) a10 + wx a11);
//   bin           step = (hi - lo) / n; j = min(n - 1, floor((z - lo) / step)), all 0 if step <= 0;
//   norm          q = (r r + g g) + b b;
//   share         ceil(p_dark n) with the FP32 p_dark widened to FP64.
// The fit is FP64.
//
// Selection on the GPU: every pixel with a depth gets the key bits(q) (q >= 0, so the unsigned
// order of the bits is the float order) and its packed index as value; a stable radix sort on q,
// then a stable radix sort on the (view, cluster) segment leave each segment's pixels in (q,
// index) order, and a pixel is dark when its rank inside its segment is below the segment's
// share.  The interval minima are 64-bit atomic minima of (bits(value) << 32 | pixel index).
//
// The fit: for a fixed Bb the residual is a convex quadratic in Binf, minimised over [0, 1] by
// clamping Sum f v / Sum f^2 (f = 1 - exp(-Bb z)); the profile residual over Bb in [0, 5] is
// scanned on a grid of 4096 points by one workgroup, and the best grid point's bracket is refined
// by bisection on the sign of the profile's derivative Sum 2 r Binf z exp(-Bb z) (with the clamped
// Binf, whose own derivative does not enter at the minimum over Binf).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "internal.h"

namespace gs {
namespace {

constexpr int kBsMaxClusters = 32;      // edges <= 33
constexpr int kBsMaxIntervals = 256;    // intervals <= 257
constexpr int kBsGrid = 4096;           // grid points of the fit's scan over Bb
constexpr double kBsBbMax = 5.0, kBsBinfMax = 1.0;
constexpr uint32_t kNoKey = 0xffffffffu;

struct BsView {
    int32_t w_in, h_in, w, h;
    int64_t in_base;                    // first input pixel of the view (layout of out_depth)
    uint32_t base;                      // first resized pixel of the view
    uint32_t pad;
};

struct BsStats {
    uint32_t zmin, zmax;                // bits of the smallest / largest resized depth > 0
    uint32_t dmin, dmax;                // bits of the smallest / largest dark-pixel depth
};

struct BsArgs {
    BsView v[GS_MAX_VIEWS];
    int32_t views, clusters, intervals;   // intervals = number of depth intervals (edges - 1 of Alg. 1)
    uint32_t total;                       // resized pixels over all views
    float p_dark;
    int32_t pad;
    const float* image;                   // packed like out_rgb
    const float* depth;                   // packed like out_depth
    float* rimg;                          // [3][total] resized image
    float* rz;                            // [total] resized depth
    uint32_t* seg_of;                     // [total] (view, cluster) segment of each pixel
    BsStats* stats;                       // [views]
    uint32_t* seg_count;                  // [views * clusters]
    uint32_t* seg_start;                  // [views * clusters]
    uint32_t* seg_sel;                    // [views * clusters] dark pixels per segment
    unsigned long long* best;             // [views][3][intervals]
};

__device__ __forceinline__ int view_of(const BsArgs& a, uint32_t g) {
    int v = 0;
    while (v + 1 < a.views && g >= a.v[v + 1].base) ++v;
    return v;
}

// 0 for -0 and for values <= 0 (the resize already clamped them), +inf for non-finite values,
// so that the bits of every key are ordered like the values.
__device__ __forceinline__ float canon(float x) {
    if (!(x > 0.0f)) return 0.0f;
    return x <= 3.402823466e38f ? x : __builtin_inff();
}

__device__ __forceinline__ int bin_of(float z, float lo, float hi, int n) {
    const float step = (hi - lo) / (float)n;
    if (!(step > 0.0f)) return 0;
    const float t = (z - lo) / step;
    const float f = floorf(t);
    return f >= (float)(n - 1) ? n - 1 : (int)f;
}

// One resize axis (see the header): source indices and weight for output coordinate i.
__device__ __forceinline__ void axis(int i, int n_in, int n_out, int& i0, int& i1, float& w) {
    const float r = (float)n_in / (float)n_out;
    float s = ((float)i + 0.5f) * r - 0.5f;
    s = s > 0.0f ? s : 0.0f;
    const float f = floorf(s);
    i0 = (int)f;
    i1 = i0 + 1 < n_in ? i0 + 1 : n_in - 1;
    w = s - f;
}

// Atomic min / max of a positive float's bits over a wave: when every active lane holds the same
// address the wave reduces first and one lane updates.
__device__ __forceinline__ void wave_minmax(uint32_t* pmin, uint32_t* pmax, bool has, uint32_t bits, int view) {
    const uint64_t act = __ballot(has);
    if (act == 0) return;
    const int lead = __builtin_ctzll(act);
    const int v0 = __shfl(view, lead);
    const bool uniform = __ballot(has && view != v0) == 0;
    if (uniform) {
        uint32_t lo = has ? bits : 0xffffffffu, hi = has ? bits : 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
        }
        if ((int)(threadIdx.x & 63) == lead) {
            atomicMin(pmin, lo);
            atomicMax(pmax, hi);
        }
    } else if (has) {
        atomicMin(pmin, bits);
        atomicMax(pmax, bits);
    }
}

__global__ __launch_bounds__(kBlock) void k_bs_init(BsArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < a.views) a.stats[i] = BsStats{0x7f800000u, 0u, 0x7f800000u, 0u};
    if (i < a.views * a.clusters) a.seg_count[i] = 0u;
    if (i < a.views * 3 * a.intervals) a.best[i] = ~0ull;
}

__global__ __launch_bounds__(kBlock) void k_bs_resize(BsArgs a) {
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    const bool in = g < a.total;
    int v = 0;
    float z = 0.0f;
    if (in) {
        v = view_of(a, g);
        const BsView vw = a.v[v];
        const uint32_t k = g - vw.base;
        const int x = (int)(k % (uint32_t)vw.w), y = (int)(k / (uint32_t)vw.w);
        const int64_t plane = (int64_t)vw.w_in * vw.h_in;
        const float* Z = a.depth + vw.in_base;
        const float* I = a.image + 3 * vw.in_base;
        float o[4];
        if (vw.w == vw.w_in && vw.h == vw.h_in) {
            const int64_t p = (int64_t)y * vw.w_in + x;
            for (int c = 0; c < 3; ++c) o[c] = I[c * plane + p];
            o[3] = Z[p];
        } else {
            int x0, x1, y0, y1;
            float wx, wy;
            axis(x, vw.w_in, vw.w, x0, x1, wx);
            axis(y, vw.h_in, vw.h, y0, y1, wy);
            const int64_t r0 = (int64_t)y0 * vw.w_in, r1 = (int64_t)y1 * vw.w_in;
            const float ux = 1.0f - wx, uy = 1.0f - wy;
            for (int c = 0; c < 4; ++c) {
                const float* A = c < 3 ? I + c * plane : Z;
                const float top = ux * A[r0 + x0] + wx * A[r0 + x1];
                const float bot = ux * A[r1 + x0] + wx * A[r1 + x1];
                o[c] = uy * top + wy * bot;
            }
        }
        for (int c = 0; c < 3; ++c) a.rimg[(size_t)c * a.total + g] = o[c] > 0.0f ? o[c] : 0.0f;
        z = o[3] > 0.0f ? o[3] : 0.0f;
        a.rz[g] = z;
    }
    const bool has = in && z > 0.0f;
    wave_minmax(&a.stats[v].zmin, &a.stats[v].zmax, has, __float_as_uint(canon(z)), v);
}

// Keys of the first sort, the segment of every pixel and the segment sizes (an LDS histogram over
// the segments of the views this workgroup touches).
__global__ __launch_bounds__(kBlock) void k_bs_keys(BsArgs a, uint32_t* keys, uint32_t* vals) {
    __shared__ uint32_t h[GS_MAX_VIEWS * kBsMaxClusters];
    const uint32_t first = blockIdx.x * kBlock;
    const uint32_t last = min(first + kBlock, a.total) - 1;
    const int s0 = view_of(a, first) * a.clusters;
    const int s1 = (view_of(a, last) + 1) * a.clusters;
    for (int i = threadIdx.x; i < s1 - s0; i += kBlock) h[i] = 0u;
    __syncthreads();
    const uint32_t g = first + threadIdx.x;
    if (g < a.total) {
        const int v = view_of(a, g);
        const float z = a.rz[g];
        uint32_t key = kNoKey, seg = kNoKey;
        if (z > 0.0f) {
            const BsStats st = a.stats[v];
            const int cl = bin_of(z, __uint_as_float(st.zmin), __uint_as_float(st.zmax), a.clusters);
            seg = (uint32_t)(v * a.clusters + cl);
            const float r = a.rimg[g], gg = a.rimg[(size_t)a.total + g], b = a.rimg[2 * (size_t)a.total + g];
            const float q = (r * r + gg * gg) + b * b;
            key = __float_as_uint(canon(q));
            atomicAdd(&h[seg - s0], 1u);
        }
        keys[g] = key;
        vals[g] = g;
        a.seg_of[g] = seg;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s1 - s0; i += kBlock)
        if (h[i]) atomicAdd(&a.seg_count[s0 + i], h[i]);
}

__global__ __launch_bounds__(kBlock) void k_bs_gather(BsArgs a, const uint32_t* n_kept, const uint32_t* vals,
                                                     uint32_t* keys_out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < *n_kept) keys_out[i] = a.seg_of[vals[i]];
}

// Segment starts and dark shares (a few thousand segments at most: one thread).
__global__ void k_bs_segscan(BsArgs a) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    const double p = (double)a.p_dark;
    for (int s = 0; s < a.views * a.clusters; ++s) {
        const uint32_t c = a.seg_count[s];
        a.seg_start[s] = run;
        a.seg_sel[s] = (uint32_t)ceil(p * (double)c);
        run += c;
    }
}

__device__ __forceinline__ bool dark_at(const BsArgs& a, uint32_t i, uint32_t n, const uint32_t* segs,
                                        uint32_t& seg) {
    if (i >= n) return false;
    seg = segs[i];
    return i - a.seg_start[seg] < a.seg_sel[seg];
}

__global__ __launch_bounds__(kBlock) void k_bs_dark_range(BsArgs a, const uint32_t* n_kept, const uint32_t* segs,
                                                         const uint32_t* vals) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    uint32_t seg = 0;
    const bool dark = dark_at(a, i, *n_kept, segs, seg);
    const int v = dark ? (int)(seg / (uint32_t)a.clusters) : 0;
    const uint32_t bits = dark ? __float_as_uint(a.rz[vals[i]]) : 0u;
    wave_minmax(&a.stats[v].dmin, &a.stats[v].dmax, dark, bits, v);
}

__global__ __launch_bounds__(kBlock) void k_bs_minima(BsArgs a, const uint32_t* n_kept, const uint32_t* segs,
                                                     const uint32_t* vals) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    uint32_t seg = 0;
    if (!dark_at(a, i, *n_kept, segs, seg)) return;
    const int v = (int)(seg / (uint32_t)a.clusters);
    const uint32_t g = vals[i];
    const BsStats st = a.stats[v];
    const int j = bin_of(a.rz[g], __uint_as_float(st.dmin), __uint_as_float(st.dmax), a.intervals);
    const unsigned long long idx = g - a.v[v].base;
    for (int c = 0; c < 3; ++c) {
        const uint32_t vb = __float_as_uint(canon(a.rimg[(size_t)c * a.total + g]));
        atomicMin(&a.best[((size_t)v * 3 + c) * a.intervals + j], ((unsigned long long)vb << 32) | idx);
    }
}

// Profile residual of the fit at Bb = b: the best Binf in [0, 1] and the residual.
__device__ double profile(const double* z, const double* val, int n, double b, double& binf) {
    double sff = 0.0, sfv = 0.0;
    for (int i = 0; i < n; ++i) {
        const double f = 1.0 - exp(-b * z[i]);
        sff = fma(f, f, sff);
        sfv = fma(f, val[i], sfv);
    }
    double B = 0.0;
    if (sff > 0.0) B = fmin(fmax(sfv / sff, 0.0), kBsBinfMax);
    double r2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = B * (1.0 - exp(-b * z[i])) - val[i];
        r2 = fma(r, r, r2);
    }
    binf = B;
    return r2;
}

// Derivative of the profile residual in Bb (Binf held at its optimum).
__device__ double profile_slope(const double* z, const double* val, int n, double b) {
    double B;
    profile(z, val, n, b, B);
    double d = 0.0;
    for (int i = 0; i < n; ++i) {
        const double e = exp(-b * z[i]);
        const double r = B * (1.0 - e) - val[i];
        d = fma(2.0 * r * B * z[i], e, d);
    }
    return d;
}

// One workgroup per (view, channel): the points in interval order, then the fit.
__global__ __launch_bounds__(kBlock) void k_bs_fit(BsArgs a, float* est, float* points, float* cost) {
    __shared__ double pz[kBsMaxIntervals], pv[kBsMaxIntervals];
    __shared__ double bc[kBlock];
    __shared__ int bk[kBlock];
    __shared__ int np;
    const int v = blockIdx.x / 3, c = blockIdx.x % 3;
    const int tid = threadIdx.x;
    const unsigned long long* best = a.best + ((size_t)v * 3 + c) * a.intervals;
    if (tid == 0) {
        int n = 0;
        for (int j = 0; j < a.intervals; ++j) {
            const unsigned long long k = best[j];
            float zz = __builtin_nanf(""), vv = __builtin_nanf("");
            if (k != ~0ull) {
                zz = a.rz[a.v[v].base + (uint32_t)(k & 0xffffffffull)];
                vv = __uint_as_float((uint32_t)(k >> 32));
                pz[n] = zz;
                pv[n] = vv;
                ++n;
            }
            if (points) {
                float* p = points + (((size_t)v * 3 + c) * a.intervals + j) * 2;
                p[0] = zz;
                p[1] = vv;
            }
        }
        np = n;
    }
    __syncthreads();
    const int n = np;
    double binf = 0.0, bb = 0.0, r2 = 0.0;
    if (n > 0) {
        // grid scan of the profile residual
        double cmin = __builtin_inf();
        int kmin = kBsGrid;
        for (int k = tid; k < kBsGrid; k += kBlock) {
            double B;
            const double r = profile(pz, pv, n, kBsBbMax * (double)k / (double)(kBsGrid - 1), B);
            if (r < cmin) {
                cmin = r;
                kmin = k;
            }
        }
        bc[tid] = cmin;
        bk[tid] = kmin;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double o = bc[tid + off];
                const int ok = bk[tid + off];
                if (o < bc[tid] || (o == bc[tid] && ok < bk[tid])) {
                    bc[tid] = o;
                    bk[tid] = ok;
                }
            }
            __syncthreads();
        }
        const int k = bk[0];
        const double bk0 = kBsBbMax * (double)k / (double)(kBsGrid - 1);
        // the bracket's lower end stays off 0, where f = 0 leaves Binf undetermined and the slope 0
        double lo = kBsBbMax * (double)(k > 0 ? k - 1 : 0) / (double)(kBsGrid - 1);
        lo = fmax(lo, 1e-6 * kBsBbMax / (double)(kBsGrid - 1));
        double hi = k < kBsGrid - 1 ? kBsBbMax * (double)(k + 1) / (double)(kBsGrid - 1) : kBsBbMax;
        bb = bk0;
        r2 = profile(pz, pv, n, bb, binf);
        // bisection on the slope's sign inside the bracket (same in every thread; thread 0 writes)
        if (profile_slope(pz, pv, n, lo) < 0.0 && profile_slope(pz, pv, n, hi) > 0.0) {
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (profile_slope(pz, pv, n, mid) < 0.0)
                    lo = mid;
                else
                    hi = mid;
            }
            double B1;
            const double b1 = 0.5 * (lo + hi);
            const double c1 = profile(pz, pv, n, b1, B1);
            if (c1 <= r2) {
                bb = b1;
                binf = B1;
                r2 = c1;
            }
        }
    }
    if (tid == 0) {
        est[(size_t)v * 6 + c] = (float)binf;
        est[(size_t)v * 6 + 3 + c] = (float)bb;
        if (cost) cost[(size_t)v * 3 + c] = (float)r2;
    }
}

// L_best = lambda sum_v (|Binf - Binf_hat|_1 + |Bb - Bb_hat|_1); its gradient is added.
__global__ void k_bs_prior(int32_t views, const float* medium, const float* est, float lambda, float* loss,
                           float* grad) {
    __shared__ float part[64];
    const int tid = threadIdx.x;
    float s = 0.0f;
    for (int i = tid; i < views * 6; i += 64) {
        const int v = i / 6, k = i % 6;                  // k < 3: B_inf channel k; else B_b channel k - 3
        const int m = k < 3 ? 6 + k : k;                 // medium slot: [Bd 0..2, Bb 3..5, Binf 6..8]
        const float d = medium[v * 9 + m] - est[v * 6 + k];
        s += fabsf(d);
        if (grad) grad[v * 9 + m] += d > 0.0f ? lambda : (d < 0.0f ? -lambda : 0.0f);
    }
    part[tid] = s;
    __syncthreads();
    if (tid == 0 && loss) {
        float t = 0.0f;
        for (int i = 0; i < 64; ++i) t += part[i];
        loss[0] = lambda * t;
    }
}

struct BsLayout {
    BsArgs a;
    int sort_parts;
    int seg_bits;
    size_t o_rimg, o_rz, o_seg, o_stats, o_count, o_start, o_sel, o_best, o_ka, o_va, o_kb, o_vb, o_hist, o_nkept;
    size_t bytes;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

int bs_layout(const gs_backscatter_options* o, int32_t n_views, const gs_camera* cams, BsLayout* L) {
    if (!o || !cams || n_views < 1 || n_views > GS_MAX_VIEWS) return GS_ERR_INVALID_ARGUMENT;
    if (!(o->p_dark > 0.0f && o->p_dark <= 1.0f)) return GS_ERR_INVALID_ARGUMENT;
    if (o->edges < 2 || o->edges > kBsMaxClusters + 1) return GS_ERR_INVALID_ARGUMENT;
    if (o->intervals < 2 || o->intervals > kBsMaxIntervals + 1) return GS_ERR_INVALID_ARGUMENT;
    if (o->resize_height < 0 || o->resize_height > 32768) return GS_ERR_INVALID_ARGUMENT;
    memset(L, 0, sizeof(*L));
    BsArgs& a = L->a;
    int64_t total = 0, in_pixels = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_camera& c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 32768 || c.height > 32768) return GS_ERR_INVALID_ARGUMENT;
        BsView& bv = a.v[v];
        bv.w_in = c.width;
        bv.h_in = c.height;
        if (o->resize_height == 0 || o->resize_height == c.height) {
            bv.w = c.width;
            bv.h = c.height;
        } else {
            const double w = floor((double)c.width * (double)o->resize_height / (double)c.height + 0.5);
            bv.w = w < 1.0 ? 1 : (int32_t)w;
            bv.h = o->resize_height;
        }
        bv.in_base = in_pixels;
        bv.base = (uint32_t)total;
        in_pixels += (int64_t)c.width * c.height;
        total += (int64_t)bv.w * bv.h;
        if (total >= (1LL << 31)) return GS_ERR_INVALID_ARGUMENT;
    }
    a.views = n_views;
    a.clusters = o->edges - 1;
    a.intervals = o->intervals - 1;
    a.total = (uint32_t)total;
    a.p_dark = o->p_dark;
    int64_t parts = (total + kSortTile - 1) / kSortTile;
    L->sort_parts = (int)(parts < 1 ? 1 : (parts > kMaxSortParts ? kMaxSortParts : parts));
    int bits = 1;
    while ((1LL << bits) < (int64_t)n_views * a.clusters) ++bits;
    L->seg_bits = bits;
    const size_t T = (size_t)total, S = (size_t)n_views * a.clusters;
    size_t at = 0;
    auto take = [&](size_t b) {
        const size_t r = at;
        at = up256(at + b);
        return r;
    };
    L->o_rimg = take(3 * T * 4);
    L->o_rz = take(T * 4);
    L->o_seg = take(T * 4);
    L->o_stats = take(sizeof(BsStats) * n_views);
    L->o_count = take(S * 4);
    L->o_start = take(S * 4);
    L->o_sel = take(S * 4);
    L->o_best = take((size_t)n_views * 3 * a.intervals * 8);
    L->o_ka = take(T * 4);
    L->o_va = take(T * 4);
    L->o_kb = take(T * 4);
    L->o_vb = take(T * 4);
    L->o_hist = take(((size_t)kMaxRadix * L->sort_parts + kMaxRadix) * 4);
    L->o_nkept = take(4);
    L->bytes = at;
    return GS_OK;
}

template <typename T>
T* off(void* base, size_t o) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + o);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

void gs_default_backscatter_options(gs_backscatter_options* o) {
    if (!o) return;
    o->p_dark = 0.01f;
    o->edges = 10;
    o->intervals = 25;
    o->resize_height = 300;
}

int gs_backscatter_workspace_query(const gs_backscatter_options* opts, int32_t n_views, const gs_camera* host_cams,
                                   size_t* workspace_bytes) {
    if (!workspace_bytes) return GS_ERR_INVALID_ARGUMENT;
    BsLayout L;
    const int rc = bs_layout(opts, n_views, host_cams, &L);
    if (rc != GS_OK) return rc;
    *workspace_bytes = L.bytes;
    return GS_OK;
}

int gs_estimate_backscatter(const gs_backscatter_options* opts, int32_t n_views, const gs_camera* host_cams,
                            const float* image, const float* depth, float* est, float* points, float* cost,
                            void* workspace, size_t workspace_bytes, gs_stream_t stream) {
    BsLayout L;
    int rc = bs_layout(opts, n_views, host_cams, &L);
    if (rc != GS_OK) return rc;
    if (!image || !depth || !est || !workspace) return GS_ERR_INVALID_ARGUMENT;
    if (workspace_bytes < L.bytes) return GS_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    BsArgs a = L.a;
    a.image = image;
    a.depth = depth;
    a.rimg = off<float>(workspace, L.o_rimg);
    a.rz = off<float>(workspace, L.o_rz);
    a.seg_of = off<uint32_t>(workspace, L.o_seg);
    a.stats = off<BsStats>(workspace, L.o_stats);
    a.seg_count = off<uint32_t>(workspace, L.o_count);
    a.seg_start = off<uint32_t>(workspace, L.o_start);
    a.seg_sel = off<uint32_t>(workspace, L.o_sel);
    a.best = off<unsigned long long>(workspace, L.o_best);
    uint32_t* ka = off<uint32_t>(workspace, L.o_ka);
    uint32_t* va = off<uint32_t>(workspace, L.o_va);
    uint32_t* kb = off<uint32_t>(workspace, L.o_kb);
    uint32_t* vb = off<uint32_t>(workspace, L.o_vb);
    uint32_t* hist = off<uint32_t>(workspace, L.o_hist);
    uint32_t* nkept = off<uint32_t>(workspace, L.o_nkept);
    const int64_t init_n = std::max<int64_t>((int64_t)a.views * 3 * a.intervals, (int64_t)a.views * a.clusters);
    hipLaunchKernelGGL(k_bs_init, dim3(blocks_for(init_n)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_bs_resize, dim3(blocks_for(a.total)), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_bs_keys, dim3(blocks_for(a.total)), dim3(kBlock), 0, s, a, ka, va);
    // stable sort of the pixels with a depth by bits(q) (31 bits: q >= 0), the others dropped
    int in_b = 0;
    if (radix_sort_u32(ka, va, kb, vb, nullptr, a.total, 0, 31, L.sort_parts, hist, &in_b, "bs_sort_q", nullptr, s,
                       1, kNoKey, nkept) != hipSuccess)
        return GS_ERR_HIP;
    uint32_t *k1 = in_b ? kb : ka, *v1 = in_b ? vb : va, *k2 = in_b ? ka : kb, *v2 = in_b ? va : vb;
    hipLaunchKernelGGL(k_bs_gather, dim3(blocks_for(a.total)), dim3(kBlock), 0, s, a, nkept, v1, k1);
    // stable sort by segment: each segment's pixels stay in (q, index) order
    int in_b2 = 0;
    if (radix_sort_u32(k1, v1, k2, v2, nkept, a.total, 0, L.seg_bits, L.sort_parts, hist, &in_b2, "bs_sort_seg",
                       nullptr, s) != hipSuccess)
        return GS_ERR_HIP;
    const uint32_t* segs = in_b2 ? k2 : k1;
    const uint32_t* vals = in_b2 ? v2 : v1;
    hipLaunchKernelGGL(k_bs_segscan, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_bs_dark_range, dim3(blocks_for(a.total)), dim3(kBlock), 0, s, a, nkept, segs, vals);
    hipLaunchKernelGGL(k_bs_minima, dim3(blocks_for(a.total)), dim3(kBlock), 0, s, a, nkept, segs, vals);
    hipLaunchKernelGGL(k_bs_fit, dim3((unsigned)a.views * 3), dim3(kBlock), 0, s, a, est, points, cost);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_backscatter_prior(int32_t n_views, const float* medium, const float* est, float lambda, float* loss,
                         float* grad_medium, gs_stream_t stream) {
    if (n_views < 1 || n_views > GS_MAX_VIEWS || !medium || !est || (!loss && !grad_medium) || !(lambda >= 0.0f))
        return GS_ERR_INVALID_ARGUMENT;
    hipLaunchKernelGGL(k_bs_prior, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), n_views, medium, est,
                       lambda, loss, grad_medium);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // extern "C"
