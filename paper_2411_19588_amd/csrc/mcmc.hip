// MCMC densification (Sec. Implementation: the densification of 3DGS replaced by the MCMC
// approach of the work the paper cites; appendix "Experimental Setup": densification every 100
// iterations, minimum opacity 0.1).  The cited work is not part of the paper, so these kernels
// implement this library's reading of it:
//   * a dead Gaussian (opacity <= dead_opacity) is moved onto a live one drawn with probability
//     proportional to opacity (relocation, in place);
//   * addition appends min(capacity, floor(1.05 n)) - n copies of Gaussians drawn the same way
//     over all n (out of place: the planes are [K][n], so a larger n is a new layout);
//   * a source drawn c times becomes N = c + 1 identical Gaussians: opacity
//     o' = 1 - (1 - o)^(1/N), so the N stacked copies have the original opacity on a ray, and
//     scales s' = s o / S(N, o') with S(N, a) = sum_{m=1..N} sum_{k<m} C(m-1, k) (-1)^k
//     a^(k+1) / sqrt(k+1), which keeps the integral of the stacked opacity profile (N capped at
//     51, o' clamped to [0.005, 1 - 2^-23]); FP64, rounded to FP32 once;
//   * every rewritten Gaussian (sources and destinations) restarts its Adam moments at 0;
//   * Langevin noise on the means between densification steps:
//     mu += lr_means * noise_lr * sigmoid(100 ((1 - o) - 0.995)) * R diag(s^2) R^T eta.
// Random numbers are inputs: one u32 per draw, eta ~ N(0, I) per mean.  A draw r picks the
// Gaussian whose integer weight interval [P_i, P_i + w_i) holds floor(r P / 2^32), with
// w_i = floor(o_i 2^24) (0 for a dead Gaussian in relocation) and P the total: integer decisions.
//
// Device work per call: the weights' exclusive prefix sums (u64) and the dead ranks by a
// three-kernel scan (block sums, one workgroup over the block sums, block-local rescan), one
// thread per draw (binary search of the prefix sums, an atomic count per source), the split of
// every drawn source, then one thread per draw copying its source's planes.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "internal.h"

namespace gs {
namespace {

constexpr int kMcItems = 4;                       // elements per thread in the scans
constexpr int kMcTile = kBlock * kMcItems;        // elements per scan block
constexpr int kMcMaxN = 51;
constexpr double kMcMinOpacity = 0.005;

struct McHeader {
    unsigned long long total;   // P, the sum of the weights
    uint32_t dead;              // dead Gaussians (relocation)
    uint32_t draws;             // draws taken (0 when P == 0)
};

// Plane sets of a Gaussian state: raw parameters, moments, activated copies.
struct McPlanes {
    float* p[5];
    float* m[5];
    float* v[5];
    float* scales;
    float* opacity;
    int32_t k[5];               // planes per group: 3, 3, 4, 1, 3 (d+1)^2
};

McPlanes planes_of(const gs_mcmc_state& s) {
    McPlanes q;
    for (int g = 0; g < 5; ++g) {
        q.p[g] = s.param[g];
        q.m[g] = s.m[g];
        q.v[g] = s.v[g];
    }
    q.scales = s.scales;
    q.opacity = s.opacity;
    q.k[0] = 3;
    q.k[1] = 3;
    q.k[2] = 4;
    q.k[3] = 1;
    q.k[4] = 3 * (s.sh_degree + 1) * (s.sh_degree + 1);
    return q;
}

__device__ __forceinline__ uint32_t weight_of(float o, float dead, int live_only) {
    if (live_only && o <= dead) return 0u;
    const float x = floorf(o * 16777216.0f);   // o 2^24 is exact; o in [0, 1]
    return x > 0.0f ? (uint32_t)x : 0u;
}

// Exclusive block scan of (u64, u32) pairs over kBlock threads; returns the block totals.
__device__ void block_scan(unsigned long long& a, uint32_t& b, unsigned long long* tot_a, uint32_t* tot_b) {
    __shared__ unsigned long long sa[kBlock / 64];
    __shared__ uint32_t sb[kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long ia = a;
    uint32_t ib = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long ya = __shfl_up(ia, d);
        const uint32_t yb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += ya;
            ib += yb;
        }
    }
    if (lane == 63) {
        sa[wv] = ia;
        sb[wv] = ib;
    }
    __syncthreads();
    unsigned long long oa = 0;
    uint32_t ob = 0;
    for (int w = 0; w < wv; ++w) {
        oa += sa[w];
        ob += sb[w];
    }
    if (tot_a) {
        unsigned long long ta = 0;
        uint32_t tb = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            ta += sa[w];
            tb += sb[w];
        }
        *tot_a = ta;
        *tot_b = tb;
    }
    a = oa + ia - a;   // exclusive
    b = ob + ib - b;
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_mc_reduce(const float* __restrict__ opacity, int64_t n, float dead,
                                                    int live_only, unsigned long long* bsum_w, uint32_t* bsum_d) {
    const int64_t base = (int64_t)blockIdx.x * kMcTile + (int64_t)threadIdx.x * kMcItems;
    unsigned long long w = 0;
    uint32_t d = 0;
#pragma unroll
    for (int k = 0; k < kMcItems; ++k) {
        const int64_t i = base + k;
        if (i < n) {
            const float o = opacity[i];
            w += weight_of(o, dead, live_only);
            d += o <= dead ? 1u : 0u;
        }
    }
    unsigned long long tw;
    uint32_t td;
    block_scan(w, d, &tw, &td);
    if (threadIdx.x == 0) {
        bsum_w[blockIdx.x] = tw;
        bsum_d[blockIdx.x] = td;
    }
}

// One workgroup: exclusive scan of the block sums in place, totals into the header.
__global__ __launch_bounds__(kBlock) void k_mc_scan_blocks(unsigned long long* bsum_w, uint32_t* bsum_d, int64_t nb,
                                                         McHeader* hdr) {
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    unsigned long long w = 0;
    uint32_t d = 0;
    for (int64_t b = b0; b < b0 + per && b < nb; ++b) {
        w += bsum_w[b];
        d += bsum_d[b];
    }
    unsigned long long tw;
    uint32_t td;
    block_scan(w, d, &tw, &td);
    for (int64_t b = b0; b < b0 + per && b < nb; ++b) {
        const unsigned long long x = bsum_w[b];
        const uint32_t y = bsum_d[b];
        bsum_w[b] = w;
        bsum_d[b] = d;
        w += x;
        d += y;
    }
    if (threadIdx.x == 0) {
        hdr->total = tw;
        hdr->dead = td;
    }
}

// Exclusive prefix sums of the weights (starts) and the dead list (indices in index order).
__global__ __launch_bounds__(kBlock) void k_mc_apply(const float* __restrict__ opacity, int64_t n, float dead,
                                                   int live_only, const unsigned long long* bsum_w,
                                                   const uint32_t* bsum_d, unsigned long long* starts,
                                                   uint32_t* dead_list) {
    const int64_t base = (int64_t)blockIdx.x * kMcTile + (int64_t)threadIdx.x * kMcItems;
    uint32_t wk[kMcItems];
    bool dk[kMcItems];
    unsigned long long w = 0;
    uint32_t d = 0;
#pragma unroll
    for (int k = 0; k < kMcItems; ++k) {
        const int64_t i = base + k;
        const float o = i < n ? opacity[i] : 2.0f;
        wk[k] = i < n ? weight_of(o, dead, live_only) : 0u;
        dk[k] = i < n && o <= dead;
        w += wk[k];
        d += dk[k] ? 1u : 0u;
    }
    block_scan(w, d, nullptr, nullptr);
    w += bsum_w[blockIdx.x];
    d += bsum_d[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kMcItems; ++k) {
        const int64_t i = base + k;
        if (i < n) {
            starts[i] = w;
            if (dead_list && dk[k]) dead_list[d] = (uint32_t)i;
        }
        w += wk[k];
        d += dk[k] ? 1u : 0u;
    }
}

// Draw j < count (count = the dead Gaussians, or `fixed`): its source by binary search of the
// prefix sums, counted per source.  dst_base >= 0: destination dst_base + j; otherwise the j-th
// dead Gaussian.
__global__ __launch_bounds__(kBlock) void k_mc_draw(const unsigned long long* __restrict__ starts, int64_t n,
                                                  const uint32_t* __restrict__ draws, int64_t fixed, McHeader* hdr,
                                                  uint32_t* src, uint32_t* counts, uint32_t* sources_out,
                                                  uint32_t* taken_out) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const unsigned long long P = hdr->total;
    const int64_t count = P == 0 ? 0 : (fixed >= 0 ? fixed : (int64_t)hdr->dead);
    if (j == 0) {
        hdr->draws = (uint32_t)count;
        if (taken_out) *taken_out = (uint32_t)count;
    }
    if (j >= count) return;
    const unsigned long long r = draws[j];
    // floor(r P / 2^32) without overflow: P = Ph 2^32 + Pl
    const unsigned long long t = r * (P >> 32) + ((r * (P & 0xffffffffull)) >> 32);
    int64_t lo = 0, hi = n;   // last i with starts[i] <= t
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (starts[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    src[j] = (uint32_t)lo;
    if (sources_out) sources_out[j] = (uint32_t)lo;
    atomicAdd(&counts[lo], 1u);
}

__device__ void zero_moments(const McPlanes& q, int64_t stride, int64_t i) {
    for (int g = 0; g < 5; ++g)
        for (int k = 0; k < q.k[g]; ++k) {
            q.m[g][(int64_t)k * stride + i] = 0.0f;
            q.v[g][(int64_t)k * stride + i] = 0.0f;
        }
}

// Every Gaussian drawn c > 0 times: split into c + 1 (opacity, scales and their raw forms), its
// moments zeroed.
__global__ __launch_bounds__(kBlock) void k_mc_split(McPlanes q, int64_t n, int64_t stride,
                                                   const uint32_t* __restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = counts[i];
    if (c == 0) return;
    const int N = (int)(c + 1 < (uint32_t)kMcMaxN ? c + 1 : (uint32_t)kMcMaxN);
    const double o = (double)q.opacity[i];
    double a = 1.0 - pow(1.0 - o, 1.0 / (double)N);
    a = fmin(fmax(a, kMcMinOpacity), 1.0 - 1.0 / 8388608.0);
    // S(N, a): binomials C(m-1, k) exact by the recurrence C(m-1, k) = C(m-1, k-1) (m-k) / k
    double S = 0.0;
    for (int m = 1; m <= N; ++m) {
        double cb = 1.0;
        for (int k = 0; k < m; ++k) {
            if (k > 0) cb = cb * (double)(m - k) / (double)k;
            const double sg = (k & 1) ? -1.0 : 1.0;
            S += cb * sg * pow(a, (double)(k + 1)) / sqrt((double)(k + 1));
        }
    }
    const double f = o / S;
    q.opacity[i] = (float)a;
    q.p[3][i] = (float)log(a / (1.0 - a));
    for (int k = 0; k < 3; ++k) {
        const double s = (double)q.scales[(int64_t)k * stride + i] * f;
        q.scales[(int64_t)k * stride + i] = (float)s;
        q.p[1][(int64_t)k * stride + i] = (float)log(s);
    }
    zero_moments(q, stride, i);
}

// Draw j: every plane of its source copied to its destination, the destination's moments zeroed.
__global__ __launch_bounds__(kBlock) void k_mc_copy(McPlanes q, int64_t stride, const McHeader* hdr,
                                                  const uint32_t* __restrict__ src, const uint32_t* __restrict__ dead_list,
                                                  int64_t dst_base) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= (int64_t)hdr->draws) return;
    const int64_t s = src[j];
    const int64_t d = dst_base >= 0 ? dst_base + j : (int64_t)dead_list[j];
    for (int g = 0; g < 5; ++g)
        for (int k = 0; k < q.k[g]; ++k) q.p[g][(int64_t)k * stride + d] = q.p[g][(int64_t)k * stride + s];
    for (int k = 0; k < 3; ++k) q.scales[(int64_t)k * stride + d] = q.scales[(int64_t)k * stride + s];
    q.opacity[d] = q.opacity[s];
    zero_moments(q, stride, d);
}

// Copy of every plane from stride n to stride n_dst (the first n Gaussians); blockIdx.y = plane.
__global__ __launch_bounds__(kBlock) void k_mc_relayout(McPlanes a, McPlanes b, int64_t n, int64_t n_dst) {
    int pl = blockIdx.y;
    const float* from = nullptr;
    float* to = nullptr;
    for (int set = 0; set < 3 && !from; ++set)
        for (int g = 0; g < 5 && !from; ++g) {
            if (pl < a.k[g]) {
                const float* const* fa = set == 0 ? (const float* const*)a.p : set == 1 ? (const float* const*)a.m
                                                                                         : (const float* const*)a.v;
                float* const* fb = set == 0 ? b.p : set == 1 ? b.m : b.v;
                from = fa[g] + (int64_t)pl * n;
                to = fb[g] + (int64_t)pl * n_dst;
            } else {
                pl -= a.k[g];
            }
        }
    if (!from) {
        if (pl < 3) {
            from = a.scales + (int64_t)pl * n;
            to = b.scales + (int64_t)pl * n_dst;
        } else {
            from = a.opacity;
            to = b.opacity;
        }
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock, t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(from) & 15) == 0) {   // 16-byte loads (and stores where aligned)
        const int64_t n4 = n / 4;
        const float4* f4 = reinterpret_cast<const float4*>(from);
        if ((reinterpret_cast<uintptr_t>(to) & 15) == 0) {
            float4* d4 = reinterpret_cast<float4*>(to);
            for (int64_t i = t0; i < n4; i += stride) d4[i] = f4[i];
        } else {
            for (int64_t i = t0; i < n4; i += stride) {
                const float4 v = f4[i];
                to[4 * i] = v.x;
                to[4 * i + 1] = v.y;
                to[4 * i + 2] = v.z;
                to[4 * i + 3] = v.w;
            }
        }
        done = 4 * n4;
    }
    for (int64_t i = done + t0; i < n; i += stride) to[i] = from[i];
}

__global__ __launch_bounds__(kBlock) void k_mc_noise(float* means, const float* __restrict__ quats,
                                                   const float* __restrict__ scales, const float* __restrict__ opacity,
                                                   const float* __restrict__ eta, int64_t n, float step) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float w = quats[i], x = quats[n + i], y = quats[2 * n + i], z = quats[3 * n + i];
    const float inv = 1.0f / sqrtf(((w * w + x * x) + y * y) + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                        2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                        2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    const float s2[3] = {scales[i] * scales[i], scales[n + i] * scales[n + i], scales[2 * n + i] * scales[2 * n + i]};
    const float e[3] = {eta[i], eta[n + i], eta[2 * n + i]};
    // R diag(s^2) R^T eta = R (s^2 * (R^T eta))
    float u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = s2[k] * ((R[k] * e[0] + R[3 + k] * e[1]) + R[6 + k] * e[2]);
    const float o = opacity[i];
    const float gate = 1.0f / (1.0f + expf(-100.0f * ((1.0f - o) - 0.995f)));
    const float sc = step * gate;
#pragma unroll
    for (int r = 0; r < 3; ++r) means[(int64_t)r * n + i] += sc * ((R[3 * r] * u[0] + R[3 * r + 1] * u[1]) + R[3 * r + 2] * u[2]);
}

struct McLayout {
    int64_t nb;
    size_t o_hdr, o_bw, o_bd, o_starts, o_dead, o_src, o_counts, bytes;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

McLayout mc_layout(int64_t n, int64_t n_draws) {
    McLayout L;
    L.nb = (n + kMcTile - 1) / kMcTile;
    if (L.nb < 1) L.nb = 1;
    size_t at = 0;
    auto take = [&](size_t b) {
        const size_t r = at;
        at = up256(at + b);
        return r;
    };
    L.o_hdr = take(sizeof(McHeader));
    L.o_bw = take((size_t)L.nb * 8);
    L.o_bd = take((size_t)L.nb * 4);
    L.o_starts = take((size_t)n * 8);
    L.o_dead = take((size_t)n * 4);
    L.o_src = take((size_t)(n_draws > 0 ? n_draws : 1) * 4);
    L.o_counts = take((size_t)n * 4);
    L.bytes = at;
    return L;
}

template <typename T>
T* off(void* base, size_t o) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + o);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

bool state_ok(const gs_mcmc_state* s) {
    if (!s || s->n < 1 || s->n > 0x7fffffffLL || s->sh_degree < 0 || s->sh_degree > 3) return false;
    for (int g = 0; g < 5; ++g)
        if (!s->param[g] || !s->m[g] || !s->v[g]) return false;
    return s->scales && s->opacity;
}

// Weights, their prefix sums, the dead list and the draws (relocation: fixed < 0).
int mc_draws(const McLayout& L, void* ws, const float* opacity, int64_t n, float dead, int live_only,
             const uint32_t* draws, int64_t fixed, uint32_t* sources_out, uint32_t* taken_out, hipStream_t s) {
    McHeader* hdr = off<McHeader>(ws, L.o_hdr);
    unsigned long long* bw = off<unsigned long long>(ws, L.o_bw);
    uint32_t* bd = off<uint32_t>(ws, L.o_bd);
    hipLaunchKernelGGL(k_mc_reduce, dim3((unsigned)L.nb), dim3(kBlock), 0, s, opacity, n, dead, live_only, bw, bd);
    hipLaunchKernelGGL(k_mc_scan_blocks, dim3(1), dim3(kBlock), 0, s, bw, bd, L.nb, hdr);
    hipLaunchKernelGGL(k_mc_apply, dim3((unsigned)L.nb), dim3(kBlock), 0, s, opacity, n, dead, live_only, bw, bd,
                       off<unsigned long long>(ws, L.o_starts), off<uint32_t>(ws, L.o_dead));
    if (launch_fill_u32(off<uint32_t>(ws, L.o_counts), 0u, n, s) != hipSuccess) return GS_ERR_HIP;
    const int64_t grid = fixed >= 0 ? fixed : n;
    hipLaunchKernelGGL(k_mc_draw, dim3(blocks_for(grid > 0 ? grid : 1)), dim3(kBlock), 0, s,
                       off<unsigned long long>(ws, L.o_starts), n, draws, fixed, hdr, off<uint32_t>(ws, L.o_src),
                       off<uint32_t>(ws, L.o_counts), sources_out, taken_out);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int64_t gs_mcmc_add_count(int64_t n, int64_t capacity, double growth) {
    if (n < 0 || capacity < 0 || !(growth >= 1.0)) return 0;
    const int64_t grown = (int64_t)floor(growth * (double)n);
    const int64_t target = grown < capacity ? grown : capacity;
    return target > n ? target - n : 0;
}

int gs_mcmc_workspace_query(int64_t n, int64_t n_draws, size_t* workspace_bytes) {
    if (!workspace_bytes || n < 1 || n_draws < 0) return GS_ERR_INVALID_ARGUMENT;
    *workspace_bytes = mc_layout(n, n_draws).bytes;
    return GS_OK;
}

int gs_mcmc_relocate(gs_mcmc_state* state, float dead_opacity, const uint32_t* draws, uint32_t* sources,
                     uint32_t* taken, void* workspace, size_t workspace_bytes, gs_stream_t stream) {
    if (!state_ok(state) || !draws || !workspace || !(dead_opacity >= 0.0f && dead_opacity < 1.0f))
        return GS_ERR_INVALID_ARGUMENT;
    const int64_t n = state->n;
    const McLayout L = mc_layout(n, n);
    if (workspace_bytes < L.bytes) return GS_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = mc_draws(L, workspace, state->opacity, n, dead_opacity, 1, draws, -1, sources, taken, s);
    if (rc != GS_OK) return rc;
    const McPlanes q = planes_of(*state);
    hipLaunchKernelGGL(k_mc_split, dim3(blocks_for(n)), dim3(kBlock), 0, s, q, n, n,
                       off<uint32_t>(workspace, L.o_counts));
    hipLaunchKernelGGL(k_mc_copy, dim3(blocks_for(n)), dim3(kBlock), 0, s, q, n, off<McHeader>(workspace, L.o_hdr),
                       off<uint32_t>(workspace, L.o_src), off<uint32_t>(workspace, L.o_dead), (int64_t)-1);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_mcmc_add(const gs_mcmc_state* src, gs_mcmc_state* dst, const uint32_t* draws, uint32_t* sources,
                uint32_t* taken, void* workspace, size_t workspace_bytes, gs_stream_t stream) {
    if (!state_ok(src) || !state_ok(dst) || !draws || !workspace) return GS_ERR_INVALID_ARGUMENT;
    if (dst->sh_degree != src->sh_degree || dst->n < src->n) return GS_ERR_INVALID_ARGUMENT;
    const int64_t n = src->n, k = dst->n - src->n;
    const McLayout L = mc_layout(n, k);
    if (workspace_bytes < L.bytes) return GS_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const McPlanes a = planes_of(*src), b = planes_of(*dst);
    const int planes = 3 * (3 + 3 + 4 + 1 + a.k[4]) + 4;
    const unsigned gx = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_mc_relayout, dim3(gx, (unsigned)planes), dim3(kBlock), 0, s, a, b, n, dst->n);
    int rc = mc_draws(L, workspace, src->opacity, n, 0.0f, 0, draws, k, sources, taken, s);
    if (rc != GS_OK) return rc;
    hipLaunchKernelGGL(k_mc_split, dim3(blocks_for(n)), dim3(kBlock), 0, s, b, n, dst->n,
                       off<uint32_t>(workspace, L.o_counts));
    if (k > 0)
        hipLaunchKernelGGL(k_mc_copy, dim3(blocks_for(k)), dim3(kBlock), 0, s, b, dst->n,
                           off<McHeader>(workspace, L.o_hdr), off<uint32_t>(workspace, L.o_src), nullptr, n);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_mcmc_noise(int64_t n, float* means, const float* quats, const float* scales, const float* opacity,
                  const float* eta, float lr_means, float noise_lr, gs_stream_t stream) {
    if (n < 0 || (n > 0 && (!means || !quats || !scales || !opacity || !eta))) return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    hipLaunchKernelGGL(k_mc_noise, dim3(blocks_for(n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream), means,
                       quats, scales, opacity, eta, n, lr_means * noise_lr);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // extern "C"
