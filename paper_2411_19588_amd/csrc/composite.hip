// Per-tile front-to-back compositing (eq. 3dgs_orig with alpha from
// eq. opacity_impact), the underwater epilogue (eq. 3dgs_uw at the depth of
// eq. Depth) and the exact adjoint.
//
// One workgroup renders one tile, one pixel per thread (16x16 = four wave64,
// or 8x8 = one wave64).  The tile's (depth-ordered) records are staged in LDS
// in batches and every lane reads the same record, so LDS reads are
// broadcasts.  A workgroup stops as soon as every pixel of the tile has
// terminated.  With depth-progressive binning the forward runs once per
// phase: per-pixel state (T, C, D, W, last contributor, terminated) carries
// over, a tile whose pixels have all terminated writes its outputs and is
// skipped by later phases.  In persistent mode a fixed grid of workgroups
// pulls tile indices from a device counter, so one launch serves every view.
//
// The adjoint walks each pixel's contributors back to front (over the phases
// in reverse) from its last contributor, recovering the transmittance by
// division (T_i = T_{i+1} / (1 - alpha_i)) instead of storing per-pixel
// lists, and reduces each Gaussian's 10 gradient terms across the wave with a
// transpose reduction before one atomic add per term.
#include "internal.h"

namespace gs {
namespace {

constexpr float kLn2 = 0.6931471805599453f;

struct FwdArgs {
    const ViewInfo* vt;
    int32_t views;
    uint32_t tiles;
    int32_t phase, last_phase;
    const gs_medium* med;
    const Record* rec;
    const uint2* ranges;      // this phase's tile ranges
    const uint32_t* vals;
    uint32_t* queue;
    uint32_t* alive;
    uint32_t* alive_count;
    float* out_rgb;
    float* out_depth;
    float* out_alpha;
    float* tfinal;
    uint32_t* nlast;
    uint8_t* done;
    float* cair;
    float* dsum;
    float* wsum;
    int64_t pixels;
    float amin, amax, tmin;
    int32_t depth_mode;
};

struct BwdArgs {
    const ViewInfo* vt;
    int32_t views;
    uint32_t tiles;
    int32_t phases;
    const gs_medium* med;
    const Record* rec;
    const uint2* ranges;      // [phases][tiles]
    const uint32_t* vals;
    uint32_t* queue;
    const float* grad_rgb;
    const float* grad_depth;
    const float* tfinal;
    const uint32_t* nlast;
    const float* cair;
    const float* dsum;
    const float* wsum;
    float* grad2d;
    float* medpart;
    int64_t pixels;
    float amin, amax, tmin;
    int32_t depth_mode;
};

// alpha exponent of one splat at one pixel: log2 of exp(-q/2), with
// q = (p - m)^T Q (p - m) and the conic pre-scaled by -log2(e)/2.
// Forward and adjoint call this same sequence, so they take identical decisions.
__device__ __forceinline__ float splat_power(const float4& ra, const float4& rb, float fpx, float fpy, float& dx,
                                             float& dy) {
    dx = fpx - ra.x;
    dy = fpy - ra.y;
    return fmaf(dx, fmaf(ra.z, dx, ra.w * dy), (rb.x * dy) * dy);
}

__device__ __forceinline__ int find_view(const ViewInfo* vt, int views, uint32_t tile) {
    int v = 0;
    while (v + 1 < views && tile >= vt[v + 1].tile_base) ++v;
    return v;
}

__device__ __forceinline__ float depth_map(float zh, int mode) {
    return mode == 1 ? 2.0f / (1.0f + expf(-0.1f * zh)) - 1.0f : zh;
}

// Sum 10 values over the 64 lanes.  Halving exchanges: at each step the lanes
// keep half of the remaining values and trade the other half with the partner
// lane, so 13 exchanges replace 60.  Afterwards lane L holds the total of value
// `which` (or which = -1).
__device__ __forceinline__ float wave_sum10(const float* v, int lane, int& which) {
    float a[5];
    const bool h5 = lane & 32;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float keep = h5 ? v[k + 5] : v[k];
        const float send = h5 ? v[k] : v[k + 5];
        a[k] = keep + __shfl_xor(send, 32);
    }
    float b[3];
    const bool h4 = lane & 16;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float lo = a[k];
        const float hi = k < 2 ? a[3 + k] : 0.0f;
        const float keep = h4 ? hi : lo;
        const float send = h4 ? lo : hi;
        b[k] = keep + __shfl_xor(send, 16);
    }
    float c[2];
    const bool h3 = lane & 8;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float lo = b[k];
        const float hi = k == 0 ? b[2] : 0.0f;
        const float keep = h3 ? hi : lo;
        const float send = h3 ? lo : hi;
        c[k] = keep + __shfl_xor(send, 8);
    }
    const bool h2 = lane & 4;
    float d = (h2 ? c[1] : c[0]) + __shfl_xor(h2 ? c[0] : c[1], 4);
    d += __shfl_xor(d, 2);
    d += __shfl_xor(d, 1);
    // value index held by this lane group
    int idx;
    if (!h4) idx = h3 ? (h2 ? -1 : 2) : (h2 ? 1 : 0);
    else idx = h3 ? -1 : (h2 ? 4 : 3);
    which = ((lane & 3) == 0 && idx >= 0) ? idx + (h5 ? 5 : 0) : -1;
    return d;
}

template <int TW, int TH, int BATCH, bool PERSISTENT>
__global__ __launch_bounds__(TW* TH) void k_composite_fwd(FwdArgs a) {
    constexpr int NT = TW * TH;
    static_assert(BATCH <= NT, "one record per thread per batch");
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x;
    for (uint32_t iter = 0;; ++iter) {
        uint32_t tile;
        if (PERSISTENT) {
            __syncthreads();
            if (tid == 0) s_tile = atomicAdd(a.queue, 1u);
            __syncthreads();
            tile = s_tile;
            if (tile >= a.tiles) return;
        } else {
            if (iter > 0) return;
            tile = blockIdx.x;
        }
        if (a.phase > 0 && a.alive[tile] == 0u) continue;   // every pixel terminated in an earlier phase
        const int v = find_view(a.vt, a.views, tile);
        const ViewInfo vi = a.vt[v];
        const uint32_t lt = tile - vi.tile_base;
        const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + tid % TW;
        const int py = (int)(lt / (uint32_t)vi.tiles_x) * TH + tid / TW;
        const bool inside = px < vi.width && py < vi.height;
        const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const uint2 rg = a.ranges[tile];
        float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, W = 0.f;
        uint32_t last = 0;
        bool done = !inside;
        if (a.phase > 0 && inside) {
            T = a.tfinal[p];
            C0 = a.cair[p];
            C1 = a.cair[a.pixels + p];
            C2 = a.cair[2 * a.pixels + p];
            D = a.dsum[p];
            W = a.wsum[p];
            last = a.nlast[p];
            done = a.done[p] != 0;
        }
        for (uint32_t b = rg.x; b < rg.y; b += BATCH) {
            if (__syncthreads_and(done)) break;
            const uint32_t idx = b + tid;
            if (tid < BATCH && idx < rg.y) {
                const Record r = a.rec[a.vals[idx]];
                sa[tid] = r.a;
                sb[tid] = r.b;
                sc[tid] = r.c;
            }
            __syncthreads();
            const int nb = min(BATCH, (int)(rg.y - b));
            if (!done) {
                for (int j = 0; j < nb; ++j) {
                    const float4 ra = sa[j], rb = sb[j];
                    float dx, dy;
                    const float pw = splat_power(ra, rb, fpx, fpy, dx, dy);
                    const float alpha = fminf(a.amax, rb.y * __builtin_amdgcn_exp2f(pw));
                    if (alpha < a.amin) continue;
                    const float Tn = T * (1.0f - alpha);
                    if (Tn < a.tmin) {
                        done = true;
                        break;
                    }
                    const float4 rc = sc[j];
                    const float w = alpha * T;
                    C0 = fmaf(w, rb.z, C0);
                    C1 = fmaf(w, rb.w, C1);
                    C2 = fmaf(w, rc.x, C2);
                    D = fmaf(w, rc.y, D);
                    W += w;
                    T = Tn;
                    last = b + j + 1;
                }
            }
            __syncthreads();
        }
        const bool any_alive = __syncthreads_or(!done);
        if (inside) {
            a.tfinal[p] = T;
            a.nlast[p] = last;
            a.done[p] = done ? 1 : 0;
            a.cair[p] = C0;
            a.cair[a.pixels + p] = C1;
            a.cair[2 * a.pixels + p] = C2;
            a.dsum[p] = D;
            a.wsum[p] = W;
        }
        if (inside && (!any_alive || a.phase == a.last_phase)) {
            const int64_t plane = (int64_t)vi.width * vi.height;
            float* rgb = a.out_rgb + 3 * vi.pix_base + (int64_t)py * vi.width + px;
            const gs_medium m = a.med[v];
            float out[3], z;
            if (W > 0.0f) {
                const float zh = D / W;
                z = depth_map(zh, a.depth_mode);
                const float Cc[3] = {C0, C1, C2};
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    out[k] = Cc[k] * expf(-m.Bd[k] * z) + m.Binf[k] * (1.0f - expf(-m.Bb[k] * z));
            } else {
                z = 0.0f;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    out[k] = a.depth_mode == 1 ? m.Binf[k] * (1.0f - expf(-m.Bb[k]))
                                               : (m.Bb[k] > 0.0f ? m.Binf[k] : 0.0f);
            }
            rgb[0] = out[0];
            rgb[plane] = out[1];
            rgb[2 * plane] = out[2];
            a.out_depth[p] = z;
            a.out_alpha[p] = W;
        }
        if (tid == 0) {
            a.alive[tile] = any_alive ? 1u : 0u;
            if (any_alive) atomicAdd(a.alive_count, 1u);
        }
    }
}

template <int TW, int TH, int BATCH, bool PERSISTENT>
__global__ __launch_bounds__(TW* TH) void k_composite_bwd(BwdArgs a) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    static_assert(BATCH <= NT, "one record per thread per batch");
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    __shared__ uint32_t se[BATCH];
    __shared__ uint32_t s_tile, s_last;
    __shared__ float s_med[NW][10];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (uint32_t iter = 0;; ++iter) {
        uint32_t tile;
        if (PERSISTENT) {
            __syncthreads();
            if (tid == 0) s_tile = atomicAdd(a.queue, 1u);
            __syncthreads();
            tile = s_tile;
            if (tile >= a.tiles) return;
        } else {
            if (iter > 0) return;
            tile = blockIdx.x;
        }
        const int v = find_view(a.vt, a.views, tile);
        const ViewInfo vi = a.vt[v];
        const uint32_t lt = tile - vi.tile_base;
        const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + tid % TW;
        const int py = (int)(lt / (uint32_t)vi.tiles_x) * TH + tid / TW;
        const bool inside = px < vi.width && py < vi.height;
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        const gs_medium m = a.med[v];
        // ---- per-pixel upstream gradient through the medium and depth
        float pm[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gW = 0.f, T = 1.0f;
        uint32_t my_last = 0;
        if (inside) {
            const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
            const int64_t plane = (int64_t)vi.width * vi.height;
            const float* g = a.grad_rgb + 3 * vi.pix_base + (int64_t)py * vi.width + px;
            const float G[3] = {g[0], g[plane], g[2 * plane]};
            const float W = a.wsum[p];
            if (W > 0.0f) {
                const float Cc[3] = {a.cair[p], a.cair[a.pixels + p], a.cair[2 * a.pixels + p]};
                const float zh = a.dsum[p] / W;
                const float z = depth_map(zh, a.depth_mode);
                float dz = a.grad_depth ? a.grad_depth[p] : 0.0f;
                float A[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    A[k] = expf(-m.Bd[k] * z);
                    const float S = expf(-m.Bb[k] * z);
                    pm[k] = -G[k] * Cc[k] * z * A[k];
                    pm[3 + k] = G[k] * m.Binf[k] * z * S;
                    pm[6 + k] = G[k] * (1.0f - S);
                    dz += G[k] * (m.Binf[k] * m.Bb[k] * S - m.Bd[k] * Cc[k] * A[k]);
                }
                const float dzh = a.depth_mode == 1 ? dz * 0.05f * (1.0f - z * z) : dz;
                gC0 = G[0] * A[0];
                gC1 = G[1] * A[1];
                gC2 = G[2] * A[2];
                gD = dzh / W;
                gW = -dzh * zh / W;
                T = a.tfinal[p];
                my_last = a.nlast[p];
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (a.depth_mode == 1) {
                        const float S = expf(-m.Bb[k]);
                        pm[6 + k] = G[k] * (1.0f - S);
                        pm[3 + k] = G[k] * m.Binf[k] * S;
                    } else {
                        pm[6 + k] = m.Bb[k] > 0.0f ? G[k] : 0.0f;
                    }
                }
            }
        }
        // ---- medium partial sums of this tile
        {
            int which;
            const float s = wave_sum10(pm, lane, which);
            if (which >= 0) s_med[wave][which] = s;
            if (tid == 0) s_last = 0;
            __syncthreads();
            if (tid < 9) {
                float t = 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w) t += s_med[w][tid];
                a.medpart[(int64_t)tile * 9 + tid] = t;
            }
            atomicMax(&s_last, my_last);
            __syncthreads();
        }
        const uint32_t block_last = s_last;
        // ---- reverse walk over the phases' ranges, last phase first
        float S = 0.0f;
        for (int ph = a.phases - 1; ph >= 0; --ph) {
            const uint2 rg = a.ranges[(size_t)ph * a.tiles + tile];
            if (rg.x >= rg.y || rg.x >= block_last) continue;
            for (uint32_t b_end = min(rg.y, block_last); b_end > rg.x;) {
                const uint32_t b0 = b_end - rg.x > (uint32_t)BATCH ? b_end - BATCH : rg.x;
                const int cnt = (int)(b_end - b0);
                if (tid < cnt) {
                    const uint32_t e = a.vals[b0 + tid];
                    const Record r = a.rec[e];
                    sa[tid] = r.a;
                    sb[tid] = r.b;
                    sc[tid] = r.c;
                    se[tid] = e;
                }
                __syncthreads();
                for (int j = cnt - 1; j >= 0; --j) {
                    bool live = inside && (b0 + (uint32_t)j) < my_last;
                    float g10[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    if (live) {
                        const float4 ra = sa[j], rb = sb[j];
                        float dx, dy;
                        const float pw = splat_power(ra, rb, fpx, fpy, dx, dy);
                        const float ev = __builtin_amdgcn_exp2f(pw);
                        const float araw = rb.y * ev;
                        const float alpha = fminf(a.amax, araw);
                        if (alpha < a.amin) {
                            live = false;
                        } else {
                            const float4 rc = sc[j];
                            const float om = 1.0f - alpha;
                            const float Ti = T / om;
                            const float w = alpha * Ti;
                            const float gf = gC0 * rb.z + gC1 * rb.w + gC2 * rc.x + gD * rc.y + gW;
                            const float dalpha = Ti * gf - S / om;
                            S = fmaf(gf, w, S);
                            T = Ti;
                            g10[6] = gC0 * w;
                            g10[7] = gC1 * w;
                            g10[8] = gC2 * w;
                            g10[9] = gD * w;
                            if (araw <= a.amax) {
                                g10[5] = dalpha * ev;
                                const float dpw = dalpha * araw * kLn2;
                                g10[2] = dpw * dx * dx;
                                g10[3] = dpw * dx * dy;
                                g10[4] = dpw * dy * dy;
                                g10[0] = -dpw * (2.0f * ra.z * dx + ra.w * dy);
                                g10[1] = -dpw * (ra.w * dx + 2.0f * rb.x * dy);
                            }
                        }
                    }
                    if (__ballot(live) != 0ull) {
                        int which;
                        const float s = wave_sum10(g10, lane, which);
                        if (which >= 0) unsafeAtomicAdd(a.grad2d + (size_t)se[j] * kGrad2D + which, s);
                    }
                }
                __syncthreads();
                b_end = b0;
            }
        }
    }
}

template <int TW, int TH, int BATCH>
hipError_t run_fwd(const FwdArgs& a, bool persistent, int grid, hipStream_t s) {
    if (persistent)
        hipLaunchKernelGGL((k_composite_fwd<TW, TH, BATCH, true>), dim3(grid), dim3(TW * TH), 0, s, a);
    else
        hipLaunchKernelGGL((k_composite_fwd<TW, TH, BATCH, false>), dim3(a.tiles), dim3(TW * TH), 0, s, a);
    return hipGetLastError();
}

template <int TW, int TH, int BATCH>
hipError_t run_bwd(const BwdArgs& a, bool persistent, int grid, hipStream_t s) {
    if (persistent)
        hipLaunchKernelGGL((k_composite_bwd<TW, TH, BATCH, true>), dim3(grid), dim3(TW * TH), 0, s, a);
    else
        hipLaunchKernelGGL((k_composite_bwd<TW, TH, BATCH, false>), dim3(a.tiles), dim3(TW * TH), 0, s, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_medium_reduce(const ViewInfo* __restrict__ vt,
                                                         const float* __restrict__ medpart,
                                                         float* __restrict__ grad_medium) {
    // one workgroup per view; deterministic: fixed per-thread strides and a fixed tree
    __shared__ float red[9][kBlock];
    const int v = blockIdx.x, tid = threadIdx.x;
    const ViewInfo vi = vt[v];
    float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint32_t t = tid; t < vi.n_tiles; t += kBlock)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += medpart[(int64_t)(vi.tile_base + t) * 9 + k];
#pragma unroll
    for (int k = 0; k < 9; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (tid < off)
#pragma unroll
            for (int k = 0; k < 9; ++k) red[k][tid] += red[k][tid + off];
        __syncthreads();
    }
    if (tid < 9) grad_medium[v * 9 + tid] = red[tid][0];
}

// Per tile: sum and max over pixels of the list entries walked (entries of the tile's
// phase ranges before the pixel's last contributor, plus the entry that stopped the walk).
template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_forward_stats(const ViewInfo* __restrict__ vt, int32_t views,
                                                         int32_t phases, uint32_t n_tiles,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ nlast,
                                                         const uint8_t* __restrict__ done,
                                                         unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_sum;
    __shared__ uint32_t s_max, s_any;
    const int tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const int v = find_view(vt, views, tile);
    const ViewInfo vi = vt[v];
    const uint32_t lt = tile - vi.tile_base;
    const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + tid % TW;
    const int py = (int)(lt / (uint32_t)vi.tiles_x) * TH + tid / TW;
    if (tid == 0) {
        s_sum = 0;
        s_max = 0;
        s_any = 0;
    }
    __syncthreads();
    if (px < vi.width && py < vi.height) {
        const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
        const uint32_t last = nlast[p];
        uint32_t walked = 0, total = 0;
        for (int ph = 0; ph < phases; ++ph) {
            const uint2 rg = ranges[(size_t)ph * n_tiles + tile];
            total += rg.y - rg.x;
            if (last > rg.x) walked += min(last, rg.y) - rg.x;
        }
        if (done[p] && walked < total) walked += 1;
        atomicAdd(&s_sum, (unsigned long long)walked);
        atomicMax(&s_max, walked);
        if (total) s_any = 1;
    }
    __syncthreads();
    if (tid == 0) {
        atomicAdd(&out[1], s_sum);
        atomicAdd(&out[2], (unsigned long long)s_max);
        if (s_any) atomicAdd(&out[3], 1ull);
    }
}

__global__ void k_stats_init(unsigned long long* out, const SavedHeader* hdr) {
    out[0] = hdr->pair_count;
    out[1] = out[2] = out[3] = 0;
}

int persistent_grid(int threads) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    return cus * (2048 / threads);
}

}  // namespace

hipError_t launch_composite_fwd(const gs_options& o, const Layout& L, int phase, const ViewInfo* vt,
                                const gs_medium* med, const Record* rec, const uint2* ranges, const uint32_t* vals,
                                SavedHeader* hdr, uint32_t* alive, float* out_rgb, float* out_depth,
                                float* out_alpha, float* tfinal, uint32_t* nlast, uint8_t* done, float* cair,
                                float* dsum, float* wsum, hipStream_t s) {
    if (L.tiles == 0) return hipSuccess;
    FwdArgs a{vt, L.views, (uint32_t)L.tiles, phase, L.phases - 1, med, rec, ranges + (size_t)phase * L.tiles, vals,
              &hdr->queue[phase], alive, &hdr->phase_alive[phase], out_rgb, out_depth, out_alpha, tfinal, nlast,
              done, cair, dsum, wsum, L.pixels, o.alpha_min, o.alpha_max, o.t_min, o.depth_mode};
    const bool pers = o.persistent != 0;
    if (o.tile_w == 8) return run_fwd<8, 8, 64>(a, pers, persistent_grid(64), s);
    switch (o.lds_batch) {
        case 64: return run_fwd<16, 16, 64>(a, pers, persistent_grid(256), s);
        case 128: return run_fwd<16, 16, 128>(a, pers, persistent_grid(256), s);
        default: return run_fwd<16, 16, 256>(a, pers, persistent_grid(256), s);
    }
}

hipError_t launch_composite_bwd(const gs_options& o, const Layout& L, const ViewInfo* vt, const gs_medium* med,
                                const Record* rec, const uint2* ranges, const uint32_t* vals, const float* grad_rgb,
                                const float* grad_depth, const float* tfinal, const uint32_t* nlast,
                                const float* cair, const float* dsum, const float* wsum, float* grad2d,
                                float* medpart, hipStream_t s) {
    if (L.tiles == 0) return hipSuccess;
    BwdArgs a{vt, L.views, (uint32_t)L.tiles, L.phases, med, rec, ranges, vals, nullptr, grad_rgb, grad_depth,
              tfinal, nlast, cair, dsum, wsum, grad2d, medpart, L.pixels, o.alpha_min, o.alpha_max, o.t_min,
              o.depth_mode};
    // the backward's persistent-mode tile counter lives after the medium partials
    a.queue = reinterpret_cast<uint32_t*>(medpart + L.tiles * 9);
    const bool pers = o.persistent != 0;
    if (pers) {
        hipError_t e = launch_fill_u32(a.queue, 0u, 1, s);
        if (e != hipSuccess) return e;
    }
    if (o.tile_w == 8) return run_bwd<8, 8, 64>(a, pers, persistent_grid(64), s);
    switch (o.lds_batch) {
        case 64: return run_bwd<16, 16, 64>(a, pers, persistent_grid(256), s);
        case 128: return run_bwd<16, 16, 128>(a, pers, persistent_grid(256), s);
        default: return run_bwd<16, 16, 256>(a, pers, persistent_grid(256), s);
    }
}

hipError_t launch_medium_reduce(const ViewInfo* vt, int32_t views, const float* medpart, float* grad_medium,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_medium_reduce, dim3(views), dim3(kBlock), 0, s, vt, medpart, grad_medium);
    return hipGetLastError();
}

hipError_t launch_forward_stats(const Layout& L, const ViewInfo* vt, const uint2* ranges, const uint32_t* nlast,
                                const uint8_t* done, const SavedHeader* hdr, unsigned long long* out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_stats_init, dim3(1), dim3(1), 0, s, out, hdr);
    if (L.tiles == 0) return hipGetLastError();
    if (L.tile_w == 8)
        hipLaunchKernelGGL((k_forward_stats<8, 8>), dim3((unsigned)L.tiles), dim3(64), 0, s, vt, L.views, L.phases,
                           (uint32_t)L.tiles, ranges, nlast, done, out);
    else
        hipLaunchKernelGGL((k_forward_stats<16, 16>), dim3((unsigned)L.tiles), dim3(256), 0, s, vt, L.views,
                           L.phases, (uint32_t)L.tiles, ranges, nlast, done, out);
    return hipGetLastError();
}

}  // namespace gs
