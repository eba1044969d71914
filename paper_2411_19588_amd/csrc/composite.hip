// Per-tile front-to-back compositing (eq. 3dgs_orig with alpha from
// eq. opacity_impact), the underwater epilogue (eq. 3dgs_uw at the depth of
// eq. Depth) and the exact adjoint.
//
// One wave64 renders one tile: a 16x16 tile gives every lane 4 pixels (rows
// y, y+4, y+8, y+12 of its column), an 8x8 tile one pixel.  The tile's
// depth-ordered records are staged in LDS in batches (one or more per lane)
// and every lane reads the same record (broadcast), so the record loads, the
// loop control, the early-exit vote and the adjoint's reduction are shared by
// the lane's pixels.  A wave stops as soon as all of its pixels have
// terminated.  With depth-progressive binning the forward runs once per phase:
// per-pixel state (T, C, D, W, last contributor, terminated) carries over, and
// a tile whose pixels have all terminated writes its outputs and is skipped by
// later phases.  In persistent mode a fixed grid of waves pulls tile indices
// from a device counter, so one launch serves every view.
//
// The adjoint walks each pixel's contributors back to front (over the phases
// in reverse) from its last contributor, recovering the transmittance by
// T_i = T_{i+1} / (1 - alpha_i) instead of storing per-pixel lists; each lane
// sums its pixels' terms for a Gaussian, the wave reduces the 10 terms with a
// transpose reduction on cross-lane swaps (v_permlane32_swap, v_permlane16_swap,
// DPP row mirrors and quad permutes), and 10 lanes issue one atomic add each.
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

__device__ __forceinline__ float dpp_f(float v, int ctrl) {
    switch (ctrl) {   // the DPP control must be a compile-time constant
        case 0x140: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
        case 0x141: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
        case 0x4E: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
        default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    }
}

// lo + hi exchanged across the two halves of the wave (lanes l and l^32): lanes < 32 get
// lo(l) + lo(l+32), lanes >= 32 get hi(l-32) + hi(l).
__device__ __forceinline__ float swap32_add(float lo, float hi) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Same across rows 0<->1 and 2<->3 (lanes l and l^16).
__device__ __forceinline__ float swap16_add(float lo, float hi) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum 10 values over the 64 lanes.  Halving exchanges: at each step a lane keeps half of
// its remaining values and adds the partner's copy of them (partners differ in lane bit
// 5, 4, 3, 2), then the last quad is summed with quad permutes.  Afterwards the lanes with
// (lane & 3) == 0 hold the totals: value `which` (or which = -1).
__device__ __forceinline__ float wave_sum10(const float* v, int lane, int& which) {
    float a[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) a[k] = swap32_add(v[k], v[k + 5]);
    float b[3];
    b[0] = swap16_add(a[0], a[3]);
    b[1] = swap16_add(a[1], a[4]);
    b[2] = swap16_add(a[2], 0.0f);
    // row mirror pairs lane i with 15 - i (bit 3 differs); half mirror pairs i with 7 - i (bit 2)
    const bool h3 = lane & 8;
    float c[2];
    {
        const float keep0 = h3 ? b[2] : b[0], send0 = h3 ? b[0] : b[2];
        const float keep1 = h3 ? 0.0f : b[1], send1 = h3 ? b[1] : 0.0f;
        c[0] = keep0 + dpp_f(send0, 0x140);
        c[1] = keep1 + dpp_f(send1, 0x140);
    }
    const bool h2 = lane & 4;
    float d = (h2 ? c[1] : c[0]) + dpp_f(h2 ? c[0] : c[1], 0x141);
    d += dpp_f(d, 0x4E);   // quad_perm [2,3,0,1]
    d += dpp_f(d, 0xB1);   // quad_perm [1,0,3,2]
    const bool h4 = lane & 16, h5 = lane & 32;
    int idx;
    if (!h4) idx = h3 ? (h2 ? -1 : 2) : (h2 ? 1 : 0);
    else idx = h3 ? -1 : (h2 ? 4 : 3);
    which = ((lane & 3) == 0 && idx >= 0) ? idx + (h5 ? 5 : 0) : -1;
    return d;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, off));
    return x;
}

// Next tile of this wave: its block index (one tile per workgroup), or the next value of the
// persistent queue.  The index is made wave-uniform explicitly (lane 0's atomic result,
// broadcast and read into a scalar register), so every branch on it is uniform and the loop
// that pulls tiles has a uniform exit; a value >= the tile count ends the loop.
template <bool PERSISTENT>
__device__ __forceinline__ uint32_t fetch_tile(uint32_t* queue, uint32_t iter) {
    if (!PERSISTENT) return iter == 0 ? (uint32_t)blockIdx.x : 0xFFFFFFFFu;
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(queue, 1u);
    return (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)t, 0));
}

template <int TW, int TH, int BATCH, bool PERSISTENT>
__global__ __launch_bounds__(64) void k_composite_fwd(FwdArgs a) {
    constexpr int PPL = TW * TH / 64;   // pixels per lane
    constexpr int ROWS = 64 / TW;       // rows covered by one pass of the wave
    static_assert(PPL >= 1 && TW * TH == 64 * PPL && BATCH % 64 == 0, "tile shape");
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    const int lane = threadIdx.x;
    for (uint32_t iter = 0;; ++iter) {
        const uint32_t tile = fetch_tile<PERSISTENT>(a.queue, iter);
        if (tile >= a.tiles) break;
        if (a.phase > 0 && a.alive[tile] == 0u) continue;   // every pixel terminated in an earlier phase
        const int v = find_view(a.vt, a.views, tile);
        const ViewInfo vi = a.vt[v];
        const uint32_t lt = tile - vi.tile_base;
        const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + lane % TW;
        const int py0 = (int)(lt / (uint32_t)vi.tiles_x) * TH + lane / TW;
        const float fpx = (float)px + 0.5f;
        const uint2 rg = a.ranges[tile];
        float T[PPL], C0[PPL], C1[PPL], C2[PPL], D[PPL], W[PPL];
        uint32_t last[PPL];
        bool done[PPL], inside[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int py = py0 + k * ROWS;
            inside[k] = px < vi.width && py < vi.height;
            const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
            T[k] = 1.0f;
            C0[k] = C1[k] = C2[k] = D[k] = W[k] = 0.0f;
            last[k] = 0;
            done[k] = !inside[k];
            if (a.phase > 0 && inside[k]) {
                T[k] = a.tfinal[p];
                C0[k] = a.cair[p];
                C1[k] = a.cair[a.pixels + p];
                C2[k] = a.cair[2 * a.pixels + p];
                D[k] = a.dsum[p];
                W[k] = a.wsum[p];
                last[k] = a.nlast[p];
                done[k] = a.done[p] != 0;
            }
        }
        for (uint32_t b = rg.x; b < rg.y; b += BATCH) {
            bool all_done = true;
#pragma unroll
            for (int k = 0; k < PPL; ++k) all_done = all_done && done[k];
            if (__all(all_done)) break;
            __syncthreads();   // the previous batch has been consumed
#pragma unroll
            for (int i = lane; i < BATCH; i += 64) {
                const uint32_t idx = b + i;
                if (idx < rg.y) {
                    const Record r = a.rec[a.vals[idx]];
                    sa[i] = r.a;
                    sb[i] = r.b;
                    sc[i] = r.c;
                }
            }
            __syncthreads();
            const int nb = min(BATCH, (int)(rg.y - b));
            for (int j = 0; j < nb; ++j) {
                const float4 ra = sa[j], rb = sb[j], rc = sc[j];
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    if (done[k]) continue;
                    float dx, dy;
                    const float pw = splat_power(ra, rb, fpx, (float)(py0 + k * ROWS) + 0.5f, dx, dy);
                    const float alpha = fminf(a.amax, rb.y * __builtin_amdgcn_exp2f(pw));
                    if (alpha < a.amin) continue;
                    const float Tn = T[k] * (1.0f - alpha);
                    if (Tn < a.tmin) {
                        done[k] = true;
                        continue;
                    }
                    const float w = alpha * T[k];
                    C0[k] = fmaf(w, rb.z, C0[k]);
                    C1[k] = fmaf(w, rb.w, C1[k]);
                    C2[k] = fmaf(w, rc.x, C2[k]);
                    D[k] = fmaf(w, rc.y, D[k]);
                    W[k] += w;
                    T[k] = Tn;
                    last[k] = b + j + 1;
                }
            }
        }
        bool mine_alive = false;
#pragma unroll
        for (int k = 0; k < PPL; ++k) mine_alive = mine_alive || !done[k];
        const bool any_alive = __any(mine_alive);
        const gs_medium m = a.med[v];
        const bool finish = !any_alive || a.phase == a.last_phase;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            if (!inside[k]) continue;
            const int py = py0 + k * ROWS;
            const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
            a.tfinal[p] = T[k];
            a.nlast[p] = last[k];
            a.done[p] = done[k] ? 1 : 0;
            a.cair[p] = C0[k];
            a.cair[a.pixels + p] = C1[k];
            a.cair[2 * a.pixels + p] = C2[k];
            a.dsum[p] = D[k];
            a.wsum[p] = W[k];
            if (!finish) continue;
            const int64_t plane = (int64_t)vi.width * vi.height;
            float* rgb = a.out_rgb + 3 * vi.pix_base + (int64_t)py * vi.width + px;
            float out[3], z;
            if (W[k] > 0.0f) {
                const float zh = D[k] / W[k];
                z = depth_map(zh, a.depth_mode);
                const float Cc[3] = {C0[k], C1[k], C2[k]};
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    out[c] = Cc[c] * expf(-m.Bd[c] * z) + m.Binf[c] * (1.0f - expf(-m.Bb[c] * z));
            } else {
                z = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    out[c] = a.depth_mode == 1 ? m.Binf[c] * (1.0f - expf(-m.Bb[c]))
                                               : (m.Bb[c] > 0.0f ? m.Binf[c] : 0.0f);
            }
            rgb[0] = out[0];
            rgb[plane] = out[1];
            rgb[2 * plane] = out[2];
            a.out_depth[p] = z;
            a.out_alpha[p] = W[k];
        }
        if (lane == 0) {
            a.alive[tile] = any_alive ? 1u : 0u;
            if (any_alive) atomicAdd(a.alive_count, 1u);
        }
    }
}

template <int TW, int TH, int BATCH, bool PERSISTENT>
__global__ __launch_bounds__(64) void k_composite_bwd(BwdArgs a) {
    constexpr int PPL = TW * TH / 64;
    constexpr int ROWS = 64 / TW;
    static_assert(PPL >= 1 && TW * TH == 64 * PPL && BATCH % 64 == 0, "tile shape");
    __shared__ float4 sa[BATCH], sb[BATCH], sc[BATCH];
    __shared__ uint32_t se[BATCH];
    const int lane = threadIdx.x;
    for (uint32_t iter = 0;; ++iter) {
        const uint32_t tile = fetch_tile<PERSISTENT>(a.queue, iter);
        if (tile >= a.tiles) break;
        const int v = find_view(a.vt, a.views, tile);
        const ViewInfo vi = a.vt[v];
        const uint32_t lt = tile - vi.tile_base;
        const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + lane % TW;
        const int py0 = (int)(lt / (uint32_t)vi.tiles_x) * TH + lane / TW;
        const float fpx = (float)px + 0.5f;
        const gs_medium m = a.med[v];
        // ---- per-pixel upstream gradient through the medium and depth
        float pm[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float gC0[PPL], gC1[PPL], gC2[PPL], gD[PPL], gW[PPL], T[PPL], S[PPL];
        uint32_t my_last[PPL];
        uint32_t lane_last = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            gC0[k] = gC1[k] = gC2[k] = gD[k] = gW[k] = S[k] = 0.0f;
            T[k] = 1.0f;
            my_last[k] = 0;
            const int py = py0 + k * ROWS;
            if (!(px < vi.width && py < vi.height)) continue;
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
                for (int c = 0; c < 3; ++c) {
                    A[c] = expf(-m.Bd[c] * z);
                    const float Sx = expf(-m.Bb[c] * z);
                    pm[c] += -G[c] * Cc[c] * z * A[c];
                    pm[3 + c] += G[c] * m.Binf[c] * z * Sx;
                    pm[6 + c] += G[c] * (1.0f - Sx);
                    dz += G[c] * (m.Binf[c] * m.Bb[c] * Sx - m.Bd[c] * Cc[c] * A[c]);
                }
                const float dzh = a.depth_mode == 1 ? dz * 0.05f * (1.0f - z * z) : dz;
                gC0[k] = G[0] * A[0];
                gC1[k] = G[1] * A[1];
                gC2[k] = G[2] * A[2];
                gD[k] = dzh / W;
                gW[k] = -dzh * zh / W;
                T[k] = a.tfinal[p];
                my_last[k] = a.nlast[p];
                lane_last = max(lane_last, my_last[k]);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (a.depth_mode == 1) {
                        const float Sx = expf(-m.Bb[c]);
                        pm[6 + c] += G[c] * (1.0f - Sx);
                        pm[3 + c] += G[c] * m.Binf[c] * Sx;
                    } else {
                        pm[6 + c] += m.Bb[c] > 0.0f ? G[c] : 0.0f;
                    }
                }
            }
        }
        // ---- medium partial sums of this tile
        {
            int which;
            const float t = wave_sum10(pm, lane, which);
            if (which >= 0 && which < 9) a.medpart[(int64_t)tile * 9 + which] = t;
        }
        const uint32_t block_last = wave_max_u32(lane_last);
        // ---- reverse walk over the phases' ranges, last phase first
        for (int ph = a.phases - 1; ph >= 0; --ph) {
            const uint2 rg = a.ranges[(size_t)ph * a.tiles + tile];
            if (rg.x >= rg.y || rg.x >= block_last) continue;
            for (uint32_t b_end = min(rg.y, block_last); b_end > rg.x;) {
                const uint32_t b0 = b_end - rg.x > (uint32_t)BATCH ? b_end - BATCH : rg.x;
                const int cnt = (int)(b_end - b0);
                __syncthreads();   // the previous batch has been consumed
#pragma unroll
                for (int i = lane; i < BATCH; i += 64) {
                    if (i < cnt) {
                        const uint32_t e = a.vals[b0 + i];
                        const Record r = a.rec[e];
                        sa[i] = r.a;
                        sb[i] = r.b;
                        sc[i] = r.c;
                        se[i] = e;
                    }
                }
                __syncthreads();
                for (int j = cnt - 1; j >= 0; --j) {
                    const float4 ra = sa[j], rb = sb[j], rc = sc[j];
                    const uint32_t idx = b0 + (uint32_t)j;
                    float g10[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    bool any = false;
#pragma unroll
                    for (int k = 0; k < PPL; ++k) {
                        if (idx >= my_last[k]) continue;
                        float dx, dy;
                        const float pw = splat_power(ra, rb, fpx, (float)(py0 + k * ROWS) + 0.5f, dx, dy);
                        const float ev = __builtin_amdgcn_exp2f(pw);
                        const float araw = rb.y * ev;
                        const float alpha = fminf(a.amax, araw);
                        if (alpha < a.amin) continue;
                        any = true;
                        const float rom = __builtin_amdgcn_rcpf(1.0f - alpha);
                        const float Ti = T[k] * rom;
                        const float w = alpha * Ti;
                        const float gf = gC0[k] * rb.z + gC1[k] * rb.w + gC2[k] * rc.x + gD[k] * rc.y + gW[k];
                        const float dalpha = Ti * gf - S[k] * rom;
                        S[k] = fmaf(gf, w, S[k]);
                        T[k] = Ti;
                        g10[6] += gC0[k] * w;
                        g10[7] += gC1[k] * w;
                        g10[8] += gC2[k] * w;
                        g10[9] += gD[k] * w;
                        if (araw <= a.amax) {
                            g10[5] += dalpha * ev;
                            const float dpw = dalpha * araw * kLn2;
                            g10[2] += dpw * dx * dx;
                            g10[3] += dpw * dx * dy;
                            g10[4] += dpw * dy * dy;
                            g10[0] -= dpw * (2.0f * ra.z * dx + ra.w * dy);
                            g10[1] -= dpw * (ra.w * dx + 2.0f * rb.x * dy);
                        }
                    }
                    if (__any(any)) {
                        int which;
                        const float t = wave_sum10(g10, lane, which);
                        if (which >= 0) unsafeAtomicAdd(a.grad2d + (size_t)se[j] * kGrad2D + which, t);
                    }
                }
                b_end = b0;
            }
        }
    }
}

template <int TW, int TH, int BATCH>
hipError_t run_fwd(const FwdArgs& a, bool persistent, int grid, hipStream_t s) {
    if (persistent)
        hipLaunchKernelGGL((k_composite_fwd<TW, TH, BATCH, true>), dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_composite_fwd<TW, TH, BATCH, false>), dim3(a.tiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int TW, int TH, int BATCH>
hipError_t run_bwd(const BwdArgs& a, bool persistent, int grid, hipStream_t s) {
    if (persistent)
        hipLaunchKernelGGL((k_composite_bwd<TW, TH, BATCH, true>), dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_composite_bwd<TW, TH, BATCH, false>), dim3(a.tiles), dim3(64), 0, s, a);
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

// Persistent grid: 16 single-wave workgroups per compute unit (4 per SIMD).
int persistent_grid(int) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    return cus * 16;
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
    if (o.tile_w == 8) return run_fwd<8, 8, 64>(a, pers, persistent_grid(64 * 4), s);
    switch (o.lds_batch) {
        case 64: return run_fwd<16, 16, 64>(a, pers, persistent_grid(64 * 4), s);
        case 128: return run_fwd<16, 16, 128>(a, pers, persistent_grid(64 * 4), s);
        default: return run_fwd<16, 16, 256>(a, pers, persistent_grid(64 * 4), s);
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
    if (o.tile_w == 8) return run_bwd<8, 8, 64>(a, pers, persistent_grid(64 * 4), s);
    switch (o.lds_batch) {
        case 64: return run_bwd<16, 16, 64>(a, pers, persistent_grid(64 * 4), s);
        case 128: return run_bwd<16, 16, 128>(a, pers, persistent_grid(64 * 4), s);
        default: return run_bwd<16, 16, 256>(a, pers, persistent_grid(64 * 4), s);
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
