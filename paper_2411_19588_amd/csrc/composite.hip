// Per-tile front-to-back compositing (eq. 3dgs_orig with alpha from
// eq. opacity_impact), the underwater epilogue (eq. 3dgs_uw at the depth of
// eq. Depth) and the exact adjoint.
//
// A tile is split among the waves of one workgroup: at 16x16 a wave owns an 8x8
// quadrant (one pixel per lane), a 16x8 half (two) or the whole tile (four pixels
// per lane: rows y, y+4, y+8, y+12 of its column); an 8x8 tile is one wave.  Every
// lane evaluates the same record at a time, which reaches the wave either from LDS
// (the workgroup stages a batch of the tile's records, each lane reads the same
// address) or through the scalar data cache (each wave fetches the record
// indices of its tile and loads one record at a time into scalar registers, one
// ahead of its use; no LDS and no workgroup barriers on the walk).  A wave stops as
// soon as all of its pixels have terminated; a terminated pixel keeps -T in its
// transmittance slot, so the blend needs no separate flag.  With depth-progressive
// binning the forward runs once per phase: the per-pixel state (T, C, D, W, last
// contributor, terminated) carries over, a wave whose pixels have all terminated
// writes its outputs, and a tile none of whose pixels is alive is skipped by later
// phases.  In persistent mode a fixed grid of workgroups pulls tile indices from a
// device counter.
//
// The adjoint walks each pixel's contributors back to front (over the phases in
// reverse) from its last contributor, recovering the transmittance by
// T_i = T_{i+1} / (1 - alpha_i) instead of storing per-pixel lists; each lane sums
// its pixels' terms for a Gaussian, the wave reduces the 10 terms with a transpose
// reduction on cross-lane swaps (v_permlane32_swap, v_permlane16_swap, DPP row
// mirrors and quad permutes), and the waves of a workgroup add their sums in LDS
// before one atomic add per term (scalar-fetch mode: one per wave).
#include <string.h>

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
    const uint32_t* order;    // persistent mode: tile of each queue position (null: index order)
    uint32_t* alive;
    uint32_t* alive_count;
    uint32_t* view_alive;     // [views]: tiles of each view left alive
    uint64_t* rowbits;        // nullable: per global tile row, the bits of the tiles left alive
    uint32_t row_words;
    // status (nullable) is set when this phase ends a forward cut short by phase_limit: a tile
    // left alive while *rank_end (the end of the depth ranks binned so far) < *visible (Gaussians
    // are left unbinned) ORs GS_STATUS_INCOMPLETE into it
    uint32_t* status;
    const uint32_t* rank_end;
    const uint32_t* visible;
    float* out_rgb;
    float* out_depth;
    float* out_alpha;
    float* out_restored;      // nullable: C_air, CHW per view
    float* tfinal;
    uint32_t* nlast;
    uint8_t* done;
    float* cair;
    float* dsum;
    float* wsum;
    int64_t pixels;
    float amin, amax, tmin;
    int32_t depth_mode, depth_output;
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
    const uint32_t* order;    // persistent mode: tile of each queue position (null: index order)
    const float* grad_rgb;
    const float* grad_depth;
    const float* grad_restored;   // nullable
    const float* tfinal;
    const uint32_t* nlast;
    const float* cair;
    const float* dsum;
    const float* wsum;
    float* grad2d;
    float* medpart;
    int64_t pixels;
    float amin, amax, tmin;
    int32_t depth_mode, depth_output;
    Guard guard;
};

// Splat fields used by the blend, in registers (scalar registers in scalar-fetch mode):
// lo = log2 of the opacity, io = its reciprocal (read by the adjoint only).
struct Splat {
    float mx, my, A, B, C, lo, r, g, b, d, io;
};

// alpha exponent of one splat at one pixel: log2 of o exp(-q/2), with
// q = (p - m)^T Q (p - m) and the conic pre-scaled by -log2(e)/2 (A, C) and -log2(e) (B),
// evaluated as (A dx^2 + log2 o) + dy (B dx + C dy) so that a lane's pixels in one column
// share the dx terms (and alpha is exp2 of it, with no product by o).  Forward and adjoint,
// and every launch shape, evaluate this same sequence of (dx, dy), so they take identical
// decisions.
struct ColTerms {
    float dx, bdx, adx2;
};

__device__ __forceinline__ ColTerms col_terms(const Splat& s, float fpx) {
    const float dx = fpx - s.mx;
    return {dx, s.B * dx, fmaf(s.A * dx, dx, s.lo)};
}

__device__ __forceinline__ float splat_power(const Splat& s, const ColTerms& c, float fpy, float& dy) {
    dy = fpy - s.my;
    return fmaf(dy, fmaf(s.C, dy, c.bdx), c.adx2);
}

typedef __attribute__((address_space(4))) const float ConstF;

// Record `e` through the scalar data cache (the index must be wave-uniform): the loads
// are from the constant address space, which the compiler emits as scalar loads.
__device__ __forceinline__ Splat load_splat_scalar(const Record* rec, uint32_t e) {
    const ConstF* p = (const ConstF*)(rec + e);
    return {p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], p[8], p[9], p[10]};
}

// Wait until a scalar-loaded splat has arrived (scalar loads complete out of order, so
// the wait is placed here, before the next record's load is issued).
__device__ __forceinline__ void splat_ready(const Splat& s) {
    asm volatile("" ::"s"(s.mx), "s"(s.my), "s"(s.A), "s"(s.B), "s"(s.C), "s"(s.lo), "s"(s.r), "s"(s.g), "s"(s.b),
                 "s"(s.d), "s"(s.io));
}

// A record staged in LDS: the forward stages (b, depth) of the third float4 and leaves io
// at 0 (it blends without it), the adjoint stages (b, depth, 1/o).
__device__ __forceinline__ Splat splat_from_lds(const float4* sa, const float4* sb, const float2* sc, int j) {
    const float4 ra = sa[j], rb = sb[j];
    const float2 rc = sc[j];
    return {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w, rc.x, rc.y, 0.0f};
}

__device__ __forceinline__ Splat splat_from_lds(const float4* sa, const float4* sb, const float4* sc, int j) {
    const float4 ra = sa[j], rb = sb[j], rc = sc[j];
    return {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w, rc.x, rc.y, rc.z};
}

__device__ __forceinline__ int find_view(const ViewInfo* vt, int views, uint32_t tile) {
    int v = 0;
    while (v + 1 < views && tile >= vt[v + 1].tile_base) ++v;
    return v;
}

// e^(-b z) of the medium terms, as the hardware exp2 of a pre-scaled argument: its relative
// error (about 1e-6 for the attenuation and backscatter exponents of a scene) is far inside
// the image and gradient tolerances, at one instruction instead of an accurate expf.
__device__ __forceinline__ float exp_neg(float b, float z) {
    return __builtin_amdgcn_exp2f(-1.4426950408889634f * (b * z));
}

__device__ __forceinline__ float depth_map(float zh, int mode) {
    return mode == 1 ? 2.0f / (1.0f + expf(-0.1f * zh)) - 1.0f : zh;
}

// Derivative of the depth image w.r.t. zhat when the image is depth_map(zhat, mode) = y:
// 0.05 (1 - y^2) for the logistic map (tanh(0.05 zhat)), 1 for the metric depth.
__device__ __forceinline__ float depth_map_slope(float y, int mode) {
    return mode == 1 ? 0.05f * (1.0f - y * y) : 1.0f;
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

// The value that lane holds after wave_sum10, or -1: lanes with (lane & 3) == 0 hold one
// total each, in an order fixed by the exchange pattern below.
__device__ __forceinline__ int sum10_slot(int lane) {
    const bool h2 = lane & 4, h3 = lane & 8, h4 = lane & 16, h5 = lane & 32;
    int idx;
    if (!h4) idx = h3 ? (h2 ? -1 : 2) : (h2 ? 1 : 0);
    else idx = h3 ? -1 : (h2 ? 4 : 3);
    return ((lane & 3) == 0 && idx >= 0) ? idx + (h5 ? 5 : 0) : -1;
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
    which = sum10_slot(lane);
    return d;
}

// Scale of the wave sum that a lane holds in the adjoint: ln 2 for the five geometry terms
// (accumulated without it), 1 otherwise; a function of the lane alone, set up once.
__device__ __forceinline__ float adjoint_scale(int lane) {
    const int which = sum10_slot(lane);
    return (which >= 0 && which < 5) ? kLn2 : 1.0f;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, off));
    return x;
}

__device__ __forceinline__ uint32_t lane_index(uint32_t chunk, uint32_t j) {
    return (uint32_t)__builtin_amdgcn_readlane((int)chunk, (int)j);
}

// How a tile is split among the waves of a workgroup: each wave owns a SW-wide block of
// 64 * PPL pixels, lane l at column l % SW and rows l / SW + k * R (k < PPL).
template <int TW, int TH, int PPL>
struct Shape {
    static constexpr int SW = (TW == 16 && PPL == 1) ? 8 : TW;
    static constexpr int R = 64 / SW;
    static constexpr int SH = R * PPL;
    static constexpr int NWX = TW / SW;
    static constexpr int NW = NWX * (TH / SH);
    static constexpr int THREADS = 64 * NW;
    static_assert(SW * R == 64 && TW % SW == 0 && TH % SH == 0 && NW >= 1 && NW <= 4, "tile split");
};

// Next tile of this workgroup: one tile per workgroup, taken in descending tile order, or the
// tile at the next position of the persistent queue (the position itself, or order[position]
// for the longest-first queue).  Descending: the kernels before a compositing pass (the tile
// sort and commit, the loss) write their outputs in ascending tile and pixel order, so the
// lines written last, still in the caches, belong to the last tiles; measured faster on every
// benchmark scene (one view at 1600x1067 and at 1080p, four orbit views).  The grid of a
// one-tile-per-workgroup launch has exactly `tiles` workgroups.  The value is wave-uniform by
// construction (read into a scalar register), so every branch on it is uniform and the loop
// that pulls tiles has a uniform exit; a position >= the tile count ends the loop.
template <int NW, bool PERSISTENT>
__device__ __forceinline__ uint32_t fetch_tile(uint32_t* queue, const uint32_t* order, uint32_t tiles, uint32_t iter,
                                               uint32_t* s_tile) {
    if (!PERSISTENT) return iter == 0 ? tiles - 1u - (uint32_t)blockIdx.x : 0xFFFFFFFFu;
    uint32_t pos;
    if (NW == 1) {
        uint32_t t = 0;
        if (threadIdx.x == 0) t = atomicAdd(queue, 1u);
        pos = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)t, 0));
    } else {
        __syncthreads();   // every wave has read the previous value
        if (threadIdx.x == 0) *s_tile = atomicAdd(queue, 1u);
        __syncthreads();
        pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)*s_tile);
    }
    if (pos >= tiles || order == nullptr) return pos;
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)order[pos]);
}

// Keys of the longest-first queue: the work of a tile is its list length in this phase
// (forward) or summed over the phases (adjoint); the key is 32 - bit_length(length), so an
// ascending stable sort puts the longest lists first in power-of-two buckets, ties in tile order.
__global__ __launch_bounds__(kBlock) void k_queue_keys(const uint2* __restrict__ ranges, int phase0, int phase1,
                                                     uint32_t tiles, uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= tiles) return;
    uint32_t len = 0;
    for (int p = phase0; p < phase1; ++p) {
        const uint2 rg = ranges[(size_t)p * tiles + t];
        len += rg.y > rg.x ? rg.y - rg.x : 0u;
    }
    keys[t] = (uint32_t)__clz(len);   // 32 - bit_length
    vals[t] = t;
}

// OR of a per-wave flag over the workgroup (a barrier; `slot` must not be reused before
// the next barrier).
template <int NW>
__device__ __forceinline__ bool block_any(bool wave_flag, uint32_t* slot) {
    if (NW == 1) return wave_flag;
    if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = wave_flag ? 1u : 0u;
    __syncthreads();
    uint32_t any = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) any |= slot[w];
    return any != 0;
}

template <int PPL>
__device__ __forceinline__ bool lane_live(const float* T) {
    bool live = false;
#pragma unroll
    for (int k = 0; k < PPL; ++k) live = live || T[k] > 0.0f;
    return live;
}

// Front-to-back blend of one splat into a lane's pixels.  T < 0 marks a terminated pixel
// (|T| is its final transmittance): its T(1 - alpha) is negative, so it neither blends nor
// changes.  `idx1` is the splat's list position + 1.
template <int PPL, int R>
__device__ __forceinline__ void blend(const Splat& s, float fpx, float fpy0, uint32_t idx1, float* T, float* C0,
                                      float* C1, float* C2, float* D, float* W, uint32_t* last, float amin,
                                      float amax, float tmin) {
    const ColTerms ct = col_terms(s, fpx);
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        float dy;
        const float pw = splat_power(s, ct, fpy0 + (float)(k * R), dy);
        const float alpha = fminf(amax, __builtin_amdgcn_exp2f(pw));
        if (alpha >= amin) {
            const float Tn = fmaf(-alpha, T[k], T[k]);   // T (1 - alpha), rounded once
            const bool use = Tn >= tmin;
            const float w = use ? alpha * T[k] : 0.0f;
            C0[k] = fmaf(w, s.r, C0[k]);
            C1[k] = fmaf(w, s.g, C1[k]);
            C2[k] = fmaf(w, s.b, C2[k]);
            D[k] = fmaf(w, s.d, D[k]);
            W[k] += w;
            T[k] = use ? Tn : -fabsf(T[k]);
            last[k] = use ? idx1 : last[k];
        }
    }
}

template <int TW, int TH, int PPL, int BATCH, bool SCALAR, bool PERSISTENT>
__global__ __launch_bounds__((Shape<TW, TH, PPL>::THREADS)) void k_composite_fwd(FwdArgs a) {
    using S = Shape<TW, TH, PPL>;
    constexpr int NW = S::NW, THREADS = S::THREADS, R = S::R;
    constexpr int LB = SCALAR ? 1 : BATCH;
    static_assert(SCALAR || BATCH % THREADS == 0 || THREADS % BATCH == 0, "batch");
    __shared__ float4 sa[LB], sb[LB];
    __shared__ float2 sc[LB];
    __shared__ uint32_t s_flag[3][NW];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ox = (wave % S::NWX) * S::SW, oy = (wave / S::NWX) * S::SH;
    for (uint32_t iter = 0;; ++iter) {
        const uint32_t tile = fetch_tile<NW, PERSISTENT>(a.queue, a.order, a.tiles, iter, &s_tile);
        if (tile >= a.tiles) break;
        if (a.phase > 0 && a.alive[tile] == 0u) continue;   // every pixel terminated in an earlier phase
        const int v = find_view(a.vt, a.views, tile);
        const ViewInfo vi = a.vt[v];
        const uint32_t lt = tile - vi.tile_base;
        const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + ox + lane % S::SW;
        const int py0 = (int)(lt / (uint32_t)vi.tiles_x) * TH + oy + lane / S::SW;
        const float fpx = (float)px + 0.5f, fpy0 = (float)py0 + 0.5f;
        const uint2 rg = a.ranges[tile];
        float T[PPL], C0[PPL], C1[PPL], C2[PPL], D[PPL], W[PPL];
        uint32_t last[PPL];
        bool inside[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int py = py0 + k * R;
            inside[k] = px < vi.width && py < vi.height;
            const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
            T[k] = inside[k] ? 1.0f : -1.0f;
            C0[k] = C1[k] = C2[k] = D[k] = W[k] = 0.0f;
            last[k] = 0;
            if (a.phase > 0 && inside[k]) {
                const float tf = a.tfinal[p];
                T[k] = a.done[p] ? -tf : tf;
                C0[k] = a.cair[p];
                C1[k] = a.cair[a.pixels + p];
                C2[k] = a.cair[2 * a.pixels + p];
                D[k] = a.dsum[p];
                W[k] = a.wsum[p];
                last[k] = a.nlast[p];
            }
        }
        const bool entry_live = __any(lane_live<PPL>(T));
        if (SCALAR) {
            // each wave walks the list on its own; records arrive through the scalar cache two
            // at a time, the next two in flight while the current two are blended
            for (uint32_t b = rg.x; b < rg.y; b += 64) {
                if (!__any(lane_live<PPL>(T))) break;
                const uint32_t n = min(64u, rg.y - b), nm = n - 1;
                const uint32_t chunk = (uint32_t)lane < n ? a.vals[b + lane] : 0u;
                Splat p0 = load_splat_scalar(a.rec, lane_index(chunk, 0));
                Splat p1 = load_splat_scalar(a.rec, lane_index(chunk, min(1u, nm)));
                for (uint32_t j = 0; j < n; j += 4) {
                    splat_ready(p0);
                    splat_ready(p1);
                    const Splat q0 = load_splat_scalar(a.rec, lane_index(chunk, min(j + 2, nm)));
                    const Splat q1 = load_splat_scalar(a.rec, lane_index(chunk, min(j + 3, nm)));
                    blend<PPL, R>(p0, fpx, fpy0, b + j + 1, T, C0, C1, C2, D, W, last, a.amin, a.amax, a.tmin);
                    if (j + 1 < n)
                        blend<PPL, R>(p1, fpx, fpy0, b + j + 2, T, C0, C1, C2, D, W, last, a.amin, a.amax, a.tmin);
                    splat_ready(q0);
                    splat_ready(q1);
                    p0 = load_splat_scalar(a.rec, lane_index(chunk, min(j + 4, nm)));
                    p1 = load_splat_scalar(a.rec, lane_index(chunk, min(j + 5, nm)));
                    if (j + 2 < n)
                        blend<PPL, R>(q0, fpx, fpy0, b + j + 3, T, C0, C1, C2, D, W, last, a.amin, a.amax, a.tmin);
                    if (j + 3 < n)
                        blend<PPL, R>(q1, fpx, fpy0, b + j + 4, T, C0, C1, C2, D, W, last, a.amin, a.amax, a.tmin);
                    if ((j & 15) == 12 && !__any(lane_live<PPL>(T))) break;
                }
            }
        } else {
            int slot = 0;
            for (uint32_t b = rg.x; b < rg.y; b += BATCH) {
                const bool wl = __any(lane_live<PPL>(T));
                // the barrier inside also tells every wave that the previous batch has been consumed
                if (!block_any<NW>(wl, s_flag[slot])) break;
                slot = slot == 0 ? 1 : 0;
                if (NW == 1) __syncthreads();
#pragma unroll
                for (int i = tid; i < BATCH; i += THREADS) {
                    const uint32_t idx = b + i;
                    if (idx < rg.y) {
                        const Record r = a.rec[a.vals[idx]];
                        sa[i] = r.a;
                        sb[i] = r.b;
                        sc[i] = make_float2(r.c.x, r.c.y);
                    }
                }
                __syncthreads();
                if (wl) {
                    // the next record is read from LDS while the current one is blended
                    const int nb = min(BATCH, (int)(rg.y - b)), nm = nb - 1;
                    Splat p = splat_from_lds(sa, sb, sc, 0);
                    for (int j = 0; j < nb; j += 2) {
                        const Splat q = splat_from_lds(sa, sb, sc, min(j + 1, nm));
                        blend<PPL, R>(p, fpx, fpy0, b + j + 1, T, C0, C1, C2, D, W, last, a.amin, a.amax, a.tmin);
                        p = splat_from_lds(sa, sb, sc, min(j + 2, nm));
                        if (j + 1 < nb)
                            blend<PPL, R>(q, fpx, fpy0, b + j + 2, T, C0, C1, C2, D, W, last, a.amin, a.amax,
                                          a.tmin);
                        if ((j & 15) == 14 && !__any(lane_live<PPL>(T))) break;
                    }
                }
            }
        }
        const bool wave_alive = __any(lane_live<PPL>(T));
        if (entry_live) {
            const gs_medium m = a.med[v];
            const bool finish = !wave_alive || a.phase == a.last_phase;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                if (!inside[k]) continue;
                const int py = py0 + k * R;
                const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
                a.tfinal[p] = fabsf(T[k]);
                a.nlast[p] = last[k];
                a.done[p] = T[k] < 0.0f ? 1 : 0;
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
                    const float zm = depth_map(zh, a.depth_mode);
                    const float Cc[3] = {C0[k], C1[k], C2[k]};
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        out[c] = Cc[c] * exp_neg(m.Bd[c], zm) + m.Binf[c] * (1.0f - exp_neg(m.Bb[c], zm));
                    z = a.depth_output == 1 ? depth_map(zh, 1) : zm;
                } else {
                    z = 0.0f;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        out[c] = a.depth_mode == 1 ? m.Binf[c] * (1.0f - exp_neg(m.Bb[c], 1.0f))
                                                   : (m.Bb[c] > 0.0f ? m.Binf[c] : 0.0f);
                }
                rgb[0] = out[0];
                rgb[plane] = out[1];
                rgb[2 * plane] = out[2];
                a.out_depth[p] = z;
                a.out_alpha[p] = W[k];
                if (a.out_restored) {
                    float* J = a.out_restored + 3 * vi.pix_base + (int64_t)py * vi.width + px;
                    J[0] = C0[k];
                    J[plane] = C1[k];
                    J[2 * plane] = C2[k];
                }
            }
        }
        const bool tile_alive = block_any<NW>(wave_alive, s_flag[2]);
        if (tid == 0) {
            a.alive[tile] = tile_alive ? 1u : 0u;
            if (tile_alive) {
                atomicAdd(a.alive_count, 1u);
                atomicAdd(a.view_alive + v, 1u);
                if (a.rowbits) {
                    const uint32_t tx = lt % (uint32_t)vi.tiles_x, ty = lt / (uint32_t)vi.tiles_x;
                    atomicOr(reinterpret_cast<unsigned long long*>(a.rowbits) +
                                 (size_t)(vi.row_base + ty) * a.row_words + (tx >> 6),
                             1ull << (tx & 63));
                }
                if (a.status && *a.rank_end < *a.visible) atomicOr(a.status, GS_STATUS_INCOMPLETE);
            }
        }
    }
}

// Adjoint of the blend of one splat for a lane's pixels, walking back to front: writes the
// lane's terms to g10 = d/d(m_x, m_y, A, B, C, o, r, g, b, depth), which must be zero on
// entry, the first five without their common factor ln 2 (applied once to the wave's sums).
// Returns whether any of the lane's pixels was reached by the splat with alpha >= alpha_min.
template <int PPL, int R>
__device__ __forceinline__ bool blend_adjoint(const Splat& s, float fpx, float fpy0, uint32_t idx,
                                              const uint32_t* my_last, float* T, float* S, const float* gC0,
                                              const float* gC1, const float* gC2, const float* gD, const float* gW,
                                              float* g10, float amin, float amax) {
    const ColTerms ct = col_terms(s, fpx);
    const float nA2 = -2.0f * s.A, nB = -s.B, nC2 = -2.0f * s.C;
    // With several pixels per lane, the exponent's derivatives are gathered per lane as
    // P = sum dpw, Q = sum dpw dy, U = sum dpw dy^2 (dx is the lane's column, the same for all
    // its pixels) and turned into the five geometry terms once per splat.  The opacity term
    // is sum dalpha exp2(q') = P / o, with dpw = dalpha * alpha_raw and alpha_raw = o exp2(q').
    constexpr bool kLaneSums = PPL >= 2;
    float P = 0.0f, Q = 0.0f, U = 0.0f;
    bool any = false;
    // Branch-free over the lane's pixels: a pixel past its last contributor, or where the splat's
    // alpha is below alpha_min, takes alpha = 0 and a raw alpha of 0, so that T (divided by
    // exactly 1) and S stay as they are and every term it adds is an exact zero.
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        float dy;
        const float pw = splat_power(s, ct, fpy0 + (float)(k * R), dy);
        const float araw = __builtin_amdgcn_exp2f(pw);
        const float alpha = fminf(amax, araw);
        const bool act = idx < my_last[k] && alpha >= amin;
        any = any || act;
        const float ae = act ? alpha : 0.0f;
        // a clamped alpha does not depend on the opacity or the exponent
        const float re = (act && araw <= amax) ? araw : 0.0f;
        const float rom = __builtin_amdgcn_rcpf(1.0f - ae);
        const float Ti = T[k] * rom;
        const float w = ae * Ti;
        const float gf = fmaf(gC0[k], s.r, fmaf(gC1[k], s.g, fmaf(gC2[k], s.b, fmaf(gD[k], s.d, gW[k]))));
        const float dalpha = fmaf(Ti, gf, -S[k] * rom);
        S[k] = fmaf(gf, w, S[k]);
        T[k] = Ti;
        g10[6] = fmaf(gC0[k], w, g10[6]);
        g10[7] = fmaf(gC1[k], w, g10[7]);
        g10[8] = fmaf(gC2[k], w, g10[8]);
        g10[9] = fmaf(gD[k], w, g10[9]);
        const float dpw = dalpha * re;   // d/d(exponent), without ln 2
        if constexpr (kLaneSums) {
            // the first pixel's terms are taken as they are (an add to zero is not free)
            const float qd = dpw * dy;
            P = k == 0 ? dpw : P + dpw;
            Q = k == 0 ? qd : Q + qd;
            U = k == 0 ? qd * dy : fmaf(qd, dy, U);
        } else {
            const float pdx = dpw * ct.dx, pdy = dpw * dy;
            g10[5] = fmaf(dpw, s.io, g10[5]);
            g10[2] = fmaf(pdx, ct.dx, g10[2]);
            g10[3] = fmaf(pdx, dy, g10[3]);
            g10[4] = fmaf(pdy, dy, g10[4]);
            g10[0] = fmaf(nA2, pdx, fmaf(nB, pdy, g10[0]));
            g10[1] = fmaf(nB, pdx, fmaf(nC2, pdy, g10[1]));
        }
    }
    if constexpr (kLaneSums) {
        const float X = ct.dx * P;   // sum over the lane's pixels of dpw dx
        g10[5] = P * s.io;
        g10[2] = fmaf(ct.dx, X, g10[2]);
        g10[3] = fmaf(ct.dx, Q, g10[3]);
        g10[4] = U;
        g10[0] = fmaf(nA2, X, fmaf(nB, Q, g10[0]));
        g10[1] = fmaf(nB, X, fmaf(nC2, Q, g10[1]));
    }
    return any;
}

// Wave sum of a lane's 10 adjoint terms; the lanes that hold a total add it to the splat's
// 2D gradient (entry e) with one atomic each.
__device__ __forceinline__ void flush_adjoint(const float* g10, int lane, float scale, float* grad2d, uint32_t e) {
    int which;
    const float t = wave_sum10(g10, lane, which) * scale;
    if (which >= 0) unsafeAtomicAdd(grad2d + (size_t)e * kGrad2D + which, t);
}

// One splat of the scalar-fetch adjoint: the lanes' terms, the wave sum and one atomic add
// per term into the splat's 2D gradient.
template <int PPL, int R>
__device__ __forceinline__ void adjoint_scalar(const BwdArgs& a, const Splat& s, uint32_t chunk, uint32_t b0, int j,
                                               float fpx, float fpy0, int lane, float scale, const uint32_t* my_last,
                                               float* T, float* Sx, const float* gC0, const float* gC1,
                                               const float* gC2, const float* gD, const float* gW) {
    float g10[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const bool any = blend_adjoint<PPL, R>(s, fpx, fpy0, b0 + (uint32_t)j, my_last, T, Sx, gC0, gC1, gC2, gD, gW,
                                           g10, a.amin, a.amax);
    if (__any(any)) flush_adjoint(g10, lane, scale, a.grad2d, lane_index(chunk, (uint32_t)j));
}

template <int TW, int TH, int PPL, int BATCH, bool SCALAR, bool PERSISTENT>
__global__ __launch_bounds__((Shape<TW, TH, PPL>::THREADS)) void k_composite_bwd(BwdArgs a) {
    using S = Shape<TW, TH, PPL>;
    constexpr int NW = S::NW, THREADS = S::THREADS, R = S::R;
    constexpr int LB = SCALAR ? 1 : BATCH;
    constexpr int RED = (!SCALAR && NW > 1) ? 64 : 1;   // records per cross-wave reduction
    __shared__ float4 sa[LB], sb[LB];
    __shared__ float4 sc[LB];
    __shared__ uint32_t se[LB];
    __shared__ float red[NW][RED][kGrad2D];
    __shared__ float s_med[NW][9];
    __shared__ uint32_t s_last[NW];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ox = (wave % S::NWX) * S::SW, oy = (wave / S::NWX) * S::SH;
    const float scale = adjoint_scale(lane);
    if (guard_set(a.guard)) return;   // the forward was truncated: no gradient (uniform exit)
    for (uint32_t iter = 0;; ++iter) {
        const uint32_t tile = fetch_tile<NW, PERSISTENT>(a.queue, a.order, a.tiles, iter, &s_tile);
        if (tile >= a.tiles) break;
        const int v = find_view(a.vt, a.views, tile);
        const ViewInfo vi = a.vt[v];
        const uint32_t lt = tile - vi.tile_base;
        const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + ox + lane % S::SW;
        const int py0 = (int)(lt / (uint32_t)vi.tiles_x) * TH + oy + lane / S::SW;
        const float fpx = (float)px + 0.5f, fpy0 = (float)py0 + 0.5f;
        const gs_medium m = a.med[v];
        // ---- per-pixel upstream gradient through the medium and depth
        float pm[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float gC0[PPL], gC1[PPL], gC2[PPL], gD[PPL], gW[PPL], T[PPL], Sx[PPL];
        uint32_t my_last[PPL];
        uint32_t lane_last = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            gC0[k] = gC1[k] = gC2[k] = gD[k] = gW[k] = Sx[k] = 0.0f;
            T[k] = 1.0f;
            my_last[k] = 0;
            const int py = py0 + k * R;
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
                float dz = 0.0f;
                float A[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A[c] = exp_neg(m.Bd[c], z);
                    const float Sb = exp_neg(m.Bb[c], z);
                    pm[c] += -G[c] * Cc[c] * z * A[c];
                    pm[3 + c] += G[c] * m.Binf[c] * z * Sb;
                    pm[6 + c] += G[c] * (1.0f - Sb);
                    dz += G[c] * (m.Binf[c] * m.Bb[c] * Sb - m.Bd[c] * Cc[c] * A[c]);
                }
                // the medium's z and the depth image, each through its own map of zhat
                float dzh = dz * depth_map_slope(z, a.depth_mode);
                if (a.grad_depth) {
                    const int dm = a.depth_output == 1 ? 1 : a.depth_mode;
                    const float zo = a.depth_output == 1 ? depth_map(zh, 1) : z;
                    dzh = fmaf(a.grad_depth[p], depth_map_slope(zo, dm), dzh);
                }
                float GJ[3] = {0.0f, 0.0f, 0.0f};
                if (a.grad_restored) {
                    const float* gj = a.grad_restored + 3 * vi.pix_base + (int64_t)py * vi.width + px;
                    GJ[0] = gj[0];
                    GJ[1] = gj[plane];
                    GJ[2] = gj[2 * plane];
                }
                gC0[k] = fmaf(G[0], A[0], GJ[0]);
                gC1[k] = fmaf(G[1], A[1], GJ[1]);
                gC2[k] = fmaf(G[2], A[2], GJ[2]);
                gD[k] = dzh / W;
                gW[k] = -dzh * zh / W;
                T[k] = a.tfinal[p];
                my_last[k] = a.nlast[p];
                lane_last = max(lane_last, my_last[k]);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (a.depth_mode == 1) {
                        const float Sb = exp_neg(m.Bb[c], 1.0f);
                        pm[6 + c] += G[c] * (1.0f - Sb);
                        pm[3 + c] += G[c] * m.Binf[c] * Sb;
                    } else {
                        pm[6 + c] += m.Bb[c] > 0.0f ? G[c] : 0.0f;
                    }
                }
            }
        }
        // ---- medium partial sums of this tile, and the furthest list position any pixel reached
        // the butterfly leaves the maximum in every lane; reading it into a scalar register makes
        // the walk's bounds and list positions scalar values (no per-splat vector index arithmetic)
        const uint32_t wave_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_u32(lane_last));
        uint32_t block_last = wave_last;
        {
            int which;
            const float t = wave_sum10(pm, lane, which);
            if (NW == 1) {
                if (which >= 0 && which < 9) a.medpart[(int64_t)tile * 9 + which] = t;
            } else {
                if (which >= 0 && which < 9) s_med[wave][which] = t;
                if (lane == 0) s_last[wave] = wave_last;
                __syncthreads();
                if (tid < 9) {
                    float acc = 0.0f;
#pragma unroll
                    for (int w = 0; w < NW; ++w) acc += s_med[w][tid];
                    a.medpart[(int64_t)tile * 9 + tid] = acc;
                }
                block_last = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) block_last = max(block_last, s_last[w]);
                block_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)block_last);
            }
        }
        // ---- reverse walk over the phases' ranges, last phase first
        if (SCALAR) {
            for (int ph = a.phases - 1; ph >= 0; --ph) {
                const uint2 rg = a.ranges[(size_t)ph * a.tiles + tile];
                if (rg.x >= rg.y || rg.x >= wave_last) continue;
                for (uint32_t b_end = min(rg.y, wave_last); b_end > rg.x;) {
                    const uint32_t b0 = b_end - rg.x > 64u ? b_end - 64u : rg.x;
                    const uint32_t n = b_end - b0;
                    const uint32_t chunk = (uint32_t)lane < n ? a.vals[b0 + lane] : 0u;
                    // records two at a time from the back, the next two in flight
                    Splat p0 = load_splat_scalar(a.rec, lane_index(chunk, n - 1));
                    Splat p1 = load_splat_scalar(a.rec, lane_index(chunk, n > 1 ? n - 2 : 0));
                    for (int j = (int)n - 1; j >= 0; j -= 4) {
                        splat_ready(p0);
                        splat_ready(p1);
                        const Splat q0 = load_splat_scalar(a.rec, lane_index(chunk, (uint32_t)max(j - 2, 0)));
                        const Splat q1 = load_splat_scalar(a.rec, lane_index(chunk, (uint32_t)max(j - 3, 0)));
                        adjoint_scalar<PPL, R>(a, p0, chunk, b0, j, fpx, fpy0, lane, scale, my_last, T, Sx, gC0, gC1,
                                               gC2, gD, gW);
                        if (j >= 1)
                            adjoint_scalar<PPL, R>(a, p1, chunk, b0, j - 1, fpx, fpy0, lane, scale, my_last, T, Sx,
                                                   gC0, gC1, gC2, gD, gW);
                        splat_ready(q0);
                        splat_ready(q1);
                        p0 = load_splat_scalar(a.rec, lane_index(chunk, (uint32_t)max(j - 4, 0)));
                        p1 = load_splat_scalar(a.rec, lane_index(chunk, (uint32_t)max(j - 5, 0)));
                        if (j >= 2)
                            adjoint_scalar<PPL, R>(a, q0, chunk, b0, j - 2, fpx, fpy0, lane, scale, my_last, T, Sx,
                                                   gC0, gC1, gC2, gD, gW);
                        if (j >= 3)
                            adjoint_scalar<PPL, R>(a, q1, chunk, b0, j - 3, fpx, fpy0, lane, scale, my_last, T, Sx,
                                                   gC0, gC1, gC2, gD, gW);
                    }
                    b_end = b0;
                }
            }
        } else {
            for (int ph = a.phases - 1; ph >= 0; --ph) {
                const uint2 rg = a.ranges[(size_t)ph * a.tiles + tile];
                if (rg.x >= rg.y || rg.x >= block_last) continue;
                for (uint32_t b_end = min(rg.y, block_last); b_end > rg.x;) {
                    const uint32_t b0 = b_end - rg.x > (uint32_t)BATCH ? b_end - BATCH : rg.x;
                    const int cnt = (int)(b_end - b0);
                    __syncthreads();   // the previous batch has been consumed
#pragma unroll
                    for (int i = tid; i < BATCH; i += THREADS) {
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
                        const uint32_t idx = b0 + (uint32_t)j;
                        float g10[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                        bool any = false;
                        if (idx < wave_last) {
                            const Splat s = splat_from_lds(sa, sb, sc, j);
                            any = blend_adjoint<PPL, R>(s, fpx, fpy0, idx, my_last, T, Sx, gC0, gC1, gC2, gD, gW,
                                                        g10, a.amin, a.amax);
                        }
                        if (NW == 1) {
                            if (__any(any)) flush_adjoint(g10, lane, scale, a.grad2d, se[j]);
                        } else {
                            const int slot = j & (RED - 1);
                            if (__any(any)) {
                                int which;
                                const float t = wave_sum10(g10, lane, which) * scale;
                                if (which >= 0) red[wave][slot][which] = t;
                            } else if (lane < kGrad2D) {
                                red[wave][slot][lane] = 0.0f;
                            }
                            if (slot == 0) {
                                // add the waves' sums of records j .. j + nrec - 1, one atomic per term
                                __syncthreads();
                                const int nrec = min(RED, cnt - j);
                                for (int i = tid; i < nrec * kGrad2D; i += THREADS) {
                                    const int r = i / kGrad2D, c = i - r * kGrad2D;
                                    float acc = 0.0f;
#pragma unroll
                                    for (int w = 0; w < NW; ++w) acc += red[w][r][c];
                                    if (acc != 0.0f) unsafeAtomicAdd(a.grad2d + (size_t)se[j + r] * kGrad2D + c, acc);
                                }
                                __syncthreads();
                            }
                        }
                    }
                    b_end = b0;
                }
            }
        }
    }
}

template <int TW, int TH, int PPL, int BATCH, bool SCALAR, bool PERSISTENT>
int occupancy_grid(bool fwd) {
    static int cached[2] = {0, 0};
    int& g = cached[fwd ? 1 : 0];
    if (g == 0) {
        int dev = 0, cus = 256, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                cus = prop.multiProcessorCount;
        }
        constexpr int threads = Shape<TW, TH, PPL>::THREADS;
        const hipError_t e =
            fwd ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, reinterpret_cast<const void*>(k_composite_fwd<TW, TH, PPL, BATCH, SCALAR, PERSISTENT>),
                      threads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, reinterpret_cast<const void*>(k_composite_bwd<TW, TH, PPL, BATCH, SCALAR, PERSISTENT>),
                      threads, 0);
        if (e != hipSuccess || per_cu < 1) per_cu = 16 / Shape<TW, TH, PPL>::NW;
        g = cus * per_cu;
    }
    return g;
}

template <int TW, int TH, int PPL, int BATCH, bool SCALAR>
hipError_t run_fwd(const FwdArgs& a, bool persistent, hipStream_t s) {
    constexpr int threads = Shape<TW, TH, PPL>::THREADS;
    if (persistent)
        hipLaunchKernelGGL((k_composite_fwd<TW, TH, PPL, BATCH, SCALAR, true>),
                           dim3(occupancy_grid<TW, TH, PPL, BATCH, SCALAR, true>(true)), dim3(threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_composite_fwd<TW, TH, PPL, BATCH, SCALAR, false>), dim3(a.tiles), dim3(threads), 0, s,
                           a);
    return hipGetLastError();
}

template <int TW, int TH, int PPL, int BATCH, bool SCALAR>
hipError_t run_bwd(const BwdArgs& a, bool persistent, hipStream_t s) {
    constexpr int threads = Shape<TW, TH, PPL>::THREADS;
    if (persistent)
        hipLaunchKernelGGL((k_composite_bwd<TW, TH, PPL, BATCH, SCALAR, true>),
                           dim3(occupancy_grid<TW, TH, PPL, BATCH, SCALAR, true>(false)), dim3(threads), 0, s, a);
    else
        hipLaunchKernelGGL((k_composite_bwd<TW, TH, PPL, BATCH, SCALAR, false>), dim3(a.tiles), dim3(threads), 0, s,
                           a);
    return hipGetLastError();
}

// Dispatch over the launch shape: tile, pixels per lane, LDS batch and record fetch.
// Unset fields take the pass's default: the forward blends two pixels per lane from LDS
// batches, the adjoint (whose per-record wave reduction and atomics are amortised over the
// lane's pixels) four pixels per lane from the scalar cache.
template <template <int, int, int, int, bool> class Run, typename Args>
hipError_t dispatch_shape(const gs_options& o, const Args& a, bool pers, bool adjoint, hipStream_t s) {
    const int fetch = o.record_fetch != GS_FETCH_DEFAULT ? o.record_fetch
                                                         : (adjoint ? kDefaultRecordFetchBwd : kDefaultRecordFetchFwd);
    const bool scalar = fetch == GS_FETCH_SCALAR;
    if (o.tile_w == 8) return scalar ? Run<8, 8, 1, 64, true>::go(a, pers, s) : Run<8, 8, 1, 64, false>::go(a, pers, s);
    const int ppl = o.pixels_per_lane != 0 ? o.pixels_per_lane
                                           : (adjoint ? kDefaultPixelsPerLaneBwd : kDefaultPixelsPerLaneFwd);
    if (scalar) {
        if (ppl == 1) return Run<16, 16, 1, 64, true>::go(a, pers, s);
        if (ppl == 2) return Run<16, 16, 2, 64, true>::go(a, pers, s);
        return Run<16, 16, 4, 64, true>::go(a, pers, s);
    }
#define GS_BATCHES(P)                                                        \
    switch (o.lds_batch) {                                                   \
        case 64: return Run<16, 16, P, 64, false>::go(a, pers, s);          \
        case 128: return Run<16, 16, P, 128, false>::go(a, pers, s);        \
        default: return Run<16, 16, P, 256, false>::go(a, pers, s);         \
    }
    if (ppl == 1) GS_BATCHES(1)
    if (ppl == 2) GS_BATCHES(2)
    GS_BATCHES(4)
#undef GS_BATCHES
}

template <int TW, int TH, int PPL, int BATCH, bool SCALAR>
struct FwdRun {
    static hipError_t go(const FwdArgs& a, bool pers, hipStream_t s) {
        return run_fwd<TW, TH, PPL, BATCH, SCALAR>(a, pers, s);
    }
};

template <int TW, int TH, int PPL, int BATCH, bool SCALAR>
struct BwdRun {
    static hipError_t go(const BwdArgs& a, bool pers, hipStream_t s) {
        return run_bwd<TW, TH, PPL, BATCH, SCALAR>(a, pers, s);
    }
};

struct MediumAdam {
    gs_adam_group g;   // count 9 * views; g.param/m/v updated when enabled
    float b1, b2, eps;
    const float* bc;
    int32_t enabled;
    Guard guard;
    const float* medium;   // [views][9] medium values (read by the prior)
    const float* prior;    // [views][6] (B_inf_hat, B_b_hat) or null
    float prior_lambda;
};

constexpr int kMedThreads = 9 * 64;   // thread t always reads component t % 9 of the [tiles][9] partials

// kMedSlices workgroups per view; deterministic: each reduces a fixed slice of the view's tiles with
// fixed per-thread strides and a fixed tree, and the last slice to finish (a per-view counter,
// zeroed with the 2D gradients at the start of the backward) adds the kMedSlices slice sums in
// slice order and takes the step.
__global__ __launch_bounds__(kMedThreads) void k_medium_reduce(const ViewInfo* __restrict__ vt,
                                                              const float* __restrict__ medpart,
                                                              float* __restrict__ medsum, uint32_t* __restrict__ done,
                                                              float* __restrict__ grad_medium, MediumAdam ad) {
    __shared__ float red[kMedThreads];
    __shared__ uint32_t s_last;
    const int v = blockIdx.x / kMedSlices, slice = blockIdx.x % kMedSlices, tid = threadIdx.x;
    const ViewInfo vi = vt[v];
    if (guard_set(ad.guard)) {   // truncated forward: no gradient and no step
        if (slice == 0 && tid < 9) grad_medium[v * 9 + tid] = 0.0f;
        return;
    }
    const uint32_t per = (vi.n_tiles + kMedSlices - 1) / kMedSlices;
    const uint32_t t0 = min(vi.n_tiles, per * (uint32_t)slice), t1 = min(vi.n_tiles, t0 + per);
    const float* p = medpart + ((int64_t)vi.tile_base + t0) * 9;
    const int64_t total = (int64_t)(t1 - t0) * 9;
    float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int64_t i = tid;
    for (; i + 7 * kMedThreads < total; i += 8 * kMedThreads)   // eight coalesced loads in flight
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += p[i + u * kMedThreads];
    for (; i < total; i += kMedThreads) a[0] += p[i];
    red[tid] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    // component c sits at c + 9 j, j < 64: a tree over j
    for (int off = 32; off > 0; off >>= 1) {
        if (tid < 9 * off) red[tid] += red[tid + 9 * off];
        __syncthreads();
    }
    float* ms = medsum + (int64_t)v * kMedSlices * 9;
    if (tid < 9) __hip_atomic_store(ms + slice * 9 + tid, red[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();   // the slice sum is visible before the counter moves
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(done + v, 1u) == (uint32_t)(kMedSlices - 1) ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (tid < 9) {
        float gm = 0.0f;
        for (int k = 0; k < kMedSlices; ++k)
            gm += __hip_atomic_load(ms + k * 9 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ad.prior && tid >= 3) {   // L_best: lambda sign(B - B_hat) on B_b (slots 3-5) and B_inf (6-8)
            const float d = ad.medium[v * 9 + tid] - ad.prior[v * 6 + (tid < 6 ? tid : tid - 6)];
            gm += d > 0.0f ? ad.prior_lambda : (d < 0.0f ? -ad.prior_lambda : 0.0f);
        }
        grad_medium[v * 9 + tid] = gm;
        if (ad.enabled) {
            const int j = v * 9 + tid;
            float m = ad.g.m[j], vv = ad.g.v[j];
            ad.g.param[j] = adam_update(ad.g.param[j], gm, m, vv, ad.g.lr, ad.b1, ad.b2, ad.eps, ad.bc[0], ad.bc[1]);
            ad.g.m[j] = m;
            ad.g.v[j] = vv;
        }
    }
}

// Per tile: sum and max over pixels of the list entries walked (entries of the tile's phase
// ranges before the pixel's last contributor, plus the entry that stopped the walk), the
// number of those entries that blended (alpha >= alpha_min, re-evaluated with the
// compositing kernel's own sequence), and the live pairs of the tile.
template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_forward_stats(const ViewInfo* __restrict__ vt, int32_t views,
                                                         int32_t phases, uint32_t n_tiles,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ vals,
                                                         const Record* __restrict__ rec,
                                                         const uint32_t* __restrict__ nlast,
                                                         const uint8_t* __restrict__ done, float amin, float amax,
                                                         unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_sum, s_blend;
    __shared__ uint32_t s_max;
    const int tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const int v = find_view(vt, views, tile);
    const ViewInfo vi = vt[v];
    const uint32_t lt = tile - vi.tile_base;
    const int px = (int)(lt % (uint32_t)vi.tiles_x) * TW + tid % TW;
    const int py = (int)(lt / (uint32_t)vi.tiles_x) * TH + tid / TW;
    if (tid == 0) {
        s_sum = 0;
        s_blend = 0;
        s_max = 0;
    }
    __syncthreads();
    uint32_t total = 0;
    for (int ph = 0; ph < phases; ++ph) {
        const uint2 rg = ranges[(size_t)ph * n_tiles + tile];
        total += rg.y - rg.x;
    }
    if (px < vi.width && py < vi.height) {
        const int64_t p = vi.pix_base + (int64_t)py * vi.width + px;
        const uint32_t last = nlast[p];
        const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
        uint32_t walked = 0, blended = 0;
        for (int ph = 0; ph < phases; ++ph) {
            const uint2 rg = ranges[(size_t)ph * n_tiles + tile];
            for (uint32_t i = rg.x; i < min(rg.y, last); ++i) {
                const Record r = rec[vals[i]];
                const Splat sp{r.a.x, r.a.y, r.a.z, r.a.w, r.b.x, r.b.y, r.b.z, r.b.w, r.c.x, r.c.y, r.c.z};
                float dy;
                const float pw = splat_power(sp, col_terms(sp, fpx), fpy, dy);
                blended += fminf(amax, __builtin_amdgcn_exp2f(pw)) >= amin;
                ++walked;
            }
        }
        if (done[p] && walked < total) walked += 1;
        atomicAdd(&s_sum, (unsigned long long)walked);
        atomicAdd(&s_blend, (unsigned long long)blended);
        atomicMax(&s_max, walked);
    }
    __syncthreads();
    if (tid == 0) {
        atomicAdd(&out[0], (unsigned long long)total);
        atomicAdd(&out[1], s_sum);
        atomicAdd(&out[2], (unsigned long long)s_max);
        if (total) atomicAdd(&out[3], 1ull);
        atomicAdd(&out[4], s_blend);
    }
}

__global__ void k_stats_init(unsigned long long* out) {
    for (int i = 0; i < 5; ++i) out[i] = 0;
}

}  // namespace

hipError_t build_queue(const Layout& L, const uint2* ranges, int p0, int p1, uint32_t* qbuf, uint32_t* hist,
                       const uint32_t** order, void* timer, hipStream_t s) {
    const uint32_t T = (uint32_t)L.tiles;
    uint32_t *ka = qbuf, *va = qbuf + T, *kb = qbuf + 2 * (size_t)T, *vb = qbuf + 3 * (size_t)T;
    timer_begin(timer, "queue_keys", s);
    hipLaunchKernelGGL(k_queue_keys, dim3((T + kBlock - 1) / kBlock), dim3(kBlock), 0, s, ranges, p0, p1, T, ka, va);
    timer_end(timer, s);
    int in_b = 0;
    const hipError_t e = radix_sort_u32(ka, va, kb, vb, nullptr, T, 0, 6, L.queue_parts, hist, &in_b, "queue_sort",
                                        timer, s);
    if (e != hipSuccess) return e;
    *order = in_b ? vb : va;
    return hipGetLastError();
}

hipError_t launch_composite_fwd(const gs_options& o, const Layout& L, int phase, int last_phase, const ViewInfo* vt,
                                const gs_medium* med, const Record* rec, const uint2* ranges, const uint32_t* vals,
                                SavedHeader* hdr, uint32_t* alive, float* out_rgb, float* out_depth,
                                float* out_alpha, float* out_restored, float* tfinal, uint32_t* nlast, uint8_t* done,
                                float* cair, float* dsum, float* wsum, const uint32_t* order, uint64_t* rowbits,
                                hipStream_t s) {
    if (L.tiles == 0) return hipSuccess;
    const bool cut = phase == last_phase && last_phase < L.phases - 1;
    FwdArgs a{vt, L.views, (uint32_t)L.tiles, phase, last_phase, med, rec, ranges + (size_t)phase * L.tiles, vals,
              &hdr->queue[phase], order, alive, &hdr->phase_alive[phase], hdr->view_alive[phase], rowbits,
              (uint32_t)L.row_words, cut ? &hdr->status : nullptr, &hdr->phase_rank[phase + 1], &hdr->visible,
              out_rgb, out_depth, out_alpha, out_restored, tfinal, nlast, done, cair, dsum, wsum, L.pixels,
              o.alpha_min, o.alpha_max, o.t_min, o.depth_mode, o.depth_output};
    return dispatch_shape<FwdRun>(o, a, o.persistent != 0, false, s);
}

hipError_t launch_composite_bwd(const gs_options& o, const Layout& L, const ViewInfo* vt, const gs_medium* med,
                                const Record* rec, const uint2* ranges, const uint32_t* vals, const float* grad_rgb,
                                const float* grad_depth, const float* grad_restored, const float* tfinal,
                                const uint32_t* nlast, const float* cair, const float* dsum, const float* wsum,
                                float* grad2d, float* medpart, const Guard& guard, const uint32_t* order,
                                hipStream_t s) {
    if (L.tiles == 0) return hipSuccess;
    BwdArgs a{vt, L.views, (uint32_t)L.tiles, L.phases, med, rec, ranges, vals, nullptr, order, grad_rgb,
              grad_depth, grad_restored, tfinal, nlast, cair, dsum, wsum, grad2d, medpart, L.pixels, o.alpha_min,
              o.alpha_max, o.t_min, o.depth_mode, o.depth_output, guard};
    // the backward's persistent-mode tile counter lives after the medium partials
    a.queue = reinterpret_cast<uint32_t*>(medpart + L.tiles * 9);
    const bool pers = o.persistent != 0;
    if (pers) {
        hipError_t e = launch_fill_u32(a.queue, 0u, 1, s);
        if (e != hipSuccess) return e;
    }
    return dispatch_shape<BwdRun>(o, a, pers, true, s);
}

hipError_t launch_medium_reduce(const ViewInfo* vt, int32_t views, const float* medpart, float* medsum,
                                uint32_t* done, float* grad_medium, const float* medium, const gs_options& o,
                                const gs_adam_group* adam, float b1, float b2, float eps, const float* bc,
                                const Guard& guard, hipStream_t s) {
    MediumAdam ad;
    memset(&ad, 0, sizeof(ad));
    ad.guard = guard;
    ad.medium = medium;
    ad.prior = o.medium_prior;
    ad.prior_lambda = o.prior_lambda;
    if (adam) {
        ad.g = *adam;
        ad.b1 = b1;
        ad.b2 = b2;
        ad.eps = eps;
        ad.bc = bc;
        ad.enabled = 1;
    }
    hipLaunchKernelGGL(k_medium_reduce, dim3(views * kMedSlices), dim3(kMedThreads), 0, s, vt, medpart, medsum, done,
                       grad_medium, ad);
    return hipGetLastError();
}

hipError_t launch_forward_stats(const gs_options& o, const Layout& L, const ViewInfo* vt, const uint2* ranges,
                                const uint32_t* vals, const Record* rec, const uint32_t* nlast, const uint8_t* done,
                                unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_stats_init, dim3(1), dim3(1), 0, s, out);
    if (L.tiles == 0) return hipGetLastError();
    if (L.tile_w == 8)
        hipLaunchKernelGGL((k_forward_stats<8, 8>), dim3((unsigned)L.tiles), dim3(64), 0, s, vt, L.views, L.phases,
                           (uint32_t)L.tiles, ranges, vals, rec, nlast, done, o.alpha_min, o.alpha_max, out);
    else
        hipLaunchKernelGGL((k_forward_stats<16, 16>), dim3((unsigned)L.tiles), dim3(256), 0, s, vt, L.views,
                           L.phases, (uint32_t)L.tiles, ranges, vals, rec, nlast, done, o.alpha_min, o.alpha_max,
                           out);
    return hipGetLastError();
}

}  // namespace gs
