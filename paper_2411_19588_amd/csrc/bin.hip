// Binning of projected Gaussians into tiles (Preliminaries, "Tiles": each
// tile lists the Gaussians whose extent reaches it, in depth order).
//
// Depth-progressive binning.  All (view, Gaussian) entries are first sorted by
// FP32 depth (stable, so equal depths keep index order); entries that touch no
// tile sort last.  The visible entries are then taken in phases of increasing
// depth rank.  Phase p emits the (tile, entry) pairs of its entries -- in phase
// 0 for every tile of each rectangle, afterwards only for tiles where some
// pixel has not yet terminated -- stable-sorts them by tile, and appends them
// to the stored pair list with per-phase tile ranges.  Concatenating a tile's
// phase ranges gives exactly the (depth, index)-ordered list of full binning,
// cut after the phase in which the tile's last pixel terminated; compositing
// never reads past that point, so the images are identical, while scenes whose
// near Gaussians saturate the tiles skip sorting almost every pair.  Every
// emission is balanced over output pairs: a workgroup writes a fixed span of
// pairs (512 in phase 0, 1024 later), whatever the sizes of the rectangles behind them.
//
// Exact tile culling (optional).  The rectangle bounds the ellipse q <= kappa,
// but a Gaussian of opacity o only blends where o exp(-q/2) >= alpha_min, and the
// ellipse covers only part of its rectangle.  A pair is dropped when an upper
// bound of the alpha exponent over the tile's pixel centres, with a margin that
// covers the FP32 rounding of the compositing kernel's own evaluation, stays
// below log2(alpha_min / o): the compositing kernel would have skipped that
// Gaussian at every pixel of the tile, so the images do not change.
#include "internal.h"

namespace gs {
namespace {

constexpr int kScanChunk = 1024;                  // depth ranks per block of the count scan
constexpr int kDownItems = kScanChunk / kBlock;   // consecutive ranks per thread of the down-sweep

// Whether the splat `r` may reach alpha >= alpha_min at a pixel centre of tile (tx, ty): false
// only when the maximum of the (concave) exponent A dx^2 + B dx dy + C dy^2 over the
// rectangle spanned by the tile's pixel centres, plus a rounding margin, is below
// log2(alpha_min) - log2(o), with log2 o as the record stores it.  The maximum is at the
// mean when it lies inside, else on an edge, where the exponent is a 1D concave quadratic
// maximised at its clamped vertex.  Anything non-finite or degenerate keeps the pair.
__device__ __forceinline__ bool tile_may_contribute(const float4& ra, const float2& rb, const ViewInfo& vi,
                                                    uint32_t tx, uint32_t ty, const CullArgs& cu) {
    const float A = ra.z, B = ra.w, C = rb.x, lo = rb.y;
    if (!(A < 0.0f && C < 0.0f)) return true;
    const float x0 = (float)(tx * (uint32_t)cu.tile_w) + 0.5f;
    const float x1 = (float)min((tx + 1) * (uint32_t)cu.tile_w, (uint32_t)vi.width) - 0.5f;
    const float y0 = (float)(ty * (uint32_t)cu.tile_h) + 0.5f;
    const float y1 = (float)min((ty + 1) * (uint32_t)cu.tile_h, (uint32_t)vi.height) - 0.5f;
    const float xl = x0 - ra.x, xr = x1 - ra.x, yl = y0 - ra.y, yr = y1 - ra.y;
    auto expo = [&](float dx, float dy) { return fmaf(dy, fmaf(C, dy, B * dx), (A * dx) * dx); };
    float best;
    if (xl <= 0.0f && xr >= 0.0f && yl <= 0.0f && yr >= 0.0f) {
        best = 0.0f;
    } else {
        // vertex of the edge quadratics, per unit offset.  A hardware reciprocal suffices: off the
        // vertex by a few ulp, a concave quadratic falls below its maximum by a second-order
        // amount (about C (eps y)^2), far inside the rounding margin below
        const float hy = -0.5f * B * __builtin_amdgcn_rcpf(C), hx = -0.5f * B * __builtin_amdgcn_rcpf(A);
        best = expo(xl, fminf(fmaxf(hy * xl, yl), yr));
        best = fmaxf(best, expo(xr, fminf(fmaxf(hy * xr, yl), yr)));
        best = fmaxf(best, expo(fminf(fmaxf(hx * yl, xl), xr), yl));
        best = fmaxf(best, expo(fminf(fmaxf(hx * yr, xl), xr), yr));
    }
    const float X = fmaxf(-xl, xr), Y = fmaxf(-yl, yr);
    const float mag = -A * X * X + fabsf(B) * X * Y - C * Y * Y;
    const float limit = cu.log2_amin - lo;
    return !(best + 4e-6f * mag + 1e-4f < limit);
}

__global__ __launch_bounds__(kBlock) void k_view_table(ViewTable t, ViewInfo* dst, SavedHeader* hdr, uint32_t* fill,
                                                      int64_t fill_count) {
    const int i = threadIdx.x;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + i; j < fill_count; j += (int64_t)gridDim.x * kBlock) fill[j] = 0u;
    if (blockIdx.x != 0) return;
    if (i < t.count) dst[i] = t.v[i];
    for (int j = i; j < GS_MAX_PHASES * GS_MAX_VIEWS; j += kBlock) (&hdr->view_alive[0][0])[j] = 0u;
    if (i == 0) {
        hdr->status = 0;
        hdr->pair_count = 0;
        hdr->pairs_needed = 0;
        hdr->visible = 0;
        hdr->stop = 0;
        for (int p = 0; p <= GS_MAX_PHASES; ++p) {
            hdr->phase_rank[p] = 0;
            hdr->queue[p] = 0;
        }
        for (int p = 0; p < GS_MAX_PHASES; ++p) {
            hdr->phase_base[p] = 0;
            hdr->phase_count[p] = 0;
            hdr->phase_alive[p] = 0;
            hdr->phase_live[p] = 0;
        }
    }
}

// The depth sort left out the entries that touch no tile (key 0xFFFFFFFF) and wrote the number V
// of visible entries it kept; phase p < phases - 1 ends at depth rank ceil(V / 2^(shift - growth p))
// (at V once the exponent reaches 0), the last phase at V.
__device__ __forceinline__ uint32_t phase_end(uint32_t V, const PhaseSched& ps, int p) {
    const int e = ps.shift - ps.growth * p;
    if (p + 1 < ps.phases && e > 0) return (uint32_t)(((uint64_t)V + (1ull << e) - 1) >> e);
    return V;
}

// Depth ranks [r0, r1) of a phase.
__device__ __forceinline__ void phase_ranks(const SavedHeader* hdr, const PhaseSched& ps, int phase, uint32_t& r0,
                                            uint32_t& r1) {
    const uint32_t V = hdr->visible;
    r0 = phase == 0 ? 0u : phase_end(V, ps, phase - 1);
    r1 = phase_end(V, ps, phase);
}

// A later phase after which no tile was left alive emits nothing: the scan kernels skip it.
__device__ __forceinline__ bool phase_empty(const SavedHeader* hdr, int phase) {
    return phase > 0 && hdr->phase_alive[phase - 1] == 0;
}

// Number of alive columns of [lo, hi] in one tile row, from the row's bit masks.
__device__ __forceinline__ uint32_t alive_in(const uint64_t* __restrict__ bits, uint32_t lo, uint32_t hi) {
    uint32_t c = 0;
    for (uint32_t w = lo >> 6; w <= (hi >> 6); ++w) {
        uint64_t m = bits[w];
        if (w == (lo >> 6)) m &= ~0ull << (lo & 63);
        if (w == (hi >> 6) && (hi & 63) != 63) m &= (2ull << (hi & 63)) - 1ull;
        c += (uint32_t)__popcll(m);
    }
    return c;
}


// Per chunk of kScanChunk depth ranks: the phase's per-entry pair counts (pcounts, written only
// inside the phase's ranks: the scan and the emission read them only there), their sum
// (blocksums[b]) and the number of non-zero ones (blocksums[nb + b]).  One rank per thread, so
// that many waves overlap the gathers of the later phases' row loops.
constexpr int kCountThreads = 1024;
constexpr int kCountItems = kScanChunk / kCountThreads;

// Unsigned division by a divisor fixed for a launch: with m = ceil(2^32 / d) (d >= 2),
// e m / 2^32 lies in [e / d, e / d + 1), so its floor is floor(e / d) or one more, which one
// product tells apart.  d = 1 is marked by m = 0.
struct DivU32 {
    uint32_t d, m;
};

inline DivU32 make_divu32(uint32_t d) {
    return {d, d > 1 ? (uint32_t)(((1ull << 32) + d - 1) / d) : 0u};
}

__device__ __forceinline__ uint32_t divu32(uint32_t e, const DivU32& v) {
    if (v.m == 0u) return e;
    uint32_t q = __umulhi(e, v.m);
    if ((uint64_t)q * v.d > (uint64_t)e) --q;
    return q;
}

__global__ __launch_bounds__(kCountThreads) void k_phase_counts(const uint32_t* __restrict__ order,
                                                               const uint32_t* __restrict__ counts,
                                                               const uint2* __restrict__ rects, int64_t nv, int64_t n,
                                                               const ViewInfo* __restrict__ vt,
                                                               const uint64_t* __restrict__ rowbits,
                                                               uint32_t row_words, const SavedHeader* __restrict__ hdr,
                                                               int phase, PhaseSched ps, DivU32 per_view,
                                                               uint32_t* __restrict__ pcounts,
                                                               uint64_t* __restrict__ blocksums, int nb) {
    __shared__ uint64_t red[kCountThreads / 64];
    __shared__ uint32_t zred[kCountThreads / 64];
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
    uint32_t r0, r1;
    phase_ranks(hdr, ps, phase, r0, r1);
    if (phase_empty(hdr, phase) || b0 + kScanChunk <= (int64_t)r0 || b0 >= (int64_t)r1) {   // nothing here
        if (tid == 0) {
            blocksums[blockIdx.x] = 0;
            blocksums[nb + blockIdx.x] = 0;
        }
        return;
    }
    const bool stop = hdr->stop != 0u;   // after an overflow every count is 0
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint32_t e[kCountItems], c[kCountItems];
#pragma unroll
    for (int k = 0; k < kCountItems; ++k) {   // all entry loads in flight before the gathers
        const int64_t r = b0 + k * kCountThreads + tid;
        e[k] = r < nv && r >= (int64_t)r0 && r < (int64_t)r1 && !stop ? order[r] : kNone;
    }
    if (phase == 0) {   // whole rectangles
#pragma unroll
        for (int k = 0; k < kCountItems; ++k) c[k] = e[k] != kNone ? counts[e[k]] : 0u;
    } else {
        // every alive tile of the rectangle (the emission marks the culled ones, as in phase 0): one
        // popcount per 64 columns of each row of the rectangle
#pragma unroll
        for (int k = 0; k < kCountItems; ++k) {
            c[k] = 0u;
            if (e[k] == kNone) continue;
            const uint32_t view = divu32(e[k], per_view);   // e[k] / n
            if (hdr->view_alive[phase - 1][view] == 0u) continue;   // every tile of the view terminated
            const uint2 rc = rects[e[k]];
            const uint32_t rb = vt[view].row_base;
            const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu, y1 = rc.y >> 16;
            for (uint32_t ty = y0; ty <= y1; ++ty) c[k] += alive_in(rowbits + (size_t)(rb + ty) * row_words, x0, x1);
        }
    }
    uint64_t s = 0;
    uint32_t z = 0;
#pragma unroll
    for (int k = 0; k < kCountItems; ++k) {
        const int64_t r = b0 + k * kCountThreads + tid;
        if (r < nv && r >= (int64_t)r0 && r < (int64_t)r1) {
            pcounts[r] = c[k];
            s += c[k];
            z += c[k] != 0u;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += (uint64_t)__shfl_xor((long long)s, off);
        z += (uint32_t)__shfl_xor((int)z, off);
    }
    if ((tid & 63) == 0) {
        red[tid >> 6] = s;
        zred[tid >> 6] = z;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t ts = 0;
        uint32_t tz = 0;
        for (int w = 0; w < kCountThreads / 64; ++w) {
            ts += red[w];
            tz += zred[w];
        }
        blocksums[blockIdx.x] = ts;
        blocksums[nb + blockIdx.x] = tz;
    }
}

// Exclusive scan over a 1024-thread workgroup of one (u64, u32) pair per thread, in place; the
// totals go to ts, tz.  Wave scans by lane shuffles, then the 16 wave totals through LDS.
__device__ __forceinline__ void block_scan_1024(uint64_t& s, uint32_t& z, uint64_t* ws, uint32_t* wz, uint64_t& ts,
                                                uint32_t& tz) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t is = s;
    uint32_t iz = z;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t ys = (uint64_t)__shfl_up((long long)is, off);
        const uint32_t yz = (uint32_t)__shfl_up((int)iz, off);
        if (lane >= off) {
            is += ys;
            iz += yz;
        }
    }
    if (lane == 63) {
        ws[wave] = is;
        wz[wave] = iz;
    }
    __syncthreads();
    uint64_t bs = 0;
    uint32_t bz = 0;
    ts = 0;
    tz = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const uint64_t a = ws[w];
        const uint32_t c = wz[w];
        bs += w < wave ? a : 0ull;
        bz += w < wave ? c : 0u;
        ts += a;
        tz += c;
    }
    __syncthreads();   // ws and wz are reused by the next scan
    s = bs + is - s;
    z = bz + iz - z;
}

// Exclusive scans of the block sums and of the block non-zero counts (one workgroup; the number
// of non-zero counts goes to blocksums[2 nb]), then the phase's ranks, base, count and capacity
// check; zero_bits (nullable) is cleared for the alive masks the phase's compositing sets (the
// phase's own emission reads the other buffer).  Groups of 8 x 1024 sums are staged in LDS by
// coalesced loads (all in flight); each thread sums 8 consecutive ones, one workgroup scan per
// group gives their bases.
__global__ __launch_bounds__(1024) void k_count_blocks(uint64_t* blocksums, int nb, SavedHeader* hdr, int phase,
                                                      PhaseSched ps, int64_t max_pairs, uint64_t* zero_bits,
                                                      int64_t zero_words) {
    constexpr int kItems = 8;
    constexpr int kGroup = 1024 * kItems;
    __shared__ uint64_t lv[kGroup];
    __shared__ uint32_t lw[kGroup];
    __shared__ uint64_t ws[16];
    __shared__ uint32_t wz[16];
    const int tid = threadIdx.x;
    if (zero_bits)
        for (int64_t i = tid; i < zero_words; i += 1024) zero_bits[i] = 0ull;
    uint64_t carry = 0;
    uint32_t zcarry = 0;
    for (int g0 = 0; g0 < nb; g0 += kGroup) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int i = k * 1024 + tid;
            lv[i] = g0 + i < nb ? blocksums[g0 + i] : 0ull;
            lw[i] = g0 + i < nb ? (uint32_t)blocksums[nb + g0 + i] : 0u;
        }
        __syncthreads();
        uint64_t s = 0;
        uint32_t z = 0;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            s += lv[tid * kItems + j];
            z += lw[tid * kItems + j];
        }
        uint64_t ts;
        uint32_t tz;
        block_scan_1024(s, z, ws, wz, ts, tz);
        uint64_t run = carry + s;
        uint32_t zrun = zcarry + z;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint64_t x = lv[tid * kItems + j];
            const uint32_t y = lw[tid * kItems + j];
            lv[tid * kItems + j] = run;
            lw[tid * kItems + j] = zrun;
            run += x;
            zrun += y;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int i = k * 1024 + tid;
            if (g0 + i < nb) {
                blocksums[g0 + i] = lv[i];
                blocksums[nb + g0 + i] = lw[i];
            }
        }
        carry += ts;
        zcarry += tz;
        __syncthreads();   // lv and lw are refilled by the next group
    }
    if (tid == 1023) blocksums[2 * nb] = zcarry;
    if (tid == 0) {   // kept for inspection: the kernels derive the ranks themselves
        uint32_t r0, r1;
        phase_ranks(hdr, ps, phase, r0, r1);
        hdr->phase_rank[phase] = r0;
        hdr->phase_rank[phase + 1] = r1;
    }
    if (tid == 1023 && !hdr->stop) {   // after an overflow the header keeps what the failing phase needed
        const uint64_t total = carry;
        const uint64_t base = hdr->pair_count;
        hdr->phase_base[phase] = (uint32_t)base;
        if (base + total > (uint64_t)max_pairs) {
            hdr->status |= GS_STATUS_PAIR_OVERFLOW;
            hdr->pairs_needed = base + total;
            hdr->stop = 1;
            hdr->phase_count[phase] = 0;
        } else {
            hdr->phase_count[phase] = (uint32_t)total;
            hdr->pair_count = (uint32_t)(base + total);
            hdr->pairs_needed = base + total;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_count_down(const uint32_t* __restrict__ pcounts, int64_t nv,
                                                      const uint64_t* __restrict__ blocksums,
                                                      const SavedHeader* __restrict__ hdr, int phase, PhaseSched ps,
                                                      uint64_t* __restrict__ offsets, uint32_t* __restrict__ emit_start,
                                                      int64_t n_spans, int nb, uint32_t* __restrict__ nzr) {
    __shared__ uint64_t part[kBlock];
    __shared__ uint32_t zpart[kBlock];
    if (phase_empty(hdr, phase)) return;   // every count is 0: no entry reads its offset
    // offsets are read inside the phase's ranks, and by the phase-0 emission up to one span past them
    uint32_t ur0, ur1;
    phase_ranks(hdr, ps, phase, ur0, ur1);
    const int64_t r0 = ur0, r1 = ur1;
    const int64_t cb = (int64_t)blockIdx.x * kScanChunk;
    if (cb + kScanChunk <= r0 || cb >= r1 + kEmitSpanLater + 1) return;
    const int tid = threadIdx.x;
    const int64_t b0 = cb + (int64_t)tid * kDownItems;   // consecutive ranks per thread
    const int64_t span = phase == 0 ? kEmitSpan0 : kEmitSpanLater;   // pairs per emission workgroup
    uint32_t c[kDownItems];
    uint64_t s = 0;
    uint32_t z = 0;
#pragma unroll
    for (int k = 0; k < kDownItems; ++k) {
        const int64_t r = b0 + k;
        c[k] = r < nv && r >= r0 && r < r1 ? pcounts[r] : 0u;
        s += c[k];
        z += c[k] != 0u;
    }
    part[tid] = s;
    zpart[tid] = z;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const uint64_t v = tid >= off ? part[tid - off] : 0ull;
        const uint32_t w = tid >= off ? zpart[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        zpart[tid] += w;
        __syncthreads();
    }
    uint64_t run = blocksums[blockIdx.x] + part[tid] - s;
    uint32_t zrun = (uint32_t)blocksums[nb + blockIdx.x] + zpart[tid] - z;
#pragma unroll
    for (int k = 0; k < kDownItems; ++k) {
        const int64_t r = b0 + k;
        if (r < nv) {
            offsets[r] = run;
            if (c[k]) {
                // later phases: the compact list of the entries with pairs, in depth order
                if (phase > 0) nzr[zrun] = (uint32_t)r;
                // emission spans whose first pair falls inside this entry's pairs [run, run + c):
                // their first entry (a depth rank in phase 0, a position in the compact list later)
                for (int64_t b = (int64_t)((run + span - 1) / span); b * span < (int64_t)(run + c[k]) && b < n_spans;
                     ++b)
                    emit_start[b] = phase == 0 ? (uint32_t)r : zrun;
                ++zrun;
            }
        }
        run += c[k];
    }
}

// Phase-0 pair emission (every tile of each rectangle).  Workgroup b writes output pairs
// [b*kEmitSpan0, (b+1)*kEmitSpan0): it stages the entries (in depth order) whose tile lists
// overlap that span in LDS -- the first one is emit_start[b] -- and each thread produces
// consecutive output slots, so writes are coalesced and every workgroup does the same amount
// of work whatever the rectangle sizes.  Entries of phase 0 all have a non-empty rectangle,
// so their offsets increase strictly and the owners of a span are a prefix of the candidates.
__global__ __launch_bounds__(kBlock) void k_emit_rects(const uint32_t* __restrict__ order,
                                                      const uint64_t* __restrict__ offsets,
                                                      const uint32_t* __restrict__ emit_start,
                                                      const uint2* __restrict__ rects, int64_t nv, int64_t n,
                                                      const ViewInfo* __restrict__ vt,
                                                      const SavedHeader* __restrict__ hdr, int phase,
                                                      CullArgs cull, uint32_t n_tiles,
                                                      uint32_t* __restrict__ tiles_out,
                                                      uint32_t* __restrict__ vals_out) {
    __shared__ int32_t s_off[kEmitSpan0 + 1];
    __shared__ uint32_t s_e[kEmitSpan0 + 1], s_base[kEmitSpan0 + 1], s_w[kEmitSpan0 + 1], s_tx[kEmitSpan0 + 1];
    __shared__ uint32_t s_xy[kEmitSpan0 + 1];
    __shared__ float s_iw[kEmitSpan0 + 1];
    __shared__ uint16_t s_view[kEmitSpan0 + 1];    // culling: view of each entry of the span
    const uint64_t K = hdr->phase_count[phase];
    const uint64_t p0 = (uint64_t)blockIdx.x * kEmitSpan0;
    if (K == 0 || p0 >= K) return;
    const uint64_t p1 = min(p0 + (uint64_t)kEmitSpan0, K);
    const int tid = threadIdx.x;
    const int64_t r0 = emit_start[blockIdx.x];
    int nent = 0;
    for (int i0 = 0; i0 < kEmitSpan0 + 1; i0 += kBlock) {
        const int i = i0 + tid;
        const int64_t r = r0 + i;
        const bool own = i < kEmitSpan0 + 1 && r < nv && (i == 0 || offsets[r] < p1);
        if (own) {
            const uint32_t e = order[r];
            const uint2 rc = rects[e];
            const ViewInfo vi = vt[e / (uint32_t)n];
            const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu;
            const uint32_t w = x1 - x0 + 1;
            s_off[i] = (int32_t)((int64_t)offsets[r] - (int64_t)p0);
            s_e[i] = e;
            s_base[i] = vi.tile_base + y0 * (uint32_t)vi.tiles_x + x0;
            s_w[i] = w;
            s_tx[i] = (uint32_t)vi.tiles_x;
            s_xy[i] = rc.x;
            s_iw[i] = 1.0f / (float)w;
            s_view[i] = (uint16_t)(e / (uint32_t)n);
        }
        nent += __syncthreads_count(own);
    }
    const int span = (int)(p1 - p0);
#pragma unroll
    for (int k = 0; k < (kEmitSpan0 / kBlock); ++k) {
        const int q = k * kBlock + tid;
        if (q >= span) break;
        int lo = 0, hi = nent;   // last i with s_off[i] <= q
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= q) lo = mid;
            else hi = mid;
        }
        const uint32_t j = (uint32_t)(q - s_off[lo]);
        const uint32_t w = s_w[lo];
        uint32_t row = (uint32_t)((float)j * s_iw[lo]);
        if (row * w > j) --row;
        else if ((row + 1) * w <= j) ++row;
        const uint32_t col = j - row * w;
        const uint32_t e = s_e[lo];
        uint32_t tile = s_base[lo] + row * s_tx[lo] + col;
        if (cull.enabled) {
            // the entry's record is read by every pair of its rectangle: cache hits after the first
            const Record* rp = cull.rec + e;
            const ViewInfo vi = vt[s_view[lo]];
            const uint32_t xy = s_xy[lo];
            if (!tile_may_contribute(rp->a, make_float2(rp->b.x, rp->b.y), vi, (xy & 0xFFFFu) + col,
                                     (xy >> 16) + row, cull))
                tile = n_tiles;
        }
        tiles_out[p0 + q] = tile;
        vals_out[p0 + q] = e;
    }
}

// Position of the k-th (from 0) set bit of m; m has more than k set bits.
__device__ __forceinline__ uint32_t select_bit(uint64_t m, uint32_t k) {
    uint32_t pos = 0, c;
    c = (uint32_t)__popc((uint32_t)m);
    if (k >= c) { k -= c; m >>= 32; pos += 32; }
    c = (uint32_t)__popc((uint32_t)m & 0xFFFFu);
    if (k >= c) { k -= c; m >>= 16; pos += 16; }
    c = (uint32_t)__popc((uint32_t)m & 0xFFu);
    if (k >= c) { k -= c; m >>= 8; pos += 8; }
    c = (uint32_t)__popc((uint32_t)m & 0xFu);
    if (k >= c) { k -= c; m >>= 4; pos += 4; }
    c = (uint32_t)__popc((uint32_t)m & 0x3u);
    if (k >= c) { k -= c; m >>= 2; pos += 2; }
    if (k >= ((uint32_t)m & 1u)) pos += 1;
    return pos;
}

// Column of the k-th (from 0) alive tile of [lo, hi] in one tile row (hi if there are fewer);
// w0 and w1 are the row's mask words lo / 64 and lo / 64 + 1, loaded by the caller.
__device__ __forceinline__ uint32_t kth_alive(const uint64_t* __restrict__ bits, uint32_t lo, uint32_t hi,
                                              uint32_t k, uint64_t w0, uint64_t w1) {
    for (uint32_t w = lo >> 6; w <= (hi >> 6); ++w) {
        uint64_t m = w == (lo >> 6) ? w0 : (w == (lo >> 6) + 1 ? w1 : bits[w]);
        if (w == (lo >> 6)) m &= ~0ull << (lo & 63);
        if (w == (hi >> 6) && (hi & 63) != 63) m &= (2ull << (hi & 63)) - 1ull;
        const uint32_t c = (uint32_t)__popcll(m);
        if (k < c) return w * 64 + select_bit(m, k);
        k -= c;
    }
    return hi;
}

// Later-phase pair emission (the alive tiles of each rectangle, rows then columns), balanced
// over output pairs like the phase-0 emission: workgroup b writes pairs [b*kEmitSpanLater,
// (b+1)*kEmitSpanLater).  It stages the entries with pairs in that span (from the compact list of the
// entries with a non-zero count, starting at emit_start[b]), splits them into rows with alive
// tiles -- one item per row, stored at its first pair in the span -- and gives each pair its row
// by a running maximum over the item positions and its column as the k-th alive one of the row.
__global__ __launch_bounds__(kBlock) void k_emit_spans(const uint32_t* __restrict__ order,
                                                      const uint64_t* __restrict__ offsets,
                                                      const uint32_t* __restrict__ nzr,
                                                      const uint64_t* __restrict__ nz_total,
                                                      const uint32_t* __restrict__ emit_start,
                                                      const uint2* __restrict__ rects, int64_t n,
                                                      const ViewInfo* __restrict__ vt,
                                                      const uint64_t* __restrict__ rowbits, uint32_t row_words,
                                                      const SavedHeader* __restrict__ hdr, int phase,
                                                      CullArgs cull, uint32_t n_tiles,
                                                      uint32_t* __restrict__ tiles_out,
                                                      uint32_t* __restrict__ vals_out) {
    __shared__ int32_t s_off[kEmitSpanLater + 1];   // entry: first pair, relative to the span
    __shared__ uint32_t s_e[kEmitSpanLater + 1];    // entry: (view, Gaussian) index
    __shared__ uint8_t s_ev[kEmitSpanLater + 1];    // entry: its view (one division per entry, not per pair)
    __shared__ int32_t s_cover[kEmitSpanLater];     // item position at its first pair, -1 elsewhere; then the running max
    __shared__ int32_t s_ist[kEmitSpanLater];       // item: first pair, relative to the span (< 0 for a row begun before)
    __shared__ uint32_t s_ilohi[kEmitSpanLater];    // item: column range lo | hi << 16
    __shared__ uint32_t s_ijy[kEmitSpanLater];      // item: entry slot | tile row << 16
    __shared__ int32_t s_wmax[kBlock / 64];
    const uint64_t K = hdr->phase_count[phase];
    const uint64_t p0 = (uint64_t)blockIdx.x * kEmitSpanLater;
    if (K == 0 || p0 >= K) return;
    const int span = (int)min((uint64_t)kEmitSpanLater, K - p0);
    const uint64_t p1 = p0 + (uint64_t)span;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint64_t i0 = emit_start[blockIdx.x], nz = *nz_total;
    // entries: every one after the first starts inside the span, and each has a pair, so at most
    // kEmitSpanLater + 1 of them
    int nent = 0;
    for (int j0 = 0; j0 < kEmitSpanLater + 1; j0 += kBlock) {
        const int j = j0 + tid;
        const uint64_t idx = i0 + (uint64_t)j;
        bool own = false;
        if (j < kEmitSpanLater + 1 && idx < nz) {
            const uint32_t r = nzr[idx];
            const uint64_t off = offsets[r];
            own = j == 0 || off < p1;
            if (own) {
                s_off[j] = (int32_t)((int64_t)off - (int64_t)p0);
                s_e[j] = order[r];
            }
        }
        nent += __syncthreads_count(own);
    }
    for (int q = tid; q < kEmitSpanLater; q += kBlock) s_cover[q] = -1;
    __syncthreads();
    // items: the rows with alive tiles of each entry that reach into the span
    for (int j = tid; j < nent; j += kBlock) {
        const uint32_t e = s_e[j];
        const uint2 rc = rects[e];
        const uint32_t view = e / (uint32_t)n;
        s_ev[j] = (uint8_t)view;
        const ViewInfo vi = vt[view];
        const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu, y1 = rc.y >> 16;
        int32_t st = s_off[j];
        for (uint32_t ty = y0; ty <= y1 && st < span; ++ty) {
            const uint32_t lo = x0, hi = x1;
            const int32_t c = (int32_t)alive_in(rowbits + (size_t)(vi.row_base + ty) * row_words, lo, hi);
            if (c == 0) continue;
            if (st + c > 0) {
                const int pos = max(st, 0);
                s_ist[pos] = st;
                s_ilohi[pos] = lo | (hi << 16);
                s_ijy[pos] = (uint32_t)j | (ty << 16);
                s_cover[pos] = pos;
            }
            st += c;
        }
    }
    __syncthreads();
    // running maximum over the span: each pair's item is the last one that starts at or before it
    constexpr int kEmitItems = kEmitSpanLater / kBlock;
    int v[kEmitItems];
    int m = -1;
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) {
        m = max(m, s_cover[tid * kEmitItems + k]);
        v[k] = m;
    }
    int x = m;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x = max(x, y);
    }
    if (lane == 63) s_wmax[tid >> 6] = x;
    __syncthreads();
    int before = __shfl_up(x, 1);
    if (lane == 0) before = -1;
    for (int w = 0; w < (tid >> 6); ++w) before = max(before, s_wmax[w]);
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) s_cover[tid * kEmitItems + k] = max(before, v[k]);
    __syncthreads();
    // Per pair, two rounds of loads: the view's fields with the splat's record, then the row's first
    // two mask words (further words, for rows of more than 128 tiles, in the loop).
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) {
        const int q = k * kBlock + tid;
        if (q >= span) break;
        const int pos = s_cover[q];
        if (pos < 0) {   // cannot happen: the first entry covers the span's first pair
            tiles_out[p0 + q] = n_tiles;
            vals_out[p0 + q] = 0u;
            continue;
        }
        const uint32_t jy = s_ijy[pos], lohi = s_ilohi[pos];
        const uint32_t e = s_e[jy & 0xFFFFu], ty = jy >> 16, lo = lohi & 0xFFFFu, hi = lohi >> 16;
        const ViewInfo vi = vt[s_ev[jy & 0xFFFFu]];
        float4 ra;
        float2 rb;
        if (cull.enabled) {
            const Record* rp = cull.rec + e;
            ra = rp->a;
            rb = make_float2(rp->b.x, rp->b.y);
        }
        const uint64_t* row = rowbits + (size_t)(vi.row_base + ty) * row_words;
        const uint64_t w0 = row[lo >> 6], w1 = (lo >> 6) < (hi >> 6) ? row[(lo >> 6) + 1] : 0ull;
        const uint32_t tx = kth_alive(row, lo, hi, (uint32_t)(q - s_ist[pos]), w0, w1);
        uint32_t tile = vi.tile_base + ty * (uint32_t)vi.tiles_x + tx;
        // a culled pair gets the out-of-range tile id: the tile sort leaves it out
        if (cull.enabled && !tile_may_contribute(ra, rb, vi, tx, ty, cull)) tile = n_tiles;
        tiles_out[p0 + q] = tile;
        vals_out[p0 + q] = e;
    }
}

// One wave per global tile row: the bit masks of the columns whose tile is still alive.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_commit(const uint32_t* __restrict__ tiles,
                                                  const SavedHeader* __restrict__ hdr, int phase, uint32_t n_tiles,
                                                  uint2* __restrict__ ranges) {
    const uint32_t K = hdr->phase_live[phase];   // culled pairs were left out by the tile sort
    const uint32_t base = hdr->phase_base[phase];
    uint2* rg = ranges + (size_t)phase * n_tiles;
    // four consecutive ids per thread (one 16-byte load; `tiles` is 16-byte aligned) and their
    // outer neighbours; a range starts or ends where the id changes
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < (K + 3) / 4; c += gridDim.x * kBlock) {
        const uint32_t i0 = 4 * c;
        uint32_t t[6];
        if (i0 + 4 <= K) {
            const uint4 v = *reinterpret_cast<const uint4*>(tiles + i0);
            t[1] = v.x;
            t[2] = v.y;
            t[3] = v.z;
            t[4] = v.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) t[1 + k] = i0 + k < K ? tiles[i0 + k] : 0xFFFFFFFFu;
        }
        t[0] = i0 > 0 ? tiles[i0 - 1] : 0xFFFFFFFFu;       // no id equals the sentinel
        t[5] = i0 + 4 < K ? tiles[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const uint32_t i = i0 + (uint32_t)(k - 1);
            if (i >= K || t[k] >= n_tiles) continue;   // tile ids are < n_tiles by construction
            if (t[k - 1] != t[k]) rg[t[k]].x = base + i;
            if (t[k + 1] != t[k]) rg[t[k]].y = base + i + 1;
        }
    }
}

// One workgroup per tile writes the keys of that tile's pairs in every phase.
__global__ __launch_bounds__(kBlock) void k_export(const uint2* __restrict__ ranges, int phases, uint32_t n_tiles,
                                                  const uint32_t* __restrict__ vals,
                                                  const uint32_t* __restrict__ depth_keys, int64_t capacity,
                                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ values) {
    const uint32_t t = blockIdx.x;
    for (int p = 0; p < phases; ++p) {
        const uint2 rg = ranges[(size_t)p * n_tiles + t];
        for (uint32_t i = rg.x + threadIdx.x; i < rg.y; i += kBlock) {
            if ((int64_t)i >= capacity) break;
            const uint32_t e = vals[i];
            keys[i] = ((uint64_t)t << 32) | (uint64_t)depth_keys[e];
            values[i] = e;
        }
    }
}

}  // namespace

hipError_t launch_view_table(const ViewTable& t, ViewInfo* dst, SavedHeader* hdr, uint32_t* fill, int64_t fill_count,
                             hipStream_t s) {
    int64_t g = (fill_count + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_view_table, dim3((unsigned)g), dim3(kBlock), 0, s, t, dst, hdr, fill, fill_count);
    return hipGetLastError();
}

int64_t count_scan_blocks(int64_t nv) { return (nv + kScanChunk - 1) / kScanChunk; }

hipError_t launch_count_scan(const uint32_t* order, const uint32_t* counts, const uint2* rects, int64_t nv,
                             int64_t n, const ViewInfo* vt, const AliveRows& ar, uint64_t* zero_bits,
                             int64_t zero_words, const PhaseSched& ps, SavedHeader* hdr, int phase,
                             uint32_t* pcounts, uint64_t* offsets, uint64_t* blocksums, int64_t max_pairs,
                             uint32_t* emit_start, hipStream_t s) {
    const int nb = (int)count_scan_blocks(nv);
    const int64_t n_spans = max_pairs / kEmitSpan0 + 2;
    if (nb > 0)
        hipLaunchKernelGGL(k_phase_counts, dim3(nb), dim3(kCountThreads), 0, s, order, counts, rects, nv, n, vt, ar.bits,
                           ar.words, hdr, phase, ps, make_divu32((uint32_t)n), pcounts, blocksums, nb);
    hipLaunchKernelGGL(k_count_blocks, dim3(1), dim3(1024), 0, s, blocksums, nb, hdr, phase, ps, max_pairs, zero_bits,
                       zero_words);
    if (nb > 0)
        hipLaunchKernelGGL(k_count_down, dim3(nb), dim3(kBlock), 0, s, pcounts, nv, blocksums, hdr, phase, ps,
                           offsets, emit_start, n_spans, nb, ar.nzr);
    return hipGetLastError();
}

hipError_t launch_emit(const uint32_t* order, const uint64_t* offsets, const uint32_t* emit_start,
                       const uint64_t* blocksums, const uint2* rects, int64_t nv, int64_t n, const ViewInfo* vt,
                       const AliveRows& ar, const SavedHeader* hdr, int phase, int64_t max_pairs,
                       const CullArgs& cull, uint32_t n_tiles, uint32_t* tiles_out, uint32_t* vals_out,
                       hipStream_t s) {
    if (nv == 0 || max_pairs == 0) return hipSuccess;
    const int64_t span = phase == 0 ? kEmitSpan0 : kEmitSpanLater;
    const unsigned grid = (unsigned)((max_pairs + span - 1) / span);
    if (phase == 0) {
        hipLaunchKernelGGL(k_emit_rects, dim3(grid), dim3(kBlock), 0, s, order, offsets, emit_start, rects, nv, n, vt,
                           hdr, phase, cull, n_tiles, tiles_out, vals_out);
    } else {
        const uint64_t* nz_total = blocksums + 2 * count_scan_blocks(nv);
        hipLaunchKernelGGL(k_emit_spans, dim3(grid), dim3(kBlock), 0, s, order, offsets, ar.nzr, nz_total,
                           emit_start, rects, n, vt, ar.bits, ar.words, hdr, phase, cull, n_tiles,
                           tiles_out, vals_out);
    }
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlock), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_commit(const uint32_t* sorted_tiles, const SavedHeader* hdr, int phase, int64_t tiles,
                         int64_t max_pairs, uint2* ranges, hipStream_t s) {
    if (max_pairs == 0) return hipSuccess;
    constexpr int64_t kMaxCommitGrid = 4096;   // grid-stride beyond 4M pairs; an empty phase costs little
    const int64_t want = (max_pairs + 4 * kBlock - 1) / (4 * kBlock);
    const unsigned grid = (unsigned)(want < kMaxCommitGrid ? want : kMaxCommitGrid);
    hipLaunchKernelGGL(k_commit, dim3(grid), dim3(kBlock), 0, s, sorted_tiles, hdr, phase, (uint32_t)tiles, ranges);
    return hipGetLastError();
}

hipError_t launch_export_keys(const Layout& L, const uint2* ranges, const uint32_t* vals, const uint32_t* depth_keys,
                              int64_t capacity, uint64_t* keys, uint32_t* values, hipStream_t s) {
    if (L.tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_export, dim3((unsigned)L.tiles), dim3(kBlock), 0, s, ranges, L.phases, (uint32_t)L.tiles,
                       vals, depth_keys, capacity, keys, values);
    return hipGetLastError();
}

}  // namespace gs
