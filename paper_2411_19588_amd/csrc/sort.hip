// Stable least-significant-digit radix sort of (u32 key, u32 value) pairs, used
// for the depth order of eq. (3dgs_orig) and for binning pairs by tile
// (Preliminaries, "Tiles").
//
// Each pass is reduce-then-scan over a FIXED number of partitions `parts`; the
// element count is read from device memory, so the launch shapes never depend
// on data and a whole forward can be captured into a graph.
//   1. k_hist:      each partition counts its digits with LDS atomics (the
//                   counts need no ranks); a wave whose valid keys all share one
//                   digit adds them with one atomic.  The next radix tile's keys
//                   are loaded while the current one is counted.
//   2. k_scan_rows: one workgroup per digit scans that digit's row of the
//                   digit-major [radix][parts] table and records the row total.
// A key of b bits takes ceil(b / 9) passes of at most 9 bits, split evenly: 8-bit
// digits use 256 counters, 9-bit digits 512 (two per thread in the block scans), so
// 17-bit tile ids (up to 131071 tiles) take two passes instead of three.
//   3. k_scatter:   each partition turns the row totals into digit bases, then
//                   re-reads its range tile by tile, ranks keys stably inside each
//                   wave (lanes that share a digit are found by intersecting one
//                   ballot per digit bit; the digit width is a template argument),
//                   combines the four waves through LDS, reorders the tile in LDS
//                   by digit and writes it out in digit runs (coalesced).  The next
//                   tile's keys and values are loaded while the current one is
//                   written out.  A radix tile holds 2048 keys, or 4096 for sorts of
//                   kLargeSortKeys keys and more (fewer, longer digit runs per tile).
#include <algorithm>
#include <string>

#include "internal.h"

namespace gs {
namespace {

__device__ __forceinline__ uint32_t load_n(const uint32_t* n_dev, uint32_t n_host) {
    return n_dev ? *n_dev : n_host;
}

// Partition p covers radix tiles [t0, t1) of TILE elements each.
template <int TILE>
__device__ __forceinline__ void part_range(uint32_t n, int parts, int p, uint32_t& t0, uint32_t& t1) {
    const uint32_t tiles = (n + TILE - 1) / TILE;
    const uint32_t per = (tiles + parts - 1) / parts;
    t0 = min(tiles, per * (uint32_t)p);
    t1 = min(tiles, t0 + per);
}

// Mask of the lanes (among `active`) whose digit equals this lane's digit: per digit bit b, the
// ballot B of the lanes with that bit set; a lane keeps B where its bit is set and ~B where it is
// clear, i.e. m &= ~(B ^ s) with s the lane's bit sign-extended (one three-input op per half).
template <int NBITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t digit, uint64_t active) {
    uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
#pragma unroll
    for (int b = 0; b < NBITS; ++b) {
        const int32_t si = (int32_t)(digit << (31 - b)) >> 31;   // the bit, sign-extended
        const uint64_t bal = __ballot(si < 0);
        const uint32_t s = (uint32_t)si;
        lo &= ~((uint32_t)bal ^ s);
        hi &= ~((uint32_t)(bal >> 32) ^ s);
    }
    return ((uint64_t)hi << 32) | lo;
}

template <int D, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_hist(const uint32_t* __restrict__ keys, const uint32_t* n_dev,
                                                uint32_t n_host, int shift, int nbits, int parts, int use_drop,
                                                uint32_t drop, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[D];
    const uint32_t n = load_n(n_dev, n_host);
    if (n == 0) return;   // nothing to sort (an empty phase): the scan and the scatter return too
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < D; i += kBlock) h[i] = 0;
    __syncthreads();
    const uint32_t mask = (1u << nbits) - 1u;
    uint32_t t0, t1;
    part_range<kBlock * ITEMS>(n, parts, blockIdx.x, t0, t1);
    uint32_t key[ITEMS];
    auto load_tile = [&](uint32_t t) {   // all loads in flight before any count
        const uint32_t base = t * (kBlock * ITEMS);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = base + k * kBlock + tid;
            key[k] = idx < n ? keys[idx] : 0u;
        }
    };
    if (t0 < t1) load_tile(t0);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t base = t * (kBlock * ITEMS);
        uint32_t cur[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) cur[k] = key[k];
        if (t + 1 < t1) load_tile(t + 1);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const bool valid = base + k * kBlock + tid < n && !(use_drop && cur[k] == drop);
            const uint32_t digit = (cur[k] >> shift) & mask;
            const uint64_t vm = __ballot(valid);
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)digit);
            const uint64_t same = __ballot(valid && digit == d0);
            if (same == vm) {   // one digit in the whole wave (runs of equal keys): one atomic
                if (vm != 0ull && lane == 0) atomicAdd(&h[d0], (uint32_t)__popcll(vm));
            } else if (valid) {
                atomicAdd(&h[digit], 1u);
            }
        }
    }
    __syncthreads();
    for (int d = tid; d < D; d += kBlock) hist[(size_t)d * parts + blockIdx.x] = h[d];
}

// Block-wide exclusive scan of one u32 per thread (256 threads = 4 waves); returns the
// total.  Inclusive scans inside each wave by lane shuffles, then the four wave totals
// through LDS (two barriers; `s` needs 4 entries).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s, uint32_t& total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) s[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const uint32_t t = s[w];
        before += w < wave ? t : 0u;
        total += t;
    }
    __syncthreads();   // `s` may be reused by the caller
    return before + inc - x;
}

// Exclusive scan of row d (parts <= kMaxSortParts entries) in place; totals[d] = row sum.
__global__ __launch_bounds__(kBlock) void k_scan_rows(uint32_t* __restrict__ hist, int parts,
                                                     uint32_t* __restrict__ totals, const uint32_t* n_dev,
                                                     uint32_t n_host) {
    __shared__ uint32_t s[kBlock / 64];
    if (load_n(n_dev, n_host) == 0) return;
    const int tid = threadIdx.x;
    uint32_t* row = hist + (size_t)blockIdx.x * parts;
    constexpr int PER = kMaxSortParts / kBlock;
    uint32_t v[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = tid * PER + k;
        v[k] = i < parts ? row[i] : 0u;
        sum += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, s, total);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = tid * PER + k;
        if (i < parts) row[i] = run;
        run += v[k];
    }
    if (tid == 0) totals[blockIdx.x] = total;
}

template <int NBITS, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                   const uint32_t* __restrict__ vout_off,
                                                   const uint32_t* n_dev, uint32_t n_host, int shift,
                                                   int parts, const uint32_t* __restrict__ hist,
                                                   const uint32_t* __restrict__ totals, int use_drop,
                                                   uint32_t drop, uint32_t* __restrict__ n_kept) {
    constexpr int D = NBITS > kRadixBits ? kMaxRadix : kRadix;
    constexpr int TILE = kBlock * ITEMS;
    constexpr int DPT = D / kBlock;   // digits per thread in the block scans: thread t owns t*DPT + j
    static_assert(DPT * kBlock == D && (DPT == 1 || DPT == 2), "256 or 512 digits");
    __shared__ uint32_t run[D];       // global write base of each digit for the next tile
    __shared__ uint32_t wcnt[4][D];   // per-wave digit counts, then per-wave digit offsets in the tile
    __shared__ uint32_t tstart[D];    // first slot of each digit in the LDS-ordered tile
    __shared__ uint32_t scan_tmp[kBlock / 64];
    __shared__ uint32_t sk[TILE], sv[TILE];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t mask = (1u << NBITS) - 1u;
    const uint32_t n = load_n(n_dev, n_host);
    if (n == 0) {
        if (n_kept && blockIdx.x == 0 && tid == 0) *n_kept = 0;
        return;
    }
    const uint32_t vbase = vout_off ? *vout_off : 0u;   // values land at vout + vbase + position
    {
        // only the pass's 2^NBITS digit rows were scanned
        uint32_t tv[DPT], sum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const uint32_t d = (uint32_t)(tid * DPT + j);
            tv[j] = d <= mask ? totals[d] : 0u;
            sum += tv[j];
        }
        uint32_t tot;
        uint32_t b = block_exclusive_scan(sum, scan_tmp, tot);
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            run[d] = b + hist[(size_t)d * parts + blockIdx.x];
            b += tv[j];
        }
        if (n_kept && blockIdx.x == 0 && tid == 0) *n_kept = tot;   // keys kept (equal to drop: left out)
    }
    uint32_t t0, t1;
    part_range<TILE>(n, parts, blockIdx.x, t0, t1);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // wave w ranks elements [tbase + w*512, tbase + (w+1)*512) of a tile in order: item k, lane l.
    uint32_t key[ITEMS], val[ITEMS];
    auto load_tile = [&](uint32_t t) {   // all loads in flight before the ranking
        const uint32_t wb = t * TILE + (uint32_t)wave * 64u * ITEMS;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wb + k * 64 + lane;
            key[k] = idx < n ? kin[idx] : 0u;
            val[k] = idx < n ? vin[idx] : 0u;
        }
    };
    if (t0 < t1) load_tile(t0);
    for (uint32_t t = t0; t < t1; ++t) {
        for (int i = tid; i < 4 * D; i += kBlock) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        const uint32_t tbase = t * TILE;
        const uint32_t wbase = tbase + (uint32_t)wave * 64u * ITEMS;
        uint32_t rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * 64 + lane;
            const bool valid = idx < n && !(use_drop && key[k] == drop);
            const uint32_t digit = (key[k] >> shift) & mask;
            const uint64_t match = match_digit<NBITS>(digit, __ballot(valid));
            const uint32_t before = wcnt[wave][digit];
            rank[k] = before + __popcll(match & lt_mask);
            if (valid && lane == __ffsll((unsigned long long)match) - 1)
                wcnt[wave][digit] = before + (uint32_t)__popcll(match);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // the thread's digits: wave offsets inside each digit, tile-local digit starts, global bases
        uint32_t cnt[DPT], csum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t x = wcnt[w][d];
                wcnt[w][d] = c;
                c += x;
            }
            cnt[j] = c;
            csum += c;
        }
        uint32_t tot;
        uint32_t ts = block_exclusive_scan(csum, scan_tmp, tot);
        uint32_t tsj[DPT], gbase[DPT];
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            tsj[j] = ts;
            tstart[d] = ts;
            ts += cnt[j];
            gbase[j] = run[d];
        }
        __syncthreads();
        // reorder the tile in LDS by digit (stable)
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * 64 + lane;
            if (idx < n && !(use_drop && key[k] == drop)) {
                const uint32_t digit = (key[k] >> shift) & mask;
                const uint32_t lp = tstart[digit] + wcnt[wave][digit] + rank[k];
                if (lp < (uint32_t)TILE) {   // always true: lp < tile count
                    sk[lp] = key[k];
                    sv[lp] = val[k];
                }
            }
        }
        if (t + 1 < t1) load_tile(t + 1);   // in flight while this tile is written out
        // LDS slot i of digit d goes to global slot (run[d] - tstart[d]) + i
#pragma unroll
        for (int j = 0; j < DPT; ++j) run[tid * DPT + j] = gbase[j] - tsj[j];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t i = k * kBlock + tid;
            if (i < tot) {   // the tile's kept keys, in digit order
                const uint32_t kk = sk[i];
                const uint32_t pos = run[(kk >> shift) & mask] + i;
                if (pos < n) {   // always true when the histogram and ranking agree
                    kout[pos] = kk;
                    vout[vbase + pos] = sv[i];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < DPT; ++j) run[tid * DPT + j] = gbase[j] + cnt[j];
        __syncthreads();
    }
}

}  // namespace

namespace {

// The passes of one sort with radix tiles of kBlock * ITEMS keys over `parts` partitions.
template <int ITEMS>
hipError_t sort_passes(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, const uint32_t* n_dev,
                       uint32_t n_host, int bit0, int nbits, int parts, uint32_t* hist, uint32_t* totals,
                       int* result_in_b, const char* tag, void* timer, hipStream_t s, int use_drop, uint32_t drop_key,
                       uint32_t* n_kept, uint32_t* final_vals, const uint32_t* final_off) {
    const std::string th = std::string(tag) + "_hist", ts = std::string(tag) + "_scan",
                      tc = std::string(tag) + "_scatter";
    // ceil(nbits / 9) passes, the bits split as evenly as possible (at most 9 per pass)
    const int passes = (nbits + kMaxRadixBits - 1) / kMaxRadixBits;
    int in_b = 0, done = 0;
    for (int q = 0; q < passes; ++q) {
        const int bits = nbits / passes + (q < nbits % passes ? 1 : 0);
        const int shift = bit0 + done;
        const uint32_t* kin = in_b ? keys_b : keys_a;
        const uint32_t* vin = in_b ? vals_b : vals_a;
        uint32_t* kout = in_b ? keys_a : keys_b;
        uint32_t* vout = in_b ? vals_a : vals_b;
        const uint32_t* voff = nullptr;
        if (q == passes - 1 && final_vals) {   // the last pass writes the values to their destination
            vout = final_vals;
            voff = final_off;
        }
        // the first pass leaves out the keys equal to drop_key; later passes sort the kept ones
        const bool first = q == 0;
        const int drop_now = first && use_drop ? 1 : 0;
        const uint32_t* n_in = (!first && n_kept) ? n_kept : n_dev;
        const bool wide = bits > kRadixBits;   // 512 digit counters
        timer_begin(timer, th.c_str(), s);
        if (wide)
            hipLaunchKernelGGL((k_hist<kMaxRadix, ITEMS>), dim3(parts), dim3(kBlock), 0, s, kin, n_in, n_host, shift,
                               bits, parts, drop_now, drop_key, hist);
        else
            hipLaunchKernelGGL((k_hist<kRadix, ITEMS>), dim3(parts), dim3(kBlock), 0, s, kin, n_in, n_host, shift,
                               bits, parts, drop_now, drop_key, hist);
        timer_end(timer, s);
        timer_begin(timer, ts.c_str(), s);
        hipLaunchKernelGGL(k_scan_rows, dim3(1u << bits), dim3(kBlock), 0, s, hist, parts, totals, n_in, n_host);
        timer_end(timer, s);
        timer_begin(timer, tc.c_str(), s);
        uint32_t* kept = first ? n_kept : nullptr;
        switch (bits) {   // the digit width is a template argument: the ranking unrolls per bit
#define GS_SCATTER(B)                                                                                                \
    case B:                                                                                                          \
        hipLaunchKernelGGL((k_scatter<B, ITEMS>), dim3(parts), dim3(kBlock), 0, s, kin, vin, kout, vout, voff, n_in,   \
                           n_host, shift, parts, hist, totals, drop_now, drop_key, kept);                            \
        break;
            GS_SCATTER(1) GS_SCATTER(2) GS_SCATTER(3) GS_SCATTER(4) GS_SCATTER(5) GS_SCATTER(6) GS_SCATTER(7)
            GS_SCATTER(8) GS_SCATTER(9)
#undef GS_SCATTER
            default: return hipErrorInvalidValue;
        }
        timer_end(timer, s);
        in_b = !in_b;
        done += bits;
    }
    *result_in_b = in_b;
    return hipGetLastError();
}

}  // namespace

hipError_t radix_sort_u32(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b,
                          const uint32_t* n_dev, uint32_t n_host, int bit0, int nbits, int parts,
                          uint32_t* hist, int* result_in_b, const char* tag, void* timer, hipStream_t s,
                          int use_drop, uint32_t drop_key, uint32_t* n_kept, uint32_t* final_vals,
                          const uint32_t* final_off) {
    if (nbits < 1 || nbits > 32 || parts < 1 || (final_vals && !final_off)) return hipErrorInvalidValue;
    uint32_t* totals = hist + (size_t)kMaxRadix * parts;
    // Large sorts take radix tiles of 4096 keys (longer digit runs per tile, so fuller write
    // segments); smaller ones 2048, which fill the device with more partitions.  The partition
    // count never exceeds the caller's, so the histogram table fits.
    if (n_host >= kLargeSortKeys) {
        constexpr int64_t tile = (int64_t)kBlock * 16;
        const int p = (int)std::min<int64_t>(parts, std::max<int64_t>(1, ((int64_t)n_host + tile - 1) / tile));
        return sort_passes<16>(keys_a, vals_a, keys_b, vals_b, n_dev, n_host, bit0, nbits, p, hist, totals,
                               result_in_b, tag, timer, s, use_drop, drop_key, n_kept, final_vals, final_off);
    }
    return sort_passes<kSortItems>(keys_a, vals_a, keys_b, vals_b, n_dev, n_host, bit0, nbits, parts, hist, totals,
                                   result_in_b, tag, timer, s, use_drop, drop_key, n_kept, final_vals, final_off);
}

}  // namespace gs
