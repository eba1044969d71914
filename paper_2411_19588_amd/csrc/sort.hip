// Stable least-significant-digit radix sort of (u32 key, u32 value) pairs, used
// for the depth order of eq. (3dgs_orig) and for binning pairs by tile
// (Preliminaries, "Tiles").
//
// Each pass is reduce-then-scan over a FIXED number of partitions `parts`; the
// element count is read from device memory, so the launch shapes never depend
// on data and a whole forward can be captured into a graph.
//   1. k_hist:    each partition counts its digits (per-wave LDS histograms).
//   2. k_scan:    exclusive scan of the digit-major [radix][parts] table.
//   3. k_scatter: each partition re-reads its range in order, ranks keys stably
//                 inside each wave64 with ballots (lanes with equal digits are
//                 found by intersecting one ballot per digit bit), combines the
//                 four waves through LDS and scatters.
#include <string>

#include "internal.h"

namespace gs {
namespace {

__device__ __forceinline__ uint32_t load_n(const uint32_t* n_dev, uint32_t n_host) {
    return n_dev ? *n_dev : n_host;
}

// Partition p covers radix tiles [t0, t1) of kSortTile elements each.
__device__ __forceinline__ void part_range(uint32_t n, int parts, int p, uint32_t& t0, uint32_t& t1) {
    const uint32_t tiles = (n + kSortTile - 1) / kSortTile;
    const uint32_t per = (tiles + parts - 1) / parts;
    t0 = min(tiles, per * (uint32_t)p);
    t1 = min(tiles, t0 + per);
}

__global__ __launch_bounds__(kBlock) void k_hist(const uint32_t* __restrict__ keys, const uint32_t* n_dev,
                                                uint32_t n_host, int shift, uint32_t mask, int parts,
                                                uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[4][kRadix];
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < 4 * kRadix; i += kBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = load_n(n_dev, n_host);
    uint32_t t0, t1;
    part_range(n, parts, blockIdx.x, t0, t1);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t base = t * kSortTile;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const uint32_t idx = base + k * kBlock + tid;
            if (idx < n) atomicAdd(&h[wave][(keys[idx] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < kRadix; d += kBlock)
        hist[(size_t)d * parts + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Exclusive scan of `count` u32 values in place by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_table(uint32_t* __restrict__ a, int count) {
    __shared__ uint32_t sums[1024];
    const int tid = threadIdx.x;
    const int per = (count + 1023) / 1024;
    const int b = tid * per, e = min(count, b + per);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += a[i];
    sums[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = tid >= off ? sums[tid - off] : 0u;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    uint32_t run = sums[tid] - s;
    for (int i = b; i < e; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                   const uint32_t* n_dev, uint32_t n_host, int shift, int nbits,
                                                   int parts, const uint32_t* __restrict__ hist) {
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wcnt[4][kRadix];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t mask = (1u << nbits) - 1u;
    const uint32_t n = load_n(n_dev, n_host);
    for (int d = tid; d < kRadix; d += kBlock) run[d] = hist[(size_t)d * parts + blockIdx.x];
    uint32_t t0, t1;
    part_range(n, parts, blockIdx.x, t0, t1);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint32_t t = t0; t < t1; ++t) {
        for (int i = tid; i < 4 * kRadix; i += kBlock) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        // wave w ranks elements [base + w*64*ITEMS, base + (w+1)*64*ITEMS) in order: item k, lane l.
        const uint32_t base = t * kSortTile + (uint32_t)wave * 64u * kSortItems;
        uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const uint32_t idx = base + k * 64 + lane;
            const bool valid = idx < n;
            key[k] = valid ? kin[idx] : 0u;
            val[k] = valid ? vin[idx] : 0u;
            const uint32_t digit = (key[k] >> shift) & mask;
            uint64_t match = __ballot(valid);
            for (int b = 0; b < nbits; ++b) {
                const bool bit = (digit >> b) & 1u;
                const uint64_t bal = __ballot(bit);
                match &= bit ? bal : ~bal;
            }
            const uint32_t before = wcnt[wave][digit];
            const uint32_t cnt = __popcll(match);
            const int leader = __ffsll((unsigned long long)match) - 1;
            rank[k] = before + __popcll(match & lt_mask);
            if (valid && lane == leader) wcnt[wave][digit] = before + cnt;
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // per digit: offsets of the four waves, then advance the running base
        for (int d = tid; d < kRadix; d += kBlock) {
            uint32_t s = run[d];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint32_t c = wcnt[w][d];
                wcnt[w][d] = s;
                s += c;
            }
            run[d] = s;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const uint32_t idx = base + k * 64 + lane;
            if (idx < n) {
                const uint32_t digit = (key[k] >> shift) & mask;
                const uint32_t pos = wcnt[wave][digit] + rank[k];
                if (pos < n) {   // always true when the histogram and ranking agree
                    kout[pos] = key[k];
                    vout[pos] = val[k];
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t radix_sort_u32(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b,
                          const uint32_t* n_dev, uint32_t n_host, int bit0, int nbits, int parts,
                          uint32_t* hist, int* result_in_b, const char* tag, void* timer, hipStream_t s) {
    const std::string th = std::string(tag) + "_hist", ts = std::string(tag) + "_scan",
                      tc = std::string(tag) + "_scatter";
    int in_b = 0;
    for (int done = 0; done < nbits; done += kRadixBits) {
        const int bits = nbits - done < kRadixBits ? nbits - done : kRadixBits;
        const int shift = bit0 + done;
        const uint32_t* kin = in_b ? keys_b : keys_a;
        const uint32_t* vin = in_b ? vals_b : vals_a;
        uint32_t* kout = in_b ? keys_a : keys_b;
        uint32_t* vout = in_b ? vals_a : vals_b;
        timer_begin(timer, th.c_str(), s);
        hipLaunchKernelGGL(k_hist, dim3(parts), dim3(kBlock), 0, s, kin, n_dev, n_host, shift,
                           (1u << bits) - 1u, parts, hist);
        timer_end(timer, s);
        timer_begin(timer, ts.c_str(), s);
        hipLaunchKernelGGL(k_scan_table, dim3(1), dim3(1024), 0, s, hist, kRadix * parts);
        timer_end(timer, s);
        timer_begin(timer, tc.c_str(), s);
        hipLaunchKernelGGL(k_scatter, dim3(parts), dim3(kBlock), 0, s, kin, vin, kout, vout, n_dev, n_host, shift,
                           bits, parts, hist);
        timer_end(timer, s);
        in_b = !in_b;
    }
    *result_in_b = in_b;
    return hipGetLastError();
}

}  // namespace gs
