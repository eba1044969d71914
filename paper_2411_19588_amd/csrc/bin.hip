// Binning of projected Gaussians into tiles (Preliminaries, "Tiles": each
// tile lists the Gaussians whose extent reaches it, in depth order).
//
// Pairs are emitted in depth order: entries (view, Gaussian) are first sorted
// by FP32 depth (stable, so equal depths keep index order), the per-entry tile
// counts are scanned in that order, and each entry writes its tiles.  A stable
// sort of the pairs by tile id then yields, per tile, the Gaussians in
// (depth, index) order -- the order of the key (tile << 32 | depth bits).
#include "internal.h"

namespace gs {
namespace {

constexpr int kScanChunk = kBlock * 16;

__global__ void k_view_table(ViewTable t, ViewInfo* dst, SavedHeader* hdr) {
    const int i = threadIdx.x;
    if (i < t.count) dst[i] = t.v[i];
    if (i == 0) {
        hdr->status = 0;
        hdr->pair_count = 0;
        hdr->pairs_needed = 0;
        hdr->queue = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_count_reduce(const uint32_t* __restrict__ counts,
                                                        const uint32_t* __restrict__ order, int64_t nv,
                                                        uint64_t* __restrict__ blocksums) {
    __shared__ uint64_t red[kBlock];
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
    uint64_t s = 0;
    for (int k = 0; k < 16; ++k) {
        const int64_t r = b0 + k * kBlock + threadIdx.x;
        if (r < nv) s += counts[order[r]];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) blocksums[blockIdx.x] = red[0];
}

// Exclusive scan of the block sums (one workgroup) and the overflow decision.
__global__ __launch_bounds__(1024) void k_count_blocks(uint64_t* blocksums, int nb, SavedHeader* hdr,
                                                      int64_t max_pairs) {
    __shared__ uint64_t sums[1024];
    const int tid = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b = tid * per, e = min(nb, b + per);
    uint64_t s = 0;
    for (int i = b; i < e; ++i) s += blocksums[i];
    sums[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = tid >= off ? sums[tid - off] : 0ull;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    uint64_t run = sums[tid] - s;
    for (int i = b; i < e; ++i) {
        const uint64_t v = blocksums[i];
        blocksums[i] = run;
        run += v;
    }
    if (tid == 1023) {
        const uint64_t total = sums[1023];
        hdr->pairs_needed = total;
        if (total > (uint64_t)max_pairs) {
            hdr->status |= GS_STATUS_PAIR_OVERFLOW;
            hdr->pair_count = 0;
        } else {
            hdr->pair_count = (uint32_t)total;
        }
    }
}

constexpr int kEmitItems = 4;
constexpr int kEmitSpan = kBlock * kEmitItems;

__global__ __launch_bounds__(kBlock) void k_count_down(const uint32_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ order, int64_t nv,
                                                      const uint64_t* __restrict__ blocksums,
                                                      uint64_t* __restrict__ offsets, uint32_t* __restrict__ emit_start,
                                                      int64_t n_spans) {
    __shared__ uint64_t part[kBlock];
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)tid * 16;   // 16 consecutive per thread
    uint32_t c[16];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t r = b0 + k;
        c[k] = r < nv ? counts[order[r]] : 0u;
        s += c[k];
    }
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const uint64_t v = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = blocksums[blockIdx.x] + part[tid] - s;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t r = b0 + k;
        if (r < nv) {
            offsets[r] = run;
            // emission spans whose first pair falls inside this entry's pairs [run, run + c)
            if (c[k]) {
                for (int64_t b = (int64_t)((run + kEmitSpan - 1) / kEmitSpan);
                     b * kEmitSpan < (int64_t)(run + c[k]) && b < n_spans; ++b)
                    emit_start[b] = (uint32_t)r;
            }
        }
        run += c[k];
    }
}

// Pair emission.  Workgroup b writes output pairs [b*kEmitSpan, (b+1)*kEmitSpan): it
// stages the entries (in depth order) whose tile lists overlap that span in LDS -- the
// first one is emit_start[b], recorded by the scan -- and each thread produces
// consecutive output slots, so writes are coalesced and every workgroup does the same
// amount of work whatever the rectangle sizes.  Visible entries (count >= 1) precede the
// others in the depth order, so offsets increase strictly over them.
__global__ __launch_bounds__(kBlock) void k_emit(const uint32_t* __restrict__ order,
                                                const uint64_t* __restrict__ offsets,
                                                const uint32_t* __restrict__ emit_start,
                                                const uint2* __restrict__ rects, int64_t nv, int64_t n,
                                                const ViewInfo* __restrict__ vt,
                                                const SavedHeader* __restrict__ hdr, uint32_t* __restrict__ tiles_out,
                                                uint32_t* __restrict__ vals_out) {
    __shared__ int32_t s_off[kEmitSpan + 1];
    __shared__ uint32_t s_e[kEmitSpan + 1], s_base[kEmitSpan + 1], s_w[kEmitSpan + 1], s_tx[kEmitSpan + 1];
    __shared__ float s_iw[kEmitSpan + 1];
    const uint64_t K = hdr->pair_count;
    const uint64_t p0 = (uint64_t)blockIdx.x * kEmitSpan;
    if (K == 0 || p0 >= K) return;
    const uint64_t p1 = min(p0 + (uint64_t)kEmitSpan, K);
    const int tid = threadIdx.x;
    const int64_t r0 = emit_start[blockIdx.x];
    // candidates r0 .. r0 + kEmitSpan: the owners of this span form a prefix of them
    int nent = 0;
    for (int i0 = 0; i0 < kEmitSpan + 1; i0 += kBlock) {
        const int i = i0 + tid;
        const int64_t r = r0 + i;
        const bool own = i < kEmitSpan + 1 && r < nv && (i == 0 || offsets[r] < p1);
        if (own) {
            const uint32_t e = order[r];
            const uint2 rc = rects[e];
            const ViewInfo vi = vt[e / (uint64_t)n];
            const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu;
            const uint32_t w = x1 - x0 + 1;
            s_off[i] = (int32_t)((int64_t)offsets[r] - (int64_t)p0);
            s_e[i] = e;
            s_base[i] = vi.tile_base + y0 * (uint32_t)vi.tiles_x + x0;
            s_w[i] = w;
            s_tx[i] = (uint32_t)vi.tiles_x;
            s_iw[i] = 1.0f / (float)w;
        }
        nent += __syncthreads_count(own);
    }
    const int span = (int)(p1 - p0);
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) {
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
        tiles_out[p0 + q] = s_base[lo] + row * s_tx[lo] + col;
        vals_out[p0 + q] = s_e[lo];
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t* __restrict__ tiles,
                                                  const SavedHeader* __restrict__ hdr, uint32_t n_tiles,
                                                  uint2* __restrict__ ranges) {
    const uint32_t K = hdr->pair_count;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= K) return;
    const uint32_t t = tiles[i];
    if (t >= n_tiles) return;   // tile ids are < n_tiles by construction
    if (i == 0 || tiles[i - 1] != t) ranges[t].x = i;
    if (i + 1 == K || tiles[i + 1] != t) ranges[t].y = i + 1;
}

__global__ __launch_bounds__(kBlock) void k_export(const uint32_t* __restrict__ tiles,
                                                  const uint32_t* __restrict__ vals,
                                                  const uint32_t* __restrict__ depth_keys,
                                                  const SavedHeader* __restrict__ hdr, int64_t capacity,
                                                  uint64_t* __restrict__ keys, uint32_t* __restrict__ values) {
    const int64_t K = min((int64_t)hdr->pair_count, capacity);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < K; i += (int64_t)gridDim.x * kBlock) {
        const uint32_t e = vals[i];
        keys[i] = ((uint64_t)tiles[i] << 32) | (uint64_t)depth_keys[e];
        values[i] = e;
    }
}

}  // namespace

hipError_t launch_view_table(const ViewTable& t, ViewInfo* dst, SavedHeader* hdr, hipStream_t s) {
    hipLaunchKernelGGL(k_view_table, dim3(1), dim3(GS_MAX_VIEWS), 0, s, t, dst, hdr);
    return hipGetLastError();
}

hipError_t launch_count_scan(const uint32_t* counts, const uint32_t* order, int64_t nv, uint64_t* offsets,
                             uint64_t* blocksums, SavedHeader* hdr, int64_t max_pairs, uint32_t* emit_start,
                             hipStream_t s) {
    const int64_t n_spans = max_pairs / kEmitSpan + 2;
    const int nb = (int)((nv + kScanChunk - 1) / kScanChunk);
    if (nb > 0) hipLaunchKernelGGL(k_count_reduce, dim3(nb), dim3(kBlock), 0, s, counts, order, nv, blocksums);
    hipLaunchKernelGGL(k_count_blocks, dim3(1), dim3(1024), 0, s, blocksums, nb, hdr, max_pairs);
    if (nb > 0)
        hipLaunchKernelGGL(k_count_down, dim3(nb), dim3(kBlock), 0, s, counts, order, nv, blocksums, offsets,
                           emit_start, n_spans);
    return hipGetLastError();
}

hipError_t launch_emit(const uint32_t* order, const uint64_t* offsets, const uint32_t* emit_start, const uint2* rects,
                       int64_t nv, int64_t n, const ViewInfo* vt, int32_t views, const SavedHeader* hdr,
                       int64_t max_pairs, uint32_t* tiles_out, uint32_t* vals_out, hipStream_t s) {
    (void)views;
    if (nv == 0 || max_pairs == 0) return hipSuccess;
    const unsigned grid = (unsigned)((max_pairs + kEmitSpan - 1) / kEmitSpan);
    hipLaunchKernelGGL(k_emit, dim3(grid), dim3(kBlock), 0, s, order, offsets, emit_start, rects, nv, n, vt, hdr,
                       tiles_out, vals_out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlock), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* sorted_tiles, const SavedHeader* hdr, int64_t tiles, int64_t max_pairs,
                         uint2* ranges, hipStream_t s) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, tiles * 2, s);
    if (e != hipSuccess || max_pairs == 0) return e;
    const unsigned grid = (unsigned)((max_pairs + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ranges, dim3(grid), dim3(kBlock), 0, s, sorted_tiles, hdr, (uint32_t)tiles, ranges);
    return hipGetLastError();
}

hipError_t launch_export_keys(const uint32_t* tiles, const uint32_t* vals, const uint32_t* depth_keys,
                              const SavedHeader* hdr, int64_t capacity, uint64_t* keys, uint32_t* values,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_export, dim3(2048), dim3(kBlock), 0, s, tiles, vals, depth_keys, hdr, capacity, keys,
                       values);
    return hipGetLastError();
}

}  // namespace gs
