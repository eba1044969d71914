// Internal declarations shared by the HIP translation units of libgsplash.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsplash.h"

namespace gs {

constexpr int kBlock = 256;              // threads per workgroup for 1D kernels (4 wave64)
constexpr int kSortItems = 8;            // keys per thread per radix tile
constexpr int kSortTile = kBlock * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxSortParts = 1024;
constexpr int kGrad2D = 10;              // per-(Gaussian, view) 2D gradient: m(2), conic'(3), o, rgb(3), depth

// Per-view layout derived from the host cameras.
struct ViewInfo {
    int32_t width, height, tiles_x, tiles_y;
    uint32_t tile_base;                  // first global tile id of the view
    uint32_t n_tiles;
    int64_t pix_base;                    // first pixel of the view in the packed outputs
};

struct ViewTable {
    ViewInfo v[GS_MAX_VIEWS];
    int32_t count;
};

// Projected splat, one per (view, Gaussian): 48 bytes, read as three float4.
//   a = (m_x, m_y, A, B)   b = (C, opacity, r, g)   c = (b, depth, -, -)
// with the conic pre-scaled so that alpha = o * exp2(A dx^2 + B dx dy + C dy^2),
// A = -log2(e)/2 Qxx, B = -log2(e) Qxy, C = -log2(e)/2 Qyy.
struct __align__(16) Record {
    float4 a, b, c;
};

// Header at the start of the saved context.
struct SavedHeader {
    uint32_t status;                     // GS_STATUS_* bits
    uint32_t pair_count;                 // pairs produced (0 if overflowed)
    uint64_t pairs_needed;               // pairs the forward wanted
    uint32_t final_buffer;               // which ping-pong buffer holds the sorted pairs (0 = A, 1 = B)
    uint32_t queue;                      // persistent-mode tile counter
    uint32_t pad[10];
};

struct Layout {
    int64_t n, nv, pixels, tiles, max_pairs;
    int32_t views;
    int32_t tile_bits, tile_passes, pair_parts, depth_parts;
    ViewTable table;
    // saved context offsets (bytes)
    size_t s_header, s_records, s_depth_keys, s_ranges, s_tiles_a, s_vals_a, s_tiles_b, s_vals_b;
    size_t s_tfinal, s_nlast, s_cair, s_dsum, s_wsum, saved_bytes;
    // workspace offsets (bytes)
    size_t w_counts, w_rects, w_dkeys, w_dvals, w_dkeys2, w_dvals2, w_offsets, w_blocksums, w_emit_start, w_hist;
    size_t w_grad2d, w_medpart, workspace_bytes;
};

int compute_layout(const gs_options* o, int64_t n, int32_t n_views, const gs_camera* cams, Layout* L);

// ---------------------------------------------------------------------------
// Kernel launchers (each enqueues on `s` and returns hipGetLastError()).
hipError_t launch_view_table(const ViewTable& t, ViewInfo* dst, SavedHeader* hdr, hipStream_t s);
hipError_t launch_project_fwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const ViewInfo* vt,
                              const gs_options& o, Record* rec, uint32_t* counts, uint2* rects,
                              uint32_t* depth_keys, uint32_t* dkeys_sort, uint32_t* dvals_sort,
                              SavedHeader* hdr, hipStream_t s);
hipError_t launch_project_bwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const gs_options& o,
                              const float* grad2d, gs_gaussian_grads grads, hipStream_t s);
// Stable LSD radix sort of (key, value) u32 pairs over bits [bit0, bit0+nbits).  n is read from n_dev
// (or n_host if n_dev is null).  Returns in *out_in_b whether the result sits in the B buffers.
hipError_t radix_sort_u32(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b,
                          const uint32_t* n_dev, uint32_t n_host, int bit0, int nbits, int parts,
                          uint32_t* hist, int* result_in_b, const char* tag, void* timer, hipStream_t s);
// Exclusive scan of counts[order[r]] into offsets (u64), total and overflow into hdr, and for each
// emission span of 1024 pairs the entry that owns its first pair (emit_start).
hipError_t launch_count_scan(const uint32_t* counts, const uint32_t* order, int64_t nv, uint64_t* offsets,
                             uint64_t* blocksums, SavedHeader* hdr, int64_t max_pairs, uint32_t* emit_start,
                             hipStream_t s);
hipError_t launch_emit(const uint32_t* order, const uint64_t* offsets, const uint32_t* emit_start, const uint2* rects,
                       int64_t nv, int64_t n, const ViewInfo* vt, int32_t views, const SavedHeader* hdr,
                       int64_t max_pairs, uint32_t* tiles_out, uint32_t* vals_out, hipStream_t s);
hipError_t launch_ranges(const uint32_t* sorted_tiles, const SavedHeader* hdr, int64_t tiles, int64_t max_pairs,
                         uint2* ranges, hipStream_t s);
hipError_t launch_composite_fwd(const gs_options& o, const Layout& L, const ViewInfo* vt, const gs_medium* med,
                                const Record* rec, const uint2* ranges, const uint32_t* vals, SavedHeader* hdr,
                                float* out_rgb, float* out_depth, float* out_alpha, float* tfinal, uint32_t* nlast,
                                float* cair, float* dsum, float* wsum, hipStream_t s);
hipError_t launch_composite_bwd(const gs_options& o, const Layout& L, const ViewInfo* vt, const gs_medium* med,
                                const Record* rec, const uint2* ranges, const uint32_t* vals, SavedHeader* hdr,
                                const float* grad_rgb, const float* grad_depth, const float* tfinal,
                                const uint32_t* nlast, const float* cair, const float* dsum, const float* wsum,
                                float* grad2d, float* medpart, hipStream_t s);
hipError_t launch_medium_reduce(const ViewInfo* vt, int32_t views, const float* medpart, float* grad_medium,
                                hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_export_keys(const uint32_t* tiles, const uint32_t* vals, const uint32_t* depth_keys,
                              const SavedHeader* hdr, int64_t capacity, uint64_t* keys, uint32_t* values,
                              hipStream_t s);

// Timer hooks (no-ops when timer == nullptr).
void timer_begin(void* timer, const char* name, hipStream_t s);
void timer_end(void* timer, hipStream_t s);

}  // namespace gs
