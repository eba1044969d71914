// Internal declarations shared by the HIP translation units of libgsplash.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsplash.h"

namespace gs {

constexpr int kBlock = 256;              // threads per workgroup for 1D kernels (4 wave64)
constexpr int kSortItems = 8;            // keys per thread per radix tile below kLargeSortKeys keys
constexpr int64_t kLargeSortKeys = 1 << 23;   // from here on, radix tiles of 16 keys per thread
constexpr int kSortTile = kBlock * kSortItems;
constexpr int kRadixBits = 8;             // digit width of most radix passes
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxRadixBits = 9;          // widest digit (a pass of a 17- or 18-bit key)
constexpr int kMaxRadix = 1 << kMaxRadixBits;
constexpr int kMaxSortParts = 1024;      // 2048 and 4096 measured no faster on 24M keys
// Pairs per emission workgroup: phase 0 (whole rectangles) 512, later phases 1024 (each measured
// fastest).
constexpr int kEmitSpan0 = kBlock * 2;
constexpr int kEmitSpanLater = kBlock * 4;
constexpr int kGrad2D = 10;              // per-(Gaussian, view) 2D gradient: m(2), conic'(3), o, rgb(3), depth
// Automatic depth-phase schedule (options phases / phase0_shift = 0), chosen by measurement: one
// view, 2 phases from the nearest 1/128 of the visible Gaussians; several views, 4 phases from
// the nearest 1/64.
constexpr int kAutoPhasesOneView = 2, kAutoShiftMin = 2, kAutoShiftMax = 12;
constexpr int kAutoPhasesViews = 4, kAutoShiftViews = 6;
constexpr int kAutoGrowth = 2;           // later phases 4x wider than the one before
// Compositing launch shape when gs_options leaves it unset (16x16 tiles).
constexpr int kDefaultPixelsPerLaneFwd = 2;   // two waves per tile
constexpr int kDefaultRecordFetchFwd = GS_FETCH_LDS;
constexpr int kDefaultPixelsPerLaneBwd = 4;   // one wave per tile
constexpr int kDefaultRecordFetchBwd = GS_FETCH_SCALAR;

// Per-view layout derived from the host cameras.
struct ViewInfo {
    int32_t width, height, tiles_x, tiles_y;
    uint32_t tile_base;                  // first global tile id of the view
    uint32_t n_tiles;
    int64_t pix_base;                    // first pixel of the view in the packed outputs
    uint32_t row_base;                   // first global tile row of the view
    uint32_t pad;
};

struct ViewTable {
    ViewInfo v[GS_MAX_VIEWS];
    int32_t count;
};

// Projected splat, one per (view, Gaussian): 48 bytes, read as three float4.
//   a = (m_x, m_y, A, B)   b = (C, log2 o, r, g)   c = (b, depth, 1/o, -)
// with the conic pre-scaled so that alpha = exp2(A dx^2 + B dx dy + C dy^2 + log2 o),
// A = -log2(e)/2 Qxx, B = -log2(e) Qxy, C = -log2(e)/2 Qyy.  An opacity o <= 0 stores
// log2 o = -inf and 1/o = 0: the splat never blends.
struct __align__(16) Record {
    float4 a, b, c;
};

// Header at the start of the saved context (device-side bookkeeping of a forward).
struct SavedHeader {
    uint32_t status;                     // GS_STATUS_* bits
    uint32_t pair_count;                 // pairs stored over all phases
    uint64_t pairs_needed;               // pairs the forward wanted (a lower bound after an overflow)
    uint32_t visible;                    // entries with at least one tile, first in the depth order
    uint32_t stop;                       // set on overflow: later phases do nothing
    uint32_t phase_rank[GS_MAX_PHASES + 1];   // phase p covers depth ranks [phase_rank[p], phase_rank[p+1])
    uint32_t phase_base[GS_MAX_PHASES];       // first stored pair of phase p
    uint32_t phase_count[GS_MAX_PHASES];      // pairs of phase p
    uint32_t phase_alive[GS_MAX_PHASES];      // tiles with an unterminated pixel after phase p
    uint32_t phase_live[GS_MAX_PHASES];       // pairs of phase p kept by the tile sort (culled ones left out)
    uint32_t queue[GS_MAX_PHASES + 1];        // persistent-mode tile counters (forward phases)
    uint32_t view_alive[GS_MAX_PHASES][GS_MAX_VIEWS];   // tiles of each view left alive after phase p
    unsigned long long stats[5];              // scratch of gs_forward_stats
    uint32_t pad[4];
};

struct Layout {
    int64_t n, nv, pixels, tiles, rows, row_words, max_pairs;
    int32_t views, phases, phase0_shift, phase_growth;
    int32_t tile_w, tile_h, tile_bits, tile_passes, pair_parts, depth_parts, queue_parts;
    ViewTable table;
    // saved context offsets (bytes)
    size_t s_header, s_records, s_depth_keys, s_ranges, s_vals, s_alive;
    size_t s_tfinal, s_nlast, s_done, s_cair, s_dsum, s_wsum, saved_bytes;
    // workspace offsets (bytes)
    size_t w_counts, w_rects, w_dkeys, w_dvals, w_dkeys2, w_dvals2, w_pcounts, w_offsets, w_blocksums, w_emit_start;
    size_t w_tiles_a, w_vals_a, w_tiles_b, w_vals_b, w_hist, w_grad2d, w_medpart, w_medsum, w_adam, w_rowbits, w_nzr,
        w_shf, w_queue;
    size_t workspace_bytes;
};

int compute_layout(const gs_options* o, int64_t n, int32_t n_views, const gs_camera* cams, Layout* L);

// The adjoint and optimizer kernels of a step do nothing when (*word & mask) != 0: the forward
// they belong to overflowed the pair capacity (its render is truncated), or an earlier step of
// a training run did (the sticky flag of the caller's training state).  word may be null.
struct Guard {
    const uint32_t* word;
    uint32_t mask;
};

__device__ __forceinline__ bool guard_set(const Guard& g) { return g.word != nullptr && (*g.word & g.mask) != 0u; }

// ---------------------------------------------------------------------------
// Kernel launchers (each enqueues on `s` and returns hipGetLastError()).
// The view table and a cleared header; fill[0, fill_count) is zeroed by the same launch.
hipError_t launch_view_table(const ViewTable& t, ViewInfo* dst, SavedHeader* hdr, uint32_t* fill, int64_t fill_count,
                             hipStream_t s);
hipError_t launch_project_fwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const ViewInfo* vt,
                              const gs_options& o, Record* rec, uint32_t* counts, uint2* rects,
                              uint32_t* depth_keys, uint32_t* dkeys_sort, uint32_t* dvals_sort,
                              SavedHeader* hdr, hipStream_t s);
// The projection adjoint; with several views `planes` (3 + 3 views floats per Gaussian) receives
// what launch_sh_views needs, and the means' and SH gradients are written by launch_sh_views.
hipError_t launch_project_bwd(const gs_gaussians& g, int32_t views, const gs_camera* cams, const gs_options& o,
                              const float* grad2d, const Record* rec, gs_gaussian_grads grads, float* planes,
                              hipStream_t s);

// One Adam step (Sec. Optimization) of one scalar: moments updated in place, returns the new
// parameter.  ibc1, ibc2 = 1 / (1 - beta^t).  The step divides by sqrt(v_hat) + eps through the
// hardware reciprocal (1 ulp); the square root is correctly rounded.
__device__ __forceinline__ float adam_update(float p, float g, float& m, float& v, float lr, float b1, float b2,
                                             float eps, float ibc1, float ibc2) {
    m = fmaf(b1, m, (1.0f - b1) * g);
    v = fmaf(b2, v, (1.0f - b2) * g * g);
    return p - (lr * (m * ibc1)) * __builtin_amdgcn_rcpf(sqrtf(v * ibc2) + eps);
}

// Adam applied inside the projection adjoint: groups means, log-scales (exp), quaternions,
// opacity logits (sigmoid), SH, in this order; bc = device [2] bias corrections of this step.
// With shf set, the adjoint steps the log-scales, quaternions and opacity logits and stores:
// one view, for launch_adam_sh, shf = [kShf][n] planes: view direction x, y, z; colour gradient
// of the unclamped channels r, g, b; inverse distance to the camera centre; the means' gradient
// without its term through the SH colour.  Several views, for launch_sh_views, shf = [3 + 3
// views][n] planes: the means' gradient without its SH term, then per view the colour gradient
// of the unclamped channels (zero where the Gaussian has no gradient in that view).
struct AdamFused {
    gs_adam_group g[5];
    float b1, b2, eps;
    const float* bc;
    float* shf;
    Guard guard;   // fused steps: skip the step when set
    float reg_o, reg_s;   // regulariser gradients added to every opacity and scale entry (set by the launchers)
};

hipError_t launch_project_bwd_adam(const gs_gaussians& g, int32_t views, const gs_camera* cams, const gs_options& o,
                                   const float* grad2d, const Record* rec, const AdamFused& adam, hipStream_t s);
constexpr int kShf = 10;
// Adam steps of the means and the SH group from what launch_project_bwd_adam stored in adam.shf:
// the gradient of SH coefficient k, channel c is Y_k(dir) gc_c, as the adjoint forms it, and the
// means' gradient gets its SH term here, from the coefficients before their update.
hipError_t launch_adam_sh(int64_t n, int sh_degree, const AdamFused& adam, hipStream_t s);
// Several views: the SH part of the adjoint from adam.shf (see AdamFused).  fused: Adam steps of
// the SH coefficients and the means; otherwise their gradients into grads.sh and grads.means.
// Gaussians per lane when n and the bases allow 4 W-byte accesses (2 measured faster than 1 or 4)
constexpr int kShViewsW = 2;
hipError_t launch_sh_views(const gs_gaussians& g, int32_t views, const gs_camera* cams,
                           const gs_gaussian_grads& grads, const AdamFused& adam, int fused, hipStream_t s);
// Zeroes p[0, count) and starts a fused step on its training state (int32[2]: step, sticky skip
// flag): when *status reports a pair overflow or state[1] is already set, state[1] |= the overflow
// bit and the step is skipped; otherwise state[0] += 1 and bc = (1 / (1 - b1^step),
// 1 / (1 - b2^step)) on the device.
hipError_t launch_zero_adam_prep(uint32_t* p, int64_t count, int32_t* state, const uint32_t* status, float b1,
                                 float b2, float* bc, hipStream_t s);
// Stable LSD radix sort of (key, value) u32 pairs over bits [bit0, bit0+nbits).  n is read from n_dev
// (or n_host if n_dev is null); with n_dev, n_host is the largest n it can hold, which picks the
// radix tile size.  Returns in *out_in_b whether the result sits in the B buffers.
// With use_drop, keys equal to drop_key are left out; with n_kept the number of kept pairs is
// written there (device), and the sorted output holds exactly those.  With final_vals, the last
// pass writes the sorted values to final_vals + *final_off (final_off on the device) instead of
// the A/B value buffers; the sorted keys are where *out_in_b says.
hipError_t radix_sort_u32(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b,
                          const uint32_t* n_dev, uint32_t n_host, int bit0, int nbits, int parts, uint32_t* hist,
                          int* out_in_b, const char* tag, void* timer, hipStream_t s, int use_drop = 0,
                          uint32_t drop_key = 0, uint32_t* n_kept = nullptr, uint32_t* final_vals = nullptr,
                          const uint32_t* final_off = nullptr);
// Depth-phase schedule.  With V visible entries (the depth sort's count of kept keys), phase
// p < phases - 1 ends at depth rank ceil(V / 2^(shift - growth p)) (at V once the exponent
// reaches 0) and the last phase at V; every kernel that needs a phase's ranks derives them from V.
struct PhaseSched {
    int32_t phases, shift, growth;
};
// Exact tile culling: a (Gaussian, tile) pair of the rectangle is dropped when no pixel centre
// of the tile can reach alpha >= alpha_min (see tile_may_contribute).
struct CullArgs {
    const Record* rec;
    float log2_amin;
    int32_t tile_w, tile_h;
    int32_t enabled;
};

// Per global tile row, after a phase: bit masks of the alive columns (`words` 64-bit words per
// row), set by that phase's compositing; and the compact list of a later phase's entries with
// pairs (depth ranks, in depth order).
struct AliveRows {
    uint64_t* bits;
    uint32_t words;
    uint32_t* nzr;   // [nv]
};
// Per-entry pair counts of phase p (by depth rank) into pcounts -- whole rectangles in phase 0,
// only the tiles alive in ar.bits in later phases, 0 outside the phase's ranks -- and their
// exclusive scan into offsets (u64), the phase's pair count and base in hdr (with the capacity
// check); for each emission span of 1024 pairs the entry that owns its first pair (its depth rank
// in phase 0, its position in the compact list `nzr` of entries with pairs later).  blocksums
// holds 2 count_scan_blocks(nv) + 1 values; the last is the length of that list.  zero_bits
// (nullable, zero_words words) is cleared for the alive masks this phase's compositing sets.
int64_t count_scan_blocks(int64_t nv);
hipError_t launch_count_scan(const uint32_t* order, const uint32_t* counts, const uint2* rects, int64_t nv,
                             int64_t n, const ViewInfo* vt, const AliveRows& ar, uint64_t* zero_bits,
                             int64_t zero_words, const PhaseSched& ps, SavedHeader* hdr, int phase,
                             uint32_t* pcounts, uint64_t* offsets, uint64_t* blocksums, int64_t max_pairs,
                             uint32_t* emit_start, hipStream_t s);
// Phase 0 writes every pair of each rectangle, later phases the pairs of the alive tiles; a culled
// pair gets the tile id n_tiles, which the tile sort's first pass leaves out.
hipError_t launch_emit(const uint32_t* order, const uint64_t* offsets, const uint32_t* emit_start,
                       const uint64_t* blocksums, const uint2* rects, int64_t nv, int64_t n, const ViewInfo* vt,
                       const AliveRows& ar, const SavedHeader* hdr, int phase, int64_t max_pairs,
                       const CullArgs& cull, uint32_t n_tiles, uint32_t* tiles_out, uint32_t* vals_out,
                       hipStream_t s);
// The phase's tile ranges from its tile-sorted keys (the tile sort wrote the values behind the
// earlier phases').
hipError_t launch_commit(const uint32_t* sorted_tiles, const SavedHeader* hdr, int phase, int64_t tiles,
                         int64_t max_pairs, uint2* ranges, hipStream_t s);
// out_restored (nullable): the in-air composite C_air per pixel, CHW per view like out_rgb.
// rowbits (nullable, zeroed beforehand): the bit of every tile left alive is set there.
// last_phase: the last phase this forward runs (tiles write their outputs there); when it
// is before the schedule's last phase, a tile left alive with Gaussians still unbinned sets
// GS_STATUS_INCOMPLETE.
hipError_t launch_composite_fwd(const gs_options& o, const Layout& L, int phase, int last_phase, const ViewInfo* vt,
                                const gs_medium* med, const Record* rec, const uint2* ranges, const uint32_t* vals,
                                SavedHeader* hdr, uint32_t* alive, float* out_rgb, float* out_depth,
                                float* out_alpha, float* out_restored, float* tfinal, uint32_t* nlast, uint8_t* done,
                                float* cair, float* dsum, float* wsum, const uint32_t* order, uint64_t* rowbits,
                                hipStream_t s);
// Longest-first order of a persistent pass (opts.persistent = 2) over the phases [p0, p1) of
// `ranges` ([phases][tiles]): per-tile keys 32 - bit_length(list length), a stable 6-bit radix
// sort, and in *order the tile ids, longest lists first (inside qbuf, 4 * tiles u32).
hipError_t build_queue(const Layout& L, const uint2* ranges, int p0, int p1, uint32_t* qbuf, uint32_t* hist,
                       const uint32_t** order, void* timer, hipStream_t s);
// grad_restored (nullable): upstream gradient of C_air, added to the colour accumulators' gradient.
hipError_t launch_composite_bwd(const gs_options& o, const Layout& L, const ViewInfo* vt, const gs_medium* med,
                                const Record* rec, const uint2* ranges, const uint32_t* vals, const float* grad_rgb,
                                const float* grad_depth, const float* grad_restored, const float* tfinal,
                                const uint32_t* nlast, const float* cair, const float* dsum, const float* wsum,
                                float* grad2d, float* medpart, const Guard& guard, const uint32_t* order,
                                hipStream_t s);
// Per-view sums of the tiles' medium partials into grad_medium [views][9]; with `adam`, also one
// Adam step of the medium parameters (group with count 9 * views) using the device bias corrections.
// When the guard is set, grad_medium is zeroed and no step is taken.
// medium: [views][9] values of the medium; with o.medium_prior set the reduction adds
// o.prior_lambda sign(B - B_hat) to the B_inf and B_b gradients before the step.
// medsum: [views][kMedSlices][9] floats of workspace; done: [views] counters, zero at the start.
constexpr int kMedSlices = 16;
hipError_t launch_medium_reduce(const ViewInfo* vt, int32_t views, const float* medpart, float* medsum,
                                uint32_t* done, float* grad_medium, const float* medium, const gs_options& o,
                                const gs_adam_group* adam, float b1, float b2, float eps, const float* bc,
                                const Guard& guard, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_export_keys(const Layout& L, const uint2* ranges, const uint32_t* vals, const uint32_t* depth_keys,
                              int64_t capacity, uint64_t* keys, uint32_t* values, hipStream_t s);
hipError_t launch_forward_stats(const gs_options& o, const Layout& L, const ViewInfo* vt, const uint2* ranges,
                                const uint32_t* vals, const Record* rec, const uint32_t* nlast, const uint8_t* done,
                                unsigned long long* out, hipStream_t s);

// Image loss (loss.hip): bytes of the per-tile partial sums, and the fused L1 + D-SSIM pass.
int loss_partial_bytes(int32_t n_views, const gs_camera* cams, size_t* bytes);
int launch_l1_dssim(int32_t n_views, const gs_camera* cams, const float* pred, const float* target, float lambda,
                    float* loss, float* grad, float* partial, size_t partial_bytes, hipStream_t s);

// Timer hooks (no-ops when timer == nullptr).
void timer_begin(void* timer, const char* name, hipStream_t s);
void timer_end(void* timer, hipStream_t s);

}  // namespace gs
