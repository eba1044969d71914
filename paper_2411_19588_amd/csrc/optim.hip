// Elementwise steps around the rasterizer: parameter activation (exp scales,
// sigmoid opacity of eq. opacity_impact), the L1 term of eq. (3DGSoriginalLoss)
// and the fused Adam update of Sec. Optimization.  All are HBM-bound streams
// with grid-stride loops.
#include <string.h>

#include "internal.h"

namespace gs {
namespace {

constexpr int kMaxGroups = 8;

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

__global__ __launch_bounds__(kBlock) void k_activate(int64_t n, const float* __restrict__ ls,
                                                    const float* __restrict__ lg, float* __restrict__ s,
                                                    float* __restrict__ o) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 3 * n; i += stride) {
        s[i] = expf(ls[i]);
        if (i < n) o[i] = sigmoidf_(lg[i]);
    }
}

__global__ __launch_bounds__(kBlock) void k_activate_bwd(int64_t n, const float* __restrict__ s,
                                                        const float* __restrict__ o, const float* __restrict__ gs_,
                                                        const float* __restrict__ go, float* __restrict__ gls,
                                                        float* __restrict__ glg) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 3 * n; i += stride) {
        gls[i] = gs_[i] * s[i];
        if (i < n) glg[i] = go[i] * o[i] * (1.0f - o[i]);
    }
}

// One group's activation (the Adam groups' encoding): 0 copy, 1 exp, 2 sigmoid.
__global__ __launch_bounds__(kBlock) void k_activation(int64_t count, int32_t act, const float* __restrict__ x,
                                                      float* __restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const float v = x[i];
        y[i] = act == 1 ? expf(v) : (act == 2 ? sigmoidf_(v) : v);
    }
}

__global__ void k_zero1(float* p) { *p = 0.0f; }

// Few large workgroups: each adds its partial loss with one atomic on the single loss word,
// and same-address atomics serialise.
constexpr int kL1Block = 1024;
constexpr int kL1MaxGrid = 256;

__global__ __launch_bounds__(kL1Block) void k_l1(int64_t count, const float* __restrict__ p,
                                                const float* __restrict__ t, float* loss, float* __restrict__ grad) {
    __shared__ float red[kL1Block / 64];
    const int64_t stride = (int64_t)gridDim.x * kL1Block;
    const float inv = 1.0f / (float)count;
    float acc = 0.0f;
    auto one = [&](float pv, float tv) {
        const float d = pv - tv;
        acc += fabsf(d);
        return d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    };
    const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(t) |
                       reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
    const int64_t n4 = vec ? count / 4 : 0;
    for (int64_t i = (int64_t)blockIdx.x * kL1Block + threadIdx.x; i < n4; i += stride) {
        const float4 pv = reinterpret_cast<const float4*>(p)[i], tv = reinterpret_cast<const float4*>(t)[i];
        const float4 g = make_float4(one(pv.x, tv.x), one(pv.y, tv.y), one(pv.z, tv.z), one(pv.w, tv.w));
        if (grad) reinterpret_cast<float4*>(grad)[i] = g;
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * kL1Block + threadIdx.x; i < count; i += stride) {
        const float g = one(p[i], t[i]);
        if (grad) grad[i] = g;
    }
    if (!loss) return;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < kL1Block / 64; ++w) s += red[w];
        unsafeAtomicAdd(loss, s * inv);
    }
}

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kAdamItems = 4;                              // float4 per thread per block
constexpr int64_t kAdamChunk = (int64_t)kBlock * kAdamItems * 4;   // scalars per workgroup

struct AdamArgs {
    gs_adam_group g[kMaxGroups];
    int32_t count;
    int32_t block0[kMaxGroups + 1];  // first workgroup of each group (one flat grid over all groups)
    float b1, b2, eps, ibc1, ibc2;   // 1 / (1 - beta^t)
    const int32_t* step_dev;         // if set, bias corrections come from this device step number
                                     // (state[0]) and the step is skipped while state[1] != 0
};

// Start of a device-counted step: a forward whose image was truncated (pair overflow, or cut
// short by phase_limit; status may be null) sets the sticky skip flag; the counter advances
// only for a step that runs.
__device__ __forceinline__ bool step_begin(int32_t* state, const uint32_t* status) {
    const uint32_t st = status ? *status : 0u;
    uint32_t skip = (uint32_t)state[GS_STATE_SKIP] | (st & GS_STATUS_TRUNCATED);
    state[GS_STATE_SKIP] = (int32_t)skip;
    if (skip) return false;
    state[GS_STATE_STEP] += 1;
    return true;
}

__global__ void k_step_prep(int32_t* state, const uint32_t* status) { (void)step_begin(state, status); }

// Zeroes p[0, count) (the 2D gradients the adjoint accumulates into) and, in workgroup 0, starts
// the device-counted step: bias corrections of the step that runs in bc.
__global__ __launch_bounds__(kBlock) void k_zero_adam_prep(uint32_t* p, int64_t count, int32_t* state,
                                                          const uint32_t* status, float b1, float b2, float* bc) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock)
        p[i] = 0u;
    if (blockIdx.x != 0 || threadIdx.x != 0 || !step_begin(state, status)) return;
    const int32_t t = state[GS_STATE_STEP];
    bc[0] = 1.0f / (1.0f - powf(b1, (float)t));
    bc[1] = 1.0f / (1.0f - powf(b2, (float)t));
}

__device__ __forceinline__ float adam_one(const gs_adam_group& G, float p, float g, float act, float& m, float& v,
                                          float& new_act, float b1, float b2, float eps, float ibc1, float ibc2) {
    if (G.activation == 1) g *= act;                        // d exp(p)/dp = exp(p)
    else if (G.activation == 2) g *= act * (1.0f - act);    // d sigmoid(p)/dp
    const float np = adam_update(p, g, m, v, G.lr, b1, b2, eps, ibc1, ibc2);
    if (G.activation == 1) new_act = expf(np);
    else if (G.activation == 2) new_act = sigmoidf_(np);
    return np;
}

// The group is selected with constant indices: indexing the by-value argument array with
// blockIdx.y would make every thread copy it to private memory.
__device__ __forceinline__ gs_adam_group select_group(const AdamArgs& a, uint32_t y) {
    switch (y) {
        case 0: return a.g[0];
        case 1: return a.g[1];
        case 2: return a.g[2];
        case 3: return a.g[3];
        case 4: return a.g[4];
        case 5: return a.g[5];
        case 6: return a.g[6];
        default: return a.g[7];
    }
}

// One flat grid: workgroup b updates scalars [chunk * kAdamChunk, (chunk + 1) * kAdamChunk) of
// the group whose block range holds b, so every group's stream gets workgroups in proportion
// to its size (the SH group is most of the bytes).
__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs a) {
    // everything read from the argument block with constant indices (no private copy)
    float ibc1 = a.ibc1, ibc2 = a.ibc2;
    if (a.step_dev) {
        if (a.step_dev[GS_STATE_SKIP] != 0) return;   // skipped step (uniform exit)
        const float t = (float)a.step_dev[GS_STATE_STEP];
        ibc1 = 1.0f / (1.0f - powf(a.b1, t));
        ibc2 = 1.0f / (1.0f - powf(a.b2, t));
    }
    uint32_t gi = 0;
    int32_t start = 0;
#pragma unroll
    for (int k = 1; k < kMaxGroups; ++k) {
        if (k < a.count && (int32_t)blockIdx.x >= a.block0[k]) {
            gi = k;
            start = a.block0[k];
        }
    }
    const gs_adam_group G = select_group(a, gi);
    const int64_t n = G.count;
    const int64_t base = (int64_t)((int32_t)blockIdx.x - start) * kAdamChunk;
    const bool vec = ((reinterpret_cast<uintptr_t>(G.param) | reinterpret_cast<uintptr_t>(G.grad) |
                       reinterpret_cast<uintptr_t>(G.m) | reinterpret_cast<uintptr_t>(G.v) |
                       reinterpret_cast<uintptr_t>(G.activated)) & 15) == 0;
    if (vec && n - base >= kAdamChunk) {
        // whole chunk: every load of the chunk issued before any arithmetic; streamed with
        // non-temporal accesses (the arrays are far larger than the caches)
        v4f p[kAdamItems], g[kAdamItems], m[kAdamItems], v[kAdamItems], ac[kAdamItems];
#pragma unroll
        for (int it = 0; it < kAdamItems; ++it) {
            const int64_t i0 = base + ((int64_t)it * kBlock + threadIdx.x) * 4;
            p[it] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(G.param + i0));
            g[it] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(G.grad + i0));
            m[it] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(G.m + i0));
            v[it] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(G.v + i0));
            ac[it] = G.activation ? __builtin_nontemporal_load(reinterpret_cast<const v4f*>(G.activated + i0))
                                  : v4f{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int it = 0; it < kAdamItems; ++it) {
            const int64_t i0 = base + ((int64_t)it * kBlock + threadIdx.x) * 4;
            v4f np, na;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float mc = m[it][c], vc = v[it][c], nac = 0.0f;
                np[c] = adam_one(G, p[it][c], g[it][c], ac[it][c], mc, vc, nac, a.b1, a.b2, a.eps, ibc1, ibc2);
                m[it][c] = mc;
                v[it][c] = vc;
                na[c] = nac;
            }
            __builtin_nontemporal_store(np, reinterpret_cast<v4f*>(G.param + i0));
            __builtin_nontemporal_store(m[it], reinterpret_cast<v4f*>(G.m + i0));
            __builtin_nontemporal_store(v[it], reinterpret_cast<v4f*>(G.v + i0));
            if (G.activation) __builtin_nontemporal_store(na, reinterpret_cast<v4f*>(G.activated + i0));
        }
        return;
    }
    // the group's last, partial chunk (or unaligned arrays): scalar loop with bounds checks
    for (int64_t j = base + threadIdx.x; j < n && j < base + kAdamChunk; j += kBlock) {
        float m = G.m[j], v = G.v[j];
        float na = 0.0f;
        const float act = G.activation ? G.activated[j] : 0.0f;
        G.param[j] = adam_one(G, G.param[j], G.grad[j], act, m, v, na, a.b1, a.b2, a.eps, ibc1, ibc2);
        G.m[j] = m;
        G.v[j] = v;
        if (G.activation) G.activated[j] = na;
    }
}

unsigned grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_zero_adam_prep(uint32_t* p, int64_t count, int32_t* state, const uint32_t* status, float b1,
                                 float b2, float* bc, hipStream_t s) {
    int64_t g = (count + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero_adam_prep, dim3((unsigned)g), dim3(kBlock), 0, s, p, count, state, status, b1, b2, bc);
    return hipGetLastError();
}

}  // namespace gs

using namespace gs;

extern "C" {

int gs_activate(int64_t n, const float* log_scales, const float* logits, float* scales, float* opacity,
                gs_stream_t stream) {
    if (n < 0 || (n > 0 && (!log_scales || !logits || !scales || !opacity))) return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    hipLaunchKernelGGL(k_activate, dim3(grid_for(3 * n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream), n,
                       log_scales, logits, scales, opacity);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_activation(int64_t count, int32_t activation, const float* x, float* y, gs_stream_t stream) {
    if (count < 0 || activation < 0 || activation > 2 || (count > 0 && (!x || !y))) return GS_ERR_INVALID_ARGUMENT;
    if (count == 0) return GS_OK;
    hipLaunchKernelGGL(k_activation, dim3(grid_for(count)), dim3(kBlock), 0, static_cast<hipStream_t>(stream), count,
                       activation, x, y);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_activate_backward(int64_t n, const float* scales, const float* opacity, const float* g_scales,
                         const float* g_opacity, float* g_log_scales, float* g_logits, gs_stream_t stream) {
    if (n < 0 || (n > 0 && (!scales || !opacity || !g_scales || !g_opacity || !g_log_scales || !g_logits)))
        return GS_ERR_INVALID_ARGUMENT;
    if (n == 0) return GS_OK;
    hipLaunchKernelGGL(k_activate_bwd, dim3(grid_for(3 * n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream), n,
                       scales, opacity, g_scales, g_opacity, g_log_scales, g_logits);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_l1_loss(int64_t count, const float* pred, const float* target, float* loss, float* grad,
               gs_stream_t stream) {
    if (count <= 0 || !pred || !target || (!loss && !grad)) return GS_ERR_INVALID_ARGUMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (loss) hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, loss);
    // at most 512 workgroups: each adds one partial sum, so the atomic tail stays short
    int64_t g = ((count + 3) / 4 + kL1Block - 1) / kL1Block;
    if (g < 1) g = 1;
    if (g > kL1MaxGrid) g = kL1MaxGrid;
    hipLaunchKernelGGL(k_l1, dim3((unsigned)g), dim3(kL1Block), 0, s, count, pred, target, loss, grad);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

static int adam_launch(const gs_adam_group* host_groups, int32_t n_groups, float beta1, float beta2, float eps,
                       int32_t step, int32_t* step_dev, const void* saved, gs_stream_t stream) {
    if (!host_groups || n_groups < 1 || n_groups > kMaxGroups || (!step_dev && step < 1))
        return GS_ERR_INVALID_ARGUMENT;
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return GS_ERR_INVALID_ARGUMENT;
    AdamArgs a;
    memset(&a, 0, sizeof(a));
    a.count = n_groups;
    for (int k = 0; k < n_groups; ++k) {
        const gs_adam_group& G = host_groups[k];
        if (G.count < 0 || G.activation < 0 || G.activation > 2) return GS_ERR_INVALID_ARGUMENT;
        if (G.count > 0 && (!G.param || !G.grad || !G.m || !G.v || (G.activation && !G.activated)))
            return GS_ERR_INVALID_ARGUMENT;
        a.g[k] = G;
    }
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.step_dev = step_dev;
    if (!step_dev) {
        a.ibc1 = (float)(1.0 / (1.0 - __builtin_pow((double)beta1, (double)step)));
        a.ibc2 = (float)(1.0 / (1.0 - __builtin_pow((double)beta2, (double)step)));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the status word is the first field of the forward context's header
    if (step_dev)
        hipLaunchKernelGGL(k_step_prep, dim3(1), dim3(1), 0, s, step_dev,
                           saved ? &static_cast<const SavedHeader*>(saved)->status : nullptr);
    int64_t blocks = 0;
    for (int k = 0; k < n_groups; ++k) {
        a.block0[k] = (int32_t)blocks;
        blocks += (host_groups[k].count + kAdamChunk - 1) / kAdamChunk;
        if (blocks >= (1LL << 31)) return GS_ERR_INVALID_ARGUMENT;
    }
    a.block0[n_groups] = (int32_t)blocks;
    if (blocks > 0) hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

int gs_adam_step(const gs_adam_group* host_groups, int32_t n_groups, float beta1, float beta2, float eps,
                 int32_t step, gs_stream_t stream) {
    return adam_launch(host_groups, n_groups, beta1, beta2, eps, step, nullptr, nullptr, stream);
}

int gs_adam_step_device(const gs_adam_group* host_groups, int32_t n_groups, float beta1, float beta2, float eps,
                        int32_t* state, const void* saved, gs_stream_t stream) {
    if (!state) return GS_ERR_INVALID_ARGUMENT;
    return adam_launch(host_groups, n_groups, beta1, beta2, eps, 0, state, saved, stream);
}

int gs_graph_begin(gs_stream_t stream) {
    if (!stream) return GS_ERR_INVALID_ARGUMENT;
    return hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal) == hipSuccess
               ? GS_OK
               : GS_ERR_HIP;
}

int gs_graph_end(gs_stream_t stream, void** graph) {
    if (!stream || !graph) return GS_ERR_INVALID_ARGUMENT;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || !g) return GS_ERR_HIP;
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return GS_ERR_HIP;
    *graph = exec;
    return GS_OK;
}

int gs_graph_launch(void* graph, gs_stream_t stream) {
    if (!graph) return GS_ERR_INVALID_ARGUMENT;
    return hipGraphLaunch(static_cast<hipGraphExec_t>(graph), static_cast<hipStream_t>(stream)) == hipSuccess
               ? GS_OK
               : GS_ERR_HIP;
}

int gs_graph_destroy(void* graph) {
    if (!graph) return GS_ERR_INVALID_ARGUMENT;
    return hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph)) == hipSuccess ? GS_OK : GS_ERR_HIP;
}

}  // extern "C"
