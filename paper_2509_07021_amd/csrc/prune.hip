// prune.hip -- the GPU steps of the memory-constrained optimisation (Sec. 3.3, Alg. 1) that act on
// the renderer's outputs: the lobe dynamic range D = |a| (1 - exp(-2 z)) (Sec. 3.3.2), a top-kappa
// selection for the factorised proximal operator, and the proximal, dual and penalty updates.
//
// Top-kappa is an MSB-first radix select on order-preserving 32-bit keys: four histogram passes
// over the candidates that still share the selected prefix, each followed by a one-thread pick of
// the digit bucket holding the kappa-th largest key. Elements equal to the threshold key are then
// taken in ascending index order through an exclusive scan of the equality flags, so the selected
// set is exactly "the kappa largest, ties to the lower index", independent of scheduling.
#include "megs_internal.hpp"

namespace megs {
namespace {

struct SelectState {
    uint32_t prefix;  // selected high digits of the threshold key
    uint32_t need;    // how many of the remaining candidates (keys matching prefix) to take
};

// Order-preserving map from float to uint32 (larger float -> larger key); -0 maps like +0.
__device__ __forceinline__ uint32_t ordered_key(float f) {
    const uint32_t b = __float_as_uint(f + 0.0f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ void k_select_init(SelectState* st, uint32_t* hist, int64_t kappa) {
    st->prefix = 0;
    st->need = (uint32_t)kappa;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
}

// Histogram of digit (key >> shift) & 255 over keys whose bits above shift + 8 equal the prefix.
__global__ __launch_bounds__(256) void k_select_hist(const float* __restrict__ score, int64_t n, int shift,
                                                     const SelectState* st, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t hi_mask = shift + 8 >= 32 ? 0u : (0xffffffffu << (shift + 8));
    const uint32_t prefix = st->prefix & hi_mask;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = ordered_key(score[i]);
        if ((key & hi_mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// One thread: from the largest digit down, find the bucket holding the need-th largest key.
__global__ void k_select_pick(SelectState* st, uint32_t* hist, int shift) {
    uint32_t need = st->need, cum = 0;
    int d = 255;
    for (; d > 0; --d) {
        if (cum + hist[d] >= need) break;
        cum += hist[d];
    }
    st->prefix |= (uint32_t)d << shift;
    st->need = need - cum;
    for (int i = 0; i < 256; ++i) hist[i] = 0;
}

__global__ void k_select_eq(const float* __restrict__ score, int64_t n, const SelectState* st, uint32_t* eq) {
    const uint32_t t = st->prefix;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        eq[i] = ordered_key(score[i]) == t;
}

__global__ void k_select_keep(const float* __restrict__ score, int64_t n, const SelectState* st,
                              const uint32_t* __restrict__ eq_rank, uint8_t* __restrict__ keep) {
    const uint32_t t = st->prefix, need = st->need;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t key = ordered_key(score[i]);
        keep[i] = key > t || (key == t && eq_rank[i] < need);
    }
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// D[l][i] = |a_l,i| (1 - exp(-2 (s + lambda)[l][i])) with |.| the Euclidean norm of the RGB amplitude.
__global__ void k_lobe_range(int64_t n, int32_t k, const float* __restrict__ s, const float* __restrict__ lam,
                             const float* __restrict__ amp, float* __restrict__ D) {
    const int64_t total = n * k;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = j / n, i = j - l * n;
        const float z = s[j] + (lam ? lam[j] : 0.0f);
        const float a0 = amp[(l * 3 + 0) * n + i], a1 = amp[(l * 3 + 1) * n + i], a2 = amp[(l * 3 + 2) * n + i];
        D[j] = sqrtf(a0 * a0 + a1 * a1 + a2 * a2) * (1.0f - expf(-2.0f * z));
    }
}

__global__ void k_prox_apply(int64_t count, const float* __restrict__ x, const float* __restrict__ lam,
                             const uint8_t* __restrict__ keep, float* __restrict__ xt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        xt[i] = keep[i] ? x[i] + lam[i] : 0.0f;
}

__global__ void k_dual(int64_t count, float* __restrict__ lam, const float* __restrict__ x,
                       const float* __restrict__ xt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        lam[i] = lam[i] + (x[i] - xt[i]);
}

__global__ void k_penalty(int64_t count, float delta, const float* __restrict__ x, const float* __restrict__ xt,
                          const float* __restrict__ lam, float* __restrict__ grad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        grad[i] = __fmaf_rn(delta, (x[i] - xt[i]) + lam[i], grad[i]);
}

inline unsigned grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace

size_t select_scratch_bytes(int64_t n) {
    const size_t a = (sizeof(SelectState) + 255) & ~(size_t)255;
    const size_t h = 256 * sizeof(uint32_t);
    const size_t e = (((size_t)(n > 0 ? n : 1) * sizeof(uint32_t)) + 255) & ~(size_t)255;
    return a + h + 2 * e + ((scan_scratch_bytes(n) + 255) & ~(size_t)255) + 256;
}

hipError_t launch_select_topk(const float* score, int64_t n, int64_t kappa, void* scratch, uint8_t* keep,
                              hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (kappa <= 0 || kappa >= n) {
        hipLaunchKernelGGL(k_fill_u8, dim3(grid_of(n)), dim3(256), 0, stream, keep, (uint8_t)(kappa > 0), n);
        return hipGetLastError();
    }
    char* p = static_cast<char*>(scratch);
    SelectState* st = reinterpret_cast<SelectState*>(p);
    p += (sizeof(SelectState) + 255) & ~(size_t)255;
    uint32_t* hist = reinterpret_cast<uint32_t*>(p);
    p += 256 * sizeof(uint32_t);
    uint32_t* eq = reinterpret_cast<uint32_t*>(p);
    p += (((size_t)n * sizeof(uint32_t)) + 255) & ~(size_t)255;
    uint32_t* rank = reinterpret_cast<uint32_t*>(p);
    p += (((size_t)n * sizeof(uint32_t)) + 255) & ~(size_t)255;
    void* scan_scratch = p;
    hipLaunchKernelGGL(k_select_init, dim3(1), dim3(256), 0, stream, st, hist, kappa);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_select_hist, dim3(grid_of(n)), dim3(256), 0, stream, score, n, shift, st, hist);
        hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(1), 0, stream, st, hist, shift);
    }
    hipLaunchKernelGGL(k_select_eq, dim3(grid_of(n)), dim3(256), 0, stream, score, n, st, eq);
    hipError_t e = launch_scan(eq, nullptr, n, rank, hist, scan_scratch, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_select_keep, dim3(grid_of(n)), dim3(256), 0, stream, score, n, st, rank, keep);
    return hipGetLastError();
}

hipError_t launch_lobe_range(int64_t n, int32_t k, const float* s, const float* lam, const float* amp, float* D,
                             hipStream_t stream) {
    if (n * k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lobe_range, dim3(grid_of(n * k)), dim3(256), 0, stream, n, k, s, lam, amp, D);
    return hipGetLastError();
}

hipError_t launch_prox_apply(int64_t count, const float* x, const float* lam, const uint8_t* keep, float* xt,
                             hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prox_apply, dim3(grid_of(count)), dim3(256), 0, stream, count, x, lam, keep, xt);
    return hipGetLastError();
}

hipError_t launch_dual(int64_t count, float* lam, const float* x, const float* xt, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dual, dim3(grid_of(count)), dim3(256), 0, stream, count, lam, x, xt);
    return hipGetLastError();
}

hipError_t launch_penalty(int64_t count, float delta, const float* x, const float* xt, const float* lam, float* grad,
                          hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_penalty, dim3(grid_of(count)), dim3(256), 0, stream, count, delta, x, xt, lam, grad);
    return hipGetLastError();
}

}  // namespace megs
