// lbm_kernels_common.hip - kernels that do not depend on the velocity set
// (fills, fixed-order sums of block partials) and the launch_* entry points
// of the C-ABI layer, which dispatch on the model and precision to the
// launchers instantiated in the lbm_kernels_<model>.hip translation units.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm_internal.h"

namespace lbm {

// Scratch of lbm_conservation_noalloc: the per-block partials of the
// conservation sums (at most 1024 blocks of D + 2 <= 5 float64 values,
// rounded up to 256 bytes) and the D + 2 reduced sums.  Every element a call
// reads is written earlier in that call, so nothing needs clearing.
constexpr size_t kStaticScratchDoubles = 1024 * 5 + 64;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

constexpr int kCommonBlock = 256;
constexpr int kMaxDevices = 64;

__global__ __launch_bounds__(kCommonBlock) void k_fill_zero(double* p, long long n) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// out[q] = sum_j part[j*stride + q] for q < count, one block, fixed order.
__global__ __launch_bounds__(kCommonBlock) void k_sum_partials(const double* __restrict__ part,
                                                               long long n, int stride, int count,
                                                               double* __restrict__ out) {
    __shared__ double sh[kCommonBlock];
    for (int q = 0; q < count; ++q) {
        double s = 0.0;
        for (long long j = threadIdx.x; j < n; j += blockDim.x) s += part[j * stride + q];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// Streaming copy: one 16-byte vector per lane, plain load, non-temporal
// store (the step's own choices); the last bytes % 16 as 4-byte words.
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kCommonBlock) void k_stream_copy(const v4f* __restrict__ src,
                                                              v4f* __restrict__ dst,
                                                              long long n16, int tail4) {
    const long long i = static_cast<long long>(blockIdx.x) * kCommonBlock + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(src[i], &dst[i]);
    if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < tail4) {
        const float* s4 = reinterpret_cast<const float*>(src + n16);
        float* d4 = reinterpret_cast<float*>(dst + n16);
        d4[threadIdx.x] = s4[threadIdx.x];
    }
}

// Calls f with a model tag and the precision as template arguments.
template <class F>
hipError_t with_model(ModelId m, Prec p, F&& f) {
    const auto pick = [&](auto M_) {
        if (p == Prec::F64) return f(M_, std::integral_constant<Prec, Prec::F64>{});
        return f(M_, std::integral_constant<Prec, Prec::F32S>{});
    };
    switch (m) {
        case ModelId::D2Q33: return pick(D2Q33{});
        case ModelId::D3Q95: return pick(D3Q95{});
        case ModelId::D3Q19: return pick(D3Q19{});
        case ModelId::D3Q15: return pick(D3Q15{});
    }
    return hipErrorInvalidValue;
}

#define LBM_DISPATCH(call)                                                        \
    with_model(m, p, [&](auto M_, auto P_) {                                      \
        return ModelKernels<decltype(M_), decltype(P_)::value>::call;             \
    })

}  // namespace

hipError_t launch_init(ModelId m, Prec p, const KParams& kp, const double* rho, const double* U,
                       const double* T, void* f, hipStream_t s) {
    return LBM_DISPATCH(init(kp, rho, U, T, f, s));
}

hipError_t launch_set_pop(ModelId m, Prec p, const KParams& kp, const double* fin, void* f,
                          hipStream_t s) {
    return LBM_DISPATCH(set_pop(kp, fin, f, s));
}

hipError_t launch_get_pop(ModelId m, Prec p, const KParams& kp, const void* f, double* fout,
                          hipStream_t s) {
    return LBM_DISPATCH(get_pop(kp, f, fout, s));
}

hipError_t launch_step(ModelId m, Prec p, const KParams& kp, const void* src, void* dst,
                       void* mom_out, hipStream_t s) {
    if (!dst && !mom_out) return hipErrorInvalidValue;
    return LBM_DISPATCH(step(kp, src, dst, mom_out, s));
}

hipError_t launch_step_aa(ModelId m, Prec p, const KParams& kp, void* f, bool push,
                          void* mom_out, hipStream_t s) {
    return LBM_DISPATCH(step_aa(kp, f, push, mom_out, s));
}

hipError_t launch_to_ab(ModelId m, Prec p, const KParams& kp, const void* f, void* out,
                        hipStream_t s) {
    return LBM_DISPATCH(to_ab(kp, f, out, s));
}

hipError_t launch_from_ab(ModelId m, Prec p, const KParams& kp, const void* f, void* out,
                          hipStream_t s) {
    return LBM_DISPATCH(from_ab(kp, f, out, s));
}

hipError_t launch_moments(ModelId m, Prec p, const KParams& kp, const void* f, double* rho,
                          double* U, double* T, hipStream_t s) {
    return LBM_DISPATCH(moments(kp, f, rho, U, T, s));
}

hipError_t launch_conservation(ModelId m, Prec p, const KParams& kp, const void* f,
                               double* partials, double* out, hipStream_t s) {
    const hipError_t e = LBM_DISPATCH(conservation(kp, f, partials, s));
    if (e != hipSuccess) return e;
    const int K = (m == ModelId::D2Q33 ? 2 : 3) + 2;
    return launch_sum_partials(partials, reduce_blocks(kp.N), K, K, out, s);
}

hipError_t launch_lambda_init(ModelId m, Prec p, const KParams& kp, const void* fn,
                              const double* dLdrho, void* lam, double* partK, hipStream_t s) {
    return LBM_DISPATCH(lambda_init(kp, fn, dLdrho, lam, partK, s));
}

hipError_t launch_adjoint_step(ModelId m, Prec p, const KParams& kp, const void* lam_src,
                               void* lam_dst, const void* mom, double* partA,
                               const void* mark_state, double* partM, hipStream_t s) {
    return LBM_DISPATCH(adjoint_step(kp, lam_src, lam_dst, mom, partA, mark_state, partM, s));
}

hipError_t launch_dT_init(ModelId m, Prec p, const KParams& kp, const void* lam0,
                          const double* rho, const double* U, const double* T, double* dT,
                          hipStream_t s) {
    return LBM_DISPATCH(dT_init(kp, lam0, rho, U, T, dT, s));
}

hipError_t static_scratch(int device, void** ptr, size_t* bytes) {
    // In host code `scratch` names a host-side stand-in; the device address
    // of each GPU's copy comes from hipGetSymbolAddress with that GPU current.
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const long long n16 = static_cast<long long>(bytes / 16);
    const int tail4 = static_cast<int>((bytes % 16) / 4);
    const long long blocks = (n16 + kCommonBlock - 1) / kCommonBlock;
    hipLaunchKernelGGL(k_stream_copy, dim3(static_cast<unsigned>(blocks > 0 ? blocks : 1)),
                       dim3(kCommonBlock), 0, s, static_cast<const v4f*>(src),
                       static_cast<v4f*>(dst), n16, tail4);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((n + kCommonBlock - 1) / kCommonBlock);
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(kCommonBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* part, long long n, int stride, int count,
                               double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kCommonBlock), 0, s, part, n, stride, count,
                       out);
    return hipGetLastError();
}

}  // namespace lbm
