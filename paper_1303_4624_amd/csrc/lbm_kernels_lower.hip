// lbm_kernels_lower.hip - the kernels of the lower-order 3D 19- and
// 15-velocity sets (order of accuracy 2, second-order Hermite equilibrium),
// float64 and FP32-shifted storage.
#include "lbm_kernels.h"

namespace lbm {
template struct ModelKernels<D3Q19, Prec::F64>;
template struct ModelKernels<D3Q19, Prec::F32S>;
template struct ModelKernels<D3Q15, Prec::F64>;
template struct ModelKernels<D3Q15, Prec::F32S>;
}  // namespace lbm
