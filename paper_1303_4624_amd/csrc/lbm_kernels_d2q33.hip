// lbm_kernels_d2q33.hip - the kernels of the 2D 33-velocity model (Table 2),
// float64 and FP32-shifted storage.
#include "lbm_kernels.h"

namespace lbm {
template struct ModelKernels<D2Q33, Prec::F64>;
template struct ModelKernels<D2Q33, Prec::F32S>;
}  // namespace lbm
