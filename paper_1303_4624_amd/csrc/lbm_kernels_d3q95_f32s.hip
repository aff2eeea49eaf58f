// lbm_kernels_d3q95_f32s.hip - the kernels of the 3D 95-velocity model (Table 3) in FP32-shifted storage
// (one translation unit per model and precision, compiled in parallel).
#include "lbm_kernels.h"

namespace lbm {
template struct ModelKernels<D3Q95, Prec::F32S>;
}  // namespace lbm
