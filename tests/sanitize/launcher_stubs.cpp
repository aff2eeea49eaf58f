// Kernel launchers for the host-only sanitizer build of the C ABI: the
// device code is not part of that build, and with no GPU present no call
// reaches a launcher (lbm_bind rejects every pointer first).  Each returns
// hipErrorNoDevice so that a call that did get here would fail loudly.
#include "lbm_internal.h"

namespace lbm {

hipError_t launch_init(ModelId, Prec, const KParams&, const double*, const double*, const double*,
                       void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_set_pop(ModelId, Prec, const KParams&, const double*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_get_pop(ModelId, Prec, const KParams&, const void*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_step(ModelId, Prec, const KParams&, const void*, void*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_step_aa(ModelId, Prec, const KParams&, void*, bool, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_to_ab(ModelId, Prec, const KParams&, const void*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_from_ab(ModelId, Prec, const KParams&, const void*, void*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_moments(ModelId, Prec, const KParams&, const void*, double*, double*, double*,
                          hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_conservation(ModelId, Prec, const KParams&, const void*, double*, double*,
                               hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_fill_zero(double*, long long, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_lambda_init(ModelId, Prec, const KParams&, const void*, const double*, void*,
                              double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_adjoint_step(ModelId, Prec, const KParams&, const void*, void*, const void*,
                               double*, const void*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_dT_init(ModelId, Prec, const KParams&, const void*, const double*,
                          const double*, const double*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_sum_partials(const double*, long long, int, int, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t static_scratch(int, void**, size_t*) { return hipErrorNoDevice; }
hipError_t launch_stream_copy(const void*, void*, size_t, hipStream_t) { return hipErrorNoDevice; }

}  // namespace lbm
