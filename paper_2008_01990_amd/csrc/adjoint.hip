// Adjoint of the eigendecomposition: placeholder until the band kernels land.
#include "common.hpp"

extern "C" int dc_stedc_backward(int, const double*, const double*, int, const double*,
                                 const double*, int, double*, double*, hipStream_t) {
    return (int)hipErrorNotSupported;
}

extern "C" int dc_stedc_backward_rank1(int, const double*, const double*, int, const double*,
                                       const double*, const double*, double*, double*,
                                       hipStream_t) {
    return (int)hipErrorNotSupported;
}
