// Structured low-rank merge product: placeholder until the SRRSC kernels land.
#include "lowrank.hpp"

hipError_t dc_lowrank_update(int, int, const double*, long long, const double*, const int*,
                             const double*, const double*, const double*, double*, long long,
                             double, int, hipStream_t) {
    return hipErrorNotSupported;
}

extern "C" int dc_merge_lowrank_ranks(int, const double*, const int*, const double*,
                                      const double*, const double*, double, int, int*,
                                      hipStream_t) {
    return (int)hipErrorNotSupported;
}
