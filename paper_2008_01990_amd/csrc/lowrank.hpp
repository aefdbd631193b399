// Structured low-rank merge product (SRRSC compression + two generated products).
#pragma once
#include "common.hpp"

hipError_t dc_lowrank_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                             const int* org, const double* tau, const double* zhat,
                             const double* scale, double* C, long long ldc, double lr_tol,
                             int lr_block, hipStream_t stream);
hipError_t dc_plain_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                           const int* org, const double* tau, const double* zhat,
                           const double* scale, double* C, long long ldc, int beta,
                           int variant, hipStream_t stream);
