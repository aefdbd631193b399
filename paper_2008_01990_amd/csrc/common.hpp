// Shared device helpers and plain-old-data descriptors of the HIP path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dcstedc.h"

#define DC_STATUS_NONFINITE (-1000)
#define DC_STATUS_EQUAL_EIG (-2000)

typedef double dc_double4 __attribute__((ext_vector_type(4)));

// Compile-time flags passed to generic lambdas.
struct dc_true_type { static constexpr bool value = true; };
struct dc_false_type { static constexpr bool value = false; };

// Reciprocal to full double precision: hardware estimate plus two
// Newton-Raphson corrections r <- r + r (1 - x r).
__device__ __forceinline__ double dc_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    return r;
}

// Reciprocal with one cubic correction: with e = 1 - x r0 (exact in the fma),
// 1/x = r0 (1 + e + e^2 + ...), and e^3 is far below double rounding for the
// hardware estimate r0, so r0 + r0 (e + e^2) is as accurate as two
// Newton-Raphson steps at three fma instead of four.
__device__ __forceinline__ double dc_rcp3(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(__builtin_fma(e, e, e), r, r);
}

// Loads through the global address space: the compiler then emits
// global_load (tracked by vmcnt only) instead of flat_load, whose lgkmcnt
// share would make every LDS wait also wait for outstanding prefetches.
typedef __attribute__((address_space(1))) const double dc_gdouble;
typedef __attribute__((address_space(1))) const int dc_gint;
__device__ __forceinline__ double dc_ldg(const double* p) { return *(dc_gdouble*)p; }
__device__ __forceinline__ int dc_ldg(const int* p) { return *(dc_gint*)p; }

__device__ __forceinline__ double dc_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double dc_wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Record a device-detected failure: the first non-convergence code wins;
// a non-finite input overrides any other code (later phases test for it).
__device__ __forceinline__ void dc_set_info(int* info, int code) {
    if (!info) return;
    if (code == DC_STATUS_NONFINITE) atomicExch(info, code);
    else atomicCAS(info, 0, code);
}

// One product C[rows, cols] (=|+=) A[rows, 0:klen] * B[0:klen, cols] in which
// B is generated on the fly (the Cauchy-like eigenvector block of
// eq. Q_Cauchy):
//    B_kc = rz[k] * cs[g] / ((rD[k] - cbase[g]) - coff[g]),
//  where g = ccol[c] if ccol is set, else col_off + c, is the generator index
//  of output column c.  The output column of C is cpos[c] when both ccol and
//  cpos are set, cpos[g] when only cpos is, and g - out_off otherwise.
struct GemmTask {
    const double* A;      // row 0 of this task inside A (column-major, lda)
    long long lda;
    const int* klen_p;    // device number of k-entries, or null (= klen)
    int klen;
    int rows;             // rows of the task
    const double* rD;     // row nodes
    const double* rz;     // row weights
    const double* cbase;  // column node bases (by generator index)
    const int* corg;      // if set, node base of g is rD[corg[g]] (cbase unused)
    const double* coff;   // column node offsets, or null (= 0)
    const double* cs;     // column scales
    const int* ncol_p;    // device number of columns, or null (= ncol)
    int ncol;
    int col_off;          // generator index of column 0 when ccol is null
    const int* ccol;      // generator index of column c, or null
    double* C;            // row 0 of this task inside C
    long long ldc;
    const int* cpos;      // output column of generator g, or null (= g - out_off)
    int out_off;          // subtracted from g when cpos is null
    int tiles_m, tiles_n; // worst-case tile grid of the task
    int beta;             // 0: overwrite, 1: accumulate
    // Register kernel only: a second k-phase accumulated into the
    // same tile after the generated one, with A2 (rows as A, lda2) and a
    // loaded B2 (row-major: B2[k ldb2 + c], c the task's column), k < klen2.
    // The epilogue's column scale multiplies it too (B2 is stored divided by
    // it).  klen2 = 0: no second phase.
    const double* A2;
    long long lda2;
    const double* B2;
    long long ldb2;
    int klen2;
};

// Host-side launcher of the generated-Cauchy product over a task list.
// tasks_dev / tile_start_dev live in device memory; tile_start has ntasks+1
// entries (exclusive prefix sum of tiles_m * tiles_n).  variant selects the
// tile shape (0 = default).
hipError_t dc_launch_cauchy_gemm(const GemmTask* tasks_dev, const int* tile_start_dev,
                                 int ntasks, int total_tiles, int variant,
                                 hipStream_t stream);
// Tasks with a second, loaded k-phase (klen2 > 0; klen may be 0, which leaves
// only the loaded phase): register kernel, variant 0 or 5 only
// (hipErrorInvalidValue otherwise).
hipError_t dc_launch_cauchy_gemm2(const GemmTask* tasks_dev, const int* tile_start_dev,
                                  int ntasks, int total_tiles, int variant,
                                  hipStream_t stream);
// Tasks built on the device, with the tile prefix and the total tile count
// in device memory: a direct launch over max_tiles (an upper bound known on
// the host) in which the tiles past the total exit at once (register
// kernel, variant 0 or 5).
hipError_t dc_launch_cauchy_gemm_bounded(const GemmTask* tasks_dev, const int* tile_start_dev,
                                         int ntasks, int max_tiles, const int* total_tiles_dev,
                                         int variant, bool two_phase, hipStream_t stream);
// Tasks whose column counts the device now knows: rewrites each task's
// tiles_n to ceil(ncol / bn) and writes the exclusive prefix of
// tiles_m * tiles_n (ntasks + 1 ints) and its sum, for a bounded launch.
hipError_t dc_launch_tile_scan(GemmTask* tasks, int ntasks, int bn, int* tile_start, int* total,
                               hipStream_t s);
// Number of merge-product tile variants (0 .. DC_TILE_VARIANTS - 1).
constexpr int DC_TILE_VARIANTS = 6;
int dc_gemm_tile_m(int variant);
int dc_gemm_tile_n(int variant);
