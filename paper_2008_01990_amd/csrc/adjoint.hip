// Reverse-mode gradient of the eigendecomposition T(d, e) = Q diag(lam) Q^T.
//
// For a loss L(lam, Q) with cotangents (lam_bar, Q_bar) and distinct
// eigenvalues, the cotangent of the matrix is
//     A_bar = Q M Q^T,   M = diag(lam_bar) + F o (Q^T Q_bar),
//     F_ij = 1 / (lam_j - lam_i) (i != j), F_ii = 0,
// and T depends on d_i through A[i][i] and on e_i through A[i][i+1] and
// A[i+1][i], so d_bar_i = A_bar[i][i], e_bar_i = A_bar[i][i+1] + A_bar[i+1][i].
//
// Only that band is ever formed.  With P = Q M,
//     d_bar_i = sum_j P_ij Q_ij,   e_bar_i = sum_j (P_ij Q_{i+1,j} + P_{i+1,j} Q_ij),
// and the product P = Q M runs through the generated-tile MFMA kernel with M
// generated per tile from (lam, lam_bar, G) and a band epilogue that reduces
// each tile of P against three rows of Q: P never reaches HBM.  Per tile the
// partial row sums are written to small buffers and summed in a fixed order
// (deterministic).
//
//   general Q_bar:  Q^T (explicit transpose, HBM-bound) -> G = Q^T Q_bar (loaded
//                   MFMA product) -> P = Q M with band epilogue: 4 n^3 flops.
//   rank-one Q_bar = u g^T:  G = (Q^T u) g^T is itself Cauchy-like inside F o G,
//                   so M is generated from (Q^T u, g, lam): 2 n^3 flops.
// Nothing of the forward tree is stored or recomputed: the final (lam, Q) is
// all the adjoint reads.
#include <cstring>
#include <vector>

#include "common.hpp"
#include "driver.hpp"

namespace {

constexpr int TT = 32;

__global__ void k_transpose(const double* __restrict__ A, long long lda, double* __restrict__ B,
                            long long ldb, int n) {
    __shared__ double t[TT][TT + 1];
    const int bx = blockIdx.x * TT, by = blockIdx.y * TT;
    const int tx = threadIdx.x, ty = threadIdx.y;     // 32 x 8
    for (int k = ty; k < TT; k += 8) {
        const int r = bx + tx, c = by + k;
        if (r < n && c < n) t[k][tx] = A[(long long)c * lda + r];
    }
    __syncthreads();
    for (int k = ty; k < TT; k += 8) {
        const int r = by + tx, c = bx + k;            // B[r, c] = A[c, r]
        if (r < n && c < n) B[(long long)c * ldb + r] = t[tx][k];
    }
}

// a_i = sum_l Q[l, i] u[l]: one wave per column.
__global__ void k_gemv_t(const double* __restrict__ Q, long long ldq, const double* __restrict__ u,
                         double* __restrict__ a, int n) {
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col >= n) return;
    const double* q = Q + (long long)col * ldq;
    double s = 0.0;
    for (int l = lane; l < n; l += 64) s += q[l] * u[l];
    s = dc_wave_sum(s);
    if (lane == 0) a[col] = s;
}

__global__ void k_band_reduce(const double* __restrict__ pd, const double* __restrict__ pu,
                              const double* __restrict__ pl, int nparts, int n,
                              double* __restrict__ dbar, double* __restrict__ ebar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sd = 0.0, se = 0.0;
    for (int p = 0; p < nparts; ++p) {
        const long long o = (long long)p * n;
        sd += pd[o + i];
        if (i + 1 < n) se += pu[o + i] + pl[o + i + 1];
    }
    dbar[i] = sd;
    if (i + 1 < n) ebar[i] = se;
}

__global__ void k_flag_to_status(const int* flag, int* status) {
    if (threadIdx.x == 0 && *flag) dc_set_info(status, DC_STATUS_EQUAL_EIG);
}

__global__ void k_zero(double* p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Common tail: P = Q M (kind 3 with band epilogue) and the band reduction.
hipError_t band_product(int n, const double* lam, const double* Q, long long ldq,
                        const double* lam_bar, const double* G, long long ldg,
                        const double* a, const double* g, double* d_bar, double* e_bar,
                        char* tmp, size_t o_task, size_t o_parts, size_t o_flag, int* status,
                        hipStream_t s) {
    const int BM = 256, BN = 128;
    const int tiles_m = (n + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    const int nparts = tiles_n * dc_band_waves_n();
    double* parts = reinterpret_cast<double*>(tmp + o_parts);
    int* flag = reinterpret_cast<int*>(tmp + o_flag);
    GemmTask T;
    std::memset(&T, 0, sizeof(T));
    T.A = Q;
    T.lda = ldq;
    T.klen = n;
    T.rows = n;
    T.ncol = n;
    T.rz = a;
    T.cs = g;
    T.Bm = G;
    T.ldb = ldg;
    T.lam = lam;
    T.lbar = lam_bar;
    T.flag = flag;
    T.Qb = Q;
    T.ldqb = ldq;
    T.nband = n;
    T.pd = parts;
    T.pu = parts + (size_t)nparts * n;
    T.pl = parts + 2 * (size_t)nparts * n;
    T.tiles_m = tiles_m;
    T.tiles_n = tiles_n;
    const int ts[2] = {0, tiles_m * tiles_n};
    hipError_t err = dc_fill_int(flag, 1, 0, s);
    if (err == hipSuccess) err = dc_write_blob(tmp + o_task, &T, sizeof(T), s);
    if (err == hipSuccess) err = dc_write_blob(tmp + o_task + 1024, ts, sizeof(ts), s);
    if (err == hipSuccess)
        err = dc_launch_adjoint_gemm(reinterpret_cast<GemmTask*>(tmp + o_task),
                                     reinterpret_cast<int*>(tmp + o_task + 1024), 1,
                                     tiles_m * tiles_n, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_band_reduce, dim3((n + 255) / 256), dim3(256), 0, s, parts,
                       parts + (size_t)nparts * n, parts + 2 * (size_t)nparts * n, nparts, n,
                       d_bar, e_bar);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_flag_to_status, dim3(1), dim3(64), 0, s, flag, status);
    return hipGetLastError();
}

size_t parts_bytes(int n) {
    const int tiles_n = (n + 127) / 128;
    return 3 * (size_t)tiles_n * dc_band_waves_n() * n * sizeof(double);
}

}  // namespace

extern "C" int dc_stedc_backward(int n, const double* lam, const double* Q, int ldq,
                                 const double* lam_bar, const double* Q_bar, int ldqb,
                                 double* d_bar, double* e_bar, hipStream_t stream) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    if (!lam) return -2;
    if (!Q) return -3;
    if (ldq < n) return -4;
    if (Q_bar && ldqb < n) return -7;
    if (!d_bar) return -8;
    if (n > 1 && !e_bar) return -9;
    int* status = nullptr;
    hipError_t err = dc_status_word(stream, &status);
    if (err != hipSuccess) return (int)err;
    err = dc_fill_int(status, 1, 0, stream);
    if (err != hipSuccess) return (int)err;
    size_t o = 0;
    const size_t o_task = o; o = al(o + 2048);
    const size_t o_flag = o; o = al(o + sizeof(int));
    const size_t o_parts = o; o = al(o + parts_bytes(n));
    const size_t o_zero = o; o = al(o + (size_t)n * sizeof(double));
    const size_t o_qt = o; o = al(o + (Q_bar ? (size_t)n * n * sizeof(double) : 0));
    const size_t o_g = o; o = al(o + (Q_bar ? (size_t)n * n * sizeof(double) : 0));
    char* tmp = nullptr;
    err = hipMallocAsync((void**)&tmp, o, stream);
    if (err != hipSuccess) return (int)err;
    double* zero = reinterpret_cast<double*>(tmp + o_zero);
    hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, stream, zero, (long long)n);
    err = hipGetLastError();
    const double* G = nullptr;
    if (err == hipSuccess && Q_bar) {
        double* Qt = reinterpret_cast<double*>(tmp + o_qt);
        double* Gw = reinterpret_cast<double*>(tmp + o_g);
        hipLaunchKernelGGL(k_transpose, dim3((n + TT - 1) / TT, (n + TT - 1) / TT), dim3(TT, 8),
                           0, stream, Q, (long long)ldq, Qt, (long long)n, n);
        err = hipGetLastError();
        // G = Q^T Q_bar: loaded-B product.
        GemmTask T;
        std::memset(&T, 0, sizeof(T));
        T.A = Qt;
        T.lda = n;
        T.klen = n;
        T.rows = n;
        T.ncol = n;
        T.Bm = Q_bar;
        T.ldb = ldqb;
        T.C = Gw;
        T.ldc = n;
        T.tiles_m = (n + 255) / 256;
        T.tiles_n = (n + 127) / 128;
        const int ts[2] = {0, T.tiles_m * T.tiles_n};
        if (err == hipSuccess) err = dc_write_blob(tmp + o_task, &T, sizeof(T), stream);
        if (err == hipSuccess) err = dc_write_blob(tmp + o_task + 1024, ts, sizeof(ts), stream);
        if (err == hipSuccess)
            err = dc_launch_loaded_gemm(reinterpret_cast<GemmTask*>(tmp + o_task),
                                        reinterpret_cast<int*>(tmp + o_task + 1024), 1, ts[1],
                                        stream);
        G = Gw;
    }
    if (err == hipSuccess)
        err = band_product(n, lam, Q, ldq, lam_bar, G, n, zero, zero, d_bar, e_bar, tmp, o_task,
                           o_parts, o_flag, status, stream);
    hipError_t e2 = hipFreeAsync(tmp, stream);
    return (int)(err != hipSuccess ? err : e2);
}

extern "C" int dc_stedc_backward_rank1(int n, const double* lam, const double* Q, int ldq,
                                       const double* lam_bar, const double* u, const double* g,
                                       double* d_bar, double* e_bar, hipStream_t stream) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    if (!lam) return -2;
    if (!Q) return -3;
    if (ldq < n) return -4;
    if (!u) return -6;
    if (!g) return -7;
    if (!d_bar) return -8;
    if (n > 1 && !e_bar) return -9;
    int* status = nullptr;
    hipError_t err = dc_status_word(stream, &status);
    if (err != hipSuccess) return (int)err;
    err = dc_fill_int(status, 1, 0, stream);
    if (err != hipSuccess) return (int)err;
    size_t o = 0;
    const size_t o_task = o; o = al(o + 2048);
    const size_t o_flag = o; o = al(o + sizeof(int));
    const size_t o_parts = o; o = al(o + parts_bytes(n));
    const size_t o_a = o; o = al(o + (size_t)n * sizeof(double));
    char* tmp = nullptr;
    err = hipMallocAsync((void**)&tmp, o, stream);
    if (err != hipSuccess) return (int)err;
    double* a = reinterpret_cast<double*>(tmp + o_a);
    hipLaunchKernelGGL(k_gemv_t, dim3((n + 3) / 4), dim3(256), 0, stream, Q, (long long)ldq, u,
                       a, n);
    err = hipGetLastError();
    if (err == hipSuccess)
        err = band_product(n, lam, Q, ldq, lam_bar, nullptr, 0, a, g, d_bar, e_bar, tmp, o_task,
                           o_parts, o_flag, status, stream);
    hipError_t e2 = hipFreeAsync(tmp, stream);
    return (int)(err != hipSuccess ? err : e2);
}
