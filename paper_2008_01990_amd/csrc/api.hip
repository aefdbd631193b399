// Single-purpose entry points of the C ABI: the short-form solve, status
// and error text, the secular solver and the merge product on explicit
// generators.
#include <map>
#include <mutex>
#include <cstring>
#include <vector>

#include "dc_internal.hpp"
#include "driver.hpp"
#include "lowrank.hpp"

namespace {

struct Blob { unsigned char b[1024]; };

__global__ void k_write_blob(unsigned char* dst, Blob blob, int nbytes) {
    for (int i = threadIdx.x; i < nbytes; i += blockDim.x) dst[i] = blob.b[i];
}

std::mutex g_status_mu;
std::map<hipStream_t, int*> g_status;

}  // namespace

hipError_t dc_status_word(hipStream_t s, int** out) {
    std::lock_guard<std::mutex> lk(g_status_mu);
    auto it = g_status.find(s);
    if (it != g_status.end()) { *out = it->second; return hipSuccess; }
    int* p = nullptr;
    hipError_t err = hipMalloc(&p, sizeof(int));
    if (err != hipSuccess) return err;
    err = hipMemset(p, 0, sizeof(int));
    if (err != hipSuccess) return err;
    g_status[s] = p;
    *out = p;
    return hipSuccess;
}

hipError_t dc_write_blob(void* dst, const void* src, int nbytes, hipStream_t s) {
    if (nbytes <= 0) return hipSuccess;
    if (nbytes > (int)sizeof(Blob)) return hipErrorInvalidValue;
    Blob b;
    std::memcpy(b.b, src, nbytes);
    hipLaunchKernelGGL(k_write_blob, dim3(1), dim3(256), 0, s,
                       static_cast<unsigned char*>(dst), b, nbytes);
    return hipGetLastError();
}

extern "C" int dc_stedc(int n, double* d, double* e, double* Q, int ldq, hipStream_t stream) {
    if (n < 0) return -1;
    if (n > 0 && !d) return -2;
    if (n > 1 && !e) return -3;
    if (n > 0 && !Q) return -4;
    if (ldq < (n > 1 ? n : 1)) return -5;
    int* st = nullptr;
    hipError_t err = dc_status_word(stream, &st);
    if (err != hipSuccess) return (int)err;
    const size_t lw = dc_stedc_workspace(n, nullptr);
    if (lw == 0) return (int)hipErrorInvalidValue;
    void* w = nullptr;
    err = hipMallocAsync(&w, lw, stream);
    if (err != hipSuccess) return (int)err;
    const int rc = dc_stedc_ex(n, d, e, Q, ldq, w, lw, st, nullptr, stream);
    hipError_t e2 = hipFreeAsync(w, stream);
    if (rc != 0) return rc;
    return (int)e2;
}

extern "C" int dc_last_info(hipStream_t stream) {
    int* st = nullptr;
    if (dc_status_word(stream, &st) != hipSuccess) return (int)hipErrorUnknown;
    if (hipStreamSynchronize(stream) != hipSuccess) return (int)hipErrorUnknown;
    int v = 0;
    if (hipMemcpy(&v, st, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return (int)hipErrorUnknown;
    return v;
}

extern "C" const char* dc_strerror(int code) {
    if (code == 0) return "success";
    if (code < 0) return "invalid argument (-code is its 1-based position)";
    return hipGetErrorString((hipError_t)code);
}

extern "C" const char* dc_status_string(int status) {
    if (status == 0) return "success";
    if (status == DC_STATUS_NONFINITE) return "non-finite value in the input";
    if (status == DC_STATUS_EQUAL_EIG) return "equal eigenvalues: adjoint term dropped";
    if (status > 0)
        return "an iteration did not converge (status - 1: first row of the leaf block, "
               "or the merge's first row plus the secular root's index, in the problem)";
    return "unknown status";
}

extern "C" int dc_secular(int K, const double* Dbar, const double* zbar, double rho, int* org,
                          double* tau, double* zhat, double* scale, int* info_dev,
                          int max_iter, hipStream_t stream) {
    if (K < 1) return -1;
    if (!Dbar) return -2;
    if (!zbar) return -3;
    if (!(rho > 0.0)) return -4;
    if (!org) return -5;
    if (!tau) return -6;
    if (!zhat) return -7;
    if (!scale) return -8;
    if (max_iter <= 0) max_iter = 200;
    const int nblk = (K + DC_ROOTS_PER_BLOCK - 1) / DC_ROOTS_PER_BLOCK;
    // task, block prefix {0, nblk} and block -> task map (all 0), generators
    const size_t off_bs = 256;
    const size_t off_cb = (off_bs + (size_t)(2 + nblk) * sizeof(int) + 255) / 256 * 256;
    char* tmp = nullptr;
    hipError_t err = hipMallocAsync((void**)&tmp, off_cb + (size_t)K * sizeof(double), stream);
    if (err != hipSuccess) return (int)err;
    SecTask T;
    std::memset(&T, 0, sizeof(T));
    T.D = Dbar;
    T.z = zbar;
    T.K = K;
    T.rho = rho;
    T.org = org;
    T.tau = tau;
    T.cbase = reinterpret_cast<double*>(tmp + off_cb);
    T.zhat = zhat;
    T.scale = scale;
    T.info = info_dev;
    int bs[2] = {0, nblk};
    err = dc_write_blob(tmp, &T, sizeof(T), stream);
    if (err == hipSuccess) err = dc_write_blob(tmp + off_bs, bs, sizeof(bs), stream);
    if (err == hipSuccess)
        err = dc_fill_int(reinterpret_cast<int*>(tmp + off_bs) + 2, nblk, 0, stream);
    if (err == hipSuccess && info_dev) err = dc_fill_int(info_dev, 1, 0, stream);
    if (err == hipSuccess)
        err = dc_launch_secular(reinterpret_cast<SecTask*>(tmp),
                                reinterpret_cast<int*>(tmp + off_bs), 1, nblk, K, max_iter,
                                stream);
    hipError_t e2 = hipFreeAsync(tmp, stream);
    return (int)(err != hipSuccess ? err : e2);
}

// Plain generated product on one task.
hipError_t dc_plain_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                           const int* org, const double* tau, const double* zhat,
                           const double* scale, double* C, long long ldc, int beta,
                           int variant, hipStream_t stream) {
    const int bm = dc_gemm_tile_m(variant), bn = dc_gemm_tile_n(variant);
    GemmTask T;
    std::memset(&T, 0, sizeof(T));
    T.A = Qnd;
    T.lda = ldq;
    T.klen = K;
    T.rows = m;
    T.rD = Dbar;
    T.rz = zhat;
    if (org) {
        T.corg = org;
        T.coff = tau;
    } else {
        T.cbase = tau;
    }
    T.cs = scale;
    T.ncol = K;
    T.C = C;
    T.ldc = ldc;
    T.tiles_m = (m + bm - 1) / bm;
    T.tiles_n = (K + bn - 1) / bn;
    T.beta = beta;
    const int tiles = T.tiles_m * T.tiles_n;
    char* tmp = nullptr;
    hipError_t err = hipMallocAsync((void**)&tmp, 512, stream);
    if (err != hipSuccess) return err;
    int ts[2] = {0, tiles};
    err = dc_write_blob(tmp, &T, sizeof(T), stream);
    if (err == hipSuccess) err = dc_write_blob(tmp + 256, ts, sizeof(ts), stream);
    if (err == hipSuccess)
        err = dc_launch_cauchy_gemm(reinterpret_cast<GemmTask*>(tmp),
                                    reinterpret_cast<int*>(tmp + 256), 1, tiles, variant, stream);
    hipError_t e2 = hipFreeAsync(tmp, stream);
    return err != hipSuccess ? err : e2;
}

extern "C" int dc_merge_update(int m, int K, const double* Qnd, int ldq, const double* Dbar,
                               const int* org, const double* tau, const double* zhat,
                               const double* scale, double* C, int ldc, double lr_tol,
                               int lr_block, hipStream_t stream) {
    if (m < 0) return -1;
    if (K < 0) return -2;
    if (m == 0 || K == 0) return 0;
    if (!Qnd) return -3;
    if (ldq < m) return -4;
    if (!Dbar) return -5;
    if (!tau) return -7;
    if (!zhat) return -8;
    if (!scale) return -9;
    if (!C) return -10;
    if (ldc < m) return -11;
    if (!(lr_tol >= 0.0)) return -12;
    if (lr_block <= 0) lr_block = 256;
    if (lr_tol > 0.0 && lr_block > dc_lowrank_max_block(org != nullptr)) return -13;
    if (lr_tol == 0.0 || K <= lr_block)
        return (int)dc_plain_update(m, K, Qnd, ldq, Dbar, org, tau, zhat, scale, C, ldc, 0, 0,
                                    stream);
    return (int)dc_lowrank_update(m, K, Qnd, ldq, Dbar, org, tau, zhat, scale, C, ldc, lr_tol,
                                  lr_block, stream);
}

extern "C" int dc_merge_update_variant(int m, int K, const double* Qnd, int ldq,
                                       const double* Dbar, const int* org, const double* tau,
                                       const double* zhat, const double* scale, double* C,
                                       int ldc, int variant, hipStream_t stream) {
    if (m <= 0 || K <= 0) return 0;
    return (int)dc_plain_update(m, K, Qnd, ldq, Dbar, org, tau, zhat, scale, C, ldc, 0,
                                variant, stream);
}
