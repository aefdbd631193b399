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
#include <map>
#include <mutex>
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

__global__ void k_fill(double* p, long long n, double v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// P = Q M on register tiles, with the band epilogue.  A workgroup of WGN
// waves covers 16 FM rows; wave wn covers 16 FN columns, and for every
// k-step of 4 it loads its A operands (16 consecutive rows of Q per MFMA)
// straight from global memory RING - 1 steps ahead and generates its M
// operands in registers:
//     M_kc = lbar_c if k == c, 0 if lam_c == lam_k (the status flag is set),
//            X_kc / (lam_c - lam_k) otherwise,
// X_kc = XR[k ldx + c] (LOADED: G stored row-major) or a_k g_c (rank one).
// The epilogue reduces each row of the wave's block of P against rows r,
// r + 1 and r - 1 of Q over its columns and writes one partial sum per
// (column group, row): the column group is wcol / (16 FN), and exactly one
// wave writes each (group, row).
template <int FM, int FN, int WGN, int RING, bool LOADED>
__global__ __launch_bounds__(WGN * 64, 2)
void k_band_reg(int n, const double* __restrict__ Q, long long ldq,
                const double* __restrict__ lam, const double* __restrict__ lbar,
                const double* __restrict__ XR, long long ldx, const double* __restrict__ av,
                const double* __restrict__ gv, double* __restrict__ pd, double* __restrict__ pu,
                double* __restrict__ pl, int tiles_m, int tiles_n, int* __restrict__ flag) {
    constexpr int WR = 16 * FM, WC = 16 * FN, BN = WGN * WC;
    constexpr int PD = RING - 1;
    // Eight consecutive blocks go to eight XCDs: give each XCD a contiguous
    // range of tiles (whole tile rows share their panel of Q in its L2).
    const int total = tiles_m * tiles_n;
    const int per_xcd = (total + 7) / 8;
    const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (t >= total) return;
    const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
    const int lane = threadIdx.x & 63, wn = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int row0 = tm * WR;
    const int wcol = tn * BN + wn * WC;
    if (wcol >= n || row0 >= n) return;      // no barriers: waves retire independently

    double lc[FN], lb[FN], gc[FN];
    int cix[FN];
    bool cval[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        cix[j] = wcol + j * 16 + lr;
        cval[j] = cix[j] < n;
        const int c = min(cix[j], n - 1);
        lc[j] = dc_ldg(lam + c);
        lb[j] = lbar ? dc_ldg(lbar + c) : 0.0;
        gc[j] = LOADED ? 0.0 : dc_ldg(gv + c);
    }
    dc_double4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = dc_double4{0.0, 0.0, 0.0, 0.0};
    bool equal_eig = false;

    // SHIFT (n >= WR): the rows move back inside the matrix, one base pointer
    // plus constant offsets; otherwise each row index is clamped.
    auto body = [&](auto shift_tag) {
        constexpr bool SHIFT = decltype(shift_tag)::value;
        const int crow = SHIFT ? min(row0, n - WR) : row0;
        const double* __restrict__ Ab = Q + (SHIFT ? crow + lr : 0);
        double a[RING][FM], dk[RING], xk[RING][LOADED ? FN : 1];
        auto issue = [&](int slot, int step) {
            const int k = min(step * 4 + lk, n - 1);
            const double* __restrict__ pk = Ab + (long long)k * ldq;
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[slot][i] = dc_ldg(pk + (SHIFT ? i * 16 : min(row0 + i * 16 + lr, n - 1)));
            dk[slot] = dc_ldg(lam + k);
            if constexpr (LOADED) {
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    xk[slot][j] = dc_ldg(XR + (long long)k * ldx + min(cix[j], n - 1));
            } else {
                xk[slot][0] = dc_ldg(av + k);
            }
        };
        auto compute = [&](int slot, int step, auto masked_tag) {
            constexpr bool MASKED = decltype(masked_tag)::value;
            const int kk = step * 4 + lk;
            const bool kok = kk < n;
            // k == c only where the step's four k meet the wave's columns
            // (a uniform test); elsewhere every k is a row of the matrix
            // (unmasked) and off the diagonal.
            const bool dstep = MASKED || (unsigned)(step * 4 + 3 - wcol) < (unsigned)(WC + 3);
            double bf[FN];
            if (dstep) {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const double den = lc[j] - dk[slot];
                    const double x = LOADED ? xk[slot][j] : xk[slot][0] * gc[j];
                    const bool diag = kk == cix[j];
                    const bool eq = den == 0.0;
                    double v = x * dc_rcp3(den);
                    v = eq ? 0.0 : v;
                    v = diag ? lb[j] : v;
                    equal_eig |= eq && !diag && kok && cval[j];
                    bf[j] = (!MASKED || kok) ? v : 0.0;
                }
            } else {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const double den = lc[j] - dk[slot];
                    const double x = LOADED ? xk[slot][j] : xk[slot][0] * gc[j];
                    const bool eq = den == 0.0;
                    const double v = x * dc_rcp3(den);
                    bf[j] = eq ? 0.0 : v;
                    equal_eig |= eq && cval[j];
                }
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[slot][i], bf[j],
                                                                     acc[i][j], 0, 0, 0);
        };
        const int nsteps = (n + 3) / 4;
        const int nfull = n / 4;
#pragma unroll
        for (int s = 0; s < PD; ++s) issue(s, s);
        int s = 0;
        for (; s + RING <= nfull; s += RING) {
#pragma unroll
            for (int j = 0; j < RING; ++j) {
                issue((j + PD) % RING, s + j + PD);
                compute(j, s + j, dc_false_type{});
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        for (; s < nsteps; s += RING) {
#pragma unroll
            for (int j = 0; j < RING; ++j) {
                issue((j + PD) % RING, s + j + PD);
                compute(j, s + j, dc_true_type{});
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        return crow;
    };
    const int crow = n >= WR ? body(dc_true_type{}) : body(dc_false_type{});

    const int part = wcol / WC;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = crow + i * 16 + lk + 4 * v;
            const bool rok = r >= row0 && r < n;
            double sd = 0.0, su = 0.0, sl = 0.0;
            if (rok) {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if (cix[j] >= n) continue;
                    const double x = acc[i][j][v];
                    const double* q = Q + (long long)cix[j] * ldq + r;
                    sd += x * q[0];
                    if (r + 1 < n) su += x * q[1];
                    if (r > 0) sl += x * q[-1];
                }
            }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                sd += __shfl_xor(sd, off, 64);
                su += __shfl_xor(su, off, 64);
                sl += __shfl_xor(sl, off, 64);
            }
            if (lr == 0 && rok) {
                const long long o = (long long)part * n + r;
                pd[o] = sd;
                pu[o] = su;
                pl[o] = sl;
            }
        }
    }
    if (equal_eig && flag) atomicOr(flag, 1);
}

constexpr int BFM = 8, BFN = 2, BWGN = 4, BRING = 3;
constexpr int BAND_WC = 16 * BFN;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Common tail: P = Q M (register tiles, band epilogue) and the band
// reduction.  XR: G row-major (general), or null with a = Q^T u, g (rank one).
hipError_t band_product(int n, const double* lam, const double* Q, long long ldq,
                        const double* lam_bar, const double* XR, long long ldx,
                        const double* a, const double* g, double* d_bar, double* e_bar,
                        char* tmp, size_t o_parts, size_t o_flag, int* status,
                        hipStream_t s) {
    const int tiles_m = (n + 16 * BFM - 1) / (16 * BFM);
    const int tiles_n = (n + BWGN * BAND_WC - 1) / (BWGN * BAND_WC);
    const int nparts = (n + BAND_WC - 1) / BAND_WC;       // column groups
    double* parts = reinterpret_cast<double*>(tmp + o_parts);
    double* pd = parts;
    double* pu = parts + (size_t)nparts * n;
    double* pl = parts + 2 * (size_t)nparts * n;
    int* flag = reinterpret_cast<int*>(tmp + o_flag);
    hipError_t err = dc_fill_int(flag, 1, 0, s);
    if (err != hipSuccess) return err;
    const int grid = (tiles_m * tiles_n + 7) / 8 * 8;
    if (XR)
        hipLaunchKernelGGL((k_band_reg<BFM, BFN, BWGN, BRING, true>), dim3(grid),
                           dim3(BWGN * 64), 0, s, n, Q, ldq, lam, lam_bar, XR, ldx, a, g, pd,
                           pu, pl, tiles_m, tiles_n, flag);
    else
        hipLaunchKernelGGL((k_band_reg<BFM, BFN, BWGN, BRING, false>), dim3(grid),
                           dim3(BWGN * 64), 0, s, n, Q, ldq, lam, lam_bar, XR, ldx, a, g, pd,
                           pu, pl, tiles_m, tiles_n, flag);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_band_reduce, dim3((n + 255) / 256), dim3(256), 0, s, pd, pu, pl,
                       nparts, n, d_bar, e_bar);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_flag_to_status, dim3(1), dim3(64), 0, s, flag, status);
    return hipGetLastError();
}

size_t parts_bytes(int n) {
    return 3 * (size_t)((n + BAND_WC - 1) / BAND_WC) * n * sizeof(double);
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
    const size_t o_ones = o; o = al(o + (size_t)n * sizeof(double));
    const size_t o_zero = o; o = al(o + (size_t)n * sizeof(double));
    const size_t o_qt = o; o = al(o + (Q_bar ? (size_t)n * n * sizeof(double) : 0));
    const size_t o_qbt = o; o = al(o + (Q_bar ? (size_t)n * n * sizeof(double) : 0));
    const size_t o_g = o; o = al(o + (Q_bar ? (size_t)n * n * sizeof(double) : 0));
    char* tmp = nullptr;
    err = hipMallocAsync((void**)&tmp, o, stream);
    if (err != hipSuccess) return (int)err;
    double* ones = reinterpret_cast<double*>(tmp + o_ones);
    double* zero = reinterpret_cast<double*>(tmp + o_zero);
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, stream, ones, (long long)n,
                       1.0);
    err = hipGetLastError();
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, stream, zero,
                           (long long)n, 0.0);
        err = hipGetLastError();
    }
    const double* XR = nullptr;
    if (err == hipSuccess && Q_bar) {
        // G^T = Q_bar^T Q through the loaded k-phase of the merge product's
        // register kernel (A2 = Q_bar^T, B2 = Q row-major; no generated phase;
        // column scales 1): G^T column-major is G row-major.
        double* Qt = reinterpret_cast<double*>(tmp + o_qt);
        double* Qbt = reinterpret_cast<double*>(tmp + o_qbt);
        double* Gt = reinterpret_cast<double*>(tmp + o_g);
        const dim3 tg((n + TT - 1) / TT, (n + TT - 1) / TT), tb(TT, 8);
        hipLaunchKernelGGL(k_transpose, tg, tb, 0, stream, Q, (long long)ldq, Qt, (long long)n,
                           n);
        err = hipGetLastError();
        if (err == hipSuccess) {
            hipLaunchKernelGGL(k_transpose, tg, tb, 0, stream, Q_bar, (long long)ldqb, Qbt,
                               (long long)n, n);
            err = hipGetLastError();
        }
        GemmTask T;
        std::memset(&T, 0, sizeof(T));
        T.klen = 0;
        T.rows = n;
        T.ncol = n;
        T.cbase = ones;
        T.cs = ones;
        T.C = Gt;
        T.ldc = n;
        T.A2 = Qbt;
        T.lda2 = n;
        T.B2 = Qt;
        T.ldb2 = n;
        T.klen2 = n;
        T.tiles_m = (n + dc_gemm_tile_m(0) - 1) / dc_gemm_tile_m(0);
        T.tiles_n = (n + dc_gemm_tile_n(0) - 1) / dc_gemm_tile_n(0);
        const int ts[2] = {0, T.tiles_m * T.tiles_n};
        if (err == hipSuccess) err = dc_write_blob(tmp + o_task, &T, sizeof(T), stream);
        if (err == hipSuccess) err = dc_write_blob(tmp + o_task + 1024, ts, sizeof(ts), stream);
        if (err == hipSuccess)
            err = dc_launch_cauchy_gemm2(reinterpret_cast<GemmTask*>(tmp + o_task),
                                         reinterpret_cast<int*>(tmp + o_task + 1024), 1, ts[1],
                                         0, stream);
        XR = Gt;
    }
    if (err == hipSuccess)
        // without Q_bar, X = a g^T with a = g = 0: M = diag(lam_bar)
        err = band_product(n, lam, Q, ldq, lam_bar, XR, n, zero, zero, d_bar, e_bar, tmp,
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
        err = band_product(n, lam, Q, ldq, lam_bar, nullptr, 0, a, g, d_bar, e_bar, tmp,
                           o_parts, o_flag, status, stream);
    hipError_t e2 = hipFreeAsync(tmp, stream);
    return (int)(err != hipSuccess ? err : e2);
}

// ---- Allocation-free rank-one adjoint ----
// The scratch of dc_stedc_backward_rank1 (the partial band sums, a = Q^T u
// and the equal-eigenvalue flag) in one fixed device array.  On the host its
// name is only a stand-in for the symbol: kernels receive the device address
// that hipGetSymbolAddress returns, looked up once per device.
namespace {

constexpr size_t NOALLOC_SCRATCH = (size_t)16 << 20;     // 16 MiB per device
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;

hipError_t scratch_address(char** out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return err;
    g_scratch_ptr[dev] = static_cast<char*>(p);
    *out = static_cast<char*>(p);
    return hipSuccess;
}

// Scratch bytes of the rank-one adjoint of order n (flag, partial sums, a).
size_t rank1_scratch_bytes(int n, size_t* o_parts, size_t* o_a) {
    size_t o = al(sizeof(int));
    *o_parts = o;
    o = al(o + parts_bytes(n));
    *o_a = o;
    return al(o + (size_t)n * sizeof(double));
}

}  // namespace

extern "C" size_t dc_stedc_backward_rank1_noalloc_max_bytes(void) { return NOALLOC_SCRATCH; }

extern "C" int dc_stedc_backward_rank1_noalloc(int n, const double* lam, const double* Q,
                                               int ldq, const double* lam_bar,
                                               const double* u, const double* g,
                                               double* d_bar, double* e_bar, int* info_dev,
                                               hipStream_t stream) {
    if (n < 0) return -1;
    if (!info_dev) return -10;
    if (n == 0) return (int)dc_fill_int(info_dev, 1, 0, stream);
    if (!lam) return -2;
    if (!Q) return -3;
    if (ldq < n) return -4;
    if (!u) return -6;
    if (!g) return -7;
    if (!d_bar) return -8;
    if (n > 1 && !e_bar) return -9;
    size_t o_parts = 0, o_a = 0;
    if (rank1_scratch_bytes(n, &o_parts, &o_a) > NOALLOC_SCRATCH) return -1;
    char* tmp = nullptr;
    hipError_t err = scratch_address(&tmp);
    if (err != hipSuccess) return (int)err;
    err = dc_fill_int(info_dev, 1, 0, stream);
    if (err != hipSuccess) return (int)err;
    double* a = reinterpret_cast<double*>(tmp + o_a);
    hipLaunchKernelGGL(k_gemv_t, dim3((n + 3) / 4), dim3(256), 0, stream, Q, (long long)ldq, u,
                       a, n);
    err = hipGetLastError();
    if (err == hipSuccess)
        err = band_product(n, lam, Q, ldq, lam_bar, nullptr, 0, a, g, d_bar, e_bar, tmp,
                           o_parts, 0, info_dev, stream);
    return (int)err;
}
