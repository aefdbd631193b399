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
//   general Q_bar:  G^T = Q_bar^T Q (an MFMA product that reads both operands
//                   down their columns: no transpose) -> P = Q M with band
//                   epilogue: 4 n^3 flops.
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

// Tile of workgroup b in a tiles_m x tiles_n grid.  Each XCD (the hardware
// places workgroup b on XCD b % 8) gets a contiguous range of the order;
// the order runs over groups of GM tile rows, column by column within a
// group, so the workgroups an XCD runs together cover a near-square patch
// (8 rows x 8 columns for 64 of them) and share both operand panels in its
// L2.  Returns false for grid padding.
template <int GM>
__device__ __forceinline__ bool grouped_tile(int b, int tiles_m, int tiles_n, int& tm, int& tn) {
    const int total = tiles_m * tiles_n;
    const int per_xcd = (total + 7) / 8;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= total || (b >> 3) >= per_xcd) return false;
    const int g = t / (GM * tiles_n);
    const int rows = min(GM, tiles_m - g * GM);
    const int w = t - g * GM * tiles_n;
    tn = w / rows;
    tm = g * GM + (w - tn * rows);
    return true;
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

// d_bar_i = sum_p pd[p][i], e_bar_i = sum_p (pu[p][i] + pl[p][i+1]) over the
// column groups p, in a fixed order: a workgroup takes 32 rows; its eight
// lanes per row sum the groups p = g, g + 8, ... (g = 0..7) in increasing
// p, and the eight partial sums are added in order of g.
constexpr int RED_ROWS = 32, RED_SPLIT = 8;
__global__ __launch_bounds__(RED_ROWS * RED_SPLIT)
void k_band_reduce(const double* __restrict__ pd, const double* __restrict__ pu,
                   const double* __restrict__ pl, int nparts, int n,
                   double* __restrict__ dbar, double* __restrict__ ebar) {
    __shared__ double sd_g[RED_SPLIT][RED_ROWS], se_g[RED_SPLIT][RED_ROWS];
    const int r = threadIdx.x % RED_ROWS, g = threadIdx.x / RED_ROWS;
    const int i = blockIdx.x * RED_ROWS + r;
    double sd = 0.0, se = 0.0;
    if (i < n) {
        for (int p = g; p < nparts; p += RED_SPLIT) {
            const long long o = (long long)p * n;
            sd += pd[o + i];
            if (i + 1 < n) se += pu[o + i] + pl[o + i + 1];
        }
    }
    sd_g[g][r] = sd;
    se_g[g][r] = se;
    __syncthreads();
    if (g == 0 && i < n) {
        double td = 0.0, te = 0.0;
#pragma unroll
        for (int q = 0; q < RED_SPLIT; ++q) {
            td += sd_g[q][r];
            te += se_g[q][r];
        }
        dbar[i] = td;
        if (i + 1 < n) ebar[i] = te;
    }
}

// distinct = 1 if lam is strictly increasing (then no two eigenvalues are
// equal and the band kernel's instance without the equality test runs),
// else 0 (unsorted, equal or NaN entries: the instance with the test).
__global__ __launch_bounds__(1024)
void k_check_distinct(const double* __restrict__ lam, int n, int* __restrict__ distinct) {
    int bad = 0;
    for (int i = threadIdx.x; i + 1 < n; i += 1024) bad |= !(lam[i] < lam[i + 1]);
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *distinct = !bad;
}

// With lam not strictly increasing: flag = 1 if two entries are equal (any
// order; one thread per entry against all the others).
__global__ __launch_bounds__(256)
void k_equal_pairs(const double* __restrict__ lam, int n, const int* __restrict__ distinct,
                   int* __restrict__ flag) {
    if (*distinct) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double v = lam[i];
    bool eq = false;
    for (int j = 0; j < n; ++j) eq |= j != i && lam[j] == v;
    if (eq) atomicOr(flag, 1);
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
//     M_kc = lbar_c if k == c, 0 if lam_c == lam_k (k_equal_pairs sets the
//            status flag), X_kc / (lam_c - lam_k) otherwise,
// X_kc = XR[k ldx + c] (LOADED: G stored row-major) or a_k g_c (rank one).
// The epilogue reduces each row of the wave's block of P against rows r,
// r + 1 and r - 1 of Q over its columns and writes one partial sum per
// (column group, row): the column group is wcol / (16 FN), and exactly one
// wave writes each (group, row).
// DISTINCT: the instance for strictly increasing lam (k_check_distinct),
// which needs no test for equal eigenvalues: off the diagonal every
// lam_c - lam_k is non-zero.  Both instances are launched; each returns at
// once unless the device flag selects it.
template <int FM, int FN, int WGN, int RING, bool LOADED, bool DISTINCT>
__global__ __launch_bounds__(WGN * 64, 2)
void k_band_reg(int n, const double* __restrict__ Q, long long ldq,
                const double* __restrict__ lam, const double* __restrict__ lbar,
                const double* __restrict__ XR, long long ldx, const double* __restrict__ av,
                const double* __restrict__ gv, double* __restrict__ pd, double* __restrict__ pu,
                double* __restrict__ pl, int tiles_m, int tiles_n,
                const int* __restrict__ distinct) {
    constexpr int WR = 16 * FM, WC = 16 * FN, BN = WGN * WC;
    constexpr int PD = RING - 1;
    if ((*distinct != 0) != DISTINCT) return;
    int tm, tn;
    if (!grouped_tile<8>(blockIdx.x, tiles_m, tiles_n, tm, tn)) return;
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
                    double v = x * dc_rcp3(den);
                    if constexpr (!DISTINCT) v = den == 0.0 ? 0.0 : v;
                    // (DISTINCT: den is 0 only on the diagonal, replaced here,
                    // and for k past n or columns past n, never used)
                    v = diag ? lb[j] : v;
                    bf[j] = (!MASKED || kok) ? v : 0.0;
                }
            } else {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const double den = lc[j] - dk[slot];
                    const double x = LOADED ? xk[slot][j] : xk[slot][0] * gc[j];
                    const double v = x * dc_rcp3(den);
                    bf[j] = (DISTINCT || den != 0.0) ? v : 0.0;
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
        if constexpr (SHIFT) {
            // Steps whose prefetches all lie below n: no clamp, running
            // pointers instead of an index product per step (the MFMA pipe
            // waits for integer VALU work as for the generation of M).
            const long long kstep = 4 * ldq, xstep = 4 * ldx;
            const double* __restrict__ pa = Ab + (long long)(PD * 4 + lk) * ldq;
            const double* __restrict__ pl = lam + PD * 4 + lk;
            const double* __restrict__ px = LOADED ? XR + (long long)(PD * 4 + lk) * ldx : av + PD * 4 + lk;
            int xc[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j) xc[j] = min(cix[j], n - 1);
            for (; s + 2 * RING - 1 <= nfull; s += RING) {
#pragma unroll
                for (int j = 0; j < RING; ++j) {
                    const int sl = (j + PD) % RING;
#pragma unroll
                    for (int i = 0; i < FM; ++i) a[sl][i] = dc_ldg(pa + i * 16);
                    dk[sl] = dc_ldg(pl);
                    if constexpr (LOADED) {
#pragma unroll
                        for (int q = 0; q < FN; ++q) xk[sl][q] = dc_ldg(px + xc[q]);
                        px += xstep;
                    } else {
                        xk[sl][0] = dc_ldg(px);
                        px += 4;
                    }
                    pa += kstep;
                    pl += 4;
                    compute(j, s + j, dc_false_type{});
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
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
}

// C = A^T B for column-major A (K x M, lda) and B (K x N, ldb); C is M x N,
// column-major (ldc).  Both operands are read down their columns, where k
// is contiguous: within a chunk of 8 values of k, lane (r, q) of a wave
// (r = lane % 16, q = lane / 16) loads k = 2q and 2q + 1 of its column (one
// 16-byte load when VEC), and the chunk's two MFMA steps take them in turn.
// An MFMA step contracts over the k its four lane rows hold; any assignment
// of k to (lane, step) that both operands share gives the same sum, so no
// transpose of either operand is needed.  Waves own 16 FM x 16 FN blocks of
// C (M >= 16 FM, N >= 16 FN); a wave's window is moved back inside the
// matrix where it would run past it (the rows or columns computed twice are
// stored once), so every load address is a wave-uniform base plus one
// per-lane offset.  A ring of RING chunk slots keeps the loads RING - 1
// chunks ahead.
typedef double dc_double2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const dc_double2 dc_gdouble2;

template <int FM, int FN, int WGM, int WGN, int RING, bool VEC>
__global__ __launch_bounds__(WGM * WGN * 64, 2)
void k_gemm_tn(int M, int N, int K, const double* __restrict__ A, long long lda,
               const double* __restrict__ B, long long ldb, double* __restrict__ C,
               long long ldc, int tiles_m, int tiles_n) {
    constexpr int WR = 16 * FM, WC = 16 * FN, BM = WGM * WR, BN = WGN * WC;
    constexpr int PD = RING - 1;
    int tm, tn;
    if (!grouped_tile<8>(blockIdx.x, tiles_m, tiles_n, tm, tn)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WGN, wn = wave - (wave / WGN) * WGN;
    const int lr = lane & 15, lq = lane >> 4;
    const int i0 = tm * BM + wm * WR, j0 = tn * BN + wn * WC;
    if (i0 >= M || j0 >= N) return;          // no barriers: waves retire independently
    const int ib = min(i0, M - WR), jb = min(j0, N - WC);
    const double* __restrict__ A0 = A + (long long)ib * lda;
    const double* __restrict__ B0 = B + (long long)jb * ldb;
    const long long oa = (long long)lr * lda + 2 * lq, ob = (long long)lr * ldb + 2 * lq;
    dc_double4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = dc_double4{0.0, 0.0, 0.0, 0.0};
    dc_double2 av[RING][FM], bv[RING][FN];
    auto ld2 = [&](const double* p) -> dc_double2 {
        if constexpr (VEC) return *(dc_gdouble2*)p;
        return dc_double2{dc_ldg(p), dc_ldg(p + 1)};
    };
    // chunk c (every k < K)
    auto issue = [&](int slot, int c) {
        const int kc = c * 8;
#pragma unroll
        for (int i = 0; i < FM; ++i) av[slot][i] = ld2(A0 + (long long)i * 16 * lda + kc + oa);
#pragma unroll
        for (int j = 0; j < FN; ++j) bv[slot][j] = ld2(B0 + (long long)j * 16 * ldb + kc + ob);
    };
    auto compute = [&](int slot) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[slot][i][s], bv[slot][j][s],
                                                                     acc[i][j], 0, 0, 0);
    };
    const int nfull = K / 8;                    // chunks with every k < K
#pragma unroll
    for (int c = 0; c < PD; ++c)
        if (c < nfull) issue(c, c);
    int c = 0;
    for (; c + RING + PD <= nfull; c += RING) {
#pragma unroll
        for (int j = 0; j < RING; ++j) {
            issue((j + PD) % RING, c + j + PD);
            compute(j);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    for (; c < nfull; c += RING) {
#pragma unroll
        for (int j = 0; j < RING; ++j) {
            if (c + j + PD < nfull) issue((j + PD) % RING, c + j + PD);
            if (c + j < nfull) compute(j);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (nfull * 8 < K) {
        // the last, partial chunk: k past K reads row K - 1 and counts 0
        const int k0 = nfull * 8 + 2 * lq;
        const bool v0 = k0 < K, v1 = k0 + 1 < K;
        const long long d0 = min(k0, K - 1) - 2 * lq, d1 = min(k0 + 1, K - 1) - 2 * lq;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const double* p = A0 + (long long)i * 16 * lda + oa;
            av[0][i] = dc_double2{v0 ? dc_ldg(p + d0) : 0.0, v1 ? dc_ldg(p + d1) : 0.0};
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const double* p = B0 + (long long)j * 16 * ldb + ob;
            bv[0][j] = dc_double2{v0 ? dc_ldg(p + d0) : 0.0, v1 ? dc_ldg(p + d1) : 0.0};
        }
        compute(0);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = jb + j * 16 + lr;
        if (col < j0) continue;
        double* Cc = C + (long long)col * ldc;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = ib + i * 16 + lq + 4 * v;
                if (r >= i0) Cc[r] = acc[i][j][v];
            }
    }
}

// The same product for matrices smaller than one wave's window: one thread
// per entry of C.
__global__ void k_gemm_tn_small(int M, int N, int K, const double* __restrict__ A, long long lda,
                                const double* __restrict__ B, long long ldb,
                                double* __restrict__ C, long long ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= M || j >= N) return;
    const double* a = A + (long long)i * lda;
    const double* b = B + (long long)j * ldb;
    double s = 0.0;
    for (int k = 0; k < K; ++k) s = __builtin_fma(a[k], b[k], s);
    C[(long long)j * ldc + i] = s;
}

constexpr int TFM = 4, TFN = 4, TWGM = 2, TWGN = 2, TRING = 2;

// G^T = Q_bar^T Q (n x n, column-major, ld n) on the TN kernel.
hipError_t gemm_tn(int n, const double* Qb, long long ldqb, const double* Q, long long ldq,
                   double* Gt, hipStream_t s) {
    constexpr int BM = TWGM * 16 * TFM, BN = TWGN * 16 * TFN;
    if (n < 16 * TFM || n < 16 * TFN) {
        hipLaunchKernelGGL(k_gemm_tn_small, dim3((n + 63) / 64, n), dim3(64), 0, s, n, n, n, Qb,
                           ldqb, Q, ldq, Gt, (long long)n);
        return hipGetLastError();
    }
    const int tiles_m = (n + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    const int grid = (tiles_m * tiles_n + 7) / 8 * 8;
    const bool vec = ldqb % 2 == 0 && ldq % 2 == 0 &&
                     (reinterpret_cast<uintptr_t>(Qb) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL((k_gemm_tn<TFM, TFN, TWGM, TWGN, TRING, true>), dim3(grid),
                           dim3(TWGM * TWGN * 64), 0, s, n, n, n, Qb, ldqb, Q, ldq, Gt,
                           (long long)n, tiles_m, tiles_n);
    else
        hipLaunchKernelGGL((k_gemm_tn<TFM, TFN, TWGM, TWGN, TRING, false>), dim3(grid),
                           dim3(TWGM * TWGN * 64), 0, s, n, n, n, Qb, ldqb, Q, ldq, Gt,
                           (long long)n, tiles_m, tiles_n);
    return hipGetLastError();
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
    int* distinct = flag + 1;                  // (the flag's slot holds 256 bytes)
    hipError_t err = dc_fill_int(flag, 1, 0, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_check_distinct, dim3(1), dim3(1024), 0, s, lam, n, distinct);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_equal_pairs, dim3((n + 255) / 256), dim3(256), 0, s, lam, n, distinct,
                       flag);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int grid = (tiles_m * tiles_n + 7) / 8 * 8;
    auto launch = [&](auto loaded, auto dist) {
        hipLaunchKernelGGL((k_band_reg<BFM, BFN, BWGN, BRING, decltype(loaded)::value,
                                       decltype(dist)::value>),
                           dim3(grid), dim3(BWGN * 64), 0, s, n, Q, ldq, lam, lam_bar, XR, ldx,
                           a, g, pd, pu, pl, tiles_m, tiles_n, distinct);
        return hipGetLastError();
    };
    if (XR) {
        err = launch(dc_true_type{}, dc_true_type{});
        if (err == hipSuccess) err = launch(dc_true_type{}, dc_false_type{});
    } else {
        err = launch(dc_false_type{}, dc_true_type{});
        if (err == hipSuccess) err = launch(dc_false_type{}, dc_false_type{});
    }
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_band_reduce, dim3((n + RED_ROWS - 1) / RED_ROWS),
                       dim3(RED_ROWS * RED_SPLIT), 0, s, pd, pu, pl, nparts, n, d_bar, e_bar);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_flag_to_status, dim3(1), dim3(64), 0, s, flag, status);
    return hipGetLastError();
}

size_t parts_bytes(int n) {
    return 3 * (size_t)((n + BAND_WC - 1) / BAND_WC) * n * sizeof(double);
}

}  // namespace

namespace {

// Workspace of the general adjoint: the equal-eigenvalue flag, the partial
// band sums, a zero vector (the rank-one generators of M when there is no
// Q_bar) and G^T = Q_bar^T Q (with Q_bar).
struct BwLayout {
    size_t flag, parts, zero, g, bytes;
};

BwLayout bw_layout(int n, bool with_qbar) {
    BwLayout L;
    size_t o = 0;
    L.flag = o; o = al(o + sizeof(int));
    L.parts = o; o = al(o + parts_bytes(n));
    L.zero = o; o = al(o + (size_t)n * sizeof(double));
    L.g = o; o = al(o + (with_qbar ? (size_t)n * n * sizeof(double) : 0));
    L.bytes = o;
    return L;
}

int backward_check(int n, const double* lam, const double* Q, int ldq, const double* Q_bar,
                   int ldqb, const double* d_bar, const double* e_bar) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    if (!lam) return -2;
    if (!Q) return -3;
    if (ldq < n) return -4;
    if (Q_bar && ldqb < n) return -7;
    if (!d_bar) return -8;
    if (n > 1 && !e_bar) return -9;
    return 0;
}

// G^T = Q_bar^T Q on the TN kernel (both operands read down their columns),
// then P = Q M with the band epilogue.  Launches only.
hipError_t backward_run(int n, const double* lam, const double* Q, int ldq,
                        const double* lam_bar, const double* Q_bar, int ldqb, double* d_bar,
                        double* e_bar, char* w, const BwLayout& L, int* status,
                        hipStream_t s) {
    double* zero = reinterpret_cast<double*>(w + L.zero);
    hipError_t err = hipSuccess;
    if (!Q_bar) {
        hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, zero, (long long)n,
                           0.0);
        err = hipGetLastError();
    }
    const double* XR = nullptr;
    if (err == hipSuccess && Q_bar) {
        double* Gt = reinterpret_cast<double*>(w + L.g);
        err = gemm_tn(n, Q_bar, ldqb, Q, ldq, Gt, s);
        XR = Gt;       // G^T column-major is G row-major, as the band kernel reads it
    }
    if (err == hipSuccess)
        // without Q_bar, X = a g^T with a = g = 0: M = diag(lam_bar)
        err = band_product(n, lam, Q, ldq, lam_bar, XR, n, zero, zero, d_bar, e_bar, w,
                           L.parts, L.flag, status, s);
    return err;
}

}  // namespace

extern "C" size_t dc_stedc_backward_workspace(int n, int with_qbar) {
    if (n < 0) return 0;
    return bw_layout(n, with_qbar != 0).bytes;
}

extern "C" int dc_stedc_backward_ex(int n, const double* lam, const double* Q, int ldq,
                                    const double* lam_bar, const double* Q_bar, int ldqb,
                                    double* d_bar, double* e_bar, void* work, size_t lwork,
                                    int* info_dev, hipStream_t stream) {
    const int bad = backward_check(n, lam, Q, ldq, Q_bar, ldqb, d_bar, e_bar);
    if (bad || n < 0) return bad;
    if (!info_dev) return -12;
    if (n == 0) return (int)dc_fill_int(info_dev, 1, 0, stream);
    const BwLayout L = bw_layout(n, Q_bar != nullptr);
    if (!work || (reinterpret_cast<uintptr_t>(work) & 255) != 0) return -10;
    if (lwork < L.bytes) return -11;
    hipError_t err = dc_fill_int(info_dev, 1, 0, stream);
    if (err == hipSuccess)
        err = backward_run(n, lam, Q, ldq, lam_bar, Q_bar, ldqb, d_bar, e_bar,
                           static_cast<char*>(work), L, info_dev, stream);
    return (int)err;
}

extern "C" int dc_stedc_backward(int n, const double* lam, const double* Q, int ldq,
                                 const double* lam_bar, const double* Q_bar, int ldqb,
                                 double* d_bar, double* e_bar, hipStream_t stream) {
    const int bad = backward_check(n, lam, Q, ldq, Q_bar, ldqb, d_bar, e_bar);
    if (bad || n <= 0) return bad;
    int* status = nullptr;
    hipError_t err = dc_status_word(stream, &status);
    if (err != hipSuccess) return (int)err;
    err = dc_fill_int(status, 1, 0, stream);
    if (err != hipSuccess) return (int)err;
    const BwLayout L = bw_layout(n, Q_bar != nullptr);
    char* tmp = nullptr;
    err = hipMallocAsync((void**)&tmp, L.bytes, stream);
    if (err != hipSuccess) return (int)err;
    err = backward_run(n, lam, Q, ldq, lam_bar, Q_bar, ldqb, d_bar, e_bar, tmp, L, status,
                       stream);
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
