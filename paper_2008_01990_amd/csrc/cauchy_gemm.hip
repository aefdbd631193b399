// Generated-tile FP64 MFMA product C = A * B with B a Cauchy-like matrix
// formed from its generators tile by tile in LDS and never written to HBM.
//
// This is the merge-step eigenvector update of eq. updateV / eq. evect,
// Q_new = Q_nd * U with U_ij = zhat_i s_j / ((D_i - D_{o_j}) - tau_j)
// (eq. Q_Cauchy, Remark 3), and the local product of Algorithm 2 step 3(b)-(c)
// in which each process builds the B sub-block it needs from the generators
// instead of receiving it (the paper's "main observation").  On one GPU the
// observation is taken to its end: no tile of U ever leaves LDS.
//
// A (the deflated basis panel) is a plain column-major matrix: the driver
// gathers the survivor columns into a contiguous panel before the product,
// so a tile load is one coalesced column segment per k and no index chases
// sit in front of the MFMA pipe.
//
// Pipeline: a workgroup owns a BM x BN tile of C and walks k in chunks of BK
// through two LDS buffers.  While the waves run the MFMAs of chunk c from one
// buffer, each thread holds the global loads of chunk c+1 in registers and
// writes them (A as loaded, U generated with one reciprocal per entry) into
// the other buffer in slices placed between the MFMA groups, so the matrix
// cores stay fed; one barrier per chunk.  Each wave owns a WTM x WTN
// sub-tile of v_mfma_f64_16x16x4_f64 blocks.
//
// Work distribution: one flat grid over the tiles of every task (every merge
// half of a tree level).  Workgroup b runs on XCD b % 8; the flat id is
// remapped so that each XCD owns a contiguous range of tiles, and within a
// task the column tile varies fastest, so the workgroups resident on one XCD
// share A row panels through that XCD's L2.
#include "common.hpp"

namespace {

constexpr int WAVE = 64;

template <int BM, int BN, int BK, int WGM, int WGN>
struct Cfg {
    static constexpr int NT = WGM * WGN * WAVE;
    static constexpr int WTM = BM / WGM;        // rows per wave
    static constexpr int WTN = BN / WGN;        // cols per wave
    static constexpr int FM = WTM / 16;         // MFMA blocks per wave (rows)
    static constexpr int FN = WTN / 16;
    static constexpr int PADA = 2;
    static constexpr int PADB = 2;
    static constexpr int LDA_S = BM + PADA;
    static constexpr int LDB_S = BN + PADB;
    static constexpr int A_PER = BM * BK / NT;  // A entries per thread per chunk
    static constexpr int B_PER = BN * BK / NT;  // U entries per thread per chunk
    static constexpr int A_KSTEP = NT / BM;
    static constexpr int B_KSTEP = NT / BN;
    static constexpr int KSTEPS = BK / 4;       // MFMA k-steps per chunk
    static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "tile split");
    static_assert(NT % BM == 0 && NT % BN == 0, "rows per pass");
    // register entry i is written to LDS after MFMA k-step slice(i)
    static constexpr int a_slice(int i) { return i * KSTEPS / A_PER; }
    static constexpr int b_slice(int i) { return i * KSTEPS / B_PER; }
};

__device__ __forceinline__ int find_task(const int* tile_start, int ntasks, int t) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int KIND, int EPI, int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(WGM * WGN * 64)
void k_cauchy_gemm(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_start,
                   int ntasks, int total_tiles) {
    using C_ = Cfg<BM, BN, BK, WGM, WGN>;
    __shared__ double As[2][BK * C_::LDA_S];
    __shared__ double Bs[2][BK * C_::LDB_S];

    // XCD-aware flat id (grid size is a multiple of 8).
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int t = (b & 7) * (nb >> 3) + (b >> 3);
    if (t >= total_tiles) return;
    const int ti = find_task(tile_start, ntasks, t);
    const GemmTask& T = tasks[ti];
    const int local = t - tile_start[ti];
    const int tm = local / T.tiles_n;
    const int tn = local - tm * T.tiles_n;
    const int ncol = T.ncol_p ? *T.ncol_p : T.ncol;
    const int row0 = tm * BM;
    const int col0 = tn * BN;
    if (col0 >= ncol || row0 >= T.rows) return;
    const int klen = T.klen_p ? *T.klen_p : T.klen;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WGN;
    const int wn = wave - wm * WGN;

    // Column generators of the B entries this thread produces (fixed column).
    const int bj = tid % BN;
    const int bk0 = tid / BN;
    const int lcol = col0 + bj;
    const bool col_ok = lcol < ncol;
    const int gcol = col_ok ? (T.ccol ? T.ccol[lcol] : T.col_off + lcol) : 0;
    const double* __restrict__ rD = T.rD;
    const double* __restrict__ rz = T.rz;
    double cb = 0.0, co = 0.0, csj = 0.0;
    if (col_ok) {
        if (KIND <= 1) {
            cb = (KIND == 0 && T.corg) ? rD[T.corg[gcol]] : T.cbase[gcol];
            co = T.coff ? T.coff[gcol] : 0.0;
        }
        if (KIND == 0) csj = T.cs[gcol];
        if (KIND == 3) {
            cb = T.lam[gcol];                       // lam_c
            co = T.lbar ? T.lbar[gcol] : 0.0;       // lbar_c
            csj = T.Bm ? 0.0 : T.cs[gcol];          // g_c of a rank-one X
        }
    }
    bool equal_eig = false;

    // A entries this thread moves: row ar, k = ak0 + i * A_KSTEP.
    const int ar = tid % BM;
    const int ak0 = tid / BM;
    const bool row_ok = row0 + ar < T.rows;
    const double* __restrict__ Acol = T.A + row0 + ar;
    const long long lda = T.lda;

    dc_double4 acc[C_::FM][C_::FN];
#pragma unroll
    for (int i = 0; i < C_::FM; ++i)
#pragma unroll
        for (int j = 0; j < C_::FN; ++j) acc[i][j] = dc_double4{0.0, 0.0, 0.0, 0.0};

    double a_reg[C_::A_PER];
    double d_reg[C_::B_PER];    // 0: row node; 1: y * vk; 2: B entry; 3: X entry
    double z_reg[C_::B_PER];    // 0: row weight; 1: skeleton node base; 3: lam_k
    double o_reg[KIND == 1 ? C_::B_PER : 1];   // kind 1: skeleton node offset
    int s_reg[KIND == 1 ? C_::B_PER : 1];      // kind 1: skeleton column (generator)

    // Interior chunks of interior tiles (the common case) load without
    // bounds checks, with strength-reduced addresses.
    const bool full_rows = row0 + BM <= T.rows;
    const long long astep = (long long)C_::A_KSTEP * lda;
    auto load = [&](int kb) {
        if (full_rows && kb + BK <= klen) {
            const double* __restrict__ pa = Acol + (long long)(kb + ak0) * lda;
#pragma unroll
            for (int i = 0; i < C_::A_PER; ++i) a_reg[i] = dc_ldg(pa + i * astep);
            if (KIND == 0) {
#pragma unroll
                for (int i = 0; i < C_::B_PER; ++i) {
                    const int k = kb + bk0 + i * C_::B_KSTEP;
                    d_reg[i] = dc_ldg(rD + k);
                    z_reg[i] = dc_ldg(rz + k);
                }
                return;
            }
        } else {
#pragma unroll
            for (int i = 0; i < C_::A_PER; ++i) {
                const int k = kb + ak0 + i * C_::A_KSTEP;
                a_reg[i] = (k < klen && row_ok) ? dc_ldg(Acol + (long long)k * lda) : 0.0;
            }
        }
#pragma unroll
        for (int i = 0; i < C_::B_PER; ++i) {
            const int k = kb + bk0 + i * C_::B_KSTEP;
            const bool ok = k < klen;
            if (KIND == 0) {
                d_reg[i] = ok ? dc_ldg(rD + k) : 0.0;
                z_reg[i] = ok ? dc_ldg(rz + k) : 0.0;
            } else if (KIND == 1) {
                const int h = ok ? dc_ldg(T.rgen + k) : 0;
                d_reg[i] = (ok && col_ok) ? dc_ldg(T.ry + k) * dc_ldg(T.vk + T.rvo[k] + lcol) : 0.0;
                z_reg[i] = ok ? dc_ldg(T.cbase + h) : 0.0;
                o_reg[i] = (ok && T.coff) ? dc_ldg(T.coff + h) : 0.0;
                s_reg[i] = ok ? h : -1;
            } else if (KIND == 2) {
                d_reg[i] = (ok && col_ok) ? dc_ldg(T.Bm + (long long)gcol * T.ldb + k) : 0.0;
            } else {
                d_reg[i] = (ok && col_ok)
                               ? (T.Bm ? dc_ldg(T.Bm + (long long)gcol * T.ldb + k)
                                       : dc_ldg(rz + k) * csj)
                               : 0.0;
                z_reg[i] = ok ? dc_ldg(T.lam + k) : 0.0;
            }
        }
    };
    // Store slice s of the registers into LDS buffer `buf` (B generated).
    auto store_slice = [&](int buf, int kb, int s) {
#pragma unroll
        for (int i = 0; i < C_::A_PER; ++i) {
            if (C_::a_slice(i) != s) continue;
            As[buf][(ak0 + i * C_::A_KSTEP) * C_::LDA_S + ar] = a_reg[i];
        }
#pragma unroll
        for (int i = 0; i < C_::B_PER; ++i) {
            if (C_::b_slice(i) != s) continue;
            const int kk = bk0 + i * C_::B_KSTEP;
            double v;
            if (KIND == 0) {
                const double den = (d_reg[i] - cb) - co;
                v = z_reg[i] * csj * dc_rcp(den);
            } else if (KIND == 1) {
                const double den = (z_reg[i] - cb) + (o_reg[i] - co);
                v = (s_reg[i] == gcol) ? 1.0 : d_reg[i] * dc_rcp(den);
            } else if (KIND == 2) {
                v = d_reg[i];
            } else {
                const double den = cb - z_reg[i];          // lam_c - lam_k
                if (kb + kk == gcol) {
                    v = co;                                // lbar_c
                } else if (den == 0.0) {
                    v = 0.0;
                    equal_eig |= (kb + kk < klen && col_ok);
                } else {
                    v = d_reg[i] * dc_rcp(den);
                }
            }
            v = (kb + kk < klen && col_ok) ? v : 0.0;
            Bs[buf][kk * C_::LDB_S + bj] = v;
        }
    };

    const int nchunks = (klen + BK - 1) / BK;
    load(0);
#pragma unroll
    for (int s = 0; s < C_::KSTEPS; ++s) store_slice(0, 0, s);
    __syncthreads();

    for (int c = 0; c < nchunks; ++c) {
        const int cur = c & 1;
        const bool more = c + 1 < nchunks;
        const int kb_next = (c + 1) * BK;
        if (more) load(kb_next);
#pragma unroll
        for (int ks = 0; ks < C_::KSTEPS; ++ks) {
            double af[C_::FM], bf[C_::FN];
            const int kr = ks * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < C_::FM; ++i)
                af[i] = As[cur][kr * C_::LDA_S + wm * C_::WTM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < C_::FN; ++j)
                bf[j] = Bs[cur][kr * C_::LDB_S + wn * C_::WTN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < C_::FM; ++i)
#pragma unroll
                for (int j = 0; j < C_::FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j],
                                                                     0, 0, 0);
            if (more) store_slice(cur ^ 1, kb_next, ks);
        }
        __syncthreads();
    }

    // Epilogue: for the FP64 16x16x4 MFMA, accumulator register v of a lane
    // holds row lane/16 + 4 v and column lane % 16 of the 16 x 16 block.
    if (EPI == 0) {
#pragma unroll
        for (int j = 0; j < C_::FN; ++j) {
            const int c = col0 + wn * C_::WTN + j * 16 + (lane & 15);
            if (c >= ncol) continue;
            const int g = T.ccol ? T.ccol[c] : T.col_off + c;
            const int oc = T.cpos ? T.cpos[T.ccol ? c : g] : g - T.out_off;
            double* Ccol = T.C + (long long)oc * T.ldc;
#pragma unroll
            for (int i = 0; i < C_::FM; ++i) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = row0 + wm * C_::WTM + i * 16 + (lane >> 4) + 4 * v;
                    if (r < T.rows) {
                        const double x = acc[i][j][v];
                        Ccol[r] = T.beta ? Ccol[r] + x : x;
                    }
                }
            }
        }
    } else {
        // Band epilogue: row sums of P o Q, P o Q(+1 row), P o Q(-1 row).
        const int part = tn * WGN + wn;
        const long long ldq = T.ldqb;
#pragma unroll
        for (int i = 0; i < C_::FM; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = row0 + wm * C_::WTM + i * 16 + (lane >> 4) + 4 * v;
                double sd = 0.0, su = 0.0, sl = 0.0;
                if (r < T.rows) {
#pragma unroll
                    for (int j = 0; j < C_::FN; ++j) {
                        const int c = col0 + wn * C_::WTN + j * 16 + (lane & 15);
                        if (c >= ncol) continue;
                        const double x = acc[i][j][v];
                        const double* q = T.Qb + (long long)c * ldq + r;
                        sd += x * q[0];
                        if (r + 1 < T.nband) su += x * q[1];
                        if (r > 0) sl += x * q[-1];
                    }
                }
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) {
                    sd += __shfl_xor(sd, off, 64);
                    su += __shfl_xor(su, off, 64);
                    sl += __shfl_xor(sl, off, 64);
                }
                if ((lane & 15) == 0 && r < T.rows) {
                    const long long o = (long long)part * T.nband + r;
                    T.pd[o] = sd;
                    T.pu[o] = su;
                    T.pl[o] = sl;
                }
            }
        }
    }
    if (KIND == 3 && equal_eig && T.flag) atomicOr(T.flag, 1);
}

template <int KIND, int EPI, int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch(const GemmTask* tasks, const int* tile_start, int ntasks, int total,
                  hipStream_t s) {
    int grid = (total + 7) & ~7;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_cauchy_gemm<KIND, EPI, BM, BN, BK, WGM, WGN>), dim3(grid),
                       dim3(WGM * WGN * 64), 0, s, tasks, tile_start, ntasks, total);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_variant(const GemmTask* tasks, const int* tile_start, int ntasks,
                          int total, int variant, hipStream_t s) {
    switch (variant) {
        case 1: return launch<KIND, 0, 128, 128, 16, 2, 2>(tasks, tile_start, ntasks, total, s);
        case 2: return launch<KIND, 0, 64, 64, 16, 1, 1>(tasks, tile_start, ntasks, total, s);
        case 3: return launch<KIND, 0, 128, 128, 32, 2, 2>(tasks, tile_start, ntasks, total, s);
        default: return launch<KIND, 0, 256, 128, 16, 4, 2>(tasks, tile_start, ntasks, total, s);
    }
}

}  // namespace

// Tile variants: 0 (default) 256 x 128, BK 16, 4 x 2 waves (two waves per
// SIMD); 1: 128 x 128, BK 16, 2 x 2 waves; 2: 64 x 64, BK 16, one wave;
// 3: 128 x 128, BK 32, 2 x 2 waves.
int dc_gemm_tile_m(int variant) {
    switch (variant) {
        case 1: case 3: return 128;
        case 2: return 64;
        default: return 256;
    }
}

int dc_gemm_tile_n(int variant) {
    switch (variant) {
        case 2: return 64;
        default: return 128;
    }
}

hipError_t dc_launch_cauchy_gemm(const GemmTask* tasks, const int* tile_start, int ntasks,
                                 int total, int variant, hipStream_t s) {
    return launch_variant<0>(tasks, tile_start, ntasks, total, variant, s);
}

hipError_t dc_launch_interp_gemm(const GemmTask* tasks, const int* tile_start, int ntasks,
                                 int total, int variant, hipStream_t s) {
    return launch_variant<1>(tasks, tile_start, ntasks, total, variant, s);
}

hipError_t dc_launch_loaded_gemm(const GemmTask* tasks, const int* tile_start, int ntasks,
                                 int total, hipStream_t s) {
    return launch<2, 0, 256, 128, 16, 4, 2>(tasks, tile_start, ntasks, total, s);
}

hipError_t dc_launch_adjoint_gemm(const GemmTask* tasks, const int* tile_start, int ntasks,
                                  int total, hipStream_t s) {
    return launch<3, 1, 256, 128, 16, 4, 2>(tasks, tile_start, ntasks, total, s);
}

int dc_band_waves_n() { return 2; }
