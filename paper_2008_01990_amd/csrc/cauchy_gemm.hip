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
// Layout: A and C column-major; a workgroup owns a BM x BN tile of C and
// streams k in chunks of BK.  Per chunk each thread prefetches into registers
// the A entries and the row generators it will place in LDS, overlapping the
// global loads with the previous chunk's MFMA work; it then writes its A
// entries and the U entries it generates (one reciprocal per entry) to LDS.
// Each wave computes a 64 x 64 sub-tile with v_mfma_f64_16x16x4_f64.
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
    // per-thread share of the A tile and of the U tile
    static constexpr int A_PER = BM * BK / NT;
    static constexpr int B_PER = BN * BK / NT;
    static_assert(BM * BK % NT == 0, "A tile split");
    static_assert(BN * BK % NT == 0, "B tile split");
    static_assert(NT % BM == 0, "A rows per pass");
    static_assert(NT % BN == 0, "B cols per pass");
    static constexpr int A_KSTEP = NT / BM;     // k advance per A pass
    static constexpr int B_KSTEP = NT / BN;
};

__device__ __forceinline__ int find_task(const int* tile_start, int ntasks, int t) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(WGM * WGN * 64)
void k_cauchy_gemm(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_start,
                   int ntasks, int total_tiles) {
    using C_ = Cfg<BM, BN, BK, WGM, WGN>;
    __shared__ double As[BK * C_::LDA_S];
    __shared__ double Bs[BK * C_::LDB_S];

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

    // Column generators of the U entries this thread produces (fixed column).
    const int bj = tid % BN;
    const int bk0 = tid / BN;
    const int gcol = col0 + bj;
    const bool col_ok = gcol < ncol;
    const double cb = col_ok ? (T.corg ? T.rD[T.corg[gcol]] : T.cbase[gcol]) : 0.0;
    const double co = (col_ok && T.coff) ? T.coff[gcol] : 0.0;
    const double csj = col_ok ? T.cs[gcol] : 0.0;

    // A entries this thread loads: row ar, k = ak0 + i * A_KSTEP.
    const int ar = tid % BM;
    const int ak0 = tid / BM;
    const int grow = row0 + ar;
    const bool row_ok = grow < T.rows;

    dc_double4 acc[C_::FM][C_::FN];
#pragma unroll
    for (int i = 0; i < C_::FM; ++i)
#pragma unroll
        for (int j = 0; j < C_::FN; ++j) acc[i][j] = dc_double4{0.0, 0.0, 0.0, 0.0};

    double a_reg[C_::A_PER];
    double d_reg[C_::B_PER];
    double z_reg[C_::B_PER];

    auto prefetch = [&](int kb) {
#pragma unroll
        for (int i = 0; i < C_::A_PER; ++i) {
            const int k = kb + ak0 + i * C_::A_KSTEP;
            double v = 0.0;
            if (k < klen && row_ok) {
                const int g = T.klist ? T.klist[k] : k;
                const int c = T.acol ? T.acol[g] : g;
                v = T.A[(long long)c * T.lda + grow];
            }
            a_reg[i] = v;
        }
#pragma unroll
        for (int i = 0; i < C_::B_PER; ++i) {
            const int k = kb + bk0 + i * C_::B_KSTEP;
            double dv = 0.0, zv = 0.0;
            if (k < klen) {
                const int g = T.klist ? T.klist[k] : k;
                dv = T.rD[g];
                zv = T.rz[g];
            }
            d_reg[i] = dv;
            z_reg[i] = zv;
        }
    };

    prefetch(0);
    for (int kb = 0; kb < klen; kb += BK) {
        // Registers -> LDS: A as loaded, U generated.
#pragma unroll
        for (int i = 0; i < C_::A_PER; ++i)
            As[(ak0 + i * C_::A_KSTEP) * C_::LDA_S + ar] = a_reg[i];
#pragma unroll
        for (int i = 0; i < C_::B_PER; ++i) {
            const int kk = bk0 + i * C_::B_KSTEP;
            const double den = (d_reg[i] - cb) - co;
            double v = z_reg[i] * csj * dc_rcp(den);
            v = (kb + kk < klen && col_ok) ? v : 0.0;
            Bs[kk * C_::LDB_S + bj] = v;
        }
        __syncthreads();
        if (kb + BK < klen) prefetch(kb + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[C_::FM], bf[C_::FN];
            const int kr = kk + (lane >> 4);
#pragma unroll
            for (int i = 0; i < C_::FM; ++i)
                af[i] = As[kr * C_::LDA_S + wm * C_::WTM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < C_::FN; ++j)
                bf[j] = Bs[kr * C_::LDB_S + wn * C_::WTN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < C_::FM; ++i)
#pragma unroll
                for (int j = 0; j < C_::FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    // Epilogue: for the FP64 16x16x4 MFMA, accumulator register v of a lane
    // holds row lane/16 + 4 v and column lane % 16 of the 16 x 16 block.
#pragma unroll
    for (int j = 0; j < C_::FN; ++j) {
        const int c = col0 + wn * C_::WTN + j * 16 + (lane & 15);
        if (c >= ncol) continue;
        const int oc = T.cpos ? T.cpos[c] : c;
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
}

template <int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch(const GemmTask* tasks, const int* tile_start, int ntasks, int total,
                  hipStream_t s) {
    int grid = (total + 7) & ~7;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_cauchy_gemm<BM, BN, BK, WGM, WGN>), dim3(grid),
                       dim3(WGM * WGN * 64), 0, s, tasks, tile_start, ntasks, total);
    return hipGetLastError();
}

}  // namespace

int dc_gemm_tile_m(int variant) {
    switch (variant) {
        case 2: return 64;
        default: return 128;
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
    switch (variant) {
        case 2: return launch<64, 64, 32, 1, 1>(tasks, tile_start, ntasks, total, s);
        case 3: return launch<128, 128, 32, 2, 2>(tasks, tile_start, ntasks, total, s);
        default: return launch<128, 128, 16, 2, 2>(tasks, tile_start, ntasks, total, s);
    }
}
