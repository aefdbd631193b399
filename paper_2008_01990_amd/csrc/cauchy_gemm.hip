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
// sub-tile of v_mfma_f64_16x16x4_f64 blocks.  Chunks whose successor is
// interior run in a loop of their own with unguarded loads, issued in the
// order the LDS writes consume them; with the late-write schedule the writes
// sit in the last k-steps, so the loads have most of a chunk to arrive
// before the first wait on them.
//
// Work distribution: one flat grid over the tiles of every task (every merge
// half of a tree level).  Workgroup b runs on XCD b % 8; the flat id is
// remapped so that each XCD runs groups of consecutive tiles (within a task
// the column tile varies fastest, so a group shares A row panels through the
// XCD's L2), with the groups dealt to the XCDs round-robin so that the two
// halves of a merge, whose depths differ, load every XCD alike.
#include "common.hpp"

namespace {

constexpr int WAVE = 64;

template <int BM, int BN, int BK, int WGM, int WGN, int SCHED>
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
    // Register entry i is written to LDS after MFMA k-step slice(i).
    // SCHED 0 spreads the writes over the chunk; SCHED 1 writes U in the
    // last two k-steps and A in the last one, so the global loads of the next
    // chunk have most of a chunk of MFMAs to arrive.
    static constexpr int a_slice(int i) {
        return SCHED == 0 ? i * KSTEPS / A_PER : KSTEPS - 1;
    }
    static constexpr int b_slice(int i) {
        return SCHED == 0 ? i * KSTEPS / B_PER
                          : (KSTEPS >= 2 ? KSTEPS - 2 + (2 * i) / B_PER : 0);
    }
};

__device__ __forceinline__ int find_task(const int* tile_start, int ntasks, int t) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Co-resident workgroups per XCD (32 CUs): the register kernel holds OCC
// waves per SIMD; the LDS kernels are limited by LDS (above 80 KB: one
// workgroup per CU) or by their waves.
template <int WAVES, int OCC>
constexpr int reg_group() { return 32 * (4 * OCC / WAVES > 0 ? 4 * OCC / WAVES : 1); }
template <int BM, int BN, int WAVES, int OCC>
constexpr int lds_group() {
    return (2 * 16 * (BM + BN + 4) * 8 > 80 * 1024 || WAVES == 8) ? 32
           : 32 * (4 * OCC / WAVES > 0 ? 4 * OCC / WAVES : 1);
}

// Flat tile id of workgroup b.  The hardware places workgroup b on XCD b % 8.
// Groups of G consecutive tiles (one XCD's co-resident workgroups, which then
// share A row panels through that XCD's L2) are dealt to the XCDs
// round-robin, so the tiles of every task, and with them the task's depth
// (which only the device knows), spread evenly over the eight XCDs.  The grid
// is a multiple of 8 G.
template <int G>
__device__ __forceinline__ int xcd_tile(int b) {
    const int i = b >> 3;
    return (i / G) * (8 * G) + (b & 7) * G + (i % G);
}

// Tile of a task for its flat local index: the task's full groups are taken
// in transposed order (8 rows of q groups), so the eight groups the XCDs run
// at one time lie q groups apart in the task, not side by side: adjacent row
// panels would put every XCD's loads on the same stretch of each A column.
template <int G>
__device__ __forceinline__ int spread_local(int local, int tiles) {
    const int q = tiles / G / 8;
    const int lg = local / G;
    if (lg >= 8 * q) return local;
    return ((lg & 7) * q + (lg >> 3)) * G + (local - lg * G);
}

template <int BM, int BN, int BK, int WGM, int WGN, int SCHED, int OCC>
__global__ __launch_bounds__(WGM * WGN * 64, OCC)
void k_cauchy_gemm(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_start,
                   int ntasks, int total_tiles) {
    using C_ = Cfg<BM, BN, BK, WGM, WGN, SCHED>;
    __shared__ double As[2][BK * C_::LDA_S];
    __shared__ double Bs[2][BK * C_::LDB_S];

    constexpr int G = lds_group<BM, BN, WGM * WGN, OCC>();
    const int t = xcd_tile<G>(blockIdx.x);
    if (t >= total_tiles) return;
    const int ti = find_task(tile_start, ntasks, t);
    const GemmTask& T = tasks[ti];
    const int local = spread_local<G>(t - tile_start[ti], tile_start[ti + 1] - tile_start[ti]);
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
        cb = T.corg ? rD[T.corg[gcol]] : T.cbase[gcol];
        co = T.coff ? T.coff[gcol] : 0.0;
        csj = T.cs[gcol];
    }

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
    double d_reg[C_::B_PER];    // row nodes
    double z_reg[C_::B_PER];    // row weights

    // Interior chunks of interior tiles (the common case) load without
    // bounds checks, with strength-reduced addresses.
    const bool full_rows = row0 + BM <= T.rows;
    const long long astep = (long long)C_::A_KSTEP * lda;
    auto load_b = [&](int kb, bool interior) {
#pragma unroll
        for (int i = 0; i < C_::B_PER; ++i) {
            const int k = kb + bk0 + i * C_::B_KSTEP;
            const bool ok = interior || k < klen;
            d_reg[i] = ok ? dc_ldg(rD + k) : 0.0;
            z_reg[i] = ok ? dc_ldg(rz + k) : 0.0;
        }
    };
    auto load_a = [&](int kb, bool interior) {
        if (interior) {
            const double* __restrict__ pa = Acol + (long long)(kb + ak0) * lda;
#pragma unroll
            for (int i = 0; i < C_::A_PER; ++i) a_reg[i] = dc_ldg(pa + i * astep);
        } else {
#pragma unroll
            for (int i = 0; i < C_::A_PER; ++i) {
                const int k = kb + ak0 + i * C_::A_KSTEP;
                a_reg[i] = (k < klen && row_ok) ? dc_ldg(Acol + (long long)k * lda) : 0.0;
            }
        }
    };
    auto load = [&](int kb) {
        const bool interior = full_rows && kb + BK <= klen;
        if (SCHED == 0) {
            load_a(kb, interior);
            load_b(kb, interior);
        } else {
            // issued in the order the LDS writes consume them
            load_b(kb, interior);
            load_a(kb, interior);
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
            const double den = (d_reg[i] - cb) - co;
            double v = z_reg[i] * csj * dc_rcp(den);
            v = (kb + kk < klen && col_ok) ? v : 0.0;
            Bs[buf][kk * C_::LDB_S + bj] = v;
        }
    };

    const int nchunks = (klen + BK - 1) / BK;
    load(0);
#pragma unroll
    for (int s = 0; s < C_::KSTEPS; ++s) store_slice(0, 0, s);
    __syncthreads();

    // One chunk: MFMAs from LDS buffer c & 1 while the next chunk's loads
    // land in registers and go to the other buffer between the k-steps.
    // FAST: the next chunk is interior (static loads, no guards).
    auto chunk = [&](int c, auto fast_tag) {
        constexpr bool FAST = decltype(fast_tag)::value;
        const int cur = c & 1;
        const bool more = FAST || c + 1 < nchunks;
        const int kb_next = (c + 1) * BK;
        if (FAST) {
            if (SCHED == 0) {
                load_a(kb_next, true);
                load_b(kb_next, true);
            } else {
                load_b(kb_next, true);
                load_a(kb_next, true);
            }
        } else if (more) {
            load(kb_next);
        }
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
    };
    int c = 0;
    if (SCHED != 0) {
        // chunks whose successor is interior: c + 2 <= klen / BK
        const int nfast = full_rows ? klen / BK - 1 : 0;
        for (; c < nfast; ++c) chunk(c, dc_true_type{});
    }
    for (; c < nchunks; ++c) chunk(c, dc_false_type{});

    // Epilogue: for the FP64 16x16x4 MFMA, accumulator register v of a lane
    // holds row lane/16 + 4 v and column lane % 16 of the 16 x 16 block.
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
}

// Register-pipelined form (no LDS, no barriers): each wave owns a
// (16 FM) x (16 FN) block of C.  Its A operands come straight from global
// memory (per MFMA, 16 consecutive rows at 4 values of k: one 128-byte
// segment per k) and its U operands are generated in registers; a ring of
// RING register slots keeps the loads PD k-steps ahead of the MFMAs.
// Indices are clamped instead of branched on (rows past the tile end are
// computed and not stored, k past klen gets U = 0), so the loop has no
// branches and no waits but the in-order load counter.  Generating U costs
// FP64 VALU time, which the MFMA pipe shares, so each generated entry should
// feed many MFMAs: one entry per FM MFMAs.
// One tile of a task (flat local index `local`); returns early for tiles and
// waves with nothing to compute.
template <int FM, int FN, int WGM, int WGN, int RING, bool P2>
__device__ __forceinline__ void reg_tile(const GemmTask& T, int local) {
    constexpr int WR = 16 * FM, WC = 16 * FN;
    constexpr int BM = WGM * WR, BN = WGN * WC;
    constexpr int PD = RING - 1;
    const int tm = local / T.tiles_n;
    const int tn = local - tm * T.tiles_n;
    const int ncol = T.ncol_p ? *T.ncol_p : T.ncol;
    const int row0 = tm * BM;
    const int col0 = tn * BN;
    if (col0 >= ncol || row0 >= T.rows) return;
    // klen may be 0 (a block with no survivor of this half): without a
    // second phase the tile is then stored as zeros, and nothing is loaded
    // from the generators.
    const int klen = T.klen_p ? *T.klen_p : T.klen;
    const int klen2 = P2 ? T.klen2 : 0;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / WGN, wn = wave - (wave / WGN) * WGN;
    const int lr = lane & 15, lk = lane >> 4;
    const int wrow = row0 + wm * WR;
    const int wcol = col0 + wn * WC;
    // no barriers: waves retire independently; a wave whose rows or columns
    // all lie past the task's end has nothing to store
    if (wrow >= T.rows || wcol >= ncol) return;

    // Column generators of this lane's U columns (clamped; global-space
    // loads: a flat load still pending at the loop header would make every
    // wait in the loop a full drain).
    double cb[FN], co[FN], cs[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int lc = min(wcol + j * 16 + lr, ncol - 1);
        const int g = T.ccol ? dc_ldg(T.ccol + lc) : T.col_off + lc;
        cb[j] = T.corg ? dc_ldg(T.rD + dc_ldg(T.corg + g)) : dc_ldg(T.cbase + g);
        co[j] = T.coff ? dc_ldg(T.coff + g) : 0.0;
        cs[j] = dc_ldg(T.cs + g);
    }
    const double* __restrict__ rD = T.rD;
    const double* __restrict__ rz = T.rz;
    const long long lda = T.lda;

    dc_double4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = dc_double4{0.0, 0.0, 0.0, 0.0};

    // SHIFT (the task has at least WR rows): the wave's rows are moved back
    // inside the matrix if they run past it, so its A rows are one base
    // pointer plus constant offsets; rows computed twice are stored once.
    // Otherwise each row index is clamped on its own.
    auto body = [&](auto shift_tag) {
        constexpr bool SHIFT = decltype(shift_tag)::value;
        const int crow = SHIFT ? min(wrow, T.rows - WR) : wrow;
        const double* __restrict__ Ab = T.A + (SHIFT ? crow + lr : 0);
        const int rlast = T.rows - 1;
        double a[RING][FM], dd[RING], zz[RING];
        auto issue = [&](int slot, int step) {
            const int k = min(step * 4 + lk, klen - 1);
            const double* __restrict__ pk = Ab + (long long)k * lda;
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[slot][i] = dc_ldg(pk + (SHIFT ? i * 16 : min(wrow + i * 16 + lr, rlast)));
            dd[slot] = dc_ldg(rD + k);
            zz[slot] = dc_ldg(rz + k);
        };
        // U entries without the column scale s_n, which the epilogue applies
        // once per output element instead of once per generated entry.
        auto compute = [&](int slot, int step, auto masked_tag) {
            constexpr bool MASKED = decltype(masked_tag)::value;
            const bool kok = step * 4 + lk < klen;
            double bf[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const double v = zz[slot] * dc_rcp3((dd[slot] - cb[j]) - co[j]);
                bf[j] = (!MASKED || kok) ? v : 0.0;
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[slot][i], bf[j],
                                                                     acc[i][j], 0, 0, 0);
        };
        if (!P2 || klen > 0) {
            const int nsteps = (klen + 3) / 4;
            const int nfull = klen / 4;      // steps with every k < klen
#pragma unroll
            for (int s = 0; s < PD; ++s) issue(s, s);
            int s = 0;
            if constexpr (SHIFT) {
                // Steps whose prefetches all lie below klen: no clamp, and
                // running pointers (one 64-bit add per step for the A rows,
                // one each for the row generators) instead of an index
                // product per step; the integer VALU work of a step was ten
                // instructions, which the MFMA pipe waits for as it waits
                // for U's generation.
                const long long kstep = 4 * lda;
                const double* __restrict__ pa = Ab + (long long)(PD * 4 + lk) * lda;
                const double* __restrict__ pdd = rD + PD * 4 + lk;
                const double* __restrict__ pzz = rz + PD * 4 + lk;
                for (; s + 2 * RING - 1 <= nfull; s += RING) {
#pragma unroll
                    for (int j = 0; j < RING; ++j) {
                        const int sl = (j + PD) % RING;
#pragma unroll
                        for (int i = 0; i < FM; ++i) a[sl][i] = dc_ldg(pa + i * 16);
                        dd[sl] = dc_ldg(pdd);
                        zz[sl] = dc_ldg(pzz);
                        pa += kstep;
                        pdd += 4;
                        pzz += 4;
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
                    // keep each step's loads in its step: hoisting them would
                    // make the ring slots overlap and force a wait for every
                    // load in flight
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
        }
        if constexpr (P2) {
          if (klen2 > 0) {
            // Second phase: A2 rows as A, B2 loaded (already divided by the
            // column scale the epilogue applies).
            const double* __restrict__ Ab2 = T.A2 + (SHIFT ? crow + lr : 0);
            const double* __restrict__ B2 = T.B2;
            const long long lda2 = T.lda2, ldb2 = T.ldb2;
            double b2[RING][FN];
            auto issue2 = [&](int slot, int step) {
                const int k = min(step * 4 + lk, klen2 - 1);
                const double* __restrict__ pk = Ab2 + (long long)k * lda2;
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    a[slot][i] = dc_ldg(pk + (SHIFT ? i * 16 : min(wrow + i * 16 + lr, rlast)));
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b2[slot][j] = dc_ldg(B2 + (long long)k * ldb2 +
                                         min(wcol + j * 16 + lr, ncol - 1));
            };
            auto compute2 = [&](int slot, int step, auto masked_tag) {
                constexpr bool MASKED = decltype(masked_tag)::value;
                const bool kok = step * 4 + lk < klen2;
                double bf[FN];
#pragma unroll
                for (int j = 0; j < FN; ++j) bf[j] = (!MASKED || kok) ? b2[slot][j] : 0.0;
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[slot][i], bf[j],
                                                                         acc[i][j], 0, 0, 0);
            };
            const int nsteps = (klen2 + 3) / 4;
            const int nfull = klen2 / 4;
#pragma unroll
            for (int s = 0; s < PD; ++s) issue2(s, s);
            int s = 0;
            if constexpr (SHIFT) {
                // as in the generated phase: unclamped steps on running pointers
                const long long kstep = 4 * lda2, bstep = 4 * ldb2;
                const double* __restrict__ pa = Ab2 + (long long)(PD * 4 + lk) * lda2;
                const double* __restrict__ pb = B2 + (long long)(PD * 4 + lk) * ldb2;
                int bc[FN];
#pragma unroll
                for (int j = 0; j < FN; ++j) bc[j] = min(wcol + j * 16 + lr, ncol - 1);
                for (; s + 2 * RING - 1 <= nfull; s += RING) {
#pragma unroll
                    for (int j = 0; j < RING; ++j) {
                        const int sl = (j + PD) % RING;
#pragma unroll
                        for (int i = 0; i < FM; ++i) a[sl][i] = dc_ldg(pa + i * 16);
#pragma unroll
                        for (int q = 0; q < FN; ++q) b2[sl][q] = dc_ldg(pb + bc[q]);
                        pa += kstep;
                        pb += bstep;
                        compute2(j, s + j, dc_false_type{});
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
            for (; s + RING <= nfull; s += RING) {
#pragma unroll
                for (int j = 0; j < RING; ++j) {
                    issue2((j + PD) % RING, s + j + PD);
                    compute2(j, s + j, dc_false_type{});
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            for (; s < nsteps; s += RING) {
#pragma unroll
                for (int j = 0; j < RING; ++j) {
                    issue2((j + PD) % RING, s + j + PD);
                    compute2(j, s + j, dc_true_type{});
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
          }
        }
        return crow;
    };
    const int crow = (klen <= 0 && (!P2 || klen2 <= 0)) ? wrow
                     : (T.rows >= WR) ? body(dc_true_type{}) : body(dc_false_type{});

#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int c = wcol + j * 16 + lr;
        if (c >= ncol) continue;
        const int g = T.ccol ? T.ccol[c] : T.col_off + c;
        const int oc = T.cpos ? T.cpos[T.ccol ? c : g] : g - T.out_off;
        double* Ccol = T.C + (long long)oc * T.ldc;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = crow + i * 16 + lk + 4 * v;
                if (r >= wrow && r < T.rows) {
                    const double x = acc[i][j][v] * cs[j];
                    Ccol[r] = T.beta ? Ccol[r] + x : x;
                }
            }
        }
    }
}


// total_p (optional): the tile count in device memory (task lists built on
// the device; the grid then covers an upper bound and the rest exit).
template <int FM, int FN, int WGM, int WGN, int RING, int OCC, bool P2>
__global__ __launch_bounds__(WGM * WGN * 64, OCC)
void k_cauchy_gemm_reg(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_start,
                       int ntasks, int total_tiles, const int* __restrict__ total_p) {
    constexpr int G = reg_group<WGM * WGN, OCC>();
    const int t = xcd_tile<G>(blockIdx.x);
    if (t >= (total_p ? *total_p : total_tiles)) return;
    const int ti = find_task(tile_start, ntasks, t);
    reg_tile<FM, FN, WGM, WGN, RING, P2>(
        tasks[ti], spread_local<G>(t - tile_start[ti], tile_start[ti + 1] - tile_start[ti]));
}

template <int FM, int FN, int WGM, int WGN, int RING, int OCC = 2, bool P2 = false>
hipError_t launch_reg(const GemmTask* tasks, const int* tile_start, int ntasks, int total,
                      hipStream_t s, const int* total_p = nullptr) {
    constexpr int G8 = 8 * reg_group<WGM * WGN, OCC>();
    const int grid = (total + G8 - 1) / G8 * G8;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_cauchy_gemm_reg<FM, FN, WGM, WGN, RING, OCC, P2>), dim3(grid),
                       dim3(WGM * WGN * 64), 0, s, tasks, tile_start, ntasks, total, total_p);
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WGM, int WGN, int SCHED, int OCC = 1>
hipError_t launch(const GemmTask* tasks, const int* tile_start, int ntasks, int total,
                  hipStream_t s) {
    constexpr int G8 = 8 * lds_group<BM, BN, WGM * WGN, OCC>();
    const int grid = (total + G8 - 1) / G8 * G8;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((k_cauchy_gemm<BM, BN, BK, WGM, WGN, SCHED, OCC>), dim3(grid),
                       dim3(WGM * WGN * 64), 0, s, tasks, tile_start, ntasks, total);
    return hipGetLastError();
}

hipError_t launch_variant(const GemmTask* tasks, const int* tile_start, int ntasks,
                          int total, int variant, hipStream_t s) {
    // the 128 x 128 LDS kernel runs two workgroups per CU; the 256 x 128 one
    // uses the late-write schedule
    switch (variant) {
        case 1: return launch<128, 128, 16, 2, 2, 0, 2>(tasks, tile_start, ntasks, total, s);
        case 2: return launch<64, 64, 16, 1, 1, 0>(tasks, tile_start, ntasks, total, s);
        case 3: return launch<128, 128, 32, 2, 2, 0>(tasks, tile_start, ntasks, total, s);
        case 4: return launch<256, 128, 16, 4, 2, 1>(tasks, tile_start, ntasks, total, s);
        case 5: return launch_reg<4, 4, 1, 1, 4>(tasks, tile_start, ntasks, total, s);
        default: return launch_reg<8, 2, 1, 4, 3>(tasks, tile_start, ntasks, total, s);
    }
}

}  // namespace

// Tile variants (the host sizes the task tiles by variant): 0 (default)
// 128 x 128, the register-pipelined kernel (waves of 128 x 32); 1: 128 x 128
// LDS kernel, BK 16, two workgroups per CU; 2: 64 x 64 LDS kernel, one wave;
// 3: 128 x 128 LDS kernel, BK 32; 4: 256 x 128 LDS kernel with the
// late-write schedule; 5: 64 x 64, register-pipelined (one 64 x 64 wave).
int dc_gemm_tile_m(int variant) {
    switch (variant) {
        case 2: case 5: return 64;
        case 4: return 256;
        default: return 128;
    }
}

int dc_gemm_tile_n(int variant) {
    switch (variant) {
        case 2: case 5: return 64;
        default: return 128;
    }
}

hipError_t dc_launch_cauchy_gemm(const GemmTask* tasks, const int* tile_start, int ntasks,
                                 int total, int variant, hipStream_t s) {
    return launch_variant(tasks, tile_start, ntasks, total, variant, s);
}

hipError_t dc_launch_cauchy_gemm2(const GemmTask* tasks, const int* tile_start, int ntasks,
                                  int total, int variant, hipStream_t s) {
    if (variant == 5) return launch_reg<4, 4, 1, 1, 4, 2, true>(tasks, tile_start, ntasks, total, s);
    if (variant == 0) return launch_reg<8, 2, 1, 4, 3, 2, true>(tasks, tile_start, ntasks, total, s);
    return hipErrorInvalidValue;
}

hipError_t dc_launch_cauchy_gemm_bounded(const GemmTask* tasks, const int* tile_start,
                                         int ntasks, int max_tiles, const int* total_p,
                                         int variant, bool two_phase, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (variant == 5)
        return two_phase ? launch_reg<4, 4, 1, 1, 4, 2, true>(tasks, tile_start, ntasks,
                                                              max_tiles, s, total_p)
                         : launch_reg<4, 4, 1, 1, 4, 2, false>(tasks, tile_start, ntasks,
                                                               max_tiles, s, total_p);
    if (variant == 0)
        return two_phase ? launch_reg<8, 2, 1, 4, 3, 2, true>(tasks, tile_start, ntasks,
                                                              max_tiles, s, total_p)
                         : launch_reg<8, 2, 1, 4, 3, 2, false>(tasks, tile_start, ntasks,
                                                               max_tiles, s, total_p);
    return hipErrorInvalidValue;
}
