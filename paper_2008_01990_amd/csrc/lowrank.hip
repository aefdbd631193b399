// Structured low-rank merge product: SRRSC compression of the off-diagonal
// blocks of U from their Cauchy generators, then two generated products.
//
// Compression (section "SRRSC low-rank approximation"): U is cut into
// contiguous b x b blocks of the sorted order (block data distribution, which
// keeps the off-diagonal low-rank property; section "Storage form affects the
// off-diagonally low-rank property").  One workgroup per off-diagonal block
// runs Schur-complement elimination on the generators alone (Theorem 1): with
// the pivot (row node d_k, column node w_k) the generators update as
//     u_l <- u_l (d_l - d_k) / (d_l - w_k),   v_l <- v_l (w_l - w_k) / (w_l - d_k),
// which also zeroes the pivot row and column, so the next complete-pivoting
// search simply scans the whole block again.  Elimination stops when every
// Schur-complement entry is at most tol.  The pivot columns are the skeleton
// T, and the interpolation matrix Z = A11^{-1} A12 is Cauchy-like with row
// generator y (eq. yk) and column generator v^(r) (Theorem 2, eq. geneZ).
// A block whose rank would exceed rmax is kept dense.
//
// Products (Algorithm 2 step 3(c), C += (A U_B) V_B, restated for one GPU):
//   1  W(:, T_IJ) = A(:, I) U_I,T_IJ                 skeleton columns, all J != I
//   2  C(:, J) = A(:, J) U_JJ + [W(:, T_IJ)]_I [I Z_IJ]_I P^T
// Step 2 is one launch of the register MFMA kernel with two k-phases per
// tile: the diagonal block with U_JJ generated, then W's columns of block J
// against the interpolation rows Y_J = [I Z_IJ]_I P^T, which are formed once
// per merge from (y, v^(r), nodes) into a small dense array (sum of ranks x b)
// and loaded.  C is written once.  A block kept dense is carried as a block
// whose skeleton is every column (identity interpolation rows).  W is laid
// out by output block J, so each J reads one contiguous column range of W
// and of Y.  U and Z never exist as matrices; W and Y are m x (sum of ranks)
// and (sum of ranks) x b.  The merges of one tree level go together: all
// compressions first (one read of all ranks), then one launch of step 1 and
// one of step 2 for every merge of the level.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

#include "dc_internal.hpp"
#include "driver.hpp"
#include "lowrank.hpp"

namespace {

constexpr int NT = 1024;
constexpr int MAX_B_OFF = 2048;   // block size limit with column offsets (merge nodes)
constexpr int MAX_B_GEN = 4096;   // block size limit with plain column nodes
constexpr int MAX_R = 128;

struct SrrscOut {
    int* rank;        // p*p: rank, -1 on the diagonal, -2 kept dense
    int* prow;        // p*p*rmax, local pivot rows
    int* pcol;        // p*p*rmax, local skeleton columns
    double* y;        // p*p*rmax
    double* vk;       // p*p*b: v^(r) of the block's columns (0 on skeletons)
};

// One compression of a launch: K nodes in p x p blocks, the generators and
// the outputs.  A launch runs the blocks of several jobs (the merges of a
// tree level): job j owns blocks [start[j], start[j + 1]) of the grid.
struct SrrscJob {
    int K, p;
    const double* D;
    const double* u0;
    const double* cbase;
    const double* coff;
    const double* v0;
    SrrscOut O;
};

// One workgroup per block (I, J).  MB: LDS capacity in generators; OFF: the
// column nodes carry an offset (w_j = cbase_j + coff_j, the merge's (origin,
// tau) form); STORE: write the skeleton and interpolation generators, else only
// count the rank (up to rmax).
template <int MB, int RG, bool OFF, bool STORE>
__global__ __launch_bounds__(NT)
void k_srrsc(const SrrscJob* __restrict__ jobs, const int* __restrict__ start, int njobs, int b,
             double tol, int rmax) {
    constexpr int JJ = (MB * RG + NT - 1) / NT;   // columns per thread
    __shared__ double sd[MB], su[MB], swb[MB], sv[MB];
    __shared__ double swo[OFF ? MB : 1];
    __shared__ double wv[NT / 64], wd[NT / 64];
    __shared__ int wi[NT / 64];
    __shared__ int spr[STORE ? MAX_R : 1], spc[STORE ? MAX_R : 1];

    int jlo = 0, jhi = njobs - 1;
    while (jlo < jhi) {
        const int mid = (jlo + jhi + 1) >> 1;
        if (start[mid] <= (int)blockIdx.x) jlo = mid; else jhi = mid - 1;
    }
    const SrrscJob& job = jobs[jlo];
    const int K = job.K, p = job.p;
    const double* __restrict__ D = job.D;
    const double* __restrict__ u0 = job.u0;
    const double* __restrict__ cbase = job.cbase;
    const double* __restrict__ coff = job.coff;
    const double* __restrict__ v0 = job.v0;
    const SrrscOut O = job.O;
    const int pair = blockIdx.x - start[jlo];
    const int I = pair / p, J = pair - (pair / p) * p;
    const int tid = threadIdx.x;
    if (I == J) {
        if (tid == 0) O.rank[pair] = -1;
        return;
    }
    const int r0 = I * b, c0 = J * b;
    const int bi = min(b, K - r0), bj = min(b, K - c0);
    for (int i = tid; i < bi; i += NT) {
        sd[i] = D[r0 + i];
        su[i] = u0[r0 + i];
    }
    for (int j = tid; j < bj; j += NT) {
        swb[j] = cbase[c0 + j];
        if constexpr (OFF) swo[j] = coff[c0 + j];
        sv[j] = v0[c0 + j];
    }
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    int k = 0;
    bool dense = false;
    for (;;) {
        // Complete pivoting: largest |A^(k)_ij| = |u_i v_j| / |d_i - w_j|,
        // ties to the smallest row-major position.  The threads form RG row
        // groups of NT / RG column slots (RG > 1 when the block has at most
        // NT / RG columns); a thread holds its columns in registers and walks
        // the rows of its group, so its own candidates arrive in increasing
        // position order.  The running maximum is kept as a fraction
        // (|u v|, |d - w|) and compared by cross-multiplication: no division
        // per entry.
        const int slots = NT / RG;
        const int cs = tid % slots, rg = tid / slots;
        double cw[JJ], co[JJ], cv[JJ];
#pragma unroll
        for (int t = 0; t < JJ; ++t) {
            const int j = cs + t * slots;
            const bool ok = j < bj;
            cw[t] = ok ? swb[j] : 0.0;
            co[t] = (OFF && ok) ? swo[j] : 0.0;
            cv[t] = ok ? fabs(sv[j]) : 0.0;     // 0 => never a candidate
        }
        // Leaders start at 0 / 1: padded slots (v = 0) and zeroed pivot rows
        // and columns never become candidates; the loop stops at tol > 0
        // anyway.  Even and odd rows of the group keep separate leaders (two
        // independent compare-select chains), merged by value then position.
        double bn = 0.0, bd = 1.0, bn1 = 0.0, bd1 = 1.0;
        int bf = INT_MAX, bf1 = INT_MAX;
        auto scan_row = [&](int i, double& n_, double& d_, int& f_) {
            const double di = sd[i], ui = fabs(su[i]);
#pragma unroll
            for (int t = 0; t < JJ; ++t) {
                if (t * slots >= bj) break;     // uniform over the workgroup
                const double a = ui * cv[t];
                const double x = fabs((di - cw[t]) - co[t]);
                const bool take = a * d_ > n_ * x;
                n_ = take ? a : n_;
                d_ = take ? x : d_;
                f_ = take ? i * bj + cs + t * slots : f_;
            }
        };
        int i = rg;
        for (; i + RG < bi; i += 2 * RG) {
            scan_row(i, bn, bd, bf);
            scan_row(i + RG, bn1, bd1, bf1);
        }
        if (i < bi) scan_row(i, bn, bd, bf);
        auto better = [](double n1, double d1, int f1, double n0, double d0, int f0) {
            const double l = n1 * d0, r = n0 * d1;
            return l > r || (l == r && f1 < f0);
        };
        if (better(bn1, bd1, bf1, bn, bd, bf)) { bn = bn1; bd = bd1; bf = bf1; }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double on = __shfl_xor(bn, off, 64);
            const double od = __shfl_xor(bd, off, 64);
            const int of = __shfl_xor(bf, off, 64);
            if (better(on, od, of, bn, bd, bf)) { bn = on; bd = od; bf = of; }
        }
        if (lane == 0) { wv[w] = bn; wd[w] = bd; wi[w] = bf; }
        __syncthreads();
        // Every wave reduces the NT / 64 wave results itself (same values,
        // same order: the same pivot everywhere), so no second barrier.
        {
            constexpr int NWV = NT / 64;
            double nn = lane < NWV ? wv[lane] : 0.0;
            double dd = lane < NWV ? wd[lane] : 1.0;
            int ff = lane < NWV ? wi[lane] : INT_MAX;
#pragma unroll
            for (int off = NWV / 2; off > 0; off >>= 1) {
                const double on = __shfl_xor(nn, off, 64);
                const double od = __shfl_xor(dd, off, 64);
                const int of = __shfl_xor(ff, off, 64);
                if (better(on, od, of, nn, dd, ff)) { nn = on; dd = od; ff = of; }
            }
            bn = __shfl(nn, 0, 64);
            bd = __shfl(dd, 0, 64);
            bf = __shfl(ff, 0, 64);
        }
        const double pmax = bn / bd;
        if (!(pmax > tol)) break;
        if (k == rmax) { dense = true; break; }
        const int pi = bf / bj;
        const int pj = bf - pi * bj;
        if constexpr (STORE) {
            if (tid == 0) { spr[k] = pi; spc[k] = pj; }
        }
        const double dk = sd[pi], wbk = swb[pj];
        const double wok = OFF ? swo[pj] : 0.0;
        // Theorem 1 generator updates (the pivot row and column become 0).
        for (int i = tid; i < bi; i += NT)
            su[i] *= (sd[i] - dk) * dc_rcp((sd[i] - wbk) - wok);
        for (int j = tid; j < bj; j += NT) {
            const double wo = OFF ? swo[j] : 0.0;
            sv[j] *= ((swb[j] - wbk) + (wo - wok)) * dc_rcp((swb[j] - dk) + wo);
        }
        ++k;
        __syncthreads();
    }
    if (tid == 0) O.rank[pair] = dense ? -2 : k;
    if constexpr (STORE) {
        if (dense) {
            // every column becomes a skeleton column: v^(r) = 0 throughout
            for (int j = tid; j < bj; j += NT) O.vk[(long long)pair * b + j] = 0.0;
            return;
        }
        const long long pb = (long long)pair * rmax;
        // Theorem 2, eq. yk: y_a = prod_{c != a} (d_c - w_a)/(w_c - w_a) * (d_a - w_a)/v0_a.
        for (int a = tid; a < k; a += NT) {
            const int ja = spc[a];
            const double wba = swb[ja], woa = OFF ? swo[ja] : 0.0;
            double y = 1.0;
            for (int c = 0; c < k; ++c) {
                if (c == a) continue;
                const double woc = OFF ? swo[spc[c]] : 0.0;
                const double num = (sd[spr[c]] - wba) - woa;
                const double den = (swb[spc[c]] - wba) + (woc - woa);
                y *= num * dc_rcp(den);
            }
            y *= ((sd[spr[a]] - wba) - woa) * dc_rcp(v0[c0 + ja]);
            O.y[pb + a] = y;
            O.prow[pb + a] = spr[a];
            O.pcol[pb + a] = ja;
        }
        for (int j = tid; j < bj; j += NT) O.vk[(long long)pair * b + j] = sv[j];
    }
}

__global__ void k_nodes(int K, const double* D, const int* org, const double* tau,
                        double* cbase, double* coff) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    if (org) {
        cbase[j] = D[org[j]];
        coff[j] = tau[j];
    } else {
        cbase[j] = tau[j];
        coff[j] = 0.0;
    }
}

// Interpolation rows [I Z_IJ] P^T of the low-rank blocks, one row per W
// column k (Theorem 2, eq. geneZ): for output column c of block column
// J = kJ[k], generator g = J b + c, the entry is 1 on the skeleton column
// itself (g == rgen[k]) and y_k v^(r)_c / (w_h - w_g) otherwise.  Stored
// row-major, Y[k b + c], divided by the column scale s_g that the product's
// epilogue multiplies back; 0 past the block's last column.
__global__ void k_build_y(long long nw, int b, int K, const double* __restrict__ ry,
                          const int* __restrict__ rgen, const long long* __restrict__ rvo,
                          const int* __restrict__ kJ, const double* __restrict__ vk,
                          const double* __restrict__ cbase, const double* __restrict__ coff,
                          const double* __restrict__ scale, double* __restrict__ Y) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nw * b) return;
    const long long k = idx / b;
    const int c = (int)(idx - k * b);
    const int g = kJ[k] * b + c;
    if (g >= K) {
        Y[idx] = 0.0;
        return;
    }
    const int h = rgen[k];
    double v = 1.0;
    if (h != g) {
        const double den = (cbase[h] - cbase[g]) + (coff ? coff[h] - coff[g] : 0.0);
        v = ry[k] * vk[rvo[k] + c] / den;
    }
    Y[idx] = v / scale[g];
}

// Column layout of the low-rank product from the SRRSC output, one
// workgroup per block pair (I, J), I != J, whose skeleton has r columns (its
// rank, or every column of block J when kept dense): W column woff + a and
// stage-1b list slot loff + a (a < r) get the skeleton column's generator
// index, the pair's v^(r) row offset, the block column J and y_a (0 for a
// dense block, whose interpolation rows are the identity).
__global__ void k_layout(int p, int b, int K, int rmax, const int* __restrict__ rank,
                         const int* __restrict__ pcol, const double* __restrict__ y,
                         const long long* __restrict__ woff, const int* __restrict__ loff,
                         int* __restrict__ rgen, long long* __restrict__ rvo,
                         int* __restrict__ kJ, double* __restrict__ ry,
                         int* __restrict__ ccol, int* __restrict__ wpos) {
    const int pair = blockIdx.x;
    const int I = pair / p, J = pair - (pair / p) * p;
    if (I == J) return;
    const int rk = rank[pair];
    const bool dense = rk == -2;
    const int r = dense ? min(b, K - J * b) : rk;
    for (int a = threadIdx.x; a < r; a += blockDim.x) {
        const long long col = woff[pair] + a;
        const int h = J * b + (dense ? a : pcol[(long long)pair * rmax + a]);
        rgen[col] = h;
        rvo[col] = (long long)pair * b;
        kJ[col] = J;
        ry[col] = dense ? 0.0 : y[(long long)pair * rmax + a];
        ccol[loff[pair] + a] = h;
        wpos[loff[pair] + a] = (int)col;
    }
}

__global__ void k_disable_tasks(GemmTask* tasks, int n, const int* zero) {
    const int i = threadIdx.x;
    if (i < n) tasks[i].ncol_p = zero;
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Compressed {
    int p = 0, b = 0, rmax = 0;
    std::vector<int> rank;
    char* dev = nullptr;          // device block holding SrrscOut arrays (not owned)
    SrrscOut out{};
};

// The SRRSC instance for a job list: column offsets present (merge nodes, b
// up to MAX_B_OFF) or plain column nodes (b up to MAX_B_GEN); store or count
// only.
template <int MB, int RG, bool OFF>
hipError_t launch_srrsc_mb(const SrrscJob* jobs, const int* start, int njobs, int blocks, int b,
                           double tol, int rmax, bool store, hipStream_t s) {
    const dim3 g((unsigned)blocks), blk(NT);
    if (store)
        hipLaunchKernelGGL((k_srrsc<MB, RG, OFF, true>), g, blk, 0, s, jobs, start, njobs, b,
                           tol, rmax);
    else
        hipLaunchKernelGGL((k_srrsc<MB, RG, OFF, false>), g, blk, 0, s, jobs, start, njobs, b,
                           tol, rmax);
    return hipGetLastError();
}

// The smallest LDS capacity that holds b (two workgroups per CU up to
// b = 1024), with the rows split among 4 or 2 thread groups when b <= 256 or
// 512.
template <bool OFF>
hipError_t launch_srrsc_off(const SrrscJob* jobs, const int* start, int njobs, int blocks,
                            int b, double tol, int rmax, bool store, hipStream_t s) {
    if (b <= 256)
        return launch_srrsc_mb<256, 4, OFF>(jobs, start, njobs, blocks, b, tol, rmax, store, s);
    if (b <= 512)
        return launch_srrsc_mb<512, 2, OFF>(jobs, start, njobs, blocks, b, tol, rmax, store, s);
    if (b <= 1024)
        return launch_srrsc_mb<1024, 1, OFF>(jobs, start, njobs, blocks, b, tol, rmax, store,
                                             s);
    if (b <= MAX_B_OFF)
        return launch_srrsc_mb<MAX_B_OFF, 1, OFF>(jobs, start, njobs, blocks, b, tol, rmax,
                                                  store, s);
    if constexpr (!OFF)
        return launch_srrsc_mb<MAX_B_GEN, 1, false>(jobs, start, njobs, blocks, b, tol, rmax,
                                                    store, s);
    return hipErrorInvalidValue;
}

hipError_t launch_srrsc(const SrrscJob* jobs, const int* start, int njobs, int blocks, int b,
                        bool offsets, double tol, int rmax, bool store, hipStream_t s) {
    if (offsets && b > MAX_B_OFF) return hipErrorInvalidValue;
    if (b > MAX_B_GEN) return hipErrorInvalidValue;
    if (blocks <= 0 || njobs <= 0) return hipSuccess;
    return offsets ? launch_srrsc_off<true>(jobs, start, njobs, blocks, b, tol, rmax, store, s)
                   : launch_srrsc_off<false>(jobs, start, njobs, blocks, b, tol, rmax, store, s);
}

// A job list in device memory: `dev` holds job_bytes(n) bytes; the list and
// the block prefix are uploaded, and the grid's block count returned.
size_t job_bytes(size_t n) {
    return al(n * sizeof(SrrscJob)) + al((n + 1) * sizeof(int));
}

hipError_t upload_jobs(const std::vector<SrrscJob>& jobs, char* dev, hipStream_t s,
                       const SrrscJob** jobs_dev, const int** start_dev, int* blocks) {
    const size_t n = jobs.size();
    std::vector<int> start(n + 1, 0);
    for (size_t i = 0; i < n; ++i) start[i + 1] = start[i] + jobs[i].p * jobs[i].p;
    std::vector<char> h(job_bytes(n));
    const size_t so = al(n * sizeof(SrrscJob));
    if (n) std::memcpy(h.data(), jobs.data(), n * sizeof(SrrscJob));
    std::memcpy(h.data() + so, start.data(), (n + 1) * sizeof(int));
    *jobs_dev = reinterpret_cast<const SrrscJob*>(dev);
    *start_dev = reinterpret_cast<const int*>(dev + so);
    *blocks = start[n];
    return dc_upload(dev, h.data(), h.size(), s);
}

// coff == nullptr: plain column nodes w_j = cbase_j.
// Bytes of the SRRSC output of a K-node problem in b x b blocks.
size_t compress_bytes(int K, int b) {
    const size_t p = (K + b - 1) / b, p2 = p * p;
    const size_t rmax = std::min(MAX_R, std::max(1, b / 2));
    return al(p2 * sizeof(int)) + 2 * al(p2 * rmax * sizeof(int)) +
           al(p2 * rmax * sizeof(double)) + al(p2 * (size_t)b * sizeof(double));
}

// The SRRSC job of every off-diagonal block, its output in `dev`
// (compress_bytes(K, b) bytes); the caller launches it and reads the ranks
// back (Cm.rank is sized for them).
SrrscJob compress_prepare(int K, int b, const double* D, const double* zhat,
                          const double* cbase, const double* coff, const double* scale,
                          Compressed& Cm, char* dev) {
    Cm.b = b;
    Cm.p = (K + b - 1) / b;
    Cm.rmax = std::min(MAX_R, std::max(1, b / 2));
    const size_t p2 = (size_t)Cm.p * Cm.p;
    size_t o = 0;
    const size_t o_rank = o; o = al(o + p2 * sizeof(int));
    const size_t o_prow = o; o = al(o + p2 * Cm.rmax * sizeof(int));
    const size_t o_pcol = o; o = al(o + p2 * Cm.rmax * sizeof(int));
    const size_t o_y = o; o = al(o + p2 * Cm.rmax * sizeof(double));
    Cm.dev = dev;
    Cm.out.rank = reinterpret_cast<int*>(Cm.dev + o_rank);
    Cm.out.prow = reinterpret_cast<int*>(Cm.dev + o_prow);
    Cm.out.pcol = reinterpret_cast<int*>(Cm.dev + o_pcol);
    Cm.out.y = reinterpret_cast<double*>(Cm.dev + o_y);
    Cm.out.vk = reinterpret_cast<double*>(Cm.dev + o);
    Cm.rank.resize(p2);
    return SrrscJob{K, Cm.p, D, zhat, cbase, coff, scale, Cm.out};
}

// Device-side task list of one launch, with its tile prefix.
struct Stage {
    std::vector<GemmTask> tasks;
    std::vector<int> start{0};
    void add(const GemmTask& t) {
        if (t.tiles_m * t.tiles_n == 0) return;
        tasks.push_back(t);
        start.push_back(start.back() + t.tiles_m * t.tiles_n);
    }
};

}  // namespace

// Device buffers of the low-rank product, kept per host thread and device
// for the process and grown on demand: stream-ordered allocation, and above
// all freeing, cost several hundred microseconds of host time per merge.
// Each use is ordered after the previous one: on the same stream by stream
// order, on another stream through an event recorded after the last use.
enum { SL_SRRSC, SL_LAYOUT, SL_W, SL_Y, SL_TASKS, NSLOT };
struct Arena {
    char* p[NSLOT] = {};
    size_t cap[NSLOT] = {};
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
};

Arena& arena() {
    thread_local std::map<int, Arena> per_device;
    int dev = 0;
    (void)hipGetDevice(&dev);
    return per_device[dev];
}

hipError_t arena_begin(Arena& A, hipStream_t s) {
    return (A.used && A.last != s) ? hipStreamWaitEvent(s, A.ev, 0) : hipSuccess;
}

hipError_t arena_get(Arena& A, int slot, size_t n, char** out) {
    if (n > A.cap[slot]) {
        if (A.p[slot]) {
            // earlier work may still read the old buffer (rare: growth)
            hipError_t err = hipDeviceSynchronize();
            if (err == hipSuccess) err = hipFree(A.p[slot]);
            if (err != hipSuccess) return err;
            A.p[slot] = nullptr;
            A.cap[slot] = 0;
        }
        const size_t want = n + n / 4;
        hipError_t err = hipMalloc((void**)&A.p[slot], want);
        if (err != hipSuccess) return err;
        A.cap[slot] = want;
    }
    *out = A.p[slot];
    return hipSuccess;
}

hipError_t arena_end(Arena& A, hipStream_t s) {
    if (!A.ev) {
        hipError_t err = hipEventCreateWithFlags(&A.ev, hipEventDisableTiming);
        if (err != hipSuccess) return err;
    }
    A.last = s;
    A.used = true;
    return hipEventRecord(A.ev, s);
}

namespace {

LrRankSummary rank_summary(const Compressed& Cm) {
    LrRankSummary R;
    const int p = Cm.p;
    for (int I = 0; I < p; ++I)
        for (int J = 0; J < p; ++J) {
            if (I == J) continue;
            const int r = Cm.rank[(size_t)I * p + J];
            ++R.blocks;
            if (r == -2) { ++R.dense; continue; }
            R.rank_sum += r;
            R.rank_max = std::max(R.rank_max, r);
        }
    return R;
}

// Host layout of one compressed merge's products, from the ranks alone (the
// skeleton columns and y stay on the device): W by output block J,
// [W_IJ for I != J], r_IJ columns each; the stage-1b column list of block
// row I, [T_IJ for J != I].  Its uploaded arrays (per-pair offsets) and its
// device-filled arrays (per W column: skeleton generator, v^(r) row, block
// column, y; the stage-1b lists) have places in the level's layout slot,
// and W and Y places in the level's W and Y slots.
struct MergePlan {
    int p = 0;
    std::vector<long long> gstart, woff;
    std::vector<int> loff, lstart;
    long long NW = 0;
    size_t up_off = 0, dev_off = 0;               // bytes, in the layout slot
    size_t o_wo = 0, o_lo = 0, up_bytes = 0;      // inside the uploaded part
    size_t o_ry = 0, o_rg = 0, o_rv = 0, o_kj = 0, o_cc = 0, o_wp = 0, dev_bytes = 0;
    size_t w_off = 0, y_off = 0;                  // elements, in the W and Y slots
};

void plan_layout(const Compressed& Cm, int K, int b, MergePlan& P) {
    const int p = Cm.p;
    P.p = p;
    auto bsz = [&](int I) { return std::min(b, K - I * b); };
    // Skeleton size of block (I, J): its rank, or every column if kept dense.
    auto rk = [&](int I, int J) {
        const int r = Cm.rank[(size_t)I * p + J];
        return r == -2 ? bsz(J) : r;
    };
    P.gstart.assign(p + 1, 0);
    P.woff.assign((size_t)p * p, 0);
    P.loff.assign((size_t)p * p, 0);
    P.lstart.assign(p + 1, 0);
    for (int J = 0; J < p; ++J) {
        long long run = 0;
        for (int I = 0; I < p; ++I)
            if (I != J && rk(I, J) > 0) { P.woff[(size_t)I * p + J] = P.gstart[J] + run; run += rk(I, J); }
        P.gstart[J + 1] = P.gstart[J] + run;
    }
    for (int I = 0; I < p; ++I) {
        int run = 0;
        for (int J = 0; J < p; ++J)
            if (I != J && rk(I, J) > 0) { P.loff[(size_t)I * p + J] = P.lstart[I] + run; run += rk(I, J); }
        P.lstart[I + 1] = P.lstart[I] + run;
    }
    P.NW = P.gstart[p];
    const size_t p2 = (size_t)p * p;
    const size_t nw1 = (size_t)std::max<long long>(P.NW, 1);
    size_t o = 0;
    P.o_wo = o; o = al(o + p2 * sizeof(long long));
    P.o_lo = o; o = al(o + p2 * sizeof(int));
    P.up_bytes = o;
    o = 0;
    P.o_ry = o; o = al(o + nw1 * sizeof(double));
    P.o_rg = o; o = al(o + nw1 * sizeof(int));
    P.o_rv = o; o = al(o + nw1 * sizeof(long long));
    P.o_kj = o; o = al(o + nw1 * sizeof(int));
    P.o_cc = o; o = al(o + nw1 * sizeof(int));
    P.o_wp = o; o = al(o + nw1 * sizeof(int));
    P.dev_bytes = o;
}

// The products of one merge as tasks of the level's two launches: (1b) the
// skeleton columns into W; then per output block J, the diagonal block
// A(:, J) U_JJ (generated) and W_J Y_J (loaded Y) accumulated in the same
// tile, so C is written once.
void add_tasks(const MergePlan& P, int K, int b, const double* cbase, const double* coff,
               const double* scale, const std::vector<LrHalf>& halves, int wrows,
               double* W, const double* Y, const int* d_ccol, const int* d_wpos, int fv,
               int sv, Stage& s1b, Stage& sf, double* flops_out) {
    const int p = P.p;
    const int BMf = dc_gemm_tile_m(fv), BNf = dc_gemm_tile_n(fv);
    const int BMs = dc_gemm_tile_m(sv), BNs = dc_gemm_tile_n(sv);
    auto bsz = [&](int I) { return std::min(b, K - I * b); };
    double flops = 0.0;
    auto tiles = [&](GemmTask& t, int bm, int bn) {
        t.tiles_m = (t.rows + bm - 1) / bm;
        t.tiles_n = (t.ncol + bn - 1) / bn;
    };
    for (const LrHalf& H : halves) {
        if (H.rows <= 0) continue;
        std::vector<int> lo(p), hi(p);
        for (int I = 0; I < p; ++I) {
            if (H.klist.empty()) {
                lo[I] = I * b;
                hi[I] = I * b + bsz(I);
            } else {
                lo[I] = (int)(std::lower_bound(H.klist.begin(), H.klist.end(), I * b) -
                              H.klist.begin());
                hi[I] = (int)(std::lower_bound(H.klist.begin(), H.klist.end(), I * b + b) -
                              H.klist.begin());
            }
        }
        GemmTask base;
        std::memset(&base, 0, sizeof(base));
        base.lda = H.lda;
        base.rows = H.rows;
        base.cbase = cbase;
        base.coff = coff;
        base.cs = scale;
        for (int I = 0; I < p; ++I) {
            GemmTask t = base;
            t.A = H.A + (long long)lo[I] * H.lda;
            t.klen = hi[I] - lo[I];
            t.rD = H.gD + lo[I];
            t.rz = H.gz + lo[I];
            // diagonal block straight into C, plus the interpolation phase
            GemmTask a = t;
            a.col_off = I * b;
            a.ncol = bsz(I);
            a.C = H.C;
            a.ldc = H.ldc;
            a.cpos = H.cpos;
            a.beta = 0;
            const long long R = P.gstart[I + 1] - P.gstart[I];
            if (R > 0) {
                a.A2 = W + H.w_row0 + P.gstart[I] * (long long)wrows;
                a.lda2 = wrows;
                a.B2 = Y + P.gstart[I] * (long long)b;
                a.ldb2 = b;
                a.klen2 = (int)R;
            }
            tiles(a, BMf, BNf);
            sf.add(a);
            flops += 2.0 * H.rows * (a.klen + a.klen2) * a.ncol;
            // 1b: skeleton columns of every J != I into W
            if (P.lstart[I + 1] > P.lstart[I]) {
                GemmTask c = t;
                c.ccol = d_ccol + P.lstart[I];
                c.cpos = d_wpos + P.lstart[I];
                c.ncol = P.lstart[I + 1] - P.lstart[I];
                c.C = W + H.w_row0;
                c.ldc = wrows;
                c.beta = 0;
                tiles(c, BMs, BNs);
                s1b.add(c);
                flops += 2.0 * H.rows * c.klen * c.ncol;
            }
        }
    }
    *flops_out = flops;
}

}  // namespace

hipError_t dc_lowrank_products(int b, double tol, std::vector<LrMerge>& ms, int variant,
                               hipStream_t s) {
    if (ms.empty()) return hipSuccess;
    Arena& A = arena();
    hipError_t err = arena_begin(A, s);
    // Every merge's compression output in its own part of one slot, so that
    // all of them are launched before their ranks come back together.
    // One launch runs the blocks of every merge; its job list follows the
    // outputs in the same slot.
    const bool offsets = ms[0].coff != nullptr;
    for (const LrMerge& M : ms)
        if ((M.coff != nullptr) != offsets) return hipErrorInvalidValue;
    std::vector<size_t> off(ms.size() + 1, 0);
    for (size_t i = 0; i < ms.size(); ++i) off[i + 1] = off[i] + al(compress_bytes(ms[i].K, b));
    char* cdev = nullptr;
    if (err == hipSuccess)
        err = arena_get(A, SL_SRRSC, off.back() + job_bytes(ms.size()), &cdev);
    std::vector<Compressed> Cm(ms.size());
    std::vector<SrrscJob> jobs;
    std::vector<DcRead> reads;
    for (size_t i = 0; i < ms.size() && err == hipSuccess; ++i) {
        const LrMerge& M = ms[i];
        jobs.push_back(compress_prepare(M.K, b, M.D, M.zhat, M.cbase, M.coff, M.scale, Cm[i],
                                        cdev + off[i]));
        reads.push_back({Cm[i].rank.data(), Cm[i].out.rank, Cm[i].rank.size() * sizeof(int)});
    }
    const SrrscJob* jd = nullptr;
    const int* sd = nullptr;
    int blocks = 0;
    if (err == hipSuccess) err = upload_jobs(jobs, cdev + off.back(), s, &jd, &sd, &blocks);
    if (err == hipSuccess)
        err = launch_srrsc(jd, sd, (int)jobs.size(), blocks, b, offsets, tol, Cm[0].rmax, true,
                           s);
    if (err == hipSuccess) err = dc_readback(reads, s);
    if (err != hipSuccess) return err;

    // Layouts of every merge, then one place for each in the level's slots:
    // the layout slot holds all uploaded parts first (one upload), then all
    // device-filled parts; W and Y hold one region per merge.
    std::vector<MergePlan> P(ms.size());
    size_t up_total = 0, dev_total = 0, w_total = 0, y_total = 0;
    for (size_t i = 0; i < ms.size(); ++i) {
        ms[i].ranks = rank_summary(Cm[i]);
        plan_layout(Cm[i], ms[i].K, b, P[i]);
        P[i].up_off = up_total;
        up_total += P[i].up_bytes;
        P[i].w_off = w_total;
        w_total += (size_t)ms[i].wrows * (size_t)P[i].NW;
        P[i].y_off = y_total;
        y_total += (size_t)P[i].NW * b;
    }
    for (size_t i = 0; i < ms.size(); ++i) {
        P[i].dev_off = up_total + dev_total;
        dev_total += P[i].dev_bytes;
    }
    char* small = nullptr;
    double* W = nullptr;
    double* Y = nullptr;
    err = arena_get(A, SL_LAYOUT, up_total + dev_total, &small);
    if (err == hipSuccess && w_total > 0)
        err = arena_get(A, SL_W, w_total * sizeof(double), reinterpret_cast<char**>(&W));
    if (err == hipSuccess && y_total > 0)
        err = arena_get(A, SL_Y, y_total * sizeof(double), reinterpret_cast<char**>(&Y));
    std::vector<char> host(up_total);
    for (size_t i = 0; i < ms.size(); ++i) {
        const size_t p2 = (size_t)P[i].p * P[i].p;
        std::memcpy(host.data() + P[i].up_off + P[i].o_wo, P[i].woff.data(),
                    p2 * sizeof(long long));
        std::memcpy(host.data() + P[i].up_off + P[i].o_lo, P[i].loff.data(), p2 * sizeof(int));
    }
    if (err == hipSuccess) err = dc_upload(small, host.data(), up_total, s);

    // Per merge: the per-column layout and the interpolation rows on the
    // device, and its tasks in the level's two launches.  The fused stage
    // needs the register kernel (variants 0 and 5).  The skeleton stage's
    // column count per block row (a sum of ranks) is rarely a multiple of
    // 128: with the default tile rule it takes 64 x 64 register tiles, which
    // waste less on the last column tile.
    const int fv = (variant == 2 || variant == 5) ? 5 : 0;
    const int sv = variant == 0 ? 5 : variant;
    Stage s1b, sf;
    for (size_t i = 0; i < ms.size() && err == hipSuccess; ++i) {
        const MergePlan& Q = P[i];
        LrMerge& M = ms[i];
        char* up = small + Q.up_off;
        char* dv = small + Q.dev_off;
        double* Wi = W ? W + Q.w_off : nullptr;
        double* Yi = Y ? Y + Q.y_off : nullptr;
        const int* d_ccol = reinterpret_cast<int*>(dv + Q.o_cc);
        const int* d_wpos = reinterpret_cast<int*>(dv + Q.o_wp);
        if (Q.NW > 0) {
            hipLaunchKernelGGL(k_layout, dim3((unsigned)((size_t)Q.p * Q.p)), dim3(128), 0, s,
                               Q.p, b, M.K, Cm[i].rmax, Cm[i].out.rank, Cm[i].out.pcol,
                               Cm[i].out.y, reinterpret_cast<long long*>(up + Q.o_wo),
                               reinterpret_cast<int*>(up + Q.o_lo),
                               reinterpret_cast<int*>(dv + Q.o_rg),
                               reinterpret_cast<long long*>(dv + Q.o_rv),
                               reinterpret_cast<int*>(dv + Q.o_kj),
                               reinterpret_cast<double*>(dv + Q.o_ry),
                               reinterpret_cast<int*>(dv + Q.o_cc),
                               reinterpret_cast<int*>(dv + Q.o_wp));
            err = hipGetLastError();
            if (err != hipSuccess) break;
            const long long ny = Q.NW * b;
            hipLaunchKernelGGL(k_build_y, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, s,
                               Q.NW, b, M.K, reinterpret_cast<double*>(dv + Q.o_ry),
                               reinterpret_cast<int*>(dv + Q.o_rg),
                               reinterpret_cast<long long*>(dv + Q.o_rv),
                               reinterpret_cast<int*>(dv + Q.o_kj), Cm[i].out.vk, M.cbase,
                               M.coff, M.scale, Yi);
            err = hipGetLastError();
            if (err != hipSuccess) break;
        }
        add_tasks(Q, M.K, b, M.cbase, M.coff, M.scale, M.halves, M.wrows, Wi, Yi, d_ccol,
                  d_wpos, fv, sv, s1b, sf, &M.flops);
    }

    // Upload the level's task lists and launch the two stages in order.
    constexpr int NS = 2;
    Stage* stages[NS] = {&s1b, &sf};
    size_t to = 0;
    std::vector<size_t> tof(NS), sof(NS);
    for (int i = 0; i < NS; ++i) {
        tof[i] = to; to = al(to + std::max<size_t>(stages[i]->tasks.size(), 1) * sizeof(GemmTask));
        sof[i] = to; to = al(to + stages[i]->start.size() * sizeof(int));
    }
    char* tdev = nullptr;
    std::vector<char> th(to);
    for (int i = 0; i < NS; ++i) {
        if (!stages[i]->tasks.empty())
            std::memcpy(th.data() + tof[i], stages[i]->tasks.data(),
                        stages[i]->tasks.size() * sizeof(GemmTask));
        std::memcpy(th.data() + sof[i], stages[i]->start.data(),
                    stages[i]->start.size() * sizeof(int));
    }
    if (err == hipSuccess) err = arena_get(A, SL_TASKS, to, &tdev);
    if (err == hipSuccess) err = dc_upload(tdev, th.data(), to, s);
    for (int i = 0; i < NS && err == hipSuccess; ++i) {
        const Stage& S = *stages[i];
        if (S.tasks.empty()) continue;
        const GemmTask* td = reinterpret_cast<GemmTask*>(tdev + tof[i]);
        const int* sd = reinterpret_cast<int*>(tdev + sof[i]);
        err = (&S == &sf)
                  ? dc_launch_cauchy_gemm2(td, sd, (int)S.tasks.size(), S.start.back(), fv, s)
                  : dc_launch_cauchy_gemm(td, sd, (int)S.tasks.size(), S.start.back(), sv, s);
    }
    const hipError_t e2 = arena_end(A, s);
    return err != hipSuccess ? err : e2;
}

hipError_t dc_lowrank_product(int K, int b, double tol, const double* D, const double* zhat,
                              const double* cbase, const double* coff, const double* scale,
                              std::vector<LrHalf>& halves, int wrows, int variant,
                              hipStream_t s, double* flops_out, LrRankSummary* ranks_out) {
    std::vector<LrMerge> ms(1);
    LrMerge& M = ms[0];
    M.K = K;
    M.D = D;
    M.zhat = zhat;
    M.cbase = cbase;
    M.coff = coff;
    M.scale = scale;
    M.halves = halves;
    M.wrows = wrows;
    const hipError_t err = dc_lowrank_products(b, tol, ms, variant, s);
    if (flops_out) *flops_out = M.flops;
    if (ranks_out) *ranks_out = M.ranks;
    return err;
}

hipError_t dc_node_arrays(int K, const double* Dbar, const int* org, const double* tau,
                          double* cbase, double* coff, hipStream_t s) {
    hipLaunchKernelGGL(k_nodes, dim3((K + 255) / 256), dim3(256), 0, s, K, Dbar, org, tau,
                       cbase, coff);
    return hipGetLastError();
}

hipError_t dc_disable_tasks(GemmTask* tasks, int n, const int* zero, hipStream_t s) {
    hipLaunchKernelGGL(k_disable_tasks, dim3(1), dim3(64), 0, s, tasks, n, zero);
    return hipGetLastError();
}

int dc_lowrank_max_block(bool offsets) { return offsets ? MAX_B_OFF : MAX_B_GEN; }

hipError_t dc_lowrank_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                             const int* org, const double* tau, const double* zhat,
                             const double* scale, double* C, long long ldc, double lr_tol,
                             int lr_block, hipStream_t stream) {
    if (lr_block > dc_lowrank_max_block(org != nullptr)) return hipErrorInvalidValue;
    // Merge generators become (base, offset) column nodes; plain column nodes
    // (org == NULL) are used as they are.
    const double* cb = tau;
    const double* co = nullptr;
    double* nodes = nullptr;
    hipError_t err = hipSuccess;
    if (org) {
        err = hipMallocAsync((void**)&nodes, 2 * (size_t)K * sizeof(double), stream);
        if (err != hipSuccess) return err;
        err = dc_node_arrays(K, Dbar, org, tau, nodes, nodes + K, stream);
        cb = nodes;
        co = nodes + K;
    }
    std::vector<LrHalf> halves(1);
    LrHalf& H = halves[0];
    H.A = Qnd;
    H.lda = ldq;
    H.rows = m;
    H.gD = Dbar;
    H.gz = zhat;
    H.C = C;
    H.ldc = ldc;
    H.cpos = nullptr;
    H.w_row0 = 0;
    if (err == hipSuccess)
        err = dc_lowrank_product(K, lr_block, lr_tol, Dbar, zhat, cb, co, scale, halves, m, 0,
                                 stream, nullptr);
    if (nodes) hipFreeAsync(nodes, stream);
    return err;
}

extern "C" int dc_merge_lowrank_ranks(int K, const double* Dbar, const int* org,
                                      const double* tau, const double* zhat,
                                      const double* scale, double lr_tol, int lr_block,
                                      int rank_cap, int* ranks_host, hipStream_t stream) {
    if (K < 1) return -1;
    if (!Dbar) return -2;
    if (!tau) return -4;
    if (!zhat) return -5;
    if (!scale) return -6;
    if (!(lr_tol > 0.0)) return -7;
    if (lr_block <= 0) lr_block = 256;
    if (lr_block > dc_lowrank_max_block(org != nullptr)) return -8;
    if (rank_cap < 0) return -9;
    if (!ranks_host) return -10;
    const double* cb = tau;
    const double* co = nullptr;
    double* nodes = nullptr;
    hipError_t err = hipSuccess;
    if (org) {
        err = hipMallocAsync((void**)&nodes, 2 * (size_t)K * sizeof(double), stream);
        if (err != hipSuccess) return (int)err;
        err = dc_node_arrays(K, Dbar, org, tau, nodes, nodes + K, stream);
        cb = nodes;
        co = nodes + K;
    }
    const int p = (K + lr_block - 1) / lr_block;
    const size_t p2 = (size_t)p * p;
    const SrrscJob* jd = nullptr;
    const int* sd = nullptr;
    int blocks = 0;
    if (rank_cap == 0) {
        // the ranks the low-rank product itself uses
        Compressed Cm;
        char* cdev = nullptr;
        const size_t cb_bytes = al(compress_bytes(K, lr_block));
        if (err == hipSuccess)
            err = hipMallocAsync((void**)&cdev, cb_bytes + job_bytes(1), stream);
        if (err == hipSuccess) {
            const std::vector<SrrscJob> jobs{
                compress_prepare(K, lr_block, Dbar, zhat, cb, co, scale, Cm, cdev)};
            err = upload_jobs(jobs, cdev + cb_bytes, stream, &jd, &sd, &blocks);
            if (err == hipSuccess)
                err = launch_srrsc(jd, sd, 1, blocks, lr_block, co != nullptr, lr_tol, Cm.rmax,
                                   true, stream);
        }
        if (err == hipSuccess)
            err = dc_readback({{ranks_host, Cm.out.rank, p2 * sizeof(int)}}, stream);
        if (cdev) hipFreeAsync(cdev, stream);
    } else {
        // count only, up to rank_cap
        char* rdev = nullptr;
        const size_t rk_bytes = al(p2 * sizeof(int));
        if (err == hipSuccess)
            err = hipMallocAsync((void**)&rdev, rk_bytes + job_bytes(1), stream);
        if (err == hipSuccess) {
            SrrscOut out{};
            out.rank = reinterpret_cast<int*>(rdev);
            const std::vector<SrrscJob> jobs{SrrscJob{K, p, Dbar, zhat, cb, co, scale, out}};
            err = upload_jobs(jobs, rdev + rk_bytes, stream, &jd, &sd, &blocks);
            if (err == hipSuccess)
                err = launch_srrsc(jd, sd, 1, blocks, lr_block, co != nullptr, lr_tol,
                                   std::min(rank_cap, lr_block), false, stream);
        }
        if (err == hipSuccess)
            err = hipMemcpyAsync(ranks_host, rdev, p2 * sizeof(int), hipMemcpyDeviceToHost,
                                 stream);
        if (rdev) hipFreeAsync(rdev, stream);
    }
    if (nodes) hipFreeAsync(nodes, stream);
    hipError_t e2 = hipStreamSynchronize(stream);
    return (int)(err != hipSuccess ? err : e2);
}
