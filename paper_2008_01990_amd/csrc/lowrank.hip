// Structured low-rank merge product: SRRSC compression of the off-diagonal
// blocks of U from their Cauchy generators, then two generated products,
// planned and launched on the device.
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
// and of Y.  U and Z never exist as matrices.
//
// Everything after the deflated size K is known runs on the device, so the
// host never waits: a decision kernel applies Algorithm 3's switch (K >=
// min_k), the compression runs on a grid bounded by the merge's order, a
// planning workgroup per merge turns the ranks into W's column layout, the
// interpolation-row generators and the two launches' task lists (and switches
// the plain product off, or leaves it on when W would not fit), and the two
// products walk their tiles with persistent grids that read the tile counts
// from device memory.  The merges of one tree level go together through every
// stage.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <vector>

#include "dc_internal.hpp"
#include "driver.hpp"
#include "lowrank.hpp"

namespace {

constexpr int NT = 1024;
constexpr int MAX_B_OFF = 2048;   // block size limit with column offsets (merge nodes)
constexpr int MAX_B_GEN = 4096;   // block size limit with plain column nodes
constexpr int MAX_R = 128;

// One workgroup per block (I, J).  MB: LDS capacity in generators; OFF: the
// column nodes carry an offset (w_j = cbase_j + coff_j, the merge's (origin,
// tau) form); STORE: write the skeleton and interpolation generators, else only
// count the rank (up to rmax).
template <int MB, int RG, bool OFF, bool STORE>
__global__ __launch_bounds__(NT)
void k_srrsc(const LrJob* __restrict__ jobs, const int* __restrict__ start, int njobs, int b,
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
    const LrJob& job = jobs[jlo];
    // the grid covers pmax x pmax blocks per job; this call's K has p blocks
    // per side (p = 0: the merge keeps the plain product)
    const int K = job.K_dev, p = job.p, pmax = job.pmax;
    const double* __restrict__ D = job.D;
    const double* __restrict__ u0 = job.zhat;
    const double* __restrict__ cbase = job.cbase;
    const double* __restrict__ coff = job.coff;
    const double* __restrict__ v0 = job.scale;
    const int loc = blockIdx.x - start[jlo];
    const int I = loc / pmax, J = loc - (loc / pmax) * pmax;
    if (I >= p || J >= p) return;
    const int pair = I * pmax + J;       // output index of block (I, J)
    const int tid = threadIdx.x;
    if (I == J) {
        if (tid == 0) job.rank[pair] = -1;
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
    if (tid == 0) job.rank[pair] = dense ? -2 : k;
    if constexpr (STORE) {
        if (dense) {
            // every column becomes a skeleton column: v^(r) = 0 throughout
            for (int j = tid; j < bj; j += NT) job.vk[(long long)pair * b + j] = 0.0;
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
            job.y[pb + a] = y;
            job.prow[pb + a] = spr[a];
            job.pcol[pb + a] = ja;
        }
        for (int j = tid; j < bj; j += NT) job.vk[(long long)pair * b + j] = sv[j];
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

// Algorithm 3's switch per merge: the low-rank product when K >= min_k and K
// exceeds one block; p = 0 keeps the plain product.
__global__ void k_lr_decide(LrJob* jobs, int njobs, int b) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    LrJob& J = jobs[j];
    const int K = J.K_p ? *J.K_p : J.K;
    J.K_dev = K;
    J.p = (K >= J.min_k && K > b) ? min((K + b - 1) / b, J.pmax) : 0;
}

__device__ __forceinline__ int lower_bound_dev(const int* a, int n, int v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void empty_task(GemmTask& t) {
    t.tiles_m = 0;
    t.tiles_n = 0;
}

// Exclusive prefix of in[0, n) into out[0, n] (out[n] = total) over one
// workgroup of NT threads; wsum (NT / 64) and carry are LDS scratch.
__device__ void block_scan_excl(const int* in, int* out, int n, int* wsum, int* carry) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) *carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += NT) {
        const int t = base + tid;
        const int v = t < n ? in[t] : 0;
        int x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int before = *carry;
        for (int q = 0; q < w; ++q) before += wsum[q];
        if (t < n) out[t] = before + x - v;
        __syncthreads();
        if (tid == NT - 1) *carry = before + x;
        __syncthreads();
    }
    if (tid == 0) out[n] = *carry;
    __syncthreads();
}

// One workgroup per merge of the level.  From the block ranks: the skeleton
// size of every block (its rank, or all its columns when kept dense), W's
// column layout by output block J (woff) and the skeleton column lists by
// block row I, the per-column generators of the interpolation rows, the
// tasks of both product launches, the flop and rank record, and the switch
// of the plain product.  When the skeleton columns would not fit W the merge
// keeps the plain product.  Block columns (and rows) are walked in segments
// of a few blocks by several threads each, whose offsets come from segment
// sums, so no thread follows a dependent chain through all p blocks.
__global__ __launch_bounds__(NT)
void k_lr_plan(LrJob* __restrict__ jobs, int b, int rmax, int bms, int bns, int bmf, int bnf) {
    extern __shared__ int sm[];
    __shared__ unsigned long long s_rsum;
    __shared__ int s_rmax, s_dense, s_carry;
    __shared__ int s_wsum[NT / 64];
    __shared__ double s_fs, s_ff;
    LrJob& J = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    const int pmax = J.pmax, p = J.p, K = J.K_dev;
    const int ntask = J.nh * pmax;
    const int* __restrict__ rank = J.rank;
    auto bsz = [&](int I) { return min(b, K - I * b); };
    auto skel = [&](int I, int c) {
        const int r = rank[I * pmax + c];
        return r == -2 ? bsz(c) : (r < 0 ? 0 : r);
    };
    int* rs = sm;                  // skeleton columns per block row (p)
    int* cs = sm + pmax;           // per block column (p)
    int* ls = sm + 2 * pmax;       // exclusive prefix of rs (p + 1)
    int* gs = ls + pmax + 1;       // exclusive prefix of cs (p + 1)
    int* seg = gs + pmax + 1;      // segment sums (NT)
    if (tid == 0) {
        s_rsum = 0;
        s_rmax = 0;
        s_dense = 0;
        s_fs = 0.0;
        s_ff = 0.0;
    }
    for (int i = tid; i < p; i += NT) {
        rs[i] = 0;
        cs[i] = 0;
    }
    __syncthreads();
    {
        unsigned long long rsum = 0;
        int rmx = 0, dn = 0;
        for (int q = tid; q < p * p; q += NT) {
            const int I = q / p, c = q - (q / p) * p;
            if (I == c) continue;
            const int rr = rank[I * pmax + c];
            const bool dense = rr == -2;
            const int r = dense ? bsz(c) : rr;
            if (dense) ++dn; else { rsum += rr; rmx = max(rmx, rr); }
            if (r > 0) {
                atomicAdd(&rs[I], r);
                atomicAdd(&cs[c], r);
            }
        }
        if (rsum) atomicAdd(&s_rsum, rsum);
        if (rmx) atomicMax(&s_rmax, rmx);
        if (dn) atomicAdd(&s_dense, dn);
    }
    __syncthreads();
    block_scan_excl(rs, ls, p, s_wsum, &s_carry);
    block_scan_excl(cs, gs, p, s_wsum, &s_carry);
    const int nw = p > 0 ? gs[p] : 0;
    const bool active = p > 0 && nw <= J.wcap;
    if (!active) {
        for (int t = tid; t < ntask; t += NT) {
            empty_task(J.tskel[t]);
            empty_task(J.tfused[t]);
        }
        if (tid == 0) *J.rec = LrRec{0, nw, 0, 0, 0, 0, 0.0, 0.0};
        return;
    }
    // T threads per block column (or row), each over L consecutive blocks.
    const int T = p >= NT ? 1 : min(64, NT / p);
    const int L = (p + T - 1) / T;
    // W's columns by output block c: block (I, c) at woff, its skeleton
    // generators, the v^(r) row of the block, the block column and y.
    for (int q = tid; q < p * T; q += NT) {
        const int c = q / T, sg = q - (q / T) * T;
        int a = 0;
        for (int I = sg * L; I < min(p, sg * L + L); ++I)
            if (I != c) a += skel(I, c);
        if (T > 1) seg[q] = a;
    }
    __syncthreads();
    for (int q = tid; q < p * T; q += NT) {
        const int c = q / T, sg = q - (q / T) * T;
        int run = gs[c];
        for (int u = 0; u < sg; ++u) run += seg[c * T + u];
        for (int I = sg * L; I < min(p, sg * L + L); ++I) {
            if (I == c) continue;
            const int pair = I * pmax + c;
            const int rr = rank[pair];
            const bool dense = rr == -2;
            const int r = dense ? bsz(c) : rr;
            J.woff[pair] = run;
            for (int a = 0; a < r; ++a) {
                const int col = run + a;
                J.rgen[col] = c * b + (dense ? a : J.pcol[(long long)pair * rmax + a]);
                J.rvo[col] = (long long)pair * b;
                J.kJ[col] = c;
                J.ry[col] = dense ? 0.0 : J.y[(long long)pair * rmax + a];
            }
            run += r;
        }
    }
    __threadfence_block();
    __syncthreads();
    // Skeleton column lists by block row I: generator and W column.
    for (int q = tid; q < p * T; q += NT) {
        const int I = q / T, sg = q - (q / T) * T;
        int a = 0;
        for (int c = sg * L; c < min(p, sg * L + L); ++c)
            if (c != I) a += skel(I, c);
        if (T > 1) seg[q] = a;
    }
    __syncthreads();
    for (int q = tid; q < p * T; q += NT) {
        const int I = q / T, sg = q - (q / T) * T;
        int run = ls[I];
        for (int u = 0; u < sg; ++u) run += seg[I * T + u];
        for (int c = sg * L; c < min(p, sg * L + L); ++c) {
            if (c == I) continue;
            const int pair = I * pmax + c;
            const int rr = rank[pair];
            const bool dense = rr == -2;
            const int r = dense ? bsz(c) : rr;
            const int w0 = J.woff[pair];
            for (int a = 0; a < r; ++a) {
                J.ccol[run + a] = c * b + (dense ? a : J.pcol[(long long)pair * rmax + a]);
                J.wpos[run + a] = w0 + a;
            }
            run += r;
        }
    }
    // Tasks: per row half and block row I, the fused task (diagonal block
    // generated, then W's columns of block I against Y) and the skeleton task.
    double fs = 0.0, ff = 0.0;
    for (int t = tid; t < ntask; t += NT) {
        const int hh = t / pmax, I = t - hh * pmax;
        if (I >= p) {
            empty_task(J.tskel[t]);
            empty_task(J.tfused[t]);
            continue;
        }
        const LrHalf& H = J.h[hh];
        int lo, hi;
        if (H.klist) {
            const int n = H.klen_p ? *H.klen_p : H.klen;
            lo = lower_bound_dev(H.klist, n, I * b);
            hi = lower_bound_dev(H.klist, n, I * b + b);
        } else {
            lo = I * b;
            hi = I * b + bsz(I);
        }
        GemmTask base;
        memset(&base, 0, sizeof(base));
        base.A = H.A + (long long)lo * H.lda;
        base.lda = H.lda;
        base.klen = hi - lo;
        base.rows = H.rows;
        base.rD = H.gD + lo;
        base.rz = H.gz + lo;
        base.cbase = J.cbase;
        base.coff = J.coff;
        base.cs = J.scale;
        GemmTask a = base;
        a.col_off = I * b;
        a.ncol = bsz(I);
        a.C = H.C;
        a.ldc = H.ldc;
        a.cpos = H.cpos;
        const int R = gs[I + 1] - gs[I];
        if (R > 0) {
            a.A2 = J.W + H.r0 + (long long)gs[I] * J.ldw;
            a.lda2 = J.ldw;
            a.B2 = J.Y + (long long)gs[I] * b;
            a.ldb2 = b;
            a.klen2 = R;
        }
        a.tiles_m = H.rows > 0 ? (H.rows + bmf - 1) / bmf : 0;
        a.tiles_n = (a.ncol + bnf - 1) / bnf;
        J.tfused[t] = a;
        ff += 2.0 * H.rows * (double)(a.klen + a.klen2) * a.ncol;
        GemmTask c = base;
        const int ncs = ls[I + 1] - ls[I];
        c.ccol = J.ccol + ls[I];
        c.cpos = J.wpos + ls[I];
        c.ncol = ncs;
        c.C = J.W + H.r0;
        c.ldc = J.ldw;
        c.tiles_m = (H.rows > 0 && ncs > 0) ? (H.rows + bms - 1) / bms : 0;
        c.tiles_n = (ncs + bns - 1) / bns;
        J.tskel[t] = c;
        fs += 2.0 * H.rows * (double)c.klen * ncs;
    }
    fs = dc_wave_sum(fs);
    ff = dc_wave_sum(ff);
    if ((tid & 63) == 0) {
        atomicAdd(&s_fs, fs);
        atomicAdd(&s_ff, ff);
    }
    __syncthreads();
    if (tid == 0) {
        for (int h = 0; h < J.nh && J.plain; ++h) J.plain[h].ncol_p = J.zero;
        *J.rec = LrRec{1, nw, p * (p - 1), (int)s_rsum, s_rmax, s_dense, s_fs, s_ff};
    }
}

// Interpolation rows [I Z_IJ] P^T of the low-rank blocks, one row per W
// column k (Theorem 2, eq. geneZ): for output column c of block column
// J = kJ[k], generator g = J b + c, the entry is 1 on the skeleton column
// itself (g == rgen[k]) and y_k v^(r)_c / (w_h - w_g) otherwise.  Stored
// row-major, Y[k b + c], divided by the column scale s_g that the product's
// epilogue multiplies back; 0 past the block's last column.  blockIdx.y is
// the merge; the blocks stride over its nw b entries.
__global__ void k_build_y(const LrJob* __restrict__ jobs, int b) {
    const LrJob& J = jobs[blockIdx.y];
    if (J.p == 0 || !J.rec->active) return;
    const long long total = (long long)J.rec->nw * b;
    const int K = J.K_dev;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long k = idx / b;
        const int c = (int)(idx - k * b);
        const int g = J.kJ[k] * b + c;
        if (g >= K) {
            J.Y[idx] = 0.0;
            continue;
        }
        const int h = J.rgen[k];
        double v = 1.0;
        if (h != g) {
            const double den = (J.cbase[h] - J.cbase[g]) + (J.coff ? J.coff[h] - J.coff[g] : 0.0);
            v = J.ry[k] * J.vk[J.rvo[k] + c] / den;
        }
        J.Y[idx] = v / J.scale[g];
    }
}

// Exclusive prefix of the tiles of a level's tasks (skeleton list, then
// fused list) and the two totals.
__global__ __launch_bounds__(NT)
void k_lr_scan(const GemmTask* __restrict__ tskel, const GemmTask* __restrict__ tfused,
               int ntasks, int* __restrict__ tile_start, int* __restrict__ totals) {
    __shared__ int wsum[NT / 64];
    __shared__ int carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int st = 0; st < 2; ++st) {
        const GemmTask* T = st ? tfused : tskel;
        int* out = tile_start + st * (ntasks + 1);
        if (tid == 0) carry = 0;
        __syncthreads();
        for (int base = 0; base < ntasks; base += NT) {
            const int t = base + tid;
            const int v = t < ntasks ? T[t].tiles_m * T[t].tiles_n : 0;
            int x = v;                                  // inclusive scan in the wave
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(x, off, 64);
                if (lane >= off) x += y;
            }
            if (lane == 63) wsum[w] = x;
            __syncthreads();
            int before = carry;
            for (int q = 0; q < w; ++q) before += wsum[q];
            if (t < ntasks) out[t] = before + x - v;
            __syncthreads();
            if (tid == NT - 1) carry = before + x;
            __syncthreads();
        }
        if (tid == 0) {
            out[ntasks] = carry;
            totals[st] = carry;
        }
        __syncthreads();
    }
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// The SRRSC instance for a job list: column offsets present (merge nodes, b
// up to MAX_B_OFF) or plain column nodes (b up to MAX_B_GEN); store or count
// only.
template <int MB, int RG, bool OFF>
hipError_t launch_srrsc_mb(const LrJob* jobs, const int* start, int njobs, int blocks, int b,
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
hipError_t launch_srrsc_off(const LrJob* jobs, const int* start, int njobs, int blocks,
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

hipError_t launch_srrsc(const LrJob* jobs, const int* start, int njobs, int blocks, int b,
                        bool offsets, double tol, int rmax, bool store, hipStream_t s) {
    if (offsets && b > MAX_B_OFF) return hipErrorInvalidValue;
    if (b > MAX_B_GEN) return hipErrorInvalidValue;
    if (blocks <= 0 || njobs <= 0) return hipSuccess;
    return offsets ? launch_srrsc_off<true>(jobs, start, njobs, blocks, b, tol, rmax, store, s)
                   : launch_srrsc_off<false>(jobs, start, njobs, blocks, b, tol, rmax, store, s);
}

// Tile shape of the two product launches (register kernel variant 5): 64 x 64
// one-wave tiles.  The k-ranges are short (one block b, plus the skeleton
// columns of the block column in the fused launch's second phase), so the
// tile's cost is dominated by generating U and loading A: a 64 x 64 wave
// feeds each generated entry to twice as many MFMAs per loaded A value as a
// 128 x 32 one (those ran the skeleton columns at 39% of peak, 64 x 64 at
// 58-65%; the fused launch took 2% less time on 64 x 64 tiles than on
// 128 x 128 tiles of 128 x 32 waves), and one-wave groups leave no slot idle
// where a row panel's last column tile is partial.
// Both launches are direct, over tile-count bounds known on the host: the
// fused launch's count depends only on the block count p <= pmax; the
// skeleton's on the ranks, and is bounded through W's capacity: a row half's
// column tiles over its p block rows number at most (wcap + 63 pmax) / 64.
// The tiles past the device's count exit at once (a launch of 65536 empty
// workgroups takes about 0.06 ms); grids of resident waves that walked or
// claimed the skeleton tiles instead fetched 1.5x as much (their tiles
// sharing an A panel ran less together) and ran 7-9% longer.
constexpr int FUSED_VARIANT = 5;
constexpr int SKEL_VARIANT = 5;

}  // namespace

int dc_lowrank_max_block(bool offsets) { return offsets ? MAX_B_OFF : MAX_B_GEN; }

int dc_lowrank_max_skel_tiles(int rows, int wcap, int pmax) {
    const int bm = dc_gemm_tile_m(SKEL_VARIANT), bn = dc_gemm_tile_n(SKEL_VARIANT);
    return ((rows + bm - 1) / bm) * ((wcap + (bn - 1) * pmax) / bn);
}

int dc_lowrank_max_fused_tiles(int rows, int m, int b, int pmax) {
    const int bm = dc_gemm_tile_m(FUSED_VARIANT), bn = dc_gemm_tile_n(FUSED_VARIANT);
    int t = 0;
    for (int I = 0; I < pmax; ++I) t += (std::min(b, m - I * b) + bn - 1) / bn;
    return t * ((rows + bm - 1) / bm);
}
int dc_lowrank_rmax(int b) { return std::min(MAX_R, std::max(1, b / 2)); }

size_t dc_lowrank_region_bytes(int pmax, int b, int wcap) {
    const size_t p2 = (size_t)pmax * pmax;
    const size_t rmax = dc_lowrank_rmax(b);
    const size_t w = std::max(wcap, 1);
    return al(p2 * sizeof(int)) * 2 + 2 * al(p2 * rmax * sizeof(int)) +
           al(p2 * rmax * sizeof(double)) + al(p2 * (size_t)b * sizeof(double)) +
           al(w * (size_t)b * sizeof(double)) + 4 * al(w * sizeof(int)) +
           al(w * sizeof(long long)) + al(w * sizeof(double)) + al(sizeof(LrRec));
}

hipError_t dc_lowrank_decide(LrJob* jobs_dev, int njobs, int b, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lr_decide, dim3((njobs + 63) / 64), dim3(64), 0, s, jobs_dev, njobs, b);
    return hipGetLastError();
}

namespace {

// The two halves of a level's pipeline: the SRRSC compression, then the
// planning, interpolation rows and the two product launches.
hipError_t lowrank_compress(LrJob* jobs_dev, int njobs, const int* srrsc_start,
                            int srrsc_blocks, int b, double tol, bool offsets, hipStream_t s) {
    return launch_srrsc(jobs_dev, srrsc_start, njobs, srrsc_blocks, b, offsets, tol,
                        dc_lowrank_rmax(b), true, s);
}

hipError_t lowrank_products(LrJob* jobs_dev, int njobs, GemmTask* tskel, GemmTask* tfused,
                            int ntasks, int* tile_start, int* totals, int b, int max_pmax,
                            int max_tiles_skel, int max_tiles_fused, hipStream_t s,
                            const hipEvent_t* ev) {
    const int rmax = dc_lowrank_rmax(b);
    const size_t lds = (size_t)(4 * max_pmax + 2 + NT) * sizeof(int);
    hipLaunchKernelGGL(k_lr_plan, dim3(njobs), dim3(NT), lds, s, jobs_dev, b, rmax,
                       dc_gemm_tile_m(SKEL_VARIANT), dc_gemm_tile_n(SKEL_VARIANT),
                       dc_gemm_tile_m(FUSED_VARIANT), dc_gemm_tile_n(FUSED_VARIANT));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_build_y, dim3(256, njobs), dim3(256), 0, s, jobs_dev, b);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_lr_scan, dim3(1), dim3(NT), 0, s, tskel, tfused, ntasks, tile_start,
                       totals);
    err = hipGetLastError();
    if (err == hipSuccess && ev) err = hipEventRecord(ev[1], s);
    if (err == hipSuccess)
        err = dc_launch_cauchy_gemm_bounded(tskel, tile_start, ntasks, max_tiles_skel, totals,
                                            SKEL_VARIANT, false, s);
    if (err == hipSuccess && ev) err = hipEventRecord(ev[2], s);
    if (err == hipSuccess)
        err = dc_launch_cauchy_gemm_bounded(tfused, tile_start + ntasks + 1, ntasks,
                                            max_tiles_fused, totals + 1, FUSED_VARIANT, true, s);
    if (err == hipSuccess && ev) err = hipEventRecord(ev[3], s);
    return err;
}

}  // namespace

hipError_t dc_lowrank_level(LrJob* jobs_dev, int njobs, const int* srrsc_start,
                            int srrsc_blocks, GemmTask* tskel, GemmTask* tfused, int ntasks,
                            int* tile_start, int* totals, int b, double tol, int max_pmax,
                            int max_tiles_skel, int max_tiles_fused, bool offsets,
                            hipStream_t s, const hipEvent_t* ev) {
    if (njobs <= 0) return hipSuccess;
    hipError_t err = ev ? hipEventRecord(ev[0], s) : hipSuccess;
    if (err == hipSuccess)
        err = lowrank_compress(jobs_dev, njobs, srrsc_start, srrsc_blocks, b, tol, offsets, s);
    if (err == hipSuccess)
        err = lowrank_products(jobs_dev, njobs, tskel, tfused, ntasks, tile_start, totals, b,
                               max_pmax, max_tiles_skel, max_tiles_fused, s, ev);
    return err;
}

hipError_t dc_node_arrays(int K, const double* Dbar, const int* org, const double* tau,
                          double* cbase, double* coff, hipStream_t s) {
    hipLaunchKernelGGL(k_nodes, dim3((K + 255) / 256), dim3(256), 0, s, K, Dbar, org, tau,
                       cbase, coff);
    return hipGetLastError();
}

// Stand-alone low-rank product C = Qnd U (one merge, one row half): the same
// device pipeline on a temporary, stream-ordered region (W is m x K; when
// the skeleton columns exceed it, the plain product launched behind the
// pipeline, which the planning kernel otherwise switches off, runs instead).
hipError_t dc_lowrank_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                             const int* org, const double* tau, const double* zhat,
                             const double* scale, double* C, long long ldc, double lr_tol,
                             int lr_block, hipStream_t stream) {
    const int b = lr_block;
    if (b > dc_lowrank_max_block(org != nullptr)) return hipErrorInvalidValue;
    const int pmax = (K + b - 1) / b;
    // Two passes with one host wait between them: the compression, whose
    // ranks give the exact number of skeleton columns NW (blocks of
    // near-full rank, as in a block-cyclic order, need several times K of
    // them), then W (m x NW), the interpolation rows and the column layout,
    // allocated at that size, and the products.
    // temporary 1: nodes | job | plain task | srrsc prefix | zero | tasks |
    // tile prefix | totals | SRRSC regions
    size_t o = 0;
    const size_t o_nodes = o; o = al(o + (org ? 2 * (size_t)K * sizeof(double) : 0));
    const size_t o_job = o; o = al(o + sizeof(LrJob));
    const size_t o_plain = o; o = al(o + sizeof(GemmTask));
    const size_t o_small = o; o = al(o + 16 * sizeof(int));
    const size_t o_tasks = o; o = al(o + 2 * (size_t)pmax * sizeof(GemmTask));
    const size_t o_ts = o; o = al(o + 2 * ((size_t)pmax + 1) * sizeof(int));
    const size_t o_reg = o; o = al(o + dc_lowrank_region_bytes(pmax, b, 1));
    char* tmp = nullptr;
    hipError_t err = hipMallocAsync((void**)&tmp, o, stream);
    if (err != hipSuccess) return err;
    const double* cb = tau;
    const double* co = nullptr;
    if (org) {
        double* nodes = reinterpret_cast<double*>(tmp + o_nodes);
        err = dc_node_arrays(K, Dbar, org, tau, nodes, nodes + K, stream);
        cb = nodes;
        co = nodes + K;
    }
    // small: [0, p^2] SRRSC prefix, a zero, the plain task's tile prefix at
    // 4, the two launches' tile totals at 8
    int* small = reinterpret_cast<int*>(tmp + o_small);
    GemmTask* plain = reinterpret_cast<GemmTask*>(tmp + o_plain);
    LrJob J;
    std::memset(&J, 0, sizeof(J));
    J.K_p = nullptr;
    J.K = K;
    J.pmax = pmax;
    J.min_k = 0;
    J.nh = 1;
    J.D = Dbar;
    J.zhat = zhat;
    J.cbase = cb;
    J.coff = co;
    J.scale = scale;
    LrHalf& H = J.h[0];
    H.A = Qnd;
    H.lda = ldq;
    H.rows = m;
    H.r0 = 0;
    H.klist = nullptr;
    H.klen_p = nullptr;
    H.klen = K;
    H.gD = Dbar;
    H.gz = zhat;
    H.C = C;
    H.ldc = ldc;
    H.cpos = nullptr;
    J.ldw = m;
    J.wrows = m;
    J.plain = plain;
    J.zero = small + 2;
    J.tskel = reinterpret_cast<GemmTask*>(tmp + o_tasks);
    J.tfused = J.tskel + pmax;
    J.K_dev = K;
    J.p = pmax;
    dc_lowrank_carve(J, tmp + o_reg, b, 1);
    // The plain product behind the pipeline (switched off by the planning
    // kernel unless the skeleton columns do not fit W).
    GemmTask T;
    std::memset(&T, 0, sizeof(T));
    const int bm = dc_gemm_tile_m(0), bn = dc_gemm_tile_n(0);
    T.A = Qnd;
    T.lda = ldq;
    T.klen = K;
    T.rows = m;
    T.rD = Dbar;
    T.rz = zhat;
    T.cbase = cb;
    T.coff = co;
    T.cs = scale;
    T.ncol = K;
    T.C = C;
    T.ldc = ldc;
    T.tiles_m = (m + bm - 1) / bm;
    T.tiles_n = (K + bn - 1) / bn;
    const int small_h[8] = {0, pmax * pmax, 0, 0, 0, T.tiles_m * T.tiles_n, 0, 0};
    LrJob* jd = reinterpret_cast<LrJob*>(tmp + o_job);
    if (err == hipSuccess) err = dc_write_blob(jd, &J, sizeof(J), stream);
    if (err == hipSuccess) err = dc_write_blob(plain, &T, sizeof(T), stream);
    if (err == hipSuccess) err = dc_write_blob(small, small_h, sizeof(small_h), stream);
    if (err == hipSuccess) err = lowrank_compress(jd, 1, small, pmax * pmax, b, lr_tol,
                                                  co != nullptr, stream);
    // NW exactly as the planning kernel counts it: a rank, or the block's
    // width where it is kept dense (-2)
    std::vector<int> rk((size_t)pmax * pmax);
    if (err == hipSuccess)
        err = hipMemcpyAsync(rk.data(), J.rank, rk.size() * sizeof(int), hipMemcpyDeviceToHost,
                             stream);
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    long long nw = 0;
    for (int I = 0; I < pmax; ++I)
        for (int c = 0; c < pmax; ++c) {
            if (I == c) continue;
            const int r = rk[(size_t)I * pmax + c];
            nw += r == -2 ? std::min(b, K - c * b) : std::max(r, 0);
        }
    // temporary 2: W and the per-W-column arrays at NW columns (none when
    // they would not fit in half the free memory: the plain product runs)
    size_t free_b = 0, total_b = 0;
    const size_t per_col = (size_t)m * sizeof(double) + (size_t)b * sizeof(double) + 64;
    const bool fits = err == hipSuccess && nw > 0 && nw < INT32_MAX &&
                      hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                      (size_t)nw * per_col <= free_b / 2;
    const int wcap = fits ? (int)nw : 0;
    char* tmp2 = nullptr;
    if (err == hipSuccess && fits) {
        size_t o2 = 0;
        const size_t o_y = o2; o2 = al(o2 + (size_t)wcap * b * sizeof(double));
        const size_t o_i = o2; o2 = al(o2 + 4 * (size_t)wcap * sizeof(int));
        const size_t o_v = o2; o2 = al(o2 + (size_t)wcap * sizeof(long long));
        const size_t o_r = o2; o2 = al(o2 + (size_t)wcap * sizeof(double));
        const size_t o_w2 = o2; o2 = al(o2 + (size_t)m * wcap * sizeof(double));
        err = hipMallocAsync((void**)&tmp2, o2, stream);
        if (err == hipSuccess) {
            J.Y = reinterpret_cast<double*>(tmp2 + o_y);
            int* ib = reinterpret_cast<int*>(tmp2 + o_i);
            J.rgen = ib;
            J.kJ = ib + wcap;
            J.ccol = ib + 2 * (size_t)wcap;
            J.wpos = ib + 3 * (size_t)wcap;
            J.rvo = reinterpret_cast<long long*>(tmp2 + o_v);
            J.ry = reinterpret_cast<double*>(tmp2 + o_r);
            J.W = reinterpret_cast<double*>(tmp2 + o_w2);
        }
    }
    J.wcap = wcap;
    if (err == hipSuccess) err = dc_write_blob(jd, &J, sizeof(J), stream);
    int* ts = reinterpret_cast<int*>(tmp + o_ts);
    if (err == hipSuccess)
        err = lowrank_products(jd, 1, J.tskel, J.tfused, pmax, ts, small + 8, b, pmax,
                               dc_lowrank_max_skel_tiles(m, std::max(wcap, 1), pmax),
                               dc_lowrank_max_fused_tiles(m, K, b, pmax), stream, nullptr);
    // plain fallback: tile prefix {0, tiles} at small[4..5]
    if (err == hipSuccess)
        err = dc_launch_cauchy_gemm(plain, small + 4, 1, T.tiles_m * T.tiles_n, 0, stream);
    const hipError_t e3 = tmp2 ? hipFreeAsync(tmp2, stream) : hipSuccess;
    const hipError_t e2 = hipFreeAsync(tmp, stream);
    return err != hipSuccess ? err : (e2 != hipSuccess ? e2 : e3);
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
    const int b = lr_block;
    const int p = (K + b - 1) / b;
    const size_t p2 = (size_t)p * p;
    // rank_cap 0: the ranks the low-rank product itself uses (full SRRSC
    // output); > 0: count only, up to rank_cap
    const size_t reg = rank_cap == 0 ? dc_lowrank_region_bytes(p, b, 1) : al(p2 * sizeof(int));
    size_t o = 0;
    const size_t o_nodes = o; o = al(o + (org ? 2 * (size_t)K * sizeof(double) : 0));
    const size_t o_job = o; o = al(o + sizeof(LrJob));
    const size_t o_start = o; o = al(o + 2 * sizeof(int));
    const size_t o_reg = o; o = al(o + reg);
    char* tmp = nullptr;
    hipError_t err = hipMallocAsync((void**)&tmp, o, stream);
    if (err != hipSuccess) return (int)err;
    const double* cb = tau;
    const double* co = nullptr;
    if (org) {
        double* nodes = reinterpret_cast<double*>(tmp + o_nodes);
        err = dc_node_arrays(K, Dbar, org, tau, nodes, nodes + K, stream);
        cb = nodes;
        co = nodes + K;
    }
    LrJob J;
    std::memset(&J, 0, sizeof(J));
    J.K = K;
    J.K_dev = K;
    J.pmax = p;
    J.p = p;
    J.D = Dbar;
    J.zhat = zhat;
    J.cbase = cb;
    J.coff = co;
    J.scale = scale;
    if (rank_cap == 0) dc_lowrank_carve(J, tmp + o_reg, b, 1);
    else J.rank = reinterpret_cast<int*>(tmp + o_reg);
    const int st[2] = {0, (int)p2};
    if (err == hipSuccess) err = dc_write_blob(tmp + o_job, &J, sizeof(J), stream);
    if (err == hipSuccess) err = dc_write_blob(tmp + o_start, st, sizeof(st), stream);
    if (err == hipSuccess)
        err = launch_srrsc(reinterpret_cast<LrJob*>(tmp + o_job),
                           reinterpret_cast<int*>(tmp + o_start), 1, (int)p2, b, co != nullptr,
                           lr_tol, rank_cap == 0 ? dc_lowrank_rmax(b) : std::min(rank_cap, b),
                           rank_cap == 0, stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(ranks_host, J.rank, p2 * sizeof(int), hipMemcpyDeviceToHost,
                             stream);
    const hipError_t e2 = hipFreeAsync(tmp, stream);
    const hipError_t e3 = hipStreamSynchronize(stream);
    return (int)(err != hipSuccess ? err : (e2 != hipSuccess ? e2 : e3));
}
