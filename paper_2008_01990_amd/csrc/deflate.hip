// Merge set-up and clean-up kernels of the divide-and-conquer tree:
// rank-one vector and deflation (eq. T3, eq. T3-def), Givens rotations of
// the basis, final eigenvalue order and deflated-column copy (eq. evect).
//
// For a merge of children with (Lambda_1, Q_1) rows [0, n1) and
// (Lambda_2, Q_2) rows [n1, m) of its diagonal block:
//   z = [last row of Q_1, sigma * first row of Q_2] / sqrt(2),  rho' = 2 |e_k|
//   D = [Lambda_1; Lambda_2] sorted by a merge of the two ascending lists.
// Deflation (tol = 8 eps max(max|D|, rho')): z-negligible entries become
// eigenpairs as they are; neighbouring survivors p < i with
// |(D_i - D_p) c s| <= tol for the Givens pair that zeroes z_p are rotated
// and p deflated.  The walk over survivors is sequential in principle (each
// test involves the last survivor, which a rotation modifies), but only along
// runs of rotations: the workgroup walks segments of the survivor list in
// parallel assuming an unrotated start, the true segment starts are settled
// by parallel rounds (a segment entered with a rotated candidate is re-walked
// only until the two walks agree on a pair that does not rotate), and the
// segments are walked again from their true starts to count and then to
// write their output.
//
// Every column of the merge block carries row-type bits: 1 if it may be
// non-zero in the top rows [0, n1), 2 in the bottom rows [n1, m).  Columns of
// Q_1 start as 1, of Q_2 as 2; a rotation of two columns gives both the union.
// The product runs separately on the top rows (k over survivors of type 1|3)
// and on the bottom rows (type 2|3): the structural zeros of diag(Q_1, Q_2)
// cost no flops.
//
// Below the root the children's eigenvectors are resident columns of B1: the
// eigenvector of local column c (the child's sorted eigenvalue c, or c - n1)
// is column cmap[c] of B1, with data only in rows rng[c] of that column; the
// other rows are structural zeros and are never read.  A merge below the
// root moves no deflated column: it overwrites the columns it deflates by
// rotation in place, gives its product columns the places of its survivors
// (packed into the panel first), and records its own map and ranges.  The
// root merge writes the caller's Q in eigenvalue order.
#include "dc_internal.hpp"

namespace {

constexpr double EPS = 2.220446049250313e-16;

// The merge of workgroup b: blk_start holds the grid's prefix (nm + 1
// entries) followed by its block -> merge map.
__device__ __forceinline__ int block_of(const int* blk_start, int nm, int b) {
    return blk_start[nm + 1 + b];
}

// Number of entries of the ascending a[0..n) strictly below x / at most x.
__device__ __forceinline__ int count_lt(const double* a, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int count_le(const double* a, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Exclusive prefix sum of one int per thread over the NT threads of the
// workgroup; *total receives the sum.  ws: NT / 64 ints of LDS.
template <int NT>
__device__ int block_excl_scan(int v, int* ws, int* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    int before = 0, tot = 0;
    for (int q = 0; q < NT / 64; ++q) {
        if (q < w) before += ws[q];
        tot += ws[q];
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

// Exclusive prefix maximum (-inf for thread 0) of one double per thread.
__device__ double block_excl_max(double v, double* ws) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(x, off, 64);
        if (lane >= off) x = fmax(x, y);
    }
    double ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = -INFINITY;
    if (lane == 63) ws[w] = x;
    __syncthreads();
    double before = -INFINITY;
    for (int q = 0; q < w; ++q) before = fmax(before, ws[q]);
    __syncthreads();
    return fmax(before, ex);
}

// State of the walk: the current candidate survivor p (unrotated, or the
// result of rotations).
struct WState {
    double D, z;
    int col, typ;
    int orig;       // 1: an unrotated survivor
};

// Pair test and rotation of the walk for candidate p = st and the next
// survivor q.  Every pass of the walk (speculative, correcting, counting,
// writing) must take the same decisions to the last bit, so that the counts
// and the writes agree: contraction into FMAs is off here, which leaves only
// IEEE operations whose results do not depend on where the code is inlined.
// (Out of line, the state structs went through scratch memory: several
// memory round trips per step.)
__device__ __forceinline__ bool walk_decide(const WState& st, const WState& q, double tol,
                                            WState& nxt, double& c, double& sn, double& dv) {
#pragma clang fp contract(off)
    // |(D_i - D_p) c s| <= tol with (c, s) = (z_i, z_p) / r, multiplied out by
    // r^2 = z_p^2 + z_i^2 so that the common case (no rotation) needs no
    // square root or reciprocal.  |z| <= 1 and surviving z are far above
    // underflow.
    const double r2 = st.z * st.z + q.z * q.z;
    if (fabs(q.D - st.D) * fabs(q.z * st.z) <= tol * r2) {
        const double r = sqrt(r2);
        const double ir = dc_rcp(r);
        c = q.z * ir;
        sn = st.z * ir;
        dv = c * c * st.D + sn * sn * q.D;
        nxt = WState{sn * sn * st.D + c * c * q.D, r, q.col, st.typ | q.typ, 0};
        return true;
    }
    nxt = q;
    return false;
}

// Writes up to 8 Prob records carried in the kernel arguments.
struct ProbPack { Prob p[8]; };
__global__ void k_write_probs(Prob* dst, int first, int count, ProbPack pack) {
    const int i = threadIdx.x;
    if (i < count) dst[first + i] = pack.p[i];
}

// Build the product and secular task records of every merge (per call: they
// hold the caller's pointers).
__global__ void k_build(const Node* __restrict__ merges, int nm, int bm, int bn, Scratch S) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nm) return;
    const Node N = merges[g];
    const Prob P = S.probs[N.prob];
    const int m = N.n1 + N.n2;
    const long long base = (long long)P.row0 + N.off;
    long long ldo;
    double* Qo = node_buf(P, N.depth, ldo);
    const int slot = N.slot;
    MergeCnt* cnt = S.cnt + slot;
    const int tn = (m + bn - 1) / bn;   // worst-case column tiles
    for (int half = 0; half < 2; ++half) {
        GemmTask T;
        memset(&T, 0, sizeof(T));
        const int r0 = half ? N.n1 : 0;
        T.A = P.B2 + (long long)N.off * P.ld2 + N.off + r0;
        T.lda = P.ld2;
        T.klen_p = half ? &cnt->nbot : &cnt->ntop;
        T.klen = 0;
        T.rows = half ? N.n2 : N.n1;
        T.rD = (half ? S.gDb : S.gDt) + base;
        T.rz = (half ? S.gzb : S.gzt) + base;
        T.cbase = S.cbase + base;
        T.corg = nullptr;
        T.coff = S.tau + base;
        T.cs = S.scale + base;
        T.ncol_p = &cnt->K;
        T.ncol = 0;
        T.C = Qo + (long long)N.off * ldo + N.off + r0;
        T.ldc = ldo;
        T.cpos = S.pos_root + base;
        T.tiles_m = (T.rows + bm - 1) / bm;
        T.tiles_n = tn;
        T.beta = 0;
        S.gtask[2 * slot + half] = T;
    }
    SecTask Q;
    Q.D = S.Dbar + base;
    Q.z = S.zbar + base;
    Q.K_p = &cnt->K;
    Q.K = 0;
    Q.row0 = N.off;
    Q.rho_p = S.rho2 + slot;
    Q.rho = 0.0;
    Q.org = S.org + base;
    Q.tau = S.tau + base;
    Q.cbase = S.cbase + base;
    Q.lam = S.lamr + base;
    Q.zhat = S.zhat + base;
    Q.scale = S.scale + base;
    Q.info = P.info;
    Q.iters = cnt->sec_iters;
    S.stask[slot] = Q;
}

// One workgroup per merge: z, sort, deflation walk, generator lists.
// Rank-one vector and sorted order of every merge of a level (eq. T3), one
// thread per eigenpair of the two children:
//   z = [last row of Q_1, sigma * first row of Q_2] / sqrt(2),
// and the merge of the two ascending spectra (Lambda_1 first on ties):
// Lambda_1[i] goes to i + #{Lambda_2 < it}, Lambda_2[j] to j + #{Lambda_1 <= it}.
__global__ __launch_bounds__(DC_ROWS_PER_BLOCK)
void k_merge_sort(const Node* __restrict__ merges, const int* __restrict__ blk_start, int nm,
                  Scratch S) {
    const int mi = block_of(blk_start, nm, blockIdx.x);
    const Node N = merges[mi];
    const Prob P = S.probs[N.prob];
    if (*P.info == DC_STATUS_NONFINITE) return;      // k_deflate handles it
    const int n1 = N.n1, n2 = N.n2, m = n1 + n2;
    const int i = (blockIdx.x - blk_start[mi]) * DC_ROWS_PER_BLOCK + threadIdx.x;
    if (i >= m) return;
    const long long base = (long long)P.row0 + N.off;
    long long ldi;
    const double* Qi = node_buf(P, N.depth + 1, ldi);
    const double* L1 = P.d + N.off;
    const double* L2 = P.d + N.off + n1;
    const double ek = P.e[N.off + n1 - 1];            // its sign only: scale-free
    const double sigma = ek < 0.0 ? -1.0 : 1.0;
    const double rs2 = 0.70710678118654752440;
    // the child's last (top) or first (bottom) row of the column, 0 outside
    // its rows
    const int col = node_cmap(S, N.depth + 1)[base + i];
    const int2 rg = node_rng(S, N.depth + 1)[base + i];
    const int row = i < n1 ? N.off + n1 - 1 : N.off + n1;
    const double q = row >= rg.x && row < rg.y ? Qi[(long long)col * ldi + row] : 0.0;
    double Dv, zv;
    int pos;
    if (i < n1) {
        Dv = L1[i];
        zv = q * rs2;
        pos = i + count_lt(L2, n2, Dv);
    } else {
        Dv = L2[i - n1];
        zv = sigma * q * rs2;
        pos = (i - n1) + count_le(L1, n1, Dv);
    }
    S.Ds[base + pos] = Dv;
    S.zs[base + pos] = zv;
    S.perm[base + pos] = i;
}

// NT threads per merge (64, 256 or 1024, by the level's largest merge): the
// walk's LDS grows with NT, and a workgroup sized for large merges holds a
// compute unit to one of the many small merges of a lower level.
template <int NT>
__global__ __launch_bounds__(NT)
void k_deflate(const Node* __restrict__ merges, Scratch S) {
    // per segment of the survivor list: speculative end state, true start
    __shared__ double oD[NT], oz[NT], iD[NT], iz[NT];
    __shared__ int ocol[NT], otyp[NT], oorg[NT], icol[NT], ityp[NT], iorg[NT];
    // per segment: its first next survivor and first speculative decision,
    // so that the usual one-step correction reads only LDS
    __shared__ double fD[NT], fz[NT];
    __shared__ int fcol[NT], ftyp[NT], fdec[NT];
    __shared__ int wsum[NT / 64];
    __shared__ double wmax[NT / 64];

    const Node N = merges[blockIdx.x];
    const Prob P = S.probs[N.prob];
    const int n1 = N.n1, n2 = N.n2, m = n1 + n2;
    const long long base = (long long)P.row0 + N.off;
    const double* L1 = P.d + N.off;          // Lambda_1 ascending
    const double* L2 = P.d + N.off + n1;     // Lambda_2 ascending
    const double ek = P.e[N.off + n1 - 1] * S.psc[N.prob];   // d is scaled, e on read
    const double rho2 = 2.0 * fabs(ek);
    const int tid = threadIdx.x;

    // A problem with non-finite input (flagged by the leaf phase) cannot be
    // ordered: every pair becomes a deflated identity column with a NaN
    // eigenvalue, which keeps every later index in range.
    if (*P.info == DC_STATUS_NONFINITE) {
        for (int k = tid; k < m; k += NT) {
            S.Dd[base + k] = NAN;
            S.dcol[base + k] = k;
            S.dtype[base + k] = k < n1 ? 1 : 2;
        }
        if (tid == 0) {
            MergeCnt* cnt = S.cnt + N.slot;
            cnt->K = 0;
            cnt->nrot = 0;
            cnt->ndefl = m;
            cnt->ntop = 0;
            cnt->nbot = 0;
            cnt->nchain = 0;
            cnt->pad_[0] = 0;
            cnt->sec_iters[0] = 0;
            cnt->sec_iters[1] = 0;
            S.rho2[N.slot] = 0.0;
        }
        return;
    }

    // (z and the merged order were written by k_merge_sort.)
    const double dmax = fmax(fmax(fabs(L1[0]), fabs(L1[n1 - 1])),
                             fmax(fabs(L2[0]), fabs(L2[n2 - 1])));
    const double tol = 8.0 * EPS * fmax(dmax, rho2);
    __syncthreads();

    // ---- Deflation walk, segmented. ----
    // z-test survivors in sorted order: SI[0..Ns).  Scratch borrowed for the
    // walk (all written again later in this merge): SI in org, speculative
    // decisions in pos_root, deflated entries keyed by the sorted position
    // that triggers them in tau / pos_defl / ktop (ktop = 0: no entry).
    int* SI = S.org + base;
    int* dspec = S.pos_root + base;
    double* tV = S.tau + base;
    int* tC = S.pos_defl + base;
    int* tT = S.ktop + base;
    const int PL = (m + NT - 1) / NT;                 // sorted positions per thread
    const int q0 = min(m, tid * PL), q1 = min(m, q0 + PL);
    auto colof = [&](int i) { return min(max(S.perm[base + i], 0), m - 1); };
    int nsl = 0;
    for (int i = q0; i < q1; ++i) nsl += !(rho2 * fabs(S.zs[base + i]) <= tol);
    int Ns = 0;
    int w0 = block_excl_scan<NT>(nsl, wsum, &Ns);
    for (int i = q0; i < q1; ++i) {
        const int c = colof(i);
        if (!(rho2 * fabs(S.zs[base + i]) <= tol)) {
            SI[w0++] = i;
            tT[i] = 0;
        } else {                                      // deflated as it is
            tV[i] = S.Ds[base + i];
            tC[i] = c;
            tT[i] = c < n1 ? 1 : 2;
        }
    }
    __syncthreads();
    // The survivors' (D, z, column) laid out in walk order, so that a walk
    // step reads index k + 1 directly (no chase through SI) and the next
    // step's loads can be issued early.  Scratch: lamr, cbase and kbot, which
    // later phases of this level write.
    double* cD = S.lamr + base;
    double* cz = S.cbase + base;
    int* cc = S.kbot + base;
    // four entries per thread and pass, loads before stores (the scratch
    // arrays may alias as far as the compiler knows, which would otherwise
    // serialise every entry's two dependent loads behind the last store)
    for (int k0 = tid; k0 < Ns; k0 += 4 * NT) {
        int ii[4];
        double dd[4], zz[4];
        int cl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ii[u] = k0 + u * NT < Ns ? SI[k0 + u * NT] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = max(ii[u], 0);
            dd[u] = S.Ds[base + i];
            zz[u] = S.zs[base + i];
            cl[u] = colof(i);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (ii[u] < 0) continue;
            cD[k0 + u * NT] = dd[u];
            cz[k0 + u * NT] = zz[u];
            cc[k0 + u * NT] = cl[u];
        }
    }
    __syncthreads();

    auto load_orig = [&](int k) {
        const int c = cc[k];
        return WState{cD[k], cz[k], c, c < n1 ? 1 : 2, 1};
    };
    // Decision for the pair (st, survivor k + 1): nxt is the next candidate;
    // on a rotation (c, s) and the deflated value are returned as well.
    auto decide = [&](const WState& st, int k, WState& nxt, double& c, double& sn,
                      double& dv, int& typi) {
        const WState q = load_orig(k + 1);
        typi = q.typ;
        return walk_decide(st, q, tol, nxt, c, sn, dv);
    };
    const int npairs = Ns > 0 ? Ns - 1 : 0;
    const int SL = npairs > 0 ? (npairs + NT - 1) / NT : 1;   // pairs per segment
    const int nseg = (npairs + SL - 1) / SL;
    const int ka = tid * SL, kb = min(npairs, ka + SL);
    const bool myseg = tid < nseg;

    // Speculative walk: every segment starts from its unrotated survivor.
    if (myseg) {
        WState st = load_orig(ka);
        WState q = load_orig(ka + 1);
        fD[tid] = q.D; fz[tid] = q.z; fcol[tid] = q.col; ftyp[tid] = q.typ;
        for (int k = ka; k < kb; ++k) {
            const WState qn = load_orig(min(k + 2, npairs));   // next step's pair
            WState nx;
            double c, sn, dv;
            dspec[k] = walk_decide(st, q, tol, nx, c, sn, dv) ? 1 : 0;
            if (k == ka) fdec[tid] = dspec[k];
            st = nx;
            q = qn;
        }
        oD[tid] = st.D; oz[tid] = st.z; ocol[tid] = st.col; otyp[tid] = st.typ;
        oorg[tid] = st.orig;
    }
    __syncthreads();
    // True segment starts: in_0 is survivor 0 and in_{sg+1} = F_sg(in_sg),
    // where F_sg keeps the speculative end state when entered with an
    // unrotated survivor and otherwise re-walks the segment until both walks
    // decline a rotation at the same pair (from there on they coincide).  The
    // recurrence is solved by rounds over all segments at once, starting from
    // in_{sg+1} = speculative end of sg: a round recomputes every F_sg from
    // the current in_sg, and another round follows only if some in_{sg+1}
    // changed.  After round r the first r + 1 starts are exact, so the rounds
    // end; a change passes on only when a re-walk never meets the speculative
    // walk, so one or two rounds usually settle it (the serial form took one
    // step per segment: 1024 dependent steps of one thread for a large merge).
    if (myseg) {
        WState in = tid == 0 ? load_orig(0)
                             : WState{oD[tid - 1], oz[tid - 1], ocol[tid - 1], otyp[tid - 1],
                                      oorg[tid - 1]};
        iD[tid] = in.D; iz[tid] = in.z; icol[tid] = in.col; ityp[tid] = in.typ;
        iorg[tid] = in.orig;
    }
    for (;;) {
        __syncthreads();
        WState out{0.0, 0.0, 0, 0, 1};
        if (myseg) {
            const int sg = tid;
            const WState in{iD[sg], iz[sg], icol[sg], ityp[sg], iorg[sg]};
            out = WState{oD[sg], oz[sg], ocol[sg], otyp[sg], oorg[sg]};
            if (!in.orig) {
                const int a = sg * SL, b = min(npairs, a + SL);
                WState nx;
                double c, sn, dv;
                const WState f{fD[sg], fz[sg], fcol[sg], ftyp[sg], 1};
                const bool rot0 = walk_decide(in, f, tol, nx, c, sn, dv);
                bool conv = !rot0 && !fdec[sg];
                WState st = nx;
                for (int k = a + 1; k < b && !conv; ++k) {
                    int ti;
                    const bool rot = decide(st, k, nx, c, sn, dv, ti);
                    st = nx;
                    if (!rot && !dspec[k]) conv = true;
                }
                if (!conv) out = st;
            }
        }
        __syncthreads();
        int changed = 0;
        if (myseg && tid + 1 < nseg) {
            const int t = tid + 1;
            if (__double_as_longlong(out.D) != __double_as_longlong(iD[t]) ||
                __double_as_longlong(out.z) != __double_as_longlong(iz[t]) ||
                out.col != icol[t] || out.typ != ityp[t] || out.orig != iorg[t]) {
                iD[t] = out.D; iz[t] = out.z; icol[t] = out.col; ityp[t] = out.typ;
                iorg[t] = out.orig;
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    __syncthreads();

    // Count, then write, from the true starts.  A rotation starts a new chain
    // exactly when its first column is an unrotated survivor.
    int cs = 0, cr = 0, nchn = 0;
    if (myseg) {
        WState st{iD[tid], iz[tid], icol[tid], ityp[tid], iorg[tid]};
        WState q = load_orig(ka + 1);
        for (int k = ka; k < kb; ++k) {
            const WState qn = load_orig(min(k + 2, npairs));
            WState nx;
            double c, sn, dv;
            if (walk_decide(st, q, tol, nx, c, sn, dv)) { ++cr; nchn += st.orig; } else ++cs;
            st = nx;
            q = qn;
        }
        cs += tid == nseg - 1;                          // the last candidate
    } else if (tid == 0 && Ns == 1) {
        cs = 1;
    }
    int K = 0, nrot = 0, nch = 0;
    int os = block_excl_scan<NT>(cs, wsum, &K);
    int orr = block_excl_scan<NT>(cr, wsum, &nrot);
    int oc = block_excl_scan<NT>(nchn, wsum, &nch);
    // rend[t]: the survivor that the column produced by rotation t becomes
    // when t ends its chain, else -1 (perm is free once the walk state is
    // laid out).  The rotation kernel writes such a column straight into
    // the survivor panel, and the gather skips it.
    int* rend = S.perm + base;
    for (int t = tid; t < nrot; t += NT) rend[t] = -1;
    __syncthreads();
    // A survivor's type bit 4 marks a chain end.  The rotation that produced
    // a rotated candidate is the last one before it: index orr - 1 (also
    // across a segment boundary, where the previous segment ended with it).
    auto put_surv = [&](const WState& st, int k, int last_rot) {
        S.Dbar[base + k] = st.D;
        S.zbar[base + k] = st.z;
        S.surv[base + k] = st.col;
        S.stype[base + k] = st.typ | (st.orig ? 0 : 4);
        if (!st.orig) rend[last_rot] = k;
    };
    if (myseg) {
        WState st{iD[tid], iz[tid], icol[tid], ityp[tid], iorg[tid]};
        WState q = load_orig(ka + 1);
        for (int k = ka; k < kb; ++k) {
            const WState qn = load_orig(min(k + 2, npairs));
            WState nx;
            double c, sn, dv;
            const int ti = q.typ;
            const bool rot = walk_decide(st, q, tol, nx, c, sn, dv);
            q = qn;
            if (rot) {
                if (st.orig) S.rch[base + oc++] = orr;
                S.rp[base + orr] = st.col;
                S.ri[base + orr] = nx.col;
                S.rc[base + orr] = c;
                S.rs[base + orr] = sn;
                S.rt[base + orr] = st.typ | (ti << 2);
                const int trig = SI[k + 1];
                tV[trig] = dv;
                tC[trig] = st.col;
                // typ_p | typ_i, the rotation flag and the rotation's index
                tT[trig] = nx.typ | 8 | (orr << 4);
                ++orr;
            } else {
                put_surv(st, os++, orr - 1);
            }
            st = nx;
        }
        if (tid == nseg - 1) put_surv(st, os, orr - 1);
    } else if (tid == 0 && Ns == 1) {
        put_surv(load_orig(0), 0, -1);
    }
    __syncthreads();

    // Deflated entries in walk order (by triggering position), then ascending:
    // an entry below the maximum of those before it is inserted backwards, in
    // order (the prefix maximum is unchanged by insertions before it), which
    // gives the walk's incremental insertion exactly.
    int cd = 0;
    for (int i = q0; i < q1; ++i) cd += tT[i] != 0;
    int nd = 0;
    int od = block_excl_scan<NT>(cd, wsum, &nd);
    for (int i = q0; i < q1; ++i) {
        if (tT[i] == 0) continue;
        S.Dd[base + od] = tV[i];
        S.dcol[base + od] = tC[i];
        S.dtype[base + od] = tT[i];
        ++od;
    }
    __syncthreads();
    const int DL = (nd + NT - 1) / NT;
    const int d0 = min(nd, tid * DL), d1 = min(nd, d0 + DL);
    double lmax = -INFINITY;
    for (int k = d0; k < d1; ++k) lmax = fmax(lmax, S.Dd[base + k]);
    double run = block_excl_max(lmax, wmax);
    int cf = 0;
    for (int k = d0; k < d1; ++k) {
        const double v = S.Dd[base + k];
        cf += v < run;
        run = fmax(run, v);
    }
    int nf = 0;
    int of = block_excl_scan<NT>(cf, wsum, &nf);
    run = block_excl_max(lmax, wmax);
    for (int k = d0; k < d1; ++k) {
        const double v = S.Dd[base + k];
        if (v < run) dspec[of++] = k;
        run = fmax(run, v);
    }
    __syncthreads();
    if (tid == 0) {
        for (int f = 0; f < nf; ++f) {
            const int k = dspec[f];
            const double v = S.Dd[base + k];
            const int c = S.dcol[base + k], t = S.dtype[base + k];
            int j = k;
            while (j > 0 && S.Dd[base + j - 1] > v) {
                S.Dd[base + j] = S.Dd[base + j - 1];
                S.dcol[base + j] = S.dcol[base + j - 1];
                S.dtype[base + j] = S.dtype[base + j - 1];
                --j;
            }
            S.Dd[base + j] = v;
            S.dcol[base + j] = c;
            S.dtype[base + j] = t;
        }
        MergeCnt* cnt = S.cnt + N.slot;
        cnt->K = K;
        cnt->nrot = nrot;
        cnt->ndefl = nd;
        cnt->nchain = nch;
        cnt->pad_[0] = 0;
        cnt->sec_iters[0] = 0;
        cnt->sec_iters[1] = 0;
        S.rho2[N.slot] = rho2;
    }
    __syncthreads();
    // Each rotation's deflated column: its entry in the final deflated list
    // (the rotation kernel writes it straight to its output column).
    for (int k = tid; k < nd; k += NT) {
        const int t = S.dtype[base + k];
        if (t & 8) S.rdk[base + (t >> 4)] = k;
    }

    // Order-preserving lists of survivors touching the top / bottom rows
    // (the survivor panel's columns), and each survivor's place in them; both
    // lists in one pass over the survivors.
    const int lane = tid & 63, wv = tid >> 6;
    __shared__ int wsum2[NT / 64];
    int run_t = 0, run_b = 0;
    for (int c0 = 0; c0 < K; c0 += NT) {
        const int j = c0 + tid;
        const int ty = j < K ? S.stype[base + j] : 0;
        const bool ft = ty & 1, fb = ty & 2;
        const unsigned long long bt = __ballot(ft), bb = __ballot(fb);
        const unsigned long long below = (1ull << lane) - 1ull;
        if (lane == 0) {
            wsum[wv] = __popcll(bt);
            wsum2[wv] = __popcll(bb);
        }
        __syncthreads();
        int ot = 0, ob = 0, tt = 0, tb = 0;
        for (int q = 0; q < NT / 64; ++q) {
            if (q < wv) {
                ot += wsum[q];
                ob += wsum2[q];
            }
            tt += wsum[q];
            tb += wsum2[q];
        }
        if (ft) {
            const int at = run_t + ot + __popcll(bt & below);
            S.ktop[base + at] = j;
            S.ptop[base + j] = at;
        }
        if (fb) {
            const int ab = run_b + ob + __popcll(bb & below);
            S.kbot[base + ab] = j;
            S.pbot[base + j] = ab;
        }
        run_t += tt;
        run_b += tb;
        __syncthreads();
    }
    if (tid == 0) {
        MergeCnt* cnt = S.cnt + N.slot;
        cnt->ntop = run_t;
        cnt->nbot = run_b;
    }
}

// Apply the pair rotations of each merge to its basis.  In the deflation
// walk a column is shared only by consecutive rotations (the rotated survivor
// becomes the next candidate), so the rotations split into independent chains
// whose first elements the walk records.  A thread owns one row of the merge
// block and DC_ROT_CHAINS chains: the first rotation of every chain is loaded
// up front, each chain is then carried through in registers, and only final
// column values are stored: the column each rotation deflates goes, zero
// outside its row type, to its output column at the root (the eigenvalue
// order is formed before the rotations run) and over the column it came from
// below the root (read by this thread, in this row, before), and the column
// that ends a chain to the survivor panel.  Entries outside a column's rows
// are structural zeros.
__device__ __forceinline__ void rot_apply(int ty, int rbit, double c, double s, double& qp,
                                          double& qi) {
    const bool inp = (ty & rbit) != 0;
    const bool ini = ((ty >> 2) & rbit) != 0;
    if (inp || ini) {
        const double a = qp, b = qi;
        qp = c * a - s * b;
        qi = s * a + c * b;
    }
}

template <bool STRIDE>
__global__ __launch_bounds__(DC_ROWS_PER_BLOCK)
void k_rotate(const Node* __restrict__ merges, const int* __restrict__ blk_start, int nm,
              Scratch S) {
    const int mi = block_of(blk_start, nm, blockIdx.x);
    const Node N = merges[mi];
    const MergeCnt C = S.cnt[N.slot];
    if (C.nrot == 0) return;
    const int m = N.n1 + N.n2;
    const int nrb = (m + DC_ROWS_PER_BLOCK - 1) / DC_ROWS_PER_BLOCK;
    const int ngb = dc_rot_group_blocks(m, STRIDE);
    const int local = blockIdx.x - blk_start[mi];
    const int gb = local / nrb;
    if (gb * DC_ROT_CHAINS >= C.nchain) return;
    const int r = (local - gb * nrb) * DC_ROWS_PER_BLOCK + threadIdx.x;
    if (r >= m) return;
    const Prob P = S.probs[N.prob];
    const long long base = (long long)P.row0 + N.off;
    long long ld, ldo;
    const double* Qi = node_buf(P, N.depth + 1, ld);
    double* Qo = node_buf(P, N.depth, ldo);
    const bool root = N.depth == 0;
    const int ra = N.off + r;                     // row of the problem
    const double* row = Qi + ra;
    const int* __restrict__ cmap = node_cmap(S, N.depth + 1) + base;
    const int2* __restrict__ rng = node_rng(S, N.depth + 1) + base;
    // local column c in this row (0 outside its rows)
    auto child = [&](int c) {
        const int col = cmap[c];
        const int2 rg = rng[c];
        return ra >= rg.x && ra < rg.y ? row[(long long)col * ld] : 0.0;
    };
    const int rbit = r < N.n1 ? 1 : 2;
    const int* __restrict__ rt = S.rt + base;
    const int* __restrict__ rend = S.perm + base;
    const int* __restrict__ ptop = S.ptop + base;
    const int* __restrict__ pbot = S.pbot + base;
    const int* __restrict__ rdk = S.rdk + base;
    const int* __restrict__ pdef = S.pos_defl + base;
    double* panel = P.B2 + (long long)N.off * P.ld2 + N.off + r;
    // the column rotation t deflates (local column p of the pair)
    auto put = [&](int t, int p, double v) {
        const long long col = root ? N.off + pdef[rdk[t]] : cmap[p];
        Qo[col * ldo + ra] = v;
    };
    const int* __restrict__ ri = S.ri + base;
    const double* __restrict__ rc = S.rc + base;
    const double* __restrict__ rs = S.rs + base;
    // Chain groups gb, gb + ngb, ...  In each, every chain's bounds and first
    // rotation are read before any store: the stores go to Q or B1, which the
    // compiler cannot tell apart from these lists, and a read after a store
    // would cost one memory round trip per chain.  The first group is peeled
    // off the loop: its list reads precede every store of the kernel, so
    // they can go through the scalar cache (in the loop they cannot).
    auto group = [&](int cg) __attribute__((always_inline)) {
        const int ch0 = cg * DC_ROT_CHAINS;
        int t0[DC_ROT_CHAINS], t1[DC_ROT_CHAINS], ty0[DC_ROT_CHAINS], p0[DC_ROT_CHAINS],
            i0[DC_ROT_CHAINS];
        double c0[DC_ROT_CHAINS], s0[DC_ROT_CHAINS];
#pragma unroll
        for (int q = 0; q < DC_ROT_CHAINS; ++q) {
            const int ch = ch0 + q;
            t0[q] = ch < C.nchain ? S.rch[base + ch] : 0;
            t1[q] = ch < C.nchain ? (ch + 1 < C.nchain ? S.rch[base + ch + 1] : C.nrot) : 0;
        }
#pragma unroll
        for (int q = 0; q < DC_ROT_CHAINS; ++q) {
            const bool live = t0[q] < t1[q];
            const int t = live ? t0[q] : 0;
            ty0[q] = live ? rt[t] : 0;
            p0[q] = S.rp[base + t];
            i0[q] = ri[t];
            c0[q] = rc[t];
            s0[q] = rs[t];
        }
        // the first rotation's two columns of every chain: loads issued together
        double vp[DC_ROT_CHAINS], vi[DC_ROT_CHAINS];
#pragma unroll
        for (int q = 0; q < DC_ROT_CHAINS; ++q) {
            vp[q] = (ty0[q] & rbit) ? child(p0[q]) : 0.0;
            vi[q] = ((ty0[q] >> 2) & rbit) ? child(i0[q]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < DC_ROT_CHAINS; ++q) {
            if (t0[q] >= t1[q]) continue;
            double a = vp[q], b = vi[q];
            int ty = ty0[q], col_i = i0[q];
            rot_apply(ty, rbit, c0[q], s0[q], a, b);
            // the deflated column of rotation t (0 outside its row type, whose
            // rows rot_apply leaves at 0)
            put(t0[q], p0[q], a);
            // the rest of a longer chain: the previous second column is this
            // rotation's first one
            for (int t = t0[q] + 1; t < t1[q]; ++t) {
                const int col_p = col_i;
                ty = rt[t];
                col_i = ri[t];
                a = b;
                b = ((ty >> 2) & rbit) ? child(col_i) : 0.0;
                rot_apply(ty, rbit, rc[t], rs[t], a, b);
                put(t, col_p, a);
            }
            // The chain's last column is a survivor: it goes straight to its
            // column of the survivor panel (the gather skips it).
            const int ks = rend[t1[q] - 1];
            if (ks >= 0 && (S.stype[base + ks] & rbit))
                panel[(long long)(rbit == 1 ? ptop[ks] : pbot[ks]) * P.ld2] = b;
        }
    };
    group(gb);
    if (STRIDE)
        for (int cg = gb + ngb; cg * DC_ROT_CHAINS < C.nchain; cg += ngb) group(cg);
}

// Final ascending order of the merged eigenvalues: roots (ascending by
// interlacing) and deflated values (ascending) meet by a merge path; ties
// place the root first.  Writes the eigenvalues into the lam array.  At the
// root, root j's product column is its place in that order; below it, the
// column of survivor j (free once the panel holds it), and the merge's map
// sends each place to its column, with the column's rows: the merge's for
// product columns and columns deflated by rotation, the child's otherwise.
__global__ __launch_bounds__(DC_ROWS_PER_BLOCK)
void k_assemble(const Node* __restrict__ merges, const int* __restrict__ blk_start, int nm,
                Scratch S) {
    const int mi = block_of(blk_start, nm, blockIdx.x);
    const Node N = merges[mi];
    const int x = (blockIdx.x - blk_start[mi]) * DC_ROWS_PER_BLOCK + threadIdx.x;
    const int m = N.n1 + N.n2;
    if (x >= m) return;
    const MergeCnt C = S.cnt[N.slot];
    const Prob P = S.probs[N.prob];
    const long long base = (long long)P.row0 + N.off;
    const double* lr = S.lamr + base;
    const double* dd = S.Dd + base;
    // Row generators of the two half products, packed in k order.
    if (x < C.ntop) {
        const int g = S.ktop[base + x];
        S.gDt[base + x] = S.Dbar[base + g];
        S.gzt[base + x] = S.zhat[base + g];
    }
    if (x < C.nbot) {
        const int g = S.kbot[base + x];
        S.gDb[base + x] = S.Dbar[base + g];
        S.gzb[base + x] = S.zhat[base + g];
    }
    const int* cin = node_cmap(S, N.depth + 1) + base;
    int* cout = node_cmap(S, N.depth) + base;
    int2* rout = node_rng(S, N.depth) + base;
    const int2 whole = make_int2(N.off, N.off + m);
    if (x < C.K) {
        const double v = lr[x];
        const int pos = x + count_lt(dd, C.ndefl, v);
        if (N.depth > 0) {
            const int col = cin[S.surv[base + x]];
            S.pos_root[base + x] = col - N.off;
            cout[pos] = col;
            rout[pos] = whole;
        } else {
            S.pos_root[base + x] = pos;
        }
        P.d[N.off + pos] = v;
    } else {
        const int k = x - C.K;
        const double v = dd[k];
        const int pos = k + count_le(lr, C.K, v);
        S.pos_defl[base + k] = pos;
        if (N.depth > 0) {
            const int c = S.dcol[base + k];
            cout[pos] = cin[c];
            rout[pos] = (S.dtype[base + k] & 8) ? whole : node_rng(S, N.depth + 1)[base + c];
        }
        P.d[N.off + pos] = v;
    }
}

// Pack the survivor columns of each merge into the product panel: column t
// of the top panel is rows [0, n1) of the basis column of top-list entry t,
// column t of the bottom panel rows [n1, m) of bottom-list entry t.
__global__ __launch_bounds__(256)
void k_gather(const Node* __restrict__ merges, const int* __restrict__ blk_start, int nm,
              bool stride, Scratch S) {
    const int mi = block_of(blk_start, nm, blockIdx.x);
    const Node N = merges[mi];
    const MergeCnt C = S.cnt[N.slot];
    const int local = blockIdx.x - blk_start[mi];
    const int ncols = max(C.ntop, C.nbot);
    if (local * DC_GATHER_COLS >= ncols) return;
    const int step = dc_gather_blocks(N.n1 + N.n2, stride) * DC_GATHER_COLS;
    const Prob P = S.probs[N.prob];
    const long long base = (long long)P.row0 + N.off;
    long long ldi;
    const double* Qi = node_buf(P, N.depth + 1, ldi);
    const int* cmap = node_cmap(S, N.depth + 1) + base;
    double* G = P.B2 + (long long)N.off * P.ld2 + N.off;
    // rows [r0, r0 + nr) of the merge block of survivor ks into panel column
    // t, zero outside the column's rows
    auto pack = [&](int ks, int t, int r0, int nr) {
        const int c = S.surv[base + ks];
        const int col = cmap[c];
        const int2 rg = node_rng(S, N.depth + 1)[base + c];
        const int lo = rg.x - N.off - r0;
        const int hi = rg.y - N.off - r0;
        const double* a = Qi + (long long)col * ldi + N.off + r0;
        double* o = G + (long long)t * P.ld2 + r0;
        for (int r = threadIdx.x; r < nr; r += 256) o[r] = r >= lo && r < hi ? a[r] : 0.0;
    };
    if (stride) {
        // Small merges: the workgroup's (at most DC_GROUPS_PER_BLOCK) column
        // groups are resolved first, one thread per (column, half) following
        // its chain of list, type, survivor, map and row-range loads at once
        // (one after another per column, those chains were most of the
        // kernel), then a wave copies each column's few rows.
        constexpr int NSL = 2 * DC_GATHER_COLS * DC_GROUPS_PER_BLOCK;
        __shared__ int s_col[NSL], s_lo[NSL], s_hi[NSL], s_t[NSL];
        const int first = local * DC_GATHER_COLS;
        const int ng = (ncols - first + step - 1) / step;
        const int nsl = min(ng, DC_GROUPS_PER_BLOCK) * 2 * DC_GATHER_COLS;
        for (int i = threadIdx.x; i < nsl; i += 256) {
            const int q = i / (2 * DC_GATHER_COLS), u = (i >> 1) % DC_GATHER_COLS, h = i & 1;
            const int t = first + q * step + u;
            int col = -1, lo = 0, hi = 0;
            if (t < (h ? C.nbot : C.ntop)) {
                const int ks = (h ? S.kbot : S.ktop)[base + t];
                // (survivors that end a rotation chain were written by the rotation)
                if (!(S.stype[base + ks] & 4)) {
                    const int c = S.surv[base + ks];
                    const int2 rg = node_rng(S, N.depth + 1)[base + c];
                    const int r0 = h ? N.n1 : 0;
                    col = cmap[c];
                    lo = rg.x - N.off - r0;
                    hi = rg.y - N.off - r0;
                }
            }
            s_col[i] = col;
            s_lo[i] = lo;
            s_hi[i] = hi;
            s_t[i] = t;
        }
        __syncthreads();
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int i = wv; i < nsl; i += 4) {
            const int col = s_col[i];
            if (col < 0) continue;
            const int h = i & 1;
            const int r0 = h ? N.n1 : 0, nr = h ? N.n2 : N.n1;
            const int lo = s_lo[i], hi = s_hi[i];
            const double* a = Qi + (long long)col * ldi + N.off + r0;
            double* o = G + (long long)s_t[i] * P.ld2 + r0;
            for (int r = lane; r < nr; r += 64) o[r] = r >= lo && r < hi ? a[r] : 0.0;
        }
        return;
    }
    for (int t0 = local * DC_GATHER_COLS; t0 < ncols; t0 += step) {
        for (int t = t0; t < t0 + DC_GATHER_COLS; ++t) {
            // (survivors that end a rotation chain were written by the rotation)
            if (t < C.ntop) {
                const int ks = S.ktop[base + t];
                if (!(S.stype[base + ks] & 4)) pack(ks, t, 0, N.n1);
            }
            if (t < C.nbot) {
                const int ks = S.kbot[base + t];
                if (!(S.stype[base + ks] & 4)) pack(ks, t, N.n1, N.n2);
            }
        }
    }
}

// Deflated eigenvectors of the root merges not produced by a rotation: the
// basis column itself, zero outside its rows, written to its place in Q.
// (Below the root deflated columns do not move; the level loop launches this
// only for the roots.)
__global__ __launch_bounds__(256)
void k_copy_deflated(const Node* __restrict__ merges, const int* __restrict__ blk_start,
                     int nm, Scratch S) {
    const int mi = block_of(blk_start, nm, blockIdx.x);
    const Node N = merges[mi];
    const MergeCnt C = S.cnt[N.slot];
    const int k0 = (blockIdx.x - blk_start[mi]) * DC_COLS_PER_BLOCK;
    if (N.depth > 0 || k0 >= C.ndefl) return;
    const Prob P = S.probs[N.prob];
    const long long base = (long long)P.row0 + N.off;
    const int m = N.n1 + N.n2;
    const int* cmap = node_cmap(S, 1) + base;
    const int2* rng = node_rng(S, 1) + base;
    long long ldi, ldo;
    const double* Qi = node_buf(P, 1, ldi);
    double* Qo = node_buf(P, 0, ldo);
    for (int k = k0; k < min(C.ndefl, k0 + DC_COLS_PER_BLOCK); ++k) {
        const int ty = S.dtype[base + k];
        if (ty & 8) continue;                // written by the rotation kernel
        const int c = S.dcol[base + k];
        const int col = cmap[c];
        const int lo = rng[c].x - N.off;
        const int hi = rng[c].y - N.off;
        const int dst = S.pos_defl[base + k];
        const double* a = Qi + (long long)col * ldi + N.off;
        double* o = Qo + (long long)(N.off + dst) * ldo + N.off;
        for (int r = threadIdx.x; r < m; r += 256) o[r] = r >= lo && r < hi ? a[r] : 0.0;
    }
}

}  // namespace

hipError_t dc_launch_set_probs(const Prob* host_probs, int count, Prob* dev, hipStream_t s) {
    for (int first = 0; first < count; first += 8) {
        ProbPack pk;
        const int c = count - first < 8 ? count - first : 8;
        for (int i = 0; i < c; ++i) pk.p[i] = host_probs[first + i];
        hipLaunchKernelGGL(k_write_probs, dim3(1), dim3(64), 0, s, dev, first, c, pk);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t dc_launch_build(const Node* merges, int nm, int bm, int bn, Scratch S,
                           hipStream_t s) {
    if (nm <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build, dim3((nm + 127) / 128), dim3(128), 0, s, merges, nm, bm, bn,
                       S);
    return hipGetLastError();
}

hipError_t dc_launch_deflate(const Node* merges, const int* row_start, int nm, int nrow_blk,
                             int max_m, Scratch S, hipStream_t s) {
    if (nm <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_sort, dim3(nrow_blk), dim3(DC_ROWS_PER_BLOCK), 0, s, merges,
                       row_start, nm, S);
    if (max_m <= 128)
        hipLaunchKernelGGL(k_deflate<64>, dim3(nm), dim3(64), 0, s, merges, S);
    else if (max_m <= 512)
        hipLaunchKernelGGL(k_deflate<256>, dim3(nm), dim3(256), 0, s, merges, S);
    else
        hipLaunchKernelGGL(k_deflate<1024>, dim3(nm), dim3(1024), 0, s, merges, S);
    return hipGetLastError();
}

hipError_t dc_launch_rotate(const Node* merges, const int* blk_start, int nm, int nblk,
                            bool stride, Scratch S, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    if (stride)
        hipLaunchKernelGGL(k_rotate<true>, dim3(nblk), dim3(DC_ROWS_PER_BLOCK), 0, s, merges,
                           blk_start, nm, S);
    else
        hipLaunchKernelGGL(k_rotate<false>, dim3(nblk), dim3(DC_ROWS_PER_BLOCK), 0, s, merges,
                           blk_start, nm, S);
    return hipGetLastError();
}

hipError_t dc_launch_assemble(const Node* merges, const int* blk_start, int nm, int nblk,
                              Scratch S, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_assemble, dim3(nblk), dim3(DC_ROWS_PER_BLOCK), 0, s, merges,
                       blk_start, nm, S);
    return hipGetLastError();
}

hipError_t dc_launch_gather(const Node* merges, const int* blk_start, int nm, int nblk,
                            bool stride, Scratch S, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(nblk), dim3(256), 0, s, merges, blk_start, nm, stride,
                       S);
    return hipGetLastError();
}

hipError_t dc_launch_copy_deflated(const Node* merges, const int* blk_start, int nm,
                                   int nblk, Scratch S, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_deflated, dim3(nblk), dim3(256), 0, s, merges, blk_start, nm,
                       S);
    return hipGetLastError();
}
