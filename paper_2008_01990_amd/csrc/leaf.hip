// Leaf eigensolver: Algorithm 1's "apply the QR algorithm" on every block of
// at most 64 rows; a wave holds 64 / LD leaves of at most LD rows each.
//
// Implicit symmetric tridiagonal QR with a Wilkinson shift (Golub & Van Loan,
// section 8.3).  The bulge chase is a chain of Givens steps that every lane
// of the leaf's lane group evaluates identically, reading the entries ahead
// of the chase from the tridiagonal in LDS and carrying the entries it has
// touched in registers, while lane r applies each rotation to row r of the
// eigenvector block (one LDS read and one write per step: the column the
// chase leaves behind).  The leaf is scaled by a power of two (exact) so that
// x^2 + y^2 of a rotation neither overflows nor underflows on the usual path;
// deflation uses the absolute threshold eps * ||T||_inf of the leaf.
//
// The leaf's diagonal carries the tear corrections of eq. T2: every boundary
// between two adjacent leaves is the split point of exactly one merge, whose
// coupling rho = |e_k| is subtracted from both rows next to it.
#include "dc_internal.hpp"

namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr int MAX_SWEEPS = 40;

// Givens rotation with c >= 0 and r carrying the sign of x, so that
// c x + s y = r and c y - s x = 0 (r = x, c = 1, s = 0 when y = 0).  The
// reciprocal square root of t = x^2 + y^2 is the hardware estimate refined
// by two Newton steps q <- q (3 - t q^2) / 2.  That branch-free form is
// taken by the whole wave unless one of its lanes has t outside the safe
// exponent range (t = 0 included); those waves take the per-lane path, with
// hypot and divisions for such lanes.
__device__ __forceinline__ void givens(double x, double y, double& c, double& s, double& r) {
    const double t = __builtin_fma(x, x, y * y);
    const bool fast = t > 0x1p-960 && t < 0x1p960;
    auto refined = [&]() {
        const double h = 0.5 * t;
        double q = __builtin_amdgcn_rsq(t);
        double e = __builtin_fma(-h * q, q, 0.5);
        q = __builtin_fma(q, e, q);
        e = __builtin_fma(-h * q, q, 0.5);
        q = __builtin_fma(q, e, q);
        q = copysign(q, x);
        c = x * q;
        s = y * q;
        r = t * q;
    };
    if (__builtin_expect(__ballot(!fast) == 0ull, 1)) {
        refined();
    } else if (y == 0.0) {
        c = 1.0;
        s = 0.0;
        r = x;
    } else if (fast) {
        refined();
    } else {
        r = copysign(hypot(x, y), x);
        c = x / r;
        s = y / r;
    }
}

// LD: leaf size bound and row stride of the eigenvector block in LDS (16,
// 32 or 64).  A wave holds 64 / LD leaves, lane group g = lane / LD solving
// leaf blockIdx.x * (64 / LD) + g with row r = lane % LD: each group computes
// its own chase in its own lanes, so one instruction of a chase step advances
// 64 / LD leaves at once (the chase's cost is instruction issue, shared by the
// waves of a SIMD).  The tridiagonal lives in
// LDS as pairs (e[k-1], d[k]): the chase reads entries ahead of it with one
// broadcast load per step and lane 0 of the group writes each finished pair
// back, so no register selects or lane permutes sit in the step.  A group that
// needs no sweep waits for the others' chases with its lanes masked off, so
// every pass of the sweep loop deflates first and chases at most once per
// group.
template <int LD>
__global__ __launch_bounds__(64)
void k_leaf(const Node* __restrict__ leaves, int nleaves, Scratch S) {
    constexpr int NPW = 64 / LD;                // leaves per wave
    __shared__ double Zall[NPW * LD * LD];      // per group: column-major, LD rows
    __shared__ double2 tdall[NPW * LD];         // per group: (e[k-1], d[k])
    __shared__ double sdall[NPW * LD];
    __shared__ int rankall[NPW * LD];

    const int lane = threadIdx.x;
    const int grp = lane / LD, r = lane - (lane / LD) * LD;
    const int li = blockIdx.x * NPW + grp;
    double* __restrict__ Z = Zall + grp * LD * LD;
    double2* __restrict__ td = tdall + grp * LD;
    double* __restrict__ sd = sdall + grp * LD;
    int* __restrict__ rank = rankall + grp * LD;
    // the group's bits of a wave ballot
    auto gbits = [&](unsigned long long m) {
        return LD == 64 ? m : (m >> (grp * LD)) & ((1ull << (LD & 63)) - 1ull);
    };

    Node L = {};
    Prob P = {};
    double esc = 1.0;
    int nl = 0;
    if (li < nleaves) {
        L = leaves[li];
        P = S.probs[L.prob];
        esc = S.psc[L.prob];                    // d is scaled in place, e on read
        nl = L.n1;
    }
    const int off = nl > 0 ? L.off : 0;

    // Load, apply the tear corrections, check for non-finite input.
    bool bad = false;
    double dv = 0.0, ev = 0.0;
    if (r < nl) {
        dv = P.d[off + r];
        bad |= !isfinite(dv);
        if (r == 0 && off > 0) {
            const double x = P.e[off - 1] * esc;
            bad |= !isfinite(x);
            dv -= fabs(x);
        }
        if (r == nl - 1 && off + nl < P.n) {
            const double x = P.e[off + nl - 1] * esc;
            bad |= !isfinite(x);
            dv -= fabs(x);
        }
        if (r < nl - 1) {
            ev = P.e[off + r] * esc;
            bad |= !isfinite(ev);
        }
    }
    if (gbits(__ballot(bad)) != 0ull && r == 0) dc_set_info(P.info, DC_STATUS_NONFINITE);
    for (int c = 0; c < nl; ++c) Z[c * LD + r] = (c == r) ? 1.0 : 0.0;

    // ||T||_inf of the leaf, then an exact power-of-two scale to [1, 2).
    double eprev = __shfl_up(ev, 1, LD);
    if (r == 0) eprev = 0.0;
    double anorm = r < nl ? fabs(dv) + fabs(ev) + fabs(eprev) : 0.0;
#pragma unroll
    for (int o = LD / 2; o > 0; o >>= 1) anorm = fmax(anorm, __shfl_xor(anorm, o, 64));
    double unscale = 1.0;
    if (anorm > 0.0 && anorm < INFINITY) {
        const int ex = (int)((__double_as_longlong(anorm) >> 52) & 0x7ff) - 1023;
        if (ex > -1000 && ex < 1000) {
            const double sc = __longlong_as_double((long long)(1023 - ex) << 52);
            unscale = __longlong_as_double((long long)(1023 + ex) << 52);
            dv *= sc;
            eprev *= sc;
            anorm *= sc;
        }
    }
    const double thresh = EPS * anorm;
    // every pair of the block is written (zeros past the leaf), so reads
    // ahead of the chase past hi see finite values
    td[r] = make_double2(eprev, dv);
    __syncthreads();

    int hi = nl - 1;
    int sweeps = 0;
    bool failed = false;
    while (true) {
        // Pairs written by lane 0 are read by the whole group below: LDS
        // operations of a wave complete in order, and the fence keeps the
        // compiler from moving those reads above the writes.
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // deflate at the bottom until the last off-diagonal is not negligible
        double ehi = hi > 0 ? td[hi].x : 0.0;
        while (hi > 0 && fabs(ehi) <= thresh) {
            if (r == 0) td[hi].x = 0.0;
            --hi;
            sweeps = 0;
            ehi = hi > 0 ? td[hi].x : 0.0;
        }
        if (hi <= 0) break;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // lo: one past the last negligible off-diagonal below hi - 1
        bool neg = false;
        if (r < hi - 1) neg = fabs(td[r + 1].x) <= thresh;
        const unsigned long long small = gbits(__ballot(neg));
        const int lo = small ? 64 - __builtin_clzll(small) : 0;
        if (lo > 0 && r == 0) td[lo].x = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (++sweeps > MAX_SWEEPS) { failed = true; break; }
        const double dhi = td[hi].y;
        const double delta = 0.5 * (td[hi - 1].y - dhi);
        const double sgn = delta >= 0.0 ? 1.0 : -1.0;
        const double mu = dhi - ehi * ehi / (delta + sgn * hypot(delta, ehi));

        // Step k rotates rows and columns k, k + 1 with the Givens rotation
        // that maps (x, y) to (rr, 0): with u = s (g - a) + 2 c f, the new
        // d[k] = a + s u, d[k+1] = g - s u (the trace is kept) and
        // e[k] = c u - f (using c^2 + s^2 = 1); rr is the new e[k-1], and
        // the rotation moves the bulge s e[k+1] one row down.  Step k reads
        // pair k + 2 (d[k+2]) and pair k + 3 (e[k+2]) for the next step,
        // before this sweep writes them, and writes pair k.  Reads are
        // clamped inside the block; past hi they feed only values the sweep
        // never uses (g and zn after the last step, en at it).
        double a = td[lo].y;                     // current d[k]
        const double2 p1 = td[lo + 1];
        double f = p1.x;                         // current e[k]
        double g = p1.y;                         // d[k+1]
        double x = a - mu, y = f;
        double en = td[min(lo + 2, LD - 1)].x;   // e[k+1]
        double zc = Z[lo * LD + r];              // current column k, this row
        double zn = Z[(lo + 1) * LD + r];
        auto step = [&](int k, auto first_tag) {
            constexpr bool FIRST = decltype(first_tag)::value;
            const int k2 = min(k + 2, LD - 1);
            const double g2 = td[k2].y;
            const double en2 = td[min(k + 3, LD - 1)].x;
            const double zn2 = Z[k2 * LD + r];
            double c, s, rr;
            givens(x, y, c, s, rr);
            const double cf = c * f;
            const double u = __builtin_fma(s, g - a, cf + cf);
            const double su = s * u;
            // the first rotation makes no off-diagonal entry: e[lo-1] stays 0
            if (r == 0) td[k] = make_double2(FIRST ? 0.0 : rr, a + su);
            x = __builtin_fma(c, u, -f);
            a = g - su;
            Z[k * LD + r] = __builtin_fma(c, zc, s * zn);
            zc = __builtin_fma(c, zn, -(s * zc));
            y = s * en;                           // the bulge
            f = c * en;
            g = g2;
            en = en2;
            zn = zn2;
        };
        step(lo, dc_true_type{});
        for (int k = lo + 1; k < hi; ++k) step(k, dc_false_type{});
        if (r == 0) td[hi] = make_double2(x, a);
        Z[hi * LD + r] = zc;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    dv = td[r].y;
    if (failed && r == 0) dc_set_info(P.info, 1 + off);
    dv *= unscale;
    if (r < nl) sd[r] = dv;
    __syncthreads();

    // Ascending order: rank of each eigenvalue, ties by index; NaN ranks as
    // +inf so the ranks always form a permutation.
    if (r < nl) {
        const double v = isnan(dv) ? INFINITY : dv;
        int q = 0;
        for (int k = 0; k < nl; ++k) {
            const double u = isnan(sd[k]) ? INFINITY : sd[k];
            q += (u < v) || (u == v && k < r);
        }
        rank[r] = q;
    }
    __syncthreads();
    if (r < nl) {
        long long ld;
        double* Qo = node_buf(P, L.depth, ld);
        P.d[off + rank[r]] = dv;
        for (int c = 0; c < nl; ++c)
            Qo[(long long)(off + rank[c]) * ld + off + r] = Z[c * LD + r];
        if (L.depth > 0) {
            // below the root: eigenvalue j in column off + j, rows of the leaf
            const long long g = (long long)P.row0 + off + r;
            node_cmap(S, L.depth)[g] = off + r;
            node_rng(S, L.depth)[g] = make_int2(off, off + nl);
        }
    }
}

// Per problem: the power of two 2^-x with max(|d|, |e|) 2^-x in [1, 2)
// (x clamped to [-1020, 1020]; 1 for an all-zero or non-finite maximum), d
// scaled by it in place; or, undoing, the eigenvalues in d divided by it.
__global__ __launch_bounds__(256)
void k_scale(Scratch S, bool undo) {
    __shared__ double wmax[4];
    __shared__ double s_sc;
    const Prob P = S.probs[blockIdx.x];
    const int n = P.n;
    const int tid = threadIdx.x;
    if (undo) {
        const double inv = 1.0 / S.psc[blockIdx.x];
        for (int i = tid; i < n; i += 256) P.d[i] *= inv;
        return;
    }
    double m = 0.0;
    for (int i = tid; i < n; i += 256) {
        m = fmax(m, fabs(P.d[i]));
        if (i < n - 1) m = fmax(m, fabs(P.e[i]));
    }
    m = dc_wave_max(m);
    if ((tid & 63) == 0) wmax[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        double sc = 1.0;
        if (m > 0.0 && m < INFINITY) {
            int ex = (int)((__double_as_longlong(m) >> 52) & 0x7ff) - 1023;
            ex = min(max(ex, -1020), 1020);
            sc = __longlong_as_double((long long)(1023 - ex) << 52);
        }
        s_sc = sc;
        S.psc[blockIdx.x] = sc;
    }
    __syncthreads();
    const double sc = s_sc;
    for (int i = tid; i < n; i += 256) P.d[i] *= sc;
}

}  // namespace

hipError_t dc_launch_scale(int nprob, bool undo, Scratch S, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(nprob), dim3(256), 0, s, S, undo);
    return hipGetLastError();
}

hipError_t dc_launch_leaf(const Node* leaves, int nleaves, int max_leaf, Scratch S,
                          hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    if (max_leaf <= 16)
        hipLaunchKernelGGL(k_leaf<16>, dim3((nleaves + 3) / 4), dim3(64), 0, s, leaves,
                           nleaves, S);
    else if (max_leaf <= 32)
        hipLaunchKernelGGL(k_leaf<32>, dim3((nleaves + 1) / 2), dim3(64), 0, s, leaves,
                           nleaves, S);
    else
        hipLaunchKernelGGL(k_leaf<64>, dim3(nleaves), dim3(64), 0, s, leaves, nleaves, S);
    return hipGetLastError();
}
