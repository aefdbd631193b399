// Leaf eigensolver: Algorithm 1's "apply the QR algorithm" on every block of
// at most 64 rows, one wave per leaf.
//
// Implicit symmetric tridiagonal QR with a Wilkinson shift (Golub & Van Loan,
// section 8.3).  The tridiagonal lives in registers, entry i in lane i; the
// bulge chase is a chain of Givens steps that every lane evaluates
// identically, reading entries ahead of the chase with readlane and carrying
// the entries the chase has touched in registers, while lane r applies each
// rotation to row r of the eigenvector block (one LDS read and one write per
// step: the column the chase leaves behind).  The leaf is scaled by a power of
// two (exact) so that x^2 + y^2 of a rotation neither overflows nor
// underflows on the usual path; deflation uses the absolute threshold
// eps * ||T||_inf of the leaf.
//
// The leaf's diagonal carries the tear corrections of eq. T2: every boundary
// between two adjacent leaves is the split point of exactly one merge, whose
// coupling rho = |e_k| is subtracted from both rows next to it.
#include "dc_internal.hpp"

namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr int MAX_SWEEPS = 40;

// Value of v in lane k (k wave-uniform).
__device__ __forceinline__ double lane_value(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double set_lane(double v, int k, double x) {
    return (int)threadIdx.x == k ? x : v;
}

// Givens rotation c = x / r, s = y / r, r = sqrt(x^2 + y^2), so that
// c x + s y = r and c y - s x = 0.  The reciprocal square root is the
// hardware estimate refined by two Newton steps q <- q (3 - t q^2) / 2 when t
// lies well inside the exponent range; hypot and divisions otherwise.
__device__ __forceinline__ void givens(double x, double y, double& c, double& s, double& r) {
    if (y == 0.0) {
        c = 1.0;
        s = 0.0;
        r = x;
        return;
    }
    const double t = __builtin_fma(x, x, y * y);
    if (t > 0x1p-960 && t < 0x1p960) {
        const double h = 0.5 * t;
        double q = __builtin_amdgcn_rsq(t);
        double e = __builtin_fma(-h * q, q, 0.5);
        q = __builtin_fma(q, e, q);
        e = __builtin_fma(-h * q, q, 0.5);
        q = __builtin_fma(q, e, q);
        c = x * q;
        s = y * q;
        r = t * q;
    } else {
        r = hypot(x, y);
        c = x / r;
        s = y / r;
    }
}

// LD: leaf size bound and row stride of the eigenvector block in LDS (16,
// 32 or 64): a block sized for the plan's leaves lets more of them share a
// compute unit, which hides the chase's latency.
template <int LD>
__global__ __launch_bounds__(64)
void k_leaf(const Node* __restrict__ leaves, Scratch S) {
    __shared__ double Z[LD * LD];   // column-major, LD rows
    __shared__ double sd[LD];
    __shared__ int rank[LD];

    const Node L = leaves[blockIdx.x];
    const Prob P = S.probs[L.prob];
    const double esc = S.psc[L.prob];        // d is scaled in place, e on read
    const int nl = L.n1;
    const int lane = threadIdx.x;
    const bool zrow = LD == 64 || lane < LD;   // lane holds a row of the block
    const int off = L.off;

    // Load, apply the tear corrections, check for non-finite input.
    bool bad = false;
    double dv = 0.0, ev = 0.0;
    if (lane < nl) {
        dv = P.d[off + lane];
        bad |= !isfinite(dv);
        if (lane == 0 && off > 0) {
            const double x = P.e[off - 1] * esc;
            bad |= !isfinite(x);
            dv -= fabs(x);
        }
        if (lane == nl - 1 && off + nl < P.n) {
            const double x = P.e[off + nl - 1] * esc;
            bad |= !isfinite(x);
            dv -= fabs(x);
        }
        if (lane < nl - 1) {
            ev = P.e[off + lane] * esc;
            bad |= !isfinite(ev);
        }
    }
    if (__ballot(bad) != 0ull && lane == 0) dc_set_info(P.info, DC_STATUS_NONFINITE);
    if (zrow)
        for (int c = 0; c < nl; ++c) Z[c * LD + lane] = (c == lane) ? 1.0 : 0.0;

    // ||T||_inf of the leaf, then an exact power-of-two scale to [1, 2).
    const double eprev = __shfl_up(ev, 1, 64);
    double rowsum = lane < nl ? fabs(dv) + fabs(ev) + (lane > 0 ? fabs(eprev) : 0.0) : 0.0;
    double anorm = lane_value(dc_wave_max(rowsum), 0);
    double unscale = 1.0;
    if (anorm > 0.0 && anorm < INFINITY) {
        const int ex = (int)((__double_as_longlong(anorm) >> 52) & 0x7ff) - 1023;
        if (ex > -1000 && ex < 1000) {
            const double sc = __longlong_as_double((long long)(1023 - ex) << 52);
            unscale = __longlong_as_double((long long)(1023 + ex) << 52);
            dv *= sc;
            ev *= sc;
            anorm *= sc;
        }
    }
    const double thresh = EPS * anorm;

    int hi = nl - 1;
    int sweeps = 0;
    bool failed = false;
    while (hi > 0) {
        const double ehi = lane_value(ev, hi - 1);
        if (fabs(ehi) <= thresh) {
            ev = set_lane(ev, hi - 1, 0.0);
            --hi;
            sweeps = 0;
            continue;
        }
        // lo: one past the last negligible off-diagonal below hi - 1
        const unsigned long long small = __ballot(lane < hi - 1 && fabs(ev) <= thresh);
        const int lo = small ? 64 - __builtin_clzll(small) : 0;
        if (lo > 0) ev = set_lane(ev, lo - 1, 0.0);
        if (++sweeps > MAX_SWEEPS) { failed = true; break; }
        const double dhi = lane_value(dv, hi);
        const double delta = 0.5 * (lane_value(dv, hi - 1) - dhi);
        const double sgn = delta >= 0.0 ? 1.0 : -1.0;
        const double mu = dhi - ehi * ehi / (delta + sgn * hypot(delta, ehi));

        // Entries ahead of the chase are read from the sweep's starting
        // values (d0, e0); the chase writes its finished entries into dv, ev.
        const double d0 = dv, e0 = ev;
        double a = lane_value(d0, lo);           // current d[k]
        double f = lane_value(e0, lo);           // current e[k]
        double x = a - mu, y = f;
        double zc = zrow ? Z[lo * LD + lane] : 0.0;   // current column k, this row
        double g = lane_value(d0, lo + 1);
        double en = lo + 1 < hi ? lane_value(e0, lo + 1) : 0.0;
        double zn = zrow ? Z[(lo + 1) * LD + lane] : 0.0;
        for (int k = lo; k < hi; ++k) {
            double g2 = 0.0, en2 = 0.0, zn2 = 0.0;
            if (k + 2 <= hi) {
                g2 = lane_value(d0, k + 2);
                zn2 = zrow ? Z[(k + 2) * LD + lane] : 0.0;
            }
            if (k + 2 < hi) en2 = lane_value(e0, k + 2);
            double c, s, r;
            givens(x, y, c, s, r);
            if (k > lo) ev = set_lane(ev, k - 1, r);
            const double cc = c * c, ss = s * s, cs = c * s;
            dv = set_lane(dv, k, cc * a + 2.0 * cs * f + ss * g);
            const double gn = ss * a - 2.0 * cs * f + cc * g;
            const double fn = cs * (g - a) + (cc - ss) * f;
            if (zrow) Z[k * LD + lane] = c * zc + s * zn;
            zc = -s * zc + c * zn;
            y = s * en;                           // the bulge (0 at the last step)
            f = c * en;
            x = fn;
            a = gn;
            g = g2;
            en = en2;
            zn = zn2;
        }
        dv = set_lane(dv, hi, a);
        ev = set_lane(ev, hi - 1, x);
        if (zrow) Z[hi * LD + lane] = zc;
    }
    if (failed && lane == 0) dc_set_info(P.info, 1 + off);
    dv *= unscale;
    if (lane < nl) sd[lane] = dv;
    __syncthreads();

    // Ascending order: rank of each eigenvalue, ties by index; NaN ranks as
    // +inf so the ranks always form a permutation.
    if (lane < nl) {
        const double v = isnan(dv) ? INFINITY : dv;
        int r = 0;
        for (int k = 0; k < nl; ++k) {
            const double u = isnan(sd[k]) ? INFINITY : sd[k];
            r += (u < v) || (u == v && k < lane);
        }
        rank[lane] = r;
    }
    __syncthreads();
    long long ld;
    double* Qo = node_buf(P, L.depth, ld);
    if (lane < nl) {
        P.d[off + rank[lane]] = dv;
        for (int c = 0; c < nl; ++c)
            Qo[(long long)(off + rank[c]) * ld + off + lane] = Z[c * LD + lane];
        if (L.depth > 0) {
            // below the root: eigenvalue j in column off + j, rows of the leaf
            const long long g = (long long)P.row0 + off + lane;
            node_cmap(S, L.depth)[g] = off + lane;
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
        hipLaunchKernelGGL(k_leaf<16>, dim3(nleaves), dim3(64), 0, s, leaves, S);
    else if (max_leaf <= 32)
        hipLaunchKernelGGL(k_leaf<32>, dim3(nleaves), dim3(64), 0, s, leaves, S);
    else
        hipLaunchKernelGGL(k_leaf<64>, dim3(nleaves), dim3(64), 0, s, leaves, S);
    return hipGetLastError();
}
