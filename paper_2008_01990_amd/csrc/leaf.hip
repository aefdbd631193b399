// Leaf eigensolver: Algorithm 1's "apply the QR algorithm" on every block of
// at most 64 rows, one wave per leaf.
//
// Implicit symmetric tridiagonal QR with a Wilkinson shift (Golub & Van Loan,
// section 8.3): the bulge chase is a chain of scalar Givens steps that every
// lane evaluates identically from LDS, while lane r applies each rotation to
// row r of the eigenvector block kept in LDS.  Deflation uses the absolute
// threshold eps * ||T||_inf of the leaf.
//
// The leaf's diagonal carries the tear corrections of eq. T2: every boundary
// between two adjacent leaves is the split point of exactly one merge, whose
// coupling rho = |e_k| is subtracted from both rows next to it.
#include "dc_internal.hpp"

namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr int MAX_SWEEPS = 40;

__global__ __launch_bounds__(64)
void k_leaf(const Node* __restrict__ leaves, Scratch S) {
    __shared__ double Z[DC_MAX_LEAF * DC_MAX_LEAF];   // column-major, 64 rows
    __shared__ double sd[DC_MAX_LEAF];
    __shared__ double se[DC_MAX_LEAF];
    __shared__ int rank[DC_MAX_LEAF];

    const Node L = leaves[blockIdx.x];
    const Prob P = S.probs[L.prob];
    const int nl = L.n1;
    const int lane = threadIdx.x;
    const int off = L.off;

    // Load, apply the tear corrections, check for non-finite input.
    bool bad = false;
    if (lane < nl) {
        double dv = P.d[off + lane];
        bad |= !isfinite(dv);
        if (lane == 0 && off > 0) {
            const double ev = P.e[off - 1];
            bad |= !isfinite(ev);
            dv -= fabs(ev);
        }
        if (lane == nl - 1 && off + nl < P.n) {
            const double ev = P.e[off + nl - 1];
            bad |= !isfinite(ev);
            dv -= fabs(ev);
        }
        sd[lane] = dv;
        if (lane < nl - 1) {
            const double ev = P.e[off + lane];
            bad |= !isfinite(ev);
            se[lane] = ev;
        }
    }
    if (__ballot(bad) != 0ull && lane == 0) dc_set_info(P.info, DC_STATUS_NONFINITE);
    for (int c = 0; c < nl; ++c) Z[c * DC_MAX_LEAF + lane] = (c == lane) ? 1.0 : 0.0;
    __syncthreads();

    // Absolute deflation threshold eps * ||T||_inf.
    double anorm = 0.0;
    for (int i = 0; i < nl; ++i) {
        double r = fabs(sd[i]);
        if (i > 0) r += fabs(se[i - 1]);
        if (i < nl - 1) r += fabs(se[i]);
        anorm = fmax(anorm, r);
    }
    const double thresh = EPS * anorm;

    int hi = nl - 1;
    int sweeps = 0;
    bool failed = false;
    while (hi > 0) {
        if (fabs(se[hi - 1]) <= thresh) {
            se[hi - 1] = 0.0;
            --hi;
            sweeps = 0;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && fabs(se[lo - 1]) > thresh) --lo;
        if (lo > 0) se[lo - 1] = 0.0;
        if (++sweeps > MAX_SWEEPS) { failed = true; break; }
        const double delta = 0.5 * (sd[hi - 1] - sd[hi]);
        const double b = se[hi - 1];
        const double sgn = delta >= 0.0 ? 1.0 : -1.0;
        const double mu = sd[hi] - b * b / (delta + sgn * hypot(delta, b));
        double x = sd[lo] - mu;
        double y = se[lo];
        double bulge = 0.0;
        for (int k = lo; k < hi; ++k) {
            if (k > lo) { x = se[k - 1]; y = bulge; }
            double c = 1.0, s = 0.0, r = x;
            if (y != 0.0) {
                r = hypot(x, y);
                c = x / r;
                s = y / r;
            }
            if (k > lo) se[k - 1] = r;
            const double a = sd[k], f = se[k], g = sd[k + 1];
            sd[k] = c * c * a + 2.0 * c * s * f + s * s * g;
            sd[k + 1] = s * s * a - 2.0 * c * s * f + c * c * g;
            se[k] = c * s * (g - a) + (c * c - s * s) * f;
            if (k + 1 < hi) {
                bulge = s * se[k + 1];
                se[k + 1] = c * se[k + 1];
            }
            if (lane < nl) {
                const double zk = Z[k * DC_MAX_LEAF + lane];
                const double zk1 = Z[(k + 1) * DC_MAX_LEAF + lane];
                Z[k * DC_MAX_LEAF + lane] = c * zk + s * zk1;
                Z[(k + 1) * DC_MAX_LEAF + lane] = -s * zk + c * zk1;
            }
        }
    }
    if (failed && lane == 0) dc_set_info(P.info, 1 + P.row0 + off);
    __syncthreads();

    // Ascending order: rank of each eigenvalue, ties by index; NaN ranks as
    // +inf so the ranks always form a permutation.
    if (lane < nl) {
        const double v = isnan(sd[lane]) ? INFINITY : sd[lane];
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
        P.d[off + rank[lane]] = sd[lane];
        for (int c = 0; c < nl; ++c)
            Qo[(long long)(off + rank[c]) * ld + off + lane] = Z[c * DC_MAX_LEAF + lane];
    }
}

}  // namespace

hipError_t dc_launch_leaf(const Node* leaves, int nleaves, Scratch S, hipStream_t s) {
    if (nleaves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaf, dim3(nleaves), dim3(64), 0, s, leaves, S);
    return hipGetLastError();
}
