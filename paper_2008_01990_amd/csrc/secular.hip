// Secular roots, Loewner recomputation and column scales of one or many
// rank-one modified diagonal problems M = diag(D) + rho z z^T (eq. rankone).
//
// Roots (eq. secular, summation restored): f(lam) = 1 + rho sum z_i^2/(D_i - lam)
// has one root in each (D_j, D_{j+1}) and one in (D_K, D_K + rho ||z||^2].
// Root j is kept as (origin o_j, offset tau_j), o_j the nearer pole, so every
// D_i - lam_j is formed as (D_i - D_{o_j}) - tau_j (Remark 3, eq. d-lambda).
// The iteration is the rational-interpolation scheme of Bunch-Nielsen-Sorensen
// in R.-C. Li's "middle way" form: the pole sums left and right of the root
// are each modelled by a constant plus one pole fitted to value and slope,
// and the quadratic of the model gives the next iterate, solved directly for
// the offset from the origin pole (so that a root within a few ulps of its
// pole is not lost to cancellation).  The terms of the root's two bracketing
// poles are formed exactly; when the middle-way iterate leaves the bracket
// (a weak origin pole, whose fitted weight is mostly that of farther poles),
// Li's fixed-weight model is tried, which keeps the origin pole's own weight;
// and the two models take turns whenever an iterate lands on the same side of
// the root as the one before it with |g| above a quarter of its previous
// value (near a weak pole the middle way creeps in, the fixed weight closes
// in; the switch on one-sided slow progress follows LAPACK's dlaed4, which
// tests for a tenth).  A switch on every slow step, whatever the side, can
// cycle between one iterate of each model, and one taken where |g| is down
// to rounding sends a root that the middle way would finish next step into
// a slow fixed-weight crawl, so neither switches.  When both models leave
// the bracket a Newton step on g is tried before bisection.  A bisection safeguard keeps each iterate
// inside a sign-change bracket.  The last root is bracketed by the last two
// poles and starts half a pole gap right of the last pole when that is inside
// its bracket; it always takes the middle way.
//
// Loewner (Gu-Eisenstat): zhat_i^2 = (lam_K - D_i)/rho
//     * prod_{j<i} (lam_j - D_i)/(D_j - D_i) * prod_{i<=j<K-1} (lam_j - D_i)/(D_{j+1} - D_i).
// Column scales: s_j = (sum_i zhat_i^2 / (D_i - lam_j)^2)^(-1/2) (eq. Q_Cauchy).
//
// Mapping: a workgroup of NW waves owns NR = 64 roots (or 64 poles for the
// Loewner product); lane r of every wave works on item r.  The other index
// (poles, or roots for Loewner) is streamed through LDS in chunks that the
// whole workgroup loads coalesced; each wave sweeps its slice of every chunk
// with broadcast LDS reads, and the NW partial sums meet in LDS.  All O(K^2)
// work is FP64 VALU with one reciprocal per term of a root's sums and one per
// two terms of the Loewner products and the scales; HBM traffic is O(K) per
// workgroup.
#include "secular.hpp"

namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr int NR = 64;          // roots per workgroup
// Two shapes: NW = 8 waves streaming chunks of CH = 1024 poles, and NW = 1
// wave with CH = 256.  The eight-wave shape splits the poles of K <= 256 over
// at most two waves and leaves the others idle, and its LDS holds a compute
// unit to five workgroups; the one-wave shape fits many more.  It is taken
// when K <= 128 (where one wave of the eight did all the work anyway), and
// for K <= 256 when the level has more blocks than one round of the
// eight-wave shape holds (about four per compute unit).
constexpr int SMALL_K = 256;
constexpr int SMALL_K_ALWAYS = 128;
constexpr int ROUND_BLOCKS = 1024;

// The task of workgroup b: block_start holds the prefix (ntasks + 1 entries)
// followed by the block -> task map.
__device__ __forceinline__ int task_of(const int* block_start, int ntasks, int b) {
    return block_start[ntasks + 1 + b];
}

struct Sums {
    double psi, dpsi, phi, dphi;
};

// Partial sums over the far poles of one staged chunk assigned to this wave,
// for a root with origin pole Do and offset tau.  sD/sz2 hold the chunk
// starting at pole c0.  The root's two bracketing poles e0 < e1 are left out
// (their terms are formed exactly by the caller); poles i < e0 lie left of
// the root (terms negative, psi), poles i > e1 right of it (terms positive,
// phi), so the slice splits at e0 and e1 instead of selecting per term.
__device__ __forceinline__ void chunk_sums(const double* sD, const double* sz2, int c0,
                                           int a, int b, double Do, double tau, int e0,
                                           int e1, Sums& s) {
    const int l_end = min(max(e0 - c0, a), b);
    const int r_beg = min(max(e1 + 1 - c0, a), b);
#pragma unroll 4
    for (int q = a; q < l_end; ++q) {
        const double r = dc_rcp3((sD[q] - Do) - tau);
        const double term = sz2[q] * r;
        s.psi += term;
        s.dpsi += term * r;
    }
#pragma unroll 4
    for (int q = r_beg; q < b; ++q) {
        const double r = dc_rcp3((sD[q] - Do) - tau);
        const double term = sz2[q] * r;
        s.phi += term;
        s.dphi += term * r;
    }
}

// Root x (offset from the origin pole) of the model
//     c + s1 / (dl - x) + s2 / (dh - x) = 0,
// poles dl < dh given as offsets from the origin (one of them is the origin
// itself, so the constant term is a single product and the root next to the
// origin comes out with full relative accuracy).  Of the quadratic's two
// roots the one inside (lo, hi) is returned (or the other if neither is).
// The iterate is only a guess that the next evaluation checks, so its two
// quotients take the refined reciprocal instead of a division.
__device__ __forceinline__ double model_root(double c, double s1, double s2, double dl,
                                             double dh, double lo, double hi) {
    const double B = c * (dl + dh) + s1 + s2;
    const double C = c * dl * dh + s1 * dh + s2 * dl;
    const double disc = fmax(B * B - 4.0 * c * C, 0.0);
    const double q = 0.5 * (B + copysign(sqrt(disc), B));
    const double r1 = q * dc_rcp3(c);
    const double r2 = C * dc_rcp3(q);
    return (r2 > lo && r2 < hi) ? r2 : r1;
}

template <int NW, int CH>
__global__ __launch_bounds__(NW * 64)
void k_secular_roots(const SecTask* __restrict__ tasks, const int* __restrict__ block_start,
                     int ntasks, int max_iter) {
    __shared__ double sD[CH], sz2[CH];
    __shared__ double red[4][NW][NR];
    __shared__ double s_tau[NR];
    __shared__ double s_do[NR];
    __shared__ int s_live;
    __shared__ double s_zz;

    const int ti = task_of(block_start, ntasks, blockIdx.x);
    const SecTask& T = tasks[ti];
    const int K = T.K_p ? *T.K_p : T.K;
    const int j0 = (blockIdx.x - block_start[ti]) * NR;
    if (j0 >= K) return;
    const double rho = T.rho_p ? *T.rho_p : T.rho;
    const double irho = 1.0 / rho;
    const double* __restrict__ D = T.D;
    const double* __restrict__ z = T.z;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = j0 + lane;
    const bool valid = j < K;
    const bool last = j == K - 1;
    // The root's bracketing poles e0 < e1, whose terms are formed exactly:
    // (j, j+1) inside, (K-2, K-1) for the last root (K = 1: the one pole).
    const int e1 = last ? K - 1 : j + 1;
    const int e0 = last ? K - 2 : j;

    // ||z||^2 bounds the last root; only the workgroup owning it needs it
    // (per-wave partials summed in a fixed order: deterministic).
    if (j0 + NR >= K) {
        double zz = 0.0;
        for (int i = tid; i < K; i += NW * 64) zz += z[i] * z[i];
        zz = dc_wave_sum(zz);
        if (lane == 0) red[0][w][0] = zz;
    }
    __syncthreads();
    if (tid == 0) {
        double zz = 0.0;
        if (j0 + NR >= K)
            for (int q = 0; q < NW; ++q) zz += red[0][q][0];
        s_zz = zz;
    }
    __syncthreads();

    // Wave 0 owns the per-root state.
    double lo = 0.0, hi = 0.0, tau = 0.0;
    double De0 = 0.0, De1 = 0.0, w0 = 0.0, w1 = 0.0;   // bracketing poles, weights z^2
    int org = 0;
    bool done = !valid;
    int iters = 0;
    double prevg = 0.0;     // g at the previous iterate
    bool fixed = false;     // next step by the fixed-weight model
    if (w == 0 && valid) {
        De1 = D[e1];
        De0 = e0 >= 0 ? D[e0] : 0.0;
        const double z1 = z[e1], z0 = e0 >= 0 ? z[e0] : 0.0;
        w1 = z1 * z1;
        w0 = z0 * z0;
        if (last) {
            hi = rho * s_zz * (1.0 + 8.0 * EPS);   // widened by a few ulps
            tau = 0.5 * hi;
            // start half a gap right of the last pole (where the root of a
            // matrix with evenly spread spectrum sits) when that is closer
            if (K > 1) tau = fmin(tau, 0.5 * (De1 - De0));
            org = j;
        } else {
            tau = 0.5 * (De1 - De0);                // midpoint, origin j frame
            org = j;
        }
    }
    if (w == 0) {
        s_tau[lane] = tau;
        s_do[lane] = valid ? D[org] : 0.0;
    }
    // When every pole fits in one chunk it is staged once for all the
    // iterations (most merges of a batch of small problems).
    const bool one_chunk = K <= CH;
    if (one_chunk)
        for (int i = tid; i < K; i += NW * 64) {
            sD[i] = D[i];
            const double zi = z[i];
            sz2[i] = zi * zi;
        }
    __syncthreads();

    for (int it = 0;; ++it) {
        // Every wave: partial sums over the far poles at the current iterate.
        Sums p{0.0, 0.0, 0.0, 0.0};
        const double Do = s_do[lane];
        const double tcur = s_tau[lane];
        if (one_chunk) {
            const int per = (K + NW - 1) / NW;    // the poles split over all waves
            const int a = min(K, w * per), b = min(K, a + per);
            if (valid) chunk_sums(sD, sz2, 0, a, b, Do, tcur, e0, e1, p);
        } else {
            for (int c0 = 0; c0 < K; c0 += CH) {
                const int cn = min(CH, K - c0);
                __syncthreads();
                for (int i = tid; i < cn; i += NW * 64) {
                    sD[i] = D[c0 + i];
                    const double zi = z[c0 + i];
                    sz2[i] = zi * zi;
                }
                __syncthreads();
                const int per = (cn + NW - 1) / NW;   // the chunk split over all waves
                const int a = min(cn, w * per), b = min(cn, a + per);
                if (valid) chunk_sums(sD, sz2, c0, a, b, Do, tcur, e0, e1, p);
            }
        }
        red[0][w][lane] = p.psi;
        red[1][w][lane] = p.dpsi;
        red[2][w][lane] = p.phi;
        red[3][w][lane] = p.dphi;
        __syncthreads();
        if (w == 0) {
            double fpsi = 0, fdpsi = 0, fphi = 0, fdphi = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                fpsi += red[0][q][lane];
                fdpsi += red[1][q][lane];
                fphi += red[2][q][lane];
                fdphi += red[3][q][lane];
            }
            // the bracketing poles' terms in the origin frame, with the
            // same refined reciprocal as the far poles' terms
            const double dl = e0 >= 0 ? De0 - Do : 0.0;   // pole offsets from the origin
            const double dh = De1 - Do;
            const double d1 = dl - tau, d2 = dh - tau;    // and from the iterate
            const double r1 = (valid && e0 >= 0) ? dc_rcp3(d1) : 0.0;
            const double r2 = valid ? dc_rcp3(d2) : 0.0;
            const double t0 = w0 * r1, dt0 = t0 * r1;
            const double t1 = w1 * r2, dt1 = t1 * r2;
            const double psi = fpsi + t0, dpsi = fdpsi + dt0;
            const double phi = fphi + t1, dphi = fdphi + dt1;
            const double aabs = (fphi - fpsi) + fabs(t0) + fabs(t1);   // sum of |terms|
            const double g = irho + psi + phi;
            const double gtol = 8.0 * EPS * (irho + aabs);
            if (!done) {
                ++iters;
                // switch models when an iterate stayed on the same side of
                // the root without shrinking |g| fourfold, unless |g| is
                // within a small multiple of the tolerance (there its size
                // and sign are rounding, not progress)
                if (iters > 1 && g * prevg > 0.0 && fabs(g) > 0.25 * fabs(prevg) &&
                    fabs(g) > 64.0 * gtol)
                    fixed = !fixed;
                prevg = g;
                if (it == 0 && !last) {
                    // Origin choice from the sign at the midpoint.
                    const double h = 0.5 * (De1 - De0);
                    if (g > 0.0) {          // root left of the midpoint
                        org = j; lo = 0.0; hi = h;
                    } else {                // root right of it: re-frame at D_{j+1}
                        org = j + 1; lo = -h; hi = 0.0; tau = -h;
                    }
                    // the midpoint itself may pass the test (roots placed
                    // halfway between poles by symmetry): a model step
                    // from a zero |g| leaves the bracket and ends in
                    // bisection at the midpoint's side
                    if (fabs(g) <= gtol) done = true;
                } else {
                    if (g > 0.0) hi = tau; else lo = tau;
                    const bool conv = fabs(g) <= gtol ||
                                      (hi - lo) <= 4.0 * EPS * fmax(fabs(lo), fabs(hi));
                    if (conv) done = true;
                }
                if (!done) {
                    if (iters > max_iter) {
                        done = true;
                        dc_set_info(T.info, T.row0 + j + 1);
                    } else {
                        // Pole offsets in the (possibly new) origin frame;
                        // their distances from the iterate are d1 and d2
                        // again (a re-framed midpoint is -h from D_{j+1} as
                        // it was h from D_j), whose reciprocals r1, r2 the
                        // fixed-weight model reuses.
                        const double Dn = (org == j) ? (last ? De1 : De0) : De1;
                        const double ol = e0 >= 0 ? De0 - Dn : 0.0, oh = De1 - Dn;
                        const double q1 = ol - tau, q2 = oh - tau;
                        double nt = lo;     // outside (lo, hi): not yet found
                        if (e0 < 0) {
                            // one pole: c + w1 / (0 - x) = 0 with c = 1/rho
                            nt = rho * w1;
                        } else {
                            if (!fixed || last) {
                                // Middle-way model: both pole sums fitted to
                                // value and slope by their bracketing pole.
                                const double s1 = dpsi * q1 * q1;
                                const double s2 = dphi * q2 * q2;
                                const double c =
                                    irho + (psi - dpsi * q1) + (phi - dphi * q2);
                                nt = model_root(c, s1, s2, ol, oh, lo, hi);
                            }
                            if (!(nt > lo && nt < hi) && !last) {
                                // Fixed-weight model: the origin pole's own
                                // term exact, everything else fitted at the
                                // other bracketing pole (a weak origin pole
                                // fools the middle way's fit).
                                const bool left = org == j;
                                const double R = irho + fpsi + fphi + (left ? t1 : t0);
                                const double Rp = fdpsi + fdphi + (left ? dt1 : dt0);
                                const double qo = left ? q2 : q1;
                                const double sf = Rp * qo * qo;
                                const double cf = R - Rp * qo;
                                nt = left ? model_root(cf, w0, sf, ol, oh, lo, hi)
                                          : model_root(cf, sf, w1, ol, oh, lo, hi);
                            }
                        }
                        if (!(nt > lo && nt < hi)) {
                            // a Newton step on g itself before bisecting:
                            // when an iterate already sits on the root to
                            // rounding the models can land just outside the
                            // bracket, and the midpoint of a bracket whose
                            // ends are orders of magnitude apart throws the
                            // root back to where it started
                            const double nn = tau - g * dc_rcp3(dpsi + dphi);
                            nt = (nn > lo && nn < hi) ? nn : 0.5 * (lo + hi);
                        }
                        tau = nt;
                    }
                }
            }
            s_tau[lane] = tau;
            if (valid) s_do[lane] = (org == j) ? (last ? De1 : De0) : De1;
            const unsigned long long live = __ballot(!done);
            if (lane == 0) s_live = live != 0ull;
        }
        __syncthreads();
        if (!s_live) break;
    }
    if (w == 0 && T.iters) {
        // per-merge iteration statistics (lanes past K count 0): a wave
        // reduction with every lane active, one atomic per wave
        int isum = iters, imax = iters;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            isum += __shfl_xor(isum, off, 64);
            imax = max(imax, __shfl_xor(imax, off, 64));
        }
        if (lane == 0) {
            atomicAdd(T.iters, isum);
            atomicMax(T.iters + 1, imax);
        }
    }
    if (w == 0 && valid) {
        const double base = (org == j) ? (last ? De1 : De0) : De1;
        T.org[j] = org;
        T.tau[j] = tau;
        if (T.cbase) T.cbase[j] = base;
        if (T.lam) T.lam[j] = base + tau;
    }
}

// zhat_i: lane r of each wave owns pole i = p0 + r; the roots are streamed in
// chunks and every wave multiplies the factors of its slice of each chunk.
template <int NW, int CH>
__global__ __launch_bounds__(NW * 64)
void k_loewner(const SecTask* __restrict__ tasks, const int* __restrict__ block_start,
               int ntasks) {
    __shared__ double sB[CH], sT[CH], sD[CH + 1];
    __shared__ double part[NW][NR];
    const int ti = task_of(block_start, ntasks, blockIdx.x);
    const SecTask& T = tasks[ti];
    const int K = T.K_p ? *T.K_p : T.K;
    const int p0 = (blockIdx.x - block_start[ti]) * NR;
    if (p0 >= K) return;
    const double rho = T.rho_p ? *T.rho_p : T.rho;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i = p0 + lane;
    const bool valid = i < K;
    const double Di = valid ? T.D[i] : 0.0;
    double prod = 1.0;
    for (int c0 = 0; c0 < K; c0 += CH) {
        const int cn = min(CH, K - c0);
        __syncthreads();
        for (int q = tid; q < cn; q += NW * 64) {
            sB[q] = T.cbase[c0 + q];
            sT[q] = T.tau[c0 + q];
        }
        for (int q = tid; q <= cn; q += NW * 64) sD[q] = (c0 + q < K) ? T.D[c0 + q] : 0.0;
        __syncthreads();
        const int per = (cn + NW - 1) / NW;   // the chunk split over all waves
        const int a = min(cn, w * per), b = min(cn, a + per);
        if (valid) {
            // Factors in pairs: one reciprocal per two denominators (a few
            // ulps per factor; the roots' own sums keep one reciprocal per
            // term, since their stopping test sits at a few ulps).
            auto factor = [&](int q, double& num, double& den) {
                const int jj = c0 + q;
                num = (sB[q] - Di) + sT[q];                         // lam_j - D_i
                den = (jj == K - 1) ? rho : ((jj < i ? sD[q] : sD[q + 1]) - Di);
            };
            int q = a;
#pragma unroll 2
            for (; q + 1 < b; q += 2) {
                double n1, d1, n2, d2;
                factor(q, n1, d1);
                factor(q + 1, n2, d2);
                prod *= (n1 * n2) * dc_rcp3(d1 * d2);
            }
            if (q < b) {
                double n1, d1;
                factor(q, n1, d1);
                prod *= n1 * dc_rcp3(d1);
            }
        }
    }
    part[w][lane] = prod;
    __syncthreads();
    if (w == 0 && valid) {
        double pr = part[0][lane];
#pragma unroll
        for (int q = 1; q < NW; ++q) pr *= part[q][lane];
        T.zhat[i] = copysign(sqrt(pr), T.z[i]);
    }
}

template <int NW, int CH>
__global__ __launch_bounds__(NW * 64)
void k_colscale(const SecTask* __restrict__ tasks, const int* __restrict__ block_start,
                int ntasks) {
    __shared__ double sD[CH], sZ[CH];
    __shared__ double part[NW][NR];
    const int ti = task_of(block_start, ntasks, blockIdx.x);
    const SecTask& T = tasks[ti];
    const int K = T.K_p ? *T.K_p : T.K;
    const int j0 = (blockIdx.x - block_start[ti]) * NR;
    if (j0 >= K) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = j0 + lane;
    const bool valid = j < K;
    const double base = valid ? T.cbase[j] : 0.0;
    const double tj = valid ? T.tau[j] : 0.0;
    double s = 0.0;
    for (int c0 = 0; c0 < K; c0 += CH) {
        const int cn = min(CH, K - c0);
        __syncthreads();
        for (int q = tid; q < cn; q += NW * 64) {
            sD[q] = T.D[c0 + q];
            sZ[q] = T.zhat[c0 + q];
        }
        __syncthreads();
        const int per = (cn + NW - 1) / NW;   // the chunk split over all waves
        const int a = min(cn, w * per), b = min(cn, a + per);
        if (valid) {
            int q = a;
#pragma unroll 2
            for (; q + 1 < b; q += 2) {
                const double x = (sD[q] - base) - tj, y = (sD[q + 1] - base) - tj;
                const double rp = dc_rcp3(x * y);
                const double v = sZ[q] * (y * rp), w = sZ[q + 1] * (x * rp);
                s += v * v + w * w;
            }
            if (q < b) {
                const double v = sZ[q] * dc_rcp3((sD[q] - base) - tj);
                s += v * v;
            }
        }
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && valid) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) t += part[q][lane];
        T.scale[j] = 1.0 / sqrt(t);
    }
}

template <int NW, int CH>
hipError_t launch_secular(const SecTask* tasks, const int* block_start, int ntasks,
                          int total_blocks, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL((k_secular_roots<NW, CH>), dim3(total_blocks), dim3(NW * 64), 0, s,
                       tasks, block_start, ntasks, max_iter);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_loewner<NW, CH>), dim3(total_blocks), dim3(NW * 64), 0, s, tasks,
                       block_start, ntasks);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_colscale<NW, CH>), dim3(total_blocks), dim3(NW * 64), 0, s, tasks,
                       block_start, ntasks);
    return hipGetLastError();
}

}  // namespace

hipError_t dc_launch_secular(const SecTask* tasks, const int* block_start, int ntasks,
                             int total_blocks, int max_k, int max_iter, hipStream_t s) {
    if (total_blocks <= 0) return hipSuccess;
    if (max_k <= SMALL_K_ALWAYS || (max_k <= SMALL_K && total_blocks > ROUND_BLOCKS))
        return launch_secular<1, SMALL_K>(tasks, block_start, ntasks, total_blocks, max_iter, s);
    return launch_secular<8, 1024>(tasks, block_start, ntasks, total_blocks, max_iter, s);
}
