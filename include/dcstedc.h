/*
 * dcstedc.h -- C ABI of the MI355X (gfx950) structured divide-and-conquer
 * symmetric tridiagonal eigensolver.
 *
 * The method is that of Liao, Li, Lu and Roman, "A parallel structured
 * divide-and-conquer algorithm for symmetric tridiagonal eigenvalue problems"
 * (IEEE TPDS 2020): Cuppen's divide and conquer (Algorithm 1) whose merge
 * step forms the eigenvectors as Q_new = diag(Q1, Q2) U (eq. updateV), with U
 * the Cauchy-like eigenvector matrix of the rank-one modified diagonal
 * problem (eq. Q_Cauchy), built from its generators and optionally replaced
 * off the diagonal by structured low-rank approximations (section "SRRSC
 * low-rank approximation"; Algorithm 2 step 3(b)-(c); Algorithm 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - FP64 throughout.  Every array argument is a DEVICE pointer owned by the
 *    caller unless stated otherwise; the library never frees caller memory.
 *  - Matrices are column-major with a leading dimension (LAPACK layout), so
 *    eigenvector j is the contiguous column j.
 *  - Calls are asynchronous on the caller's stream.  Argument errors are
 *    detected synchronously on the host: the call returns -i for the i-th
 *    (1-based) invalid argument and launches nothing.  Errors the device
 *    detects are written to a device status word (decoded by
 *    dc_status_string; return codes are decoded by dc_strerror):
 *        0        success
 *        j > 0    an iteration did not converge; j - 1 is a row of the
 *                 problem: the first row of the leaf block whose QR sweeps
 *                 ran out, or the merge's first row plus the index of the
 *                 first secular root that reached max_iter (for dc_secular
 *                 alone: the root's index)
 *        -1000    a non-finite value in the input
 *        -2000    equal eigenvalues met by the adjoint (dc_stedc_backward)
 *    The short forms keep that word in library-owned memory per stream
 *    (read it with dc_last_info after synchronising); the _ex forms write it
 *    to the caller's info_dev.
 *  - A positive return value is a HIP runtime error code.
 *  - The short forms allocate stream-ordered workspace; only the _ex forms
 *    with caller workspace allocate nothing and may be captured in a graph.
 *  - Host threads: solves may be issued from several threads (on separate
 *    streams, with separate workspaces).  The tree plans, captured graphs
 *    and tuning tables are shared under locks; the records read by
 *    dc_last_stats belong to the calling thread.  The instrumentation
 *    (dc_profile_enable / dc_profile_read) and dc_autotune_batched, which
 *    uses it, are process-wide: call them while no other thread solves.
 */
#ifndef DCSTEDC_H
#define DCSTEDC_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Tuning and path options.  A NULL dc_opts* means the defaults below. */
typedef struct dc_opts {
    int leaf;        /* largest block solved directly by tridiagonal QR
                        (Algorithm 1, "size of T is small enough");
                        1..64, default 32 */
    double lr_tol;   /* absolute tolerance of the structured low-rank merge
                        (0 = plain merge, the default) */
    int lr_block;    /* block size b of the low-rank merge; 0 (the
                        default) = automatic: the value dc_autotune_batched
                        chose for this problem, else 256 */
    int lr_min_k;    /* use the low-rank merge only when the deflated size K
                        reaches this (Algorithm 3's "size of M is large");
                        0 (the default) = automatic: tuned, else 2048 */
    int max_iter;    /* secular iteration cap (default 200: enough for pure
                        bisection to reach 4-ulp relative accuracy) */
    int gemm_tile;   /* merge-product tile variant for every level:
                        0 = automatic (the tuned choice when one exists,
                        else 64 x 64 tiles for levels of merges up to 512
                        rows and the 128 x 128 register kernel above);
                        1 128 x 128 LDS kernel, two workgroups per CU;
                        2 64 x 64 LDS; 3 128 x 128 LDS, k-step 32;
                        4 256 x 128 LDS; 5 64 x 64 register kernel.
                        Other values are invalid options. */
} dc_opts;

void dc_opts_default(dc_opts* opt);

/*
 * dc_stedc -- all eigenpairs of the symmetric tridiagonal T(d, e),
 * T[i][i] = d[i], T[i][i+1] = T[i+1][i] = e[i] (section "Preliminaries",
 * eq. t; Algorithm 1's input and output).
 *   n    order, n >= 0 (n == 0: nothing happens)
 *   d    in: diagonal (n); out: eigenvalues in ascending order
 *   e    in: off-diagonal (n-1); left unchanged
 *   Q    out: ldq x n, column j the unit eigenvector of d[j]
 *   ldq  >= max(1, n)
 * T is scaled internally by the power of two that brings max(|d|, |e|) into
 * [1, 2), and the eigenvalues are scaled back: exact, so the result does not
 * depend on the magnitude of T (any finite T).
 * Returns 0, -i for a bad argument i, or a HIP error.
 */
int dc_stedc(int n, double* d, double* e, double* Q, int ldq, hipStream_t stream);

/* Workspace in bytes that dc_stedc_ex needs for order n. */
size_t dc_stedc_workspace(int n, const dc_opts* opt);

/*
 * dc_stedc_ex -- dc_stedc with caller workspace and status word.
 *   work, lwork  device workspace of at least dc_stedc_workspace(n, opt)
 *                bytes, 256-byte aligned
 *   info_dev     device int; receives the status (see above)
 * It allocates nothing and performs no host synchronisation, with or
 * without the low-rank product (graph-capturable): with opt->lr_tol > 0 the
 * switch of Algorithm 3, the SRRSC compression, W's layout and the product
 * task lists are decided and built on the device, in regions of the
 * workspace (dc_stedc_workspace includes them for the options' lr_block and
 * lr_min_k, or for every automatic choice when those are 0); W itself
 * occupies the merge's square of Q below the root (Q is written only by the
 * root merge) and of the workspace basis at the root.
 * The first call for a given (n, options) builds and uploads the tree plan
 * synchronously; call dc_stedc_workspace first (it builds the plan) before
 * capturing.
 */
int dc_stedc_ex(int n, double* d, double* e, double* Q, int ldq, void* work,
                size_t lwork, int* info_dev, const dc_opts* opt,
                hipStream_t stream);

/*
 * dc_stedc_batched -- many independent problems of uneven size, solved
 * together: every tree level of every problem runs as one launch per phase.
 *   count           number of problems
 *   n_host, ldq_host  HOST arrays (count) of orders and leading dimensions
 *   d, e, Q         HOST arrays (count) of DEVICE pointers, as in dc_stedc
 *   work, lwork     device workspace >= dc_stedc_batched_workspace(...)
 *   info_dev        DEVICE int array (count), one status per problem
 * The level schedule is captured into a HIP graph on first use for a given
 * (count, sizes, options, pointers) signature and replayed afterwards.
 */
size_t dc_stedc_batched_workspace(int count, const int* n_host, const dc_opts* opt);
int dc_stedc_batched(int count, const int* n_host, double* const* d,
                     double* const* e, double* const* Q, const int* ldq_host,
                     void* work, size_t lwork, int* info_dev,
                     const dc_opts* opt, hipStream_t stream);

/*
 * dc_secular -- the rank-one modified diagonal eigenproblem
 * M = diag(D) + rho z z^T (eq. rankone) on its deflated generators.
 *   K        size, K >= 1
 *   Dbar     poles, strictly increasing (K)
 *   zbar     weights, all non-zero (K); rho > 0
 *   org      out: origin pole of root j (K, int): lam_j = Dbar[org_j] + tau_j
 *   tau      out: offset of root j from its origin (K) (eq. secular with
 *            Remark 3's stable differences, eq. d-lambda)
 *   zhat     out: Loewner-recomputed weights (K) (Gu-Eisenstat)
 *   scale    out: column normalisers s_j (K) (eq. Q_Cauchy)
 *   info_dev device int status, or NULL
 */
int dc_secular(int K, const double* Dbar, const double* zbar, double rho,
               int* org, double* tau, double* zhat, double* scale,
               int* info_dev, int max_iter, hipStream_t stream);

/*
 * dc_merge_update -- the merge-step eigenvector update C = Qnd * U
 * (eq. updateV, eq. evect) with U generated from its generators and never
 * stored: U_ij = zhat_i scale_j / ((Dbar_i - Dbar_{org_j}) - tau_j)
 * (eq. Q_Cauchy with Remark 3's differences).  With org == NULL the column
 * nodes are tau itself: U_ij = zhat_i scale_j / (Dbar_i - tau_j) (general
 * Cauchy-like generators as in the paper's Examples 0 and 1).
 *   m, K         Qnd is m x K (ldq >= m), U is K x K, C is m x K (ldc >= m)
 *   lr_tol       0: plain product.  > 0: off-diagonal lr_block x lr_block
 *                blocks of U are replaced by SRRSC approximations with
 *                absolute entry error <= lr_tol (eq. sid; Algorithm 2 step
 *                3(b)-(c)); diagonal blocks stay exact.
 *   lr_block     block size for lr_tol > 0 (<= 0: default 256); at most
 *                2048 with org, 4096 with org == NULL (else returns -13)
 * With lr_tol > 0 it allocates its temporaries stream-ordered
 * (hipMallocAsync / hipFreeAsync on the stream) and waits for the stream
 * once, after the compression, to size the skeleton columns W (m x the sum
 * of the ranks, a block kept dense counting its width) exactly; when W
 * would take more than half the free device memory the plain product runs
 * instead.
 */
int dc_merge_update(int m, int K, const double* Qnd, int ldq,
                    const double* Dbar, const int* org, const double* tau,
                    const double* zhat, const double* scale, double* C,
                    int ldc, double lr_tol, int lr_block, hipStream_t stream);

/*
 * dc_merge_lowrank_ranks -- SRRSC ranks of the lr_block x lr_block blocks
 * of U (section "SRRSC low-rank approximation", complete pivoting, stop when
 * every Schur-complement entry is <= lr_tol; Table "rank" reports such ranks
 * for Example 1's B).  For the generators of dc_merge_update, writes nb*nb
 * ints row-major to ranks_host (HOST), nb = ceil(K / lr_block): the rank of
 * off-diagonal block (I, J), -1 on the diagonal, -2 where the rank exceeds
 * the cap.
 *   rank_cap   0: the cap of the low-rank product itself (min(128,
 *              lr_block/2)), i.e. the ranks dc_merge_update would use;
 *              > 0: count ranks up to min(rank_cap, lr_block) without
 *              forming the factors.
 * lr_block limits as dc_merge_update (else -8).  Synchronises the stream.
 */
int dc_merge_lowrank_ranks(int K, const double* Dbar, const int* org,
                           const double* tau, const double* zhat,
                           const double* scale, double lr_tol, int lr_block,
                           int rank_cap, int* ranks_host, hipStream_t stream);

/*
 * dc_autotune -- choose the merge-product tile variant per level size by
 * timing (the batched driver's "autotuned tiles"; the paper leaves the local
 * product's blocking to the implementation).  For each size bucket
 * m = 64, 128, ..., min(max_n, 8192) it times every variant on a level of
 * max_n / m synthetic m x m merges (HIP events on `stream`) and keeps the
 * fastest; larger levels use the largest bucket's choice.  The table is per
 * device; solves planned afterwards use it (earlier plans and captured
 * graphs stay as they were).  Allocates and synchronises: not for use inside
 * graph capture.  max_n = 0 clears the device's table and every table made
 * by dc_autotune_batched on it (back to the default rule: 64 x 64 tiles up
 * to 512 rows, 128 x 128 above).  A variant replaces the default rule's
 * choice only when it is at least 3 % faster.  Returns 0, -1 for max_n < 0,
 * or a HIP error code.
 */
int dc_autotune(int max_n, hipStream_t stream);

/*
 * dc_autotune_batched -- tile choice measured on the caller's own batch.
 * Arguments as dc_stedc_batched (lr options included; gemm_tile must be 0).
 * Solves the batch twice with every level forced to each tile variant,
 * times each level's product phase with HIP events on `stream`, and keeps,
 * per level, the fastest variant (the default rule's unless another is at
 * least 3 % faster).  The per-level table applies to later plans with the
 * same device, leaf and sizes (dc_stedc_ex for count == 1), and takes
 * precedence over dc_autotune's buckets.  With opt->lr_tol > 0 it then
 * times whole solves over b in {128, 256, 512} and the switch in
 * {1024, 2048, 4096} (only for the fields the caller left at 0) and keeps
 * the fastest pair (256 / 2048 unless another is at least 3 % faster) for
 * later solves of the same device, leaf and sizes whose fields are 0.  On return d and e hold the inputs
 * again; Q, info_dev and work hold no defined result.  Allocates (a copy of
 * the diagonals) and synchronises: not for graph capture.  Returns 0, the
 * argument codes of dc_stedc_batched (-10 also for gemm_tile != 0), or a
 * HIP error code.
 */
int dc_autotune_batched(int count, const int* n_host, double* const* d,
                        double* const* e, double* const* Q, const int* ldq_host,
                        void* work, size_t lwork, int* info_dev,
                        const dc_opts* opt, hipStream_t stream);

/*
 * dc_autotune_levels -- copies the per-level variants that
 * dc_autotune_batched chose for (current device, leaf, sizes) to
 * variant_out[0..cap) (HOST; level 0 = the deepest merges) and returns the
 * number of levels, 0 when that batch was not tuned, -1 for bad arguments.
 */
int dc_autotune_levels(int count, const int* n_host, int leaf, int* variant_out, int cap);

/*
 * dc_autotune_lowrank -- the low-rank block size and switch that
 * dc_autotune_batched chose for (current device, leaf, sizes): writes them to
 * *block_out, *min_k_out (HOST) and returns 1; 0 when none was chosen, -1 for
 * bad arguments.
 */
int dc_autotune_lowrank(int count, const int* n_host, int leaf, int* block_out,
                        int* min_k_out);

/*
 * dc_autotune_table -- copies the current device's tuned variant per size
 * bucket (bucket b: largest merge in (2^(b-1), 2^b]; -1 = not tuned) to
 * variant_out[0..cap) (HOST) and returns the number of buckets.
 */
int dc_autotune_table(int* variant_out, int cap);

/*
 * dc_stedc_backward -- reverse-mode gradient of (lam, Q) = eig(T(d, e)).
 * With M = diag(lam_bar) + F o (Q^T Q_bar), F_ij = 1/(lam_j - lam_i)
 * (i != j, 0 on the diagonal), A_bar = Q M Q^T and
 *   d_bar_i = A_bar[i][i],  e_bar_i = A_bar[i][i+1] + A_bar[i+1][i].
 * Only the band of A_bar is formed.
 *   lam, Q     the forward result (Q ldq x n, column-major)
 *   lam_bar    cotangent of lam (n) or NULL (= 0)
 *   Q_bar      cotangent of Q (ldqb x n) or NULL (= 0)
 *   d_bar      out (n);  e_bar  out (n-1)
 * Equal eigenvalues make F undefined: such pairs get F_ij = 0 and the status
 * word is set to -2000 (read with dc_last_info).
 * With Q_bar, G^T = Q_bar^T Q is formed first, by an MFMA product that reads
 * both operands down their columns (no transposed copies); P = Q M then runs
 * on register tiles with M generated and only the band reduced.  Temporaries
 * (G^T, n x n, with Q_bar; O(n^2 / 32) partial sums) are allocated
 * stream-ordered and freed on the stream: not for graph capture (use
 * dc_stedc_backward_ex).
 */
int dc_stedc_backward(int n, const double* lam, const double* Q, int ldq,
                      const double* lam_bar, const double* Q_bar, int ldqb,
                      double* d_bar, double* e_bar, hipStream_t stream);

/* Workspace in bytes that dc_stedc_backward_ex needs for order n, with
 * (with_qbar != 0) or without a Q_bar. */
size_t dc_stedc_backward_workspace(int n, int with_qbar);

/*
 * dc_stedc_backward_ex -- dc_stedc_backward with caller workspace and status
 * word: the same gradient (same kernels, same result bit for bit).
 *   work, lwork  device workspace of at least
 *                dc_stedc_backward_workspace(n, Q_bar != NULL) bytes,
 *                256-byte aligned (else -10; too small: -11)
 *   info_dev     device int (else -12); cleared, then -2000 when equal
 *                eigenvalues were met
 * It allocates nothing and never waits for the device: graph-capturable.
 */
int dc_stedc_backward_ex(int n, const double* lam, const double* Q, int ldq,
                         const double* lam_bar, const double* Q_bar, int ldqb,
                         double* d_bar, double* e_bar, void* work, size_t lwork,
                         int* info_dev, hipStream_t stream);

/*
 * dc_stedc_backward_rank1 -- the same gradient when Q_bar = u g^T has rank
 * one (for instance a loss sum_i c_i (u^T q_i)^2, where g_i = 2 c_i u^T q_i).
 * Then F o (Q^T Q_bar) is itself Cauchy-like, (Q^T u)_i g_j / (lam_j -
 * lam_i), and M is generated from (Q^T u, g, lam) inside the register-tile
 * product P = Q M.  Temporaries are allocated stream-ordered, as above.
 *   u (n), g (n) device vectors; lam_bar may be NULL.
 */
int dc_stedc_backward_rank1(int n, const double* lam, const double* Q, int ldq,
                            const double* lam_bar, const double* u,
                            const double* g, double* d_bar, double* e_bar,
                            hipStream_t stream);

/*
 * dc_stedc_backward_rank1_noalloc -- dc_stedc_backward_rank1 for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * training or serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and result, plus the caller's device status word info_dev
 * (cleared, then -2000 on equal eigenvalues).  It allocates nothing: its
 * scratch (the partial band sums, Q^T u and a flag) is a fixed 16 MiB device
 * array per GPU, held until the process ends, which limits n to 4712
 * (dc_stedc_backward_rank1_noalloc_max_bytes() gives the size; a larger n
 * returns -1 and launches nothing).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (on different streams or host threads) race
 * and must be ordered by the caller.
 */
int dc_stedc_backward_rank1_noalloc(int n, const double* lam, const double* Q, int ldq,
                                    const double* lam_bar, const double* u,
                                    const double* g, double* d_bar, double* e_bar,
                                    int* info_dev, hipStream_t stream);
size_t dc_stedc_backward_rank1_noalloc_max_bytes(void);

/* Status word of the last short-form call on `stream`; synchronises it. */
int dc_last_info(hipStream_t stream);

/* Human-readable text for a return code: 0, -i (bad argument i) or a
 * positive HIP runtime error code. */
const char* dc_strerror(int code);

/* Human-readable text for a device status word (0, j > 0, -1000, -2000). */
const char* dc_status_string(int status);

/*
 * dc_stats -- per-merge record of the last dc_stedc / dc_stedc_ex /
 * dc_stedc_batched call on the calling host thread (copied back synchronously
 * when requested; for a batch, the merges of every problem by tree level):
 * order m, deflated size K, number of pair rotations, path (0 plain,
 * 1 low-rank), and the product's algorithmic flop count.
 */
typedef struct dc_merge_stat {
    int level, m, K, nrot, path;
    double flops;
    /* low-rank merges: off-diagonal blocks, sum and maximum of the ranks of
       the compressed ones, blocks kept dense (0 on the plain path) */
    int lr_blocks, lr_rank_sum, lr_rank_max, lr_dense;
    /* low-rank merges: executed flops of the skeleton-column product and of
       the fused product (diagonal blocks plus interpolation rows); their sum
       is flops */
    double lr_flops_skeleton, lr_flops_fused;
    /* rows of the first child (the second has m - n1); survivors with
       non-zeros in the first child's rows and in the second's; problem index
       (0 for dc_stedc / dc_stedc_ex) */
    int n1, ntop, nbot, prob;
    /* secular iterations of the merge's K roots: sum and maximum */
    int sec_iters_sum, sec_iters_max;
} dc_merge_stat;

/* Copies up to cap records into out (HOST); returns the number available. */
int dc_last_stats(dc_merge_stat* out, int cap);

/*
 * Instrumentation.  dc_profile_enable(1) makes later dc_stedc / dc_stedc_ex
 * calls record HIP events on the caller's stream at the phase boundaries of
 * every tree level; dc_profile_read waits for them and writes, for each
 * level from the deepest to the root, six durations in milliseconds
 * (deflation, rotations, secular/Loewner/scale, eigenvalue order, merge
 * product, deflated-column copy) into ms (HOST, 6 per level, up to cap
 * values); it returns the number of levels.  Not for use under graph capture.
 */
int dc_profile_enable(int on);
int dc_profile_read(double* ms, int cap);
/* With profiling on: for each level, three durations in milliseconds of its
 * low-rank product phase (compression and planning, skeleton-column
 * product, fused product), 0 for levels without a low-rank merge; returns
 * the number of levels. */
int dc_profile_read_lowrank(double* ms, int cap);

#ifdef __cplusplus
}
#endif
#endif /* DCSTEDC_H */
