// Structured low-rank merge product (SRRSC compression + generated products).
#pragma once
#include <vector>

#include "common.hpp"

// One row half of a merge product: C[rows, :] = A[rows, panel] * U[panel, :],
// where panel column t holds the basis column of survivor klist[t] (klist
// ascending; empty means the identity 0..K-1) and gD / gz are the row
// generators in panel order.
struct LrHalf {
    const double* A = nullptr;
    long long lda = 0;
    int rows = 0;
    std::vector<int> klist;
    const double* gD = nullptr;
    const double* gz = nullptr;
    double* C = nullptr;
    long long ldc = 0;
    const int* cpos = nullptr;   // output column of generator g (null: g)
    long long w_row0 = 0;        // row offset of this half inside W
};

// Low-rank product over the given halves (host-synchronising: reads the
// ranks).  cbase/coff are the column nodes w_j = cbase_j + coff_j (coff null:
// plain nodes w_j = cbase_j), scale the column scales.  wrows
// is the row count of the skeleton panel W (sum of the halves' rows).
// Ranks of the off-diagonal blocks of one low-rank product: block count,
// sum and maximum of the ranks of the compressed blocks, blocks kept dense.
struct LrRankSummary {
    int blocks = 0, rank_sum = 0, rank_max = 0, dense = 0;
};

hipError_t dc_lowrank_product(int K, int b, double tol, const double* D, const double* zhat,
                              const double* cbase, const double* coff, const double* scale,
                              std::vector<LrHalf>& halves, int wrows, int variant,
                              hipStream_t s, double* flops_out,
                              LrRankSummary* ranks_out = nullptr);

// One merge of dc_lowrank_products: its generators and halves as for
// dc_lowrank_product; flops and ranks are filled in.
struct LrMerge {
    int K = 0;
    const double* D = nullptr;
    const double* zhat = nullptr;
    const double* cbase = nullptr;
    const double* coff = nullptr;
    const double* scale = nullptr;
    std::vector<LrHalf> halves;
    int wrows = 0;
    double flops = 0.0;
    LrRankSummary ranks;
};

// Low-rank products of several merges (one tree level) on one stream: every
// compression is launched first and all ranks are read in one round trip,
// then each merge's products follow in turn (host-synchronising once).
hipError_t dc_lowrank_products(int b, double tol, std::vector<LrMerge>& ms, int variant,
                               hipStream_t s);

// Largest block size b of the compression: with column offsets (merge nodes)
// or with plain column nodes.
int dc_lowrank_max_block(bool offsets);

hipError_t dc_lowrank_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                             const int* org, const double* tau, const double* zhat,
                             const double* scale, double* C, long long ldc, double lr_tol,
                             int lr_block, hipStream_t stream);
hipError_t dc_plain_update(int m, int K, const double* Qnd, long long ldq, const double* Dbar,
                           const int* org, const double* tau, const double* zhat,
                           const double* scale, double* C, long long ldc, int beta,
                           int variant, hipStream_t stream);
hipError_t dc_node_arrays(int K, const double* Dbar, const int* org, const double* tau,
                          double* cbase, double* coff, hipStream_t s);
hipError_t dc_disable_tasks(GemmTask* tasks, int n, const int* zero, hipStream_t s);
