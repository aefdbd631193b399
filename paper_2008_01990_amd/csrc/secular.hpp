// Descriptors of the secular / Loewner / column-scale kernels.
#pragma once
#include "common.hpp"

// One rank-one modified diagonal problem diag(D) + rho z z^T.
struct SecTask {
    const double* D;      // poles, strictly increasing
    const double* z;      // weights
    const int* K_p;       // device size, or null (= K)
    int K;
    int row0;             // first row of the merge inside its problem: a root j
                          // that does not converge reports status row0 + j + 1
    const double* rho_p;  // device rho, or null (= rho)
    double rho;
    int* org;             // out: origin pole of each root
    double* tau;          // out: offset from the origin pole
    double* cbase;        // out: D[org_j]
    double* lam;          // out (optional): D[org_j] + tau_j
    double* zhat;         // out: Loewner weights
    double* scale;        // out: column scales
    int* info;            // status word, or null
    int* iters;           // out (optional): [0] sum, [1] maximum of the roots'
                          // iteration counts (accumulated: cleared by the caller)
};

// block_start: exclusive prefix sum (ntasks + 1 entries, device) of
// ceil(Kmax / 64) per task, followed by the task of each of the total_blocks
// workgroups; the three kernels run in sequence.  max_k bounds
// every task's K (it selects the workgroup shape).
hipError_t dc_launch_secular(const SecTask* tasks, const int* block_start, int ntasks,
                             int total_blocks, int max_k, int max_iter, hipStream_t s);
