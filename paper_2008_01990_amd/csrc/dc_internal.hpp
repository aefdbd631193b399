// Descriptors shared by the tree driver and its kernels.
//
// A plan describes the divide-and-conquer tree of one or many problems with
// pointer-free records (offsets and sizes only), uploaded once.  Per call the
// caller's pointers reach the device through kernel arguments (the Prob table
// is written by a kernel whose arguments carry it), so a captured graph holds
// no pointer to host memory.
#pragma once
#include "secular.hpp"

#define DC_MAX_LEAF 64

struct Prob {
    double* d;          // in: diagonal; out: eigenvalues (also the level's lam array)
    const double* e;    // off-diagonal (n - 1)
    double* Q;          // output eigenvectors, column-major
    long long ldq;
    double* B1;         // working basis of every merge below the root (workspace)
    long long ld1;
    double* B2;         // packed survivor panels of the merge products
    long long ld2;
    int n;
    int row0;           // first row of this problem in the concatenated row space
    int* info;          // status word
    int pad_;
};

// A tree node: a merge (n2 > 0) or a leaf (n2 == 0, size n1).
struct Node {
    int prob;
    int off;            // first row inside its problem
    int n1, n2;
    int depth;          // 0 at the root (writes Q); below it the basis lives in B1
    int slot;           // merge index across the plan (per-merge scalars)
};

// Per-merge counters, one record per merge slot.
struct MergeCnt {
    int K;              // deflated size (secular problem order)
    int nrot;           // pair rotations
    int ndefl;          // deflated eigenpairs
    int ntop;           // survivors with non-zeros in the top rows
    int nbot;           // survivors with non-zeros in the bottom rows
    int nchain;         // rotation chains (a chain shares columns only inside itself)
    int pad_[2];        // pad_[0] stays 0: a disabled product task points here
    int sec_iters[2];   // secular iterations of the merge's roots: sum, maximum
};

// Per-row scratch (indexed by prob.row0 + node.off + local index) and
// per-merge records, all inside the caller's workspace.
struct Scratch {
    double *Ds, *zs;            // sorted poles / weights (m)
    double *Dbar, *zbar;        // survivors (K)
    double *tau, *cbase, *lamr, *zhat, *scale;   // roots and eigenvector generators (K)
    double *Dd;                 // deflated eigenvalues, ascending (m - K)
    double *gDt, *gzt;          // row generators of the top-half product (ntop)
    double *gDb, *gzb;          // row generators of the bottom-half product (nbot)
    double *rc, *rs;            // rotation cosines / sines
    int *perm;                  // sorted position -> local column
    int *surv, *stype;          // survivor -> local column, row-type bits
    int *org;                   // root origin (K)
    int *dcol, *dtype;          // deflated -> local column, row-type bits (1 top rows,
                                //   2 bottom rows; 8: deflated by rotation t = dtype >> 4)
    int *rp, *ri, *rt;          // rotation column pair and row-type bits (p | i << 2)
    int *rch;                   // first rotation of each rotation chain
    int *ktop, *kbot;           // generator lists of the top and bottom row halves
    int *ptop, *pbot;           // place of each survivor in those lists
    int *rdk;                   // deflated-list entry of the column rotation t deflates
    // Resident columns below the root.  The eigenvector of a node's sorted
    // eigenvalue j lives in column cmap[off + j] of B1 (a column of the
    // node's own range [off, off + m)) and holds data only in rows
    // [rng[off + j].x, rng[off + j].y); the other rows of the node's range
    // are structural zeros (stale memory, never read).  A merge reads its
    // children's map and ranges (parity of depth + 1) and writes its own
    // (parity of depth).
    int *cmap0, *cmap1;
    int2 *rng0, *rng1;
    int *pos_root, *pos_defl;   // output column of each root / deflated pair
    MergeCnt* cnt;              // per merge slot
    double* rho2;               // per merge slot: 2 |e_k|
    double* psc;                // per problem: power-of-two scale of d and e
    Prob* probs;
    GemmTask* gtask;            // two per merge slot
    SecTask* stask;             // one per merge slot
};

// Output buffer of a node: the caller's Q at the root, B1 below it (the
// children of every merge are therefore in B1).
__host__ __device__ inline double* node_buf(const Prob& P, int depth, long long& ld) {
    if (depth > 0) { ld = P.ld1; return P.B1; }
    ld = P.ldq;
    return P.Q;
}

__host__ __device__ inline int* node_cmap(const Scratch& S, int depth) {
    return (depth & 1) ? S.cmap1 : S.cmap0;
}

__host__ __device__ inline int2* node_rng(const Scratch& S, int depth) {
    return (depth & 1) ? S.rng1 : S.rng0;
}

// Kernel launchers (deflate.hip / leaf.hip).
// Scaling by powers of two: undo = false picks, per problem, the power of two
// that brings max(|d|, |e|) into [1, 2), stores it in S.psc and scales d in
// place (e stays as given; its readers apply S.psc); undo = true divides the
// eigenvalues in d by it again.
hipError_t dc_launch_scale(int nprob, bool undo, Scratch S, hipStream_t s);
// Every leaf has at most max_leaf (<= DC_MAX_LEAF) rows.
hipError_t dc_launch_leaf(const Node* leaves, int nleaves, int max_leaf, Scratch S,
                          hipStream_t s);
hipError_t dc_launch_build(const Node* merges, int nmerges, int bm, int bn, Scratch S,
                           hipStream_t s);
// k_merge_sort over row blocks (row_start: per-merge prefix of ceil(m /
// DC_ROWS_PER_BLOCK) blocks, nrow_blk in total), then k_deflate per merge.
hipError_t dc_launch_deflate(const Node* merges, const int* row_start, int nm, int nrow_blk,
                             int max_m, Scratch S, hipStream_t s);
hipError_t dc_launch_rotate(const Node* merges, const int* blk_start, int nm, int nblk,
                            bool stride, Scratch S, hipStream_t s);
hipError_t dc_launch_assemble(const Node* merges, const int* blk_start, int nm, int nblk,
                              Scratch S, hipStream_t s);
hipError_t dc_launch_gather(const Node* merges, const int* blk_start, int nm, int nblk,
                            bool stride, Scratch S, hipStream_t s);
hipError_t dc_launch_copy_deflated(const Node* merges, const int* blk_start, int nm,
                                   int nblk, Scratch S, hipStream_t s);
hipError_t dc_launch_set_probs(const Prob* host_probs, int count, Prob* dev, hipStream_t s);

// Rows handled per block by the rotation and assembly kernels, and columns
// per block of the deflated-column copy.
#define DC_ROWS_PER_BLOCK 256
#define DC_COLS_PER_BLOCK 4
#define DC_GATHER_COLS 4
// Column groups (of DC_GATHER_COLS) and chain groups (of DC_ROT_CHAINS) per
// workgroup of the gather and rotation kernels, taken with a stride: the
// grids are sized for the worst case (every column a survivor, m / 2
// chains), and most merges of a batch of random problems have few of either
// (batched 256 problems 6.46 -> 6.07 ms).  Only levels whose merges all
// have fewer than DC_STRIDE_MAX_M rows stride: a workgroup's next group
// waits for its stores (the wait for loads also counts them), which slowed
// the rotations and gathers of the large Clement merges, where every group
// is busy; the rotation kernel has a separate instance for such levels.
#define DC_GROUPS_PER_BLOCK 8
#define DC_STRIDE_MAX_M 4096
#define DC_ROT_CHAINS 8     // rotation chains per block of the rotation kernel
#define DC_ROOTS_PER_BLOCK 64

// Workgroups per merge of order m: the gather's, and the rotation kernel's
// per row block.
__host__ __device__ inline int dc_strided_blocks(int groups, bool stride) {
    if (groups < 1) return 1;
    return stride ? (groups + DC_GROUPS_PER_BLOCK - 1) / DC_GROUPS_PER_BLOCK : groups;
}
__host__ __device__ inline int dc_gather_blocks(int m, bool stride) {
    return dc_strided_blocks((m + DC_GATHER_COLS - 1) / DC_GATHER_COLS, stride);
}
__host__ __device__ inline int dc_rot_group_blocks(int m, bool stride) {
    return dc_strided_blocks((m / 2 + DC_ROT_CHAINS - 1) / DC_ROT_CHAINS, stride);
}
