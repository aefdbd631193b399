// Structured low-rank merge product (SRRSC compression + generated products),
// planned and launched on the device: no host read sits between its kernels,
// so a tree level that takes it can be captured in a graph.
#pragma once
#include <vector>

#include "common.hpp"

// One row half of a merge product: C[rows, :] = A[rows, panel] * U[panel, :],
// where panel column t holds the basis column of survivor klist[t] (klist
// ascending; null means the identity 0..K-1) and gD / gz are the row
// generators in panel order.
struct LrHalf {
    const double* A;
    long long lda;
    int rows;
    int r0;               // first row of the half inside the merge (and W)
    const int* klist;     // survivor list of the half, or null (= 0..K-1)
    const int* klen_p;    // device length of klist, or null (= klen)
    int klen;
    const double* gD;
    const double* gz;
    double* C;
    long long ldc;
    const int* cpos;      // output column of generator g (null: g)
};

// Per-merge record of the low-rank path, written on the device.
struct LrRec {
    int active;           // 1: the merge took the low-rank product
    int nw;               // W columns: sum of the skeleton sizes
    int blocks, rank_sum, rank_max, dense;   // off-diagonal blocks
    double flops_skel, flops_fused;          // executed product flops
};

// Everything the device pipeline of one low-rank merge reads and writes.
// The driver fills these on the device (they hold the call's pointers);
// the stand-alone entry points fill them on the host.
struct LrJob {
    const int* K_p;       // device K, or null (= K)
    int K;
    int pmax;             // block grid bound: ceil(max K / b)
    int min_k;            // take the low-rank product when K >= min_k and K > b
    int nh;               // number of row halves (1 or 2)
    const double *D, *zhat, *cbase, *coff, *scale;   // generators (coff null: plain nodes)
    LrHalf h[2];
    double* W;            // skeleton columns: wrows x wcap, leading dimension ldw
    long long ldw;
    int wrows, wcap;
    GemmTask* plain;      // nh plain product tasks, disabled when the merge switches
    const int* zero;      // an int 0 for the disabled tasks' column count
    // SRRSC output (pmax^2 blocks, rmax skeleton columns each)
    int* rank;
    int* prow;
    int* pcol;
    double* y;
    double* vk;           // pmax^2 x b: v^(r) of each block's columns
    int* woff;            // pmax^2: first W column of block (I, J)
    // per W column (wcap): interpolation rows and the skeleton column lists
    double* Y;            // wcap x b, row-major
    int* rgen;
    long long* rvo;
    int* kJ;
    double* ry;
    int* ccol;
    int* wpos;
    GemmTask* tskel;      // nh * pmax skeleton tasks
    GemmTask* tfused;     // nh * pmax fused tasks
    LrRec* rec;
    // set on the device before compression
    int K_dev, p;         // this call's K and block count (p = 0: plain path)
};

// Largest block size b of the compression: with column offsets (merge nodes)
// or with plain column nodes.
int dc_lowrank_max_block(bool offsets);
// Skeleton-column cap of one block: min(128, b / 2).
int dc_lowrank_rmax(int b);

// Device bytes of one merge's low-rank regions (SRRSC output, layout, Y,
// record) for block grid pmax, block b and W capacity wcap.
size_t dc_lowrank_region_bytes(int pmax, int b, int wcap);
// Points the job's region pointers into `dev` (dc_lowrank_region_bytes;
// J.pmax must be set).
__host__ __device__ inline void dc_lowrank_carve(LrJob& J, char* dev, int b, int wcap) {
    const size_t p2 = (size_t)J.pmax * J.pmax;
    const size_t rmax = b / 2 < 128 ? (b / 2 > 1 ? b / 2 : 1) : 128;
    const size_t w = wcap > 1 ? wcap : 1;
    auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t o = 0;
    J.rank = reinterpret_cast<int*>(dev + o); o = a(o + p2 * sizeof(int));
    J.woff = reinterpret_cast<int*>(dev + o); o = a(o + p2 * sizeof(int));
    J.prow = reinterpret_cast<int*>(dev + o); o = a(o + p2 * rmax * sizeof(int));
    J.pcol = reinterpret_cast<int*>(dev + o); o = a(o + p2 * rmax * sizeof(int));
    J.y = reinterpret_cast<double*>(dev + o); o = a(o + p2 * rmax * sizeof(double));
    J.vk = reinterpret_cast<double*>(dev + o); o = a(o + p2 * (size_t)b * sizeof(double));
    J.Y = reinterpret_cast<double*>(dev + o); o = a(o + w * (size_t)b * sizeof(double));
    J.rgen = reinterpret_cast<int*>(dev + o); o = a(o + w * sizeof(int));
    J.kJ = reinterpret_cast<int*>(dev + o); o = a(o + w * sizeof(int));
    J.ccol = reinterpret_cast<int*>(dev + o); o = a(o + w * sizeof(int));
    J.wpos = reinterpret_cast<int*>(dev + o); o = a(o + w * sizeof(int));
    J.rvo = reinterpret_cast<long long*>(dev + o); o = a(o + w * sizeof(long long));
    J.ry = reinterpret_cast<double*>(dev + o); o = a(o + w * sizeof(double));
    J.rec = reinterpret_cast<LrRec*>(dev + o);
}


// Algorithm 3's switch on the device: sets K_dev and p (0: plain product)
// of every job from its device K.
hipError_t dc_lowrank_decide(LrJob* jobs_dev, int njobs, int b, hipStream_t s);

// The pipeline over njobs jobs in device memory (one tree level), after
// K_dev and p are set:
//   SRRSC on the pmax^2 block grid of every job -> layout, tasks, records and
//   the plain-task switch-off -> interpolation rows -> skeleton product into
//   W -> fused product into C.
// srrsc_start: device prefix of pmax^2 over the jobs (njobs + 1), srrsc_blocks
// its total; tskel / tfused: the level's task lists (job j's nh * pmax tasks
// at its own offset), ntasks in all; tile_start: device scratch of
// 2 (ntasks + 1) ints; totals: 2 ints; max_pmax: largest pmax;
// max_tiles_skel / max_tiles_fused: upper bounds of the two launches' tiles
// (the sums of dc_lowrank_max_skel_tiles / _fused_tiles over the jobs'
// halves);
// offsets: the column nodes carry offsets (merge generators).  ev (optional,
// 4 events) is recorded before the compression, before the skeleton product,
// before the fused product and after it.
hipError_t dc_lowrank_level(LrJob* jobs_dev, int njobs, const int* srrsc_start,
                            int srrsc_blocks, GemmTask* tskel, GemmTask* tfused, int ntasks,
                            int* tile_start, int* totals, int b, double tol, int max_pmax,
                            int max_tiles_skel, int max_tiles_fused, bool offsets,
                            hipStream_t s, const hipEvent_t* ev);
// Upper bound of the skeleton launch's tiles for one row half of `rows` rows
// whose W holds at most wcap columns, over pmax blocks.
int dc_lowrank_max_skel_tiles(int rows, int wcap, int pmax);
// Upper bound of the fused launch's tiles for one row half of `rows` rows of
// a merge of order m (K <= m) over pmax blocks of b.
int dc_lowrank_max_fused_tiles(int rows, int m, int b, int pmax);

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
