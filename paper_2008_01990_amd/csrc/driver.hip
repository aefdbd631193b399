// Divide-and-conquer tree driver (Algorithm 1, with Algorithm 3's choice of
// merge product) and the dc_stedc family of entry points.
//
// Plan: every problem is split at k = m / 2 until a block has at most
// `leaf` rows.  Merges are grouped by tree depth; all merges of one depth
// (of every problem of a batch) form one level, processed as one launch per
// phase:
//   deflate -> secular roots / Loewner / scales -> assemble (eigenvalue
//   order) -> rotate and gather -> deflated copy -> [low-rank pipeline]
//   -> generated-Cauchy product (top and bottom row halves).
// Leaves run first, all in one launch.  Below the root, eigenvectors stay
// where they were formed, in the workspace basis B1: a merge writes the
// columns it deflates by rotation over the columns they came from and its
// product columns over the columns of the survivors (already packed into the
// product panel); the columns it deflates untouched do not move.  A map per
// node (sorted eigenvalue -> column of B1) and a row range per column record
// the layout.  Only the root merge writes Q, in eigenvalue order: the
// permutation is materialised once.
//
// Nothing here synchronises with the device after the plan exists: the
// level loop only launches kernels, with data-dependent sizes (the deflated
// K of each merge, the low-rank ranks) read by the kernels from device memory
// and grids sized for the worst case or walking device-held tile counts.
//
// Merges whose order reaches the low-rank switch are candidates: each has
// low-rank regions in the workspace sized by its order, and its skeleton
// columns W go into its square of the buffer it does not write (Q below the
// root, B1 at the root once the deflated columns are in Q).
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "dc_internal.hpp"
#include "driver.hpp"
#include "lowrank.hpp"

namespace {

struct Level {
    int first;          // first merge (slot) of the level
    int nm;
    int tiles;          // worst-case product tiles
    int sec_blocks, row_blocks, copy_blocks, gather_blocks, rot_blocks;
    int max_m;          // largest merge of the level
    int depth;          // tree depth of its merges (0: the roots, which write Q)
    bool stride;        // gather and rotation workgroups take strided groups
    int variant, bm, bn;   // product tile shape of the level
    int off_tile, off_sec, off_row, off_copy, off_gather, off_rot;   // prefix offsets
};

// Low-rank candidates of one plan for one (block size, switch): merges whose
// order reaches the switch and exceeds one block (and spans at most
// DC_LR_MAX_PMAX blocks), in level order.  The
// device table and the per-level SRRSC block prefixes are uploaded once; the
// workspace offsets are relative to the low-rank part of the workspace.
constexpr int DC_LR_MAX_PMAX = 3072;

struct LrCand {
    int merge;          // index of the merge (slot)
    int pmax;           // ceil(m / b)
    int task0;          // first task of the candidate in the task lists
    int pad_;
    long long reg;      // byte offset of its regions
};

struct LrLevel {
    int first = 0, njobs = 0;      // candidates of the level
    int srrsc_blocks = 0;          // sum of pmax^2
    int start_off = 0;             // its SRRSC prefix in d_start (njobs + 1 ints)
    int task0 = 0, ntasks = 0;     // its tasks in the task lists
    int ts_off = 0;                // its tile prefix scratch (2 (ntasks + 1) ints)
    int max_pmax = 0;
    int tiles_skel = 0, tiles_fused = 0;   // tile bounds of its two launches
};

struct LrPlan {
    int b = 0, min_k = 0;
    std::vector<LrCand> cands;
    std::vector<LrLevel> levels;   // one per plan level
    std::vector<int> cand_of_merge;
    size_t o_jobs = 0, o_tskel = 0, o_tfused = 0, o_ts = 0, o_tot = 0, o_reg = 0, bytes = 0;
    LrCand* d_cands = nullptr;
    int* d_start = nullptr;
    ~LrPlan() {
        if (d_cands) hipFree(d_cands);
        if (d_start) hipFree(d_start);
    }
};

struct Plan {
    std::vector<int> sizes;
    int leaf, tile;
    std::vector<Node> leaves, merges;   // merges ordered by level, deepest first
    std::vector<Level> levels;
    std::vector<int> prefix;            // all per-level prefix sums
    std::vector<long long> row0, buf_off, pan_off;
    long long rows = 0;                 // sum of n
    long long buf_elems = 0;            // sum of n^2 (working bases B1)
    long long pan_elems = 0;            // sum of panel_ld(n) n (survivor panels)
    Node* d_nodes = nullptr;            // leaves then merges
    int* d_prefix = nullptr;
    int device = -1;
    std::map<std::pair<int, int>, std::unique_ptr<LrPlan>> lr;   // by (b, min_k)
    ~Plan() {
        if (d_nodes) hipFree(d_nodes);
        if (d_prefix) hipFree(d_prefix);
    }
};

// Leading dimension of a problem's survivor-panel buffer: a whole number of
// 128-byte lines plus one, so the k-columns of a panel (read together by the
// product's tiles) do not sit a power of two apart and share L2 sets.
int panel_ld(int n) { return ((std::max(n, 1) + 15) & ~15) + 16; }

void split(std::vector<std::vector<Node>>& by_depth, std::vector<Node>& leaves, int prob,
           int off, int m, int depth, int leaf) {
    if (m <= leaf) {
        leaves.push_back(Node{prob, off, m, 0, depth, -1});
        return;
    }
    const int k = m / 2;
    split(by_depth, leaves, prob, off, k, depth + 1, leaf);
    split(by_depth, leaves, prob, off + k, m - k, depth + 1, leaf);
    if ((int)by_depth.size() <= depth) by_depth.resize(depth + 1);
    by_depth[depth].push_back(Node{prob, off, k, m - k, depth, -1});
}

// Tile variants chosen by dc_autotune, per device, by the size bucket of a
// level's largest merge: bucket b holds sizes in (2^(b-1), 2^b].
// dc_autotune_batched keeps, per (device, leaf, sizes), one variant per level
// of that plan; it takes precedence over the bucket table.
constexpr int NBUCKET = 24;
std::mutex g_tune_mu;
std::map<int, std::vector<int>> g_tuned;
std::map<std::vector<int>, std::vector<int>> g_level_tuned;
// dc_autotune_batched with lr_tol > 0: low-rank block size and switch per
// (device, leaf, sizes).
std::map<std::vector<int>, std::pair<int, int>> g_lr_tuned;
int g_tune_epoch = 0;

int size_bucket(int m) {
    int b = 0;
    while (b < NBUCKET - 1 && (1 << b) < m) ++b;
    return b;
}

// Product tile shape of a level: a forced variant, the tuned choice for the
// level's largest merge, or by default 64 x 64 tiles for levels of merges up
// to 256 (more tiles per merge) and the 128 x 128 register kernel above.
int level_variant(int forced, int max_m, const std::vector<int>* tuned) {
    if (forced > 0) return forced;
    if (tuned && (*tuned)[size_bucket(max_m)] >= 0) return (*tuned)[size_bucket(max_m)];
    if (max_m <= 512) return 5;
    return 0;
}

std::unique_ptr<Plan> make_plan(const std::vector<int>& sizes, int leaf, int tile,
                                const std::vector<int>* tuned,
                                const std::vector<int>* per_level) {
    auto P = std::make_unique<Plan>();
    P->sizes = sizes;
    P->leaf = leaf;
    P->tile = tile;
    std::vector<std::vector<Node>> by_depth;
    for (size_t p = 0; p < sizes.size(); ++p) {
        P->row0.push_back(P->rows);
        P->buf_off.push_back(P->buf_elems);
        P->pan_off.push_back(P->pan_elems);
        P->rows += sizes[p];
        P->buf_elems += (long long)sizes[p] * sizes[p];
        P->pan_elems += (long long)panel_ld(sizes[p]) * sizes[p];
        if (sizes[p] > 0) split(by_depth, P->leaves, (int)p, 0, sizes[p], 0, leaf);
    }
    for (int dep = (int)by_depth.size() - 1; dep >= 0; --dep) {
        Level L{};
        L.depth = dep;
        L.first = (int)P->merges.size();
        for (Node N : by_depth[dep]) {
            N.slot = (int)P->merges.size();
            P->merges.push_back(N);
        }
        L.nm = (int)P->merges.size() - L.first;
        if (L.nm == 0) continue;
        L.max_m = 0;
        for (int i = 0; i < L.nm; ++i)
            L.max_m = std::max(L.max_m, P->merges[L.first + i].n1 + P->merges[L.first + i].n2);
        const size_t li = P->levels.size();
        L.variant = tile <= 0 && per_level && li < per_level->size()
                        ? (*per_level)[li]
                        : level_variant(tile, L.max_m, tuned);
        L.bm = dc_gemm_tile_m(L.variant);
        L.bn = dc_gemm_tile_n(L.variant);
        const int bm = L.bm, bn = L.bn;
        auto& pre = P->prefix;
        L.off_tile = (int)pre.size();
        int acc = 0;
        for (int i = 0; i < L.nm; ++i) {
            const Node& N = P->merges[L.first + i];
            const int m = N.n1 + N.n2;
            const int tn = (m + bn - 1) / bn;
            pre.push_back(acc);
            acc += ((N.n1 + bm - 1) / bm) * tn;
            pre.push_back(acc);
            acc += ((N.n2 + bm - 1) / bm) * tn;
        }
        pre.push_back(acc);
        L.tiles = acc;
        // Each grid's prefix (nm + 1 entries) is followed by its block -> merge
        // map (one entry per block), so a workgroup finds its merge with one
        // load instead of a binary search of dependent loads.
        auto add_map = [&](int off) {
            for (int i = 0; i < L.nm; ++i)
                for (int b = pre[off + i]; b < pre[off + i + 1]; ++b) pre.push_back(i);
        };
        auto add = [&](int per, int& off, int& total) {
            off = (int)pre.size();
            int a = 0;
            for (int i = 0; i < L.nm; ++i) {
                const Node& N = P->merges[L.first + i];
                pre.push_back(a);
                a += (N.n1 + N.n2 + per - 1) / per;
            }
            pre.push_back(a);
            total = a;
            add_map(off);
        };
        add(DC_ROOTS_PER_BLOCK, L.off_sec, L.sec_blocks);
        add(DC_ROWS_PER_BLOCK, L.off_row, L.row_blocks);
        add(DC_COLS_PER_BLOCK, L.off_copy, L.copy_blocks);
        auto add_fn = [&](auto blocks_of, int& off, int& total) {
            off = (int)pre.size();
            int a = 0;
            for (int i = 0; i < L.nm; ++i) {
                const Node& N = P->merges[L.first + i];
                pre.push_back(a);
                a += blocks_of(N.n1 + N.n2);
            }
            pre.push_back(a);
            total = a;
            add_map(off);
        };
        L.stride = L.max_m < DC_STRIDE_MAX_M;
        const bool st = L.stride;
        add_fn([st](int m) { return dc_gather_blocks(m, st); }, L.off_gather, L.gather_blocks);
        // rotations: (row blocks) x (chain groups); at most m/2 chains
        add_fn([st](int m) {
            return ((m + DC_ROWS_PER_BLOCK - 1) / DC_ROWS_PER_BLOCK) * dc_rot_group_blocks(m, st);
        }, L.off_rot, L.rot_blocks);
        P->levels.push_back(L);
    }
    return P;
}

hipError_t upload(Plan& P) {
    hipError_t err = hipGetDevice(&P.device);
    if (err != hipSuccess) return err;
    std::vector<Node> all(P.leaves);
    all.insert(all.end(), P.merges.begin(), P.merges.end());
    if (!all.empty()) {
        err = hipMalloc(&P.d_nodes, all.size() * sizeof(Node));
        if (err != hipSuccess) return err;
        err = hipMemcpy(P.d_nodes, all.data(), all.size() * sizeof(Node), hipMemcpyHostToDevice);
        if (err != hipSuccess) return err;
    }
    if (!P.prefix.empty()) {
        err = hipMalloc(&P.d_prefix, P.prefix.size() * sizeof(int));
        if (err != hipSuccess) return err;
        err = hipMemcpy(P.d_prefix, P.prefix.data(), P.prefix.size() * sizeof(int),
                        hipMemcpyHostToDevice);
    }
    return err;
}

std::mutex g_plan_mu;
std::map<std::vector<int>, std::unique_ptr<Plan>> g_plans;

// Plans are keyed by (device, leaf, tile option, tuning epoch, sizes).  A new
// tuning leaves older plans (and graphs captured on them) valid.
hipError_t get_plan(const std::vector<int>& sizes, int leaf, int variant, Plan** out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    int epoch = 0;
    std::vector<int> tuned, per_level;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        epoch = g_tune_epoch;
        auto t = g_tuned.find(dev);
        if (t != g_tuned.end()) tuned = t->second;
        std::vector<int> lkey{dev, leaf};
        lkey.insert(lkey.end(), sizes.begin(), sizes.end());
        auto pl = g_level_tuned.find(lkey);
        if (pl != g_level_tuned.end()) per_level = pl->second;
    }
    std::vector<int> key{dev, leaf, variant, epoch};
    key.insert(key.end(), sizes.begin(), sizes.end());
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.get();
        return hipSuccess;
    }
    auto P = make_plan(sizes, leaf, variant, tuned.empty() ? nullptr : &tuned,
                       per_level.empty() ? nullptr : &per_level);
    err = upload(*P);
    if (err != hipSuccess) return err;
    *out = P.get();
    g_plans[key] = std::move(P);
    return hipSuccess;
}

// Workspace layout.
struct Layout {
    size_t bytes = 0;
    size_t probs, gtask, stask, cnt, rho2, psc, dbl, ints, rng, tiles, bufs, lr;
    int nd = 16, ni = 19;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Candidates, tasks and regions of the low-rank path for block b and switch
// min_k (host side; the device tables are uploaded by get_lr_plan).
std::unique_ptr<LrPlan> make_lr(const Plan& P, int b, int min_k, std::vector<int>* starts) {
    auto L = std::make_unique<LrPlan>();
    L->b = b;
    L->min_k = min_k;
    L->cand_of_merge.assign(P.merges.size(), -1);
    L->levels.resize(P.levels.size());
    int ntask = 0, ts = 0;
    size_t reg = 0;
    for (size_t li = 0; li < P.levels.size(); ++li) {
        const Level& Lv = P.levels[li];
        LrLevel& LL = L->levels[li];
        LL.first = (int)L->cands.size();
        LL.task0 = ntask;
        LL.start_off = starts ? (int)starts->size() : 0;
        int acc = 0;
        for (int i = 0; i < Lv.nm; ++i) {
            const Node& N = P.merges[Lv.first + i];
            const int m = N.n1 + N.n2;
            // (the planning kernel keeps 4 pmax ints of its block grid in LDS)
            if (m < min_k || m <= b || (m + b - 1) / b > DC_LR_MAX_PMAX) continue;
            LrCand c{};
            c.merge = Lv.first + i;
            c.pmax = (m + b - 1) / b;
            c.task0 = ntask;
            c.reg = (long long)reg;
            reg += align256(dc_lowrank_region_bytes(c.pmax, b, m));
            ntask += 2 * c.pmax;
            if (starts) starts->push_back(acc);
            acc += c.pmax * c.pmax;
            LL.max_pmax = std::max(LL.max_pmax, c.pmax);
            for (int rows : {N.n1, N.n2}) {
                LL.tiles_skel += dc_lowrank_max_skel_tiles(rows, m, c.pmax);
                LL.tiles_fused += dc_lowrank_max_fused_tiles(rows, m, b, c.pmax);
            }
            L->cand_of_merge[c.merge] = (int)L->cands.size();
            L->cands.push_back(c);
        }
        LL.njobs = (int)L->cands.size() - LL.first;
        if (starts && LL.njobs > 0) starts->push_back(acc);
        LL.srrsc_blocks = acc;
        LL.ntasks = ntask - LL.task0;
        LL.ts_off = ts;
        if (LL.njobs > 0) ts += 2 * (LL.ntasks + 1);
    }
    size_t o = 0;
    L->o_jobs = o; o = align256(o + L->cands.size() * sizeof(LrJob));
    L->o_tskel = o; o = align256(o + (size_t)ntask * sizeof(GemmTask));
    L->o_tfused = o; o = align256(o + (size_t)ntask * sizeof(GemmTask));
    L->o_ts = o; o = align256(o + (size_t)ts * sizeof(int));
    L->o_tot = o; o = align256(o + 2 * P.levels.size() * sizeof(int));
    L->o_reg = o; o += reg;
    L->bytes = L->cands.empty() ? 0 : o;
    return L;
}

Layout layout(const Plan& P, const LrPlan* LP = nullptr) {
    Layout L;
    size_t o = 0;
    const size_t nm = std::max<size_t>(P.merges.size(), 1);
    const size_t R = std::max<long long>(P.rows, 1);
    L.probs = o; o = align256(o + P.sizes.size() * sizeof(Prob));
    L.gtask = o; o = align256(o + 2 * nm * sizeof(GemmTask));
    L.stask = o; o = align256(o + nm * sizeof(SecTask));
    L.cnt = o; o = align256(o + nm * sizeof(MergeCnt));
    L.rho2 = o; o = align256(o + nm * sizeof(double));
    L.psc = o; o = align256(o + std::max<size_t>(P.sizes.size(), 1) * sizeof(double));
    L.dbl = o; o = align256(o + L.nd * R * sizeof(double));
    L.ints = o; o = align256(o + L.ni * R * sizeof(int));
    L.rng = o; o = align256(o + 2 * R * sizeof(int2));
    // per level: the actual tile prefix of its 2 nm product tasks and the total
    L.tiles = o; o = align256(o + (2 * nm + 2 * (P.levels.size() + 1)) * sizeof(int));
    L.bufs = o; o = align256(o + (P.buf_elems + P.pan_elems) * sizeof(double));
    L.lr = o; o = align256(o + (LP ? LP->bytes : 0));
    L.bytes = o;
    return L;
}

// The low-rank tables of (plan, b, min_k), made and uploaded on first use
// (synchronously: call the workspace query before capturing a graph).
hipError_t get_lr_plan(Plan& P, int b, int min_k, LrPlan** out) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto key = std::make_pair(b, min_k);
    auto it = P.lr.find(key);
    if (it != P.lr.end()) {
        *out = it->second.get();
        return hipSuccess;
    }
    std::vector<int> starts;
    auto L = make_lr(P, b, min_k, &starts);
    hipError_t err = hipSuccess;
    if (!L->cands.empty()) {
        err = hipMalloc(&L->d_cands, L->cands.size() * sizeof(LrCand));
        if (err == hipSuccess)
            err = hipMemcpy(L->d_cands, L->cands.data(), L->cands.size() * sizeof(LrCand),
                            hipMemcpyHostToDevice);
        if (err == hipSuccess) err = hipMalloc(&L->d_start, starts.size() * sizeof(int));
        if (err == hipSuccess)
            err = hipMemcpy(L->d_start, starts.data(), starts.size() * sizeof(int),
                            hipMemcpyHostToDevice);
    }
    if (err != hipSuccess) return err;
    *out = L.get();
    P.lr[key] = std::move(L);
    return hipSuccess;
}

Scratch carve(const Plan& P, const Layout& L, char* w) {
    Scratch S;
    const size_t R = std::max<long long>(P.rows, 1);
    double* db = reinterpret_cast<double*>(w + L.dbl);
    double** dp[] = {&S.Ds, &S.zs, &S.Dbar, &S.zbar, &S.tau, &S.cbase, &S.lamr, &S.zhat,
                     &S.scale, &S.Dd, &S.rc, &S.rs, &S.gDt, &S.gzt, &S.gDb, &S.gzb};
    for (int i = 0; i < L.nd; ++i) *dp[i] = db + i * R;
    int* ib = reinterpret_cast<int*>(w + L.ints);
    int** ip[] = {&S.perm, &S.surv, &S.stype, &S.org, &S.dcol, &S.dtype, &S.rp, &S.ri,
                  &S.rt, &S.ktop, &S.kbot, &S.pos_root, &S.pos_defl, &S.rch, &S.ptop,
                  &S.pbot, &S.rdk, &S.cmap0, &S.cmap1};
    for (int i = 0; i < L.ni; ++i) *ip[i] = ib + i * R;
    S.rng0 = reinterpret_cast<int2*>(w + L.rng);
    S.rng1 = S.rng0 + R;
    S.cnt = reinterpret_cast<MergeCnt*>(w + L.cnt);
    S.rho2 = reinterpret_cast<double*>(w + L.rho2);
    S.psc = reinterpret_cast<double*>(w + L.psc);
    S.probs = reinterpret_cast<Prob*>(w + L.probs);
    S.gtask = reinterpret_cast<GemmTask*>(w + L.gtask);
    S.stask = reinterpret_cast<SecTask*>(w + L.stask);
    return S;
}

__global__ void k_fill_int(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Optional instrumentation: HIP events on the caller's stream at the phase
// boundaries of every level, in launch order (deflate, secular, assemble,
// rotate and gather, deflated copy, product), and inside the product phase of a level
// with low-rank merges (before the compression, the skeleton launch and the
// fused launch, and after it).  Off by default; never enabled under graph
// capture.
constexpr int NPHASE = 6;
// marks before the phases in launch order: 0 deflate, 1 secular, 2 assemble,
// 3 rotate (and gather), 4 deflated copy, 5 product; NPHASE after it
constexpr int MARK_ROTATE = 3, MARK_COPY = 4, MARK_PRODUCT = 5;
bool g_prof = false;
std::vector<hipEvent_t> g_ev, g_lr_ev;
std::vector<char> g_lr_rec;            // level recorded its low-rank events
int g_ev_levels = 0;

hipError_t prof_event(std::vector<hipEvent_t>& v, size_t idx, hipEvent_t* out) {
    while (v.size() <= idx) {
        hipEvent_t ev;
        hipError_t err = hipEventCreate(&ev);
        if (err != hipSuccess) return err;
        v.push_back(ev);
    }
    *out = v[idx];
    return hipSuccess;
}

hipError_t prof_mark(int level, int phase, hipStream_t s) {
    if (!g_prof) return hipSuccess;
    hipEvent_t ev;
    hipError_t err = prof_event(g_ev, (size_t)level * (NPHASE + 1) + phase, &ev);
    return err == hipSuccess ? hipEventRecord(ev, s) : err;
}

// The four low-rank events of a level (null when not profiling).
hipError_t prof_lr_events(int level, hipEvent_t* ev4, bool* on) {
    *on = g_prof;
    if (!g_prof) return hipSuccess;
    for (int k = 0; k < 4; ++k) {
        hipError_t err = prof_event(g_lr_ev, (size_t)level * 4 + k, &ev4[k]);
        if (err != hipSuccess) return err;
    }
    if (g_lr_rec.size() <= (size_t)level) g_lr_rec.resize(level + 1, 0);
    g_lr_rec[level] = 1;
    return hipSuccess;
}

}  // namespace

namespace {

// Actual tile grids of a level's plain product tasks, once the device knows
// each merge's K: every task's tiles_n becomes ceil(ncol / bn) (its rows
// are fixed), and tile_start / *total their exclusive prefix and sum.  One
// workgroup.
constexpr int SCAN_NT = 1024;
__global__ __launch_bounds__(SCAN_NT)
void k_tile_scan(GemmTask* __restrict__ tasks, int ntasks, int bn, int* __restrict__ tile_start,
                 int* __restrict__ total) {
    __shared__ int wsum[SCAN_NT / 64];
    __shared__ int carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ntasks; base += SCAN_NT) {
        const int t = base + tid;
        int v = 0;
        if (t < ntasks) {
            GemmTask& T = tasks[t];
            const int ncol = T.ncol_p ? *T.ncol_p : T.ncol;
            const int tn = (ncol + bn - 1) / bn;
            T.tiles_n = tn;
            v = T.tiles_m * tn;
        }
        int x = v;                                      // inclusive scan in the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int before = carry;
        for (int q = 0; q < w; ++q) before += wsum[q];
        if (t < ntasks) tile_start[t] = before + x - v;
        __syncthreads();
        if (tid == SCAN_NT - 1) carry = before + x;
        __syncthreads();
    }
    if (tid == 0) {
        tile_start[ntasks] = carry;
        *total = carry;
    }
}

}  // namespace

hipError_t dc_launch_tile_scan(GemmTask* tasks, int ntasks, int bn, int* tile_start, int* total,
                               hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(SCAN_NT), 0, s, tasks, ntasks, bn, tile_start,
                       total);
    return hipGetLastError();
}

namespace {

// The low-rank jobs of every candidate of the plan: the call's pointers
// (problem buffers, scratch, workspace) and the candidate's regions.  W is
// the candidate's square of the buffer it does not write: Q below the root
// (Q receives nothing before the root merge), B1 at the root (its square is
// dead once the deflated columns are in Q, before the product runs).
__global__ void k_lr_build(const LrCand* __restrict__ cands, int ncand,
                           const Node* __restrict__ merges, Scratch S, char* regbase,
                           LrJob* jobs, GemmTask* tskel, GemmTask* tfused, int b, int min_k) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncand) return;
    const LrCand C = cands[c];
    const Node N = merges[C.merge];
    const Prob P = S.probs[N.prob];
    const long long base = (long long)P.row0 + N.off;
    const int m = N.n1 + N.n2;
    long long ldo;
    double* Qo = node_buf(P, N.depth, ldo);
    const long long ldw = N.depth > 0 ? P.ldq : P.ld1;
    double* Wb = N.depth > 0 ? P.Q : P.B1;
    MergeCnt* cnt = S.cnt + N.slot;
    LrJob J;
    memset(&J, 0, sizeof(J));
    J.K_p = &cnt->K;
    J.pmax = C.pmax;
    J.min_k = min_k;
    J.nh = 2;
    J.D = S.Dbar + base;
    J.zhat = S.zhat + base;
    J.cbase = S.cbase + base;
    J.coff = S.tau + base;
    J.scale = S.scale + base;
    for (int h = 0; h < 2; ++h) {
        LrHalf& H = J.h[h];
        const int r0 = h ? N.n1 : 0;
        H.A = P.B2 + (long long)N.off * P.ld2 + N.off + r0;
        H.lda = P.ld2;
        H.rows = h ? N.n2 : N.n1;
        H.r0 = r0;
        H.klist = (h ? S.kbot : S.ktop) + base;
        H.klen_p = h ? &cnt->nbot : &cnt->ntop;
        H.gD = (h ? S.gDb : S.gDt) + base;
        H.gz = (h ? S.gzb : S.gzt) + base;
        H.C = Qo + (long long)N.off * ldo + N.off + r0;
        H.ldc = ldo;
        H.cpos = S.pos_root + base;
    }
    J.W = Wb + (long long)N.off * ldw + N.off;
    J.ldw = ldw;
    J.wrows = m;
    J.wcap = m;
    J.plain = S.gtask + 2 * N.slot;
    J.zero = &cnt->pad_[0];
    J.tskel = tskel + C.task0;
    J.tfused = tfused + C.task0;
    dc_lowrank_carve(J, regbase + C.reg, b, m);
    jobs[c] = J;
}

// Algorithm 3's switch and the structured product for the candidates of one
// level, all on the device (graph-capturable).
hipError_t lowrank_level(const LrPlan& LP, int li, char* lrbase, double tol, hipStream_t s) {
    const LrLevel& LL = LP.levels[li];
    LrJob* jobs = reinterpret_cast<LrJob*>(lrbase + LP.o_jobs) + LL.first;
    GemmTask* tskel = reinterpret_cast<GemmTask*>(lrbase + LP.o_tskel) + LL.task0;
    GemmTask* tfused = reinterpret_cast<GemmTask*>(lrbase + LP.o_tfused) + LL.task0;
    int* ts = reinterpret_cast<int*>(lrbase + LP.o_ts) + LL.ts_off;
    int* tot = reinterpret_cast<int*>(lrbase + LP.o_tot) + 2 * li;
    hipError_t err = dc_lowrank_decide(jobs, LL.njobs, LP.b, s);
    if (err != hipSuccess) return err;
    hipEvent_t ev[4];
    bool prof = false;
    err = prof_lr_events(li, ev, &prof);
    if (err != hipSuccess) return err;
    return dc_lowrank_level(jobs, LL.njobs, LP.d_start + LL.start_off, LL.srrsc_blocks, tskel,
                            tfused, LL.ntasks, ts, tot, LP.b, tol, LL.max_pmax,
                            LL.tiles_skel, LL.tiles_fused, true, s, prof ? ev : nullptr);
}

hipError_t run_plan(const Plan& P, const LrPlan* LP, const std::vector<Prob>& probs,
                    char* work, const dc_opts& o, hipStream_t s) {
    const Layout L = layout(P, LP);
    Scratch S = carve(P, L, work);
    char* lrbase = work + L.lr;
    hipError_t err = dc_launch_set_probs(probs.data(), (int)probs.size(), S.probs, s);
    if (err != hipSuccess) return err;
    // Exact power-of-two scaling of every problem to max(|d|, |e|) in [1, 2)
    // (results are unchanged where nothing under- or overflows; it keeps the
    // squared pole distances of the secular and scale steps in range).
    err = dc_launch_scale((int)probs.size(), false, S, s);
    if (err != hipSuccess) return err;
    const Node* d_leaves = P.d_nodes;
    const Node* d_merges = P.d_nodes + P.leaves.size();
    for (const Level& Lv : P.levels) {
        err = dc_launch_build(d_merges + Lv.first, Lv.nm, Lv.bm, Lv.bn, S, s);
        if (err != hipSuccess) return err;
    }
    const bool lr = LP && o.lr_tol > 0.0 && !LP->cands.empty();
    if (lr) {
        const int nc = (int)LP->cands.size();
        hipLaunchKernelGGL(k_lr_build, dim3((nc + 63) / 64), dim3(64), 0, s, LP->d_cands, nc,
                           d_merges, S, lrbase + LP->o_reg,
                           reinterpret_cast<LrJob*>(lrbase + LP->o_jobs),
                           reinterpret_cast<GemmTask*>(lrbase + LP->o_tskel),
                           reinterpret_cast<GemmTask*>(lrbase + LP->o_tfused), LP->b,
                           LP->min_k);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    err = dc_launch_leaf(d_leaves, (int)P.leaves.size(), P.leaf, S, s);
    if (err != hipSuccess) return err;
    g_ev_levels = (int)P.levels.size();
    if (g_prof) g_lr_rec.assign(P.levels.size(), 0);
    for (int li = 0; li < (int)P.levels.size(); ++li) {
        const Level& Lv = P.levels[li];
        const Node* mg = d_merges + Lv.first;
#define DC_TRY(x) do { err = (x); if (err != hipSuccess) return err; } while (0)
        DC_TRY(prof_mark(li, 0, s));
        DC_TRY(dc_launch_deflate(mg, P.d_prefix + Lv.off_row, Lv.nm, Lv.row_blocks, Lv.max_m,
                                 S, s));
        DC_TRY(prof_mark(li, 1, s));
        DC_TRY(dc_launch_secular(S.stask + Lv.first, P.d_prefix + Lv.off_sec, Lv.nm,
                                 Lv.sec_blocks, Lv.max_m, o.max_iter, s));
        DC_TRY(prof_mark(li, 2, s));
        DC_TRY(dc_launch_assemble(mg, P.d_prefix + Lv.off_row, Lv.nm, Lv.row_blocks, S, s));
        // With the eigenvalue order formed, the rotations write the columns
        // they deflate straight to their output columns and the survivors
        // that end their chains to the panel; the gather packs the others.
        DC_TRY(prof_mark(li, MARK_ROTATE, s));
        DC_TRY(dc_launch_rotate(mg, P.d_prefix + Lv.off_rot, Lv.nm, Lv.rot_blocks, Lv.stride,
                                S, s));
        DC_TRY(dc_launch_gather(mg, P.d_prefix + Lv.off_gather, Lv.nm, Lv.gather_blocks,
                                Lv.stride, S, s));
        // At the root the remaining deflated columns go to Q before the
        // product, whose low-rank form keeps its skeleton columns in B1's
        // square; below the root they stay where they are.
        DC_TRY(prof_mark(li, MARK_COPY, s));
        if (Lv.depth == 0)
            DC_TRY(dc_launch_copy_deflated(mg, P.d_prefix + Lv.off_copy, Lv.nm,
                                           Lv.copy_blocks, S, s));
        DC_TRY(prof_mark(li, MARK_PRODUCT, s));
        if (lr && LP->levels[li].njobs > 0)
            DC_TRY(lowrank_level(*LP, li, lrbase, o.lr_tol, s));
        if ((Lv.stride || Lv.nm >= 16) && Lv.max_m >= 1024 &&
            (Lv.variant == 0 || Lv.variant == 5)) {
            // Levels of merges from 1024 to 4095 rows, or of many merges
            // reaching 4096 and more (the top of a batch of random problems,
            // whose K is a few percent of m): the tiles of the actual K,
            // compacted on the device; the workgroups of the worst-case grid
            // past their total exit at once instead of searching the task
            // list first (batched 256 problems: the two top levels' products
            // 0.37 -> 0.29 ms; on the levels of smaller merges the scan's own
            // launch cost more than it saved, and a level of a few large
            // merges has little to compact).
            int* act = reinterpret_cast<int*>(work + L.tiles) + 2 * Lv.first + 2 * li;
            DC_TRY(dc_launch_tile_scan(S.gtask + 2 * Lv.first, 2 * Lv.nm, Lv.bn, act,
                                       act + 2 * Lv.nm + 1, s));
            DC_TRY(dc_launch_cauchy_gemm_bounded(S.gtask + 2 * Lv.first, act, 2 * Lv.nm,
                                                 Lv.tiles, act + 2 * Lv.nm + 1, Lv.variant,
                                                 false, s));
        } else {
            DC_TRY(dc_launch_cauchy_gemm(S.gtask + 2 * Lv.first, P.d_prefix + Lv.off_tile,
                                         2 * Lv.nm, Lv.tiles, Lv.variant, s));
        }
        DC_TRY(prof_mark(li, NPHASE, s));
#undef DC_TRY
    }
    return dc_launch_scale((int)probs.size(), true, S, s);
}

thread_local const Plan* t_last_plan = nullptr;
thread_local const LrPlan* t_last_lr = nullptr;
thread_local char* t_last_work = nullptr;

}  // namespace

// Fields left at 0 (automatic) take the defaults here; resolve_for may
// replace the low-rank ones by tuned values.
constexpr int DC_DEFAULT_LR_BLOCK = 256;
constexpr int DC_DEFAULT_LR_MIN_K = 2048;

dc_opts dc_resolve_opts(const dc_opts* opt) {
    dc_opts o;
    dc_opts_default(&o);
    if (opt) {
        if (opt->leaf > 0) o.leaf = opt->leaf;
        o.lr_tol = opt->lr_tol;
        if (opt->lr_block > 0) o.lr_block = opt->lr_block;
        if (opt->lr_min_k > 0) o.lr_min_k = opt->lr_min_k;
        if (opt->max_iter > 0) o.max_iter = opt->max_iter;
        o.gemm_tile = opt->gemm_tile;
    }
    if (o.lr_block <= 0) o.lr_block = DC_DEFAULT_LR_BLOCK;
    if (o.lr_min_k <= 0) o.lr_min_k = DC_DEFAULT_LR_MIN_K;
    return o;
}

// Options for a solve of these sizes: the low-rank block size and switch
// the caller left at 0 take the values dc_autotune_batched chose for this
// (device, leaf, sizes), if any, else the defaults.
static dc_opts resolve_for(const dc_opts* opt, const std::vector<int>& sizes) {
    dc_opts o = dc_resolve_opts(opt);
    if (!opt || !(o.lr_tol > 0.0) || (opt->lr_block > 0 && opt->lr_min_k > 0)) return o;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return o;
    std::vector<int> key{dev, o.leaf};
    key.insert(key.end(), sizes.begin(), sizes.end());
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_lr_tuned.find(key);
    if (it == g_lr_tuned.end()) return o;
    if (opt->lr_block <= 0) o.lr_block = it->second.first;
    if (opt->lr_min_k <= 0) o.lr_min_k = it->second.second;
    return o;
}

hipError_t dc_fill_int(int* p, int n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

extern "C" void dc_opts_default(dc_opts* o) {
    if (!o) return;
    o->leaf = 32;
    o->lr_tol = 0.0;
    o->lr_block = 0;                    // automatic: tuned, else 256
    o->lr_min_k = 0;                    // automatic: tuned, else 2048
    o->max_iter = 200;
    o->gemm_tile = 0;
}

static int check_opts(const dc_opts& o) {
    if (o.leaf < 1 || o.leaf > DC_MAX_LEAF) return 1;
    if (!(o.lr_tol >= 0.0)) return 1;
    if (o.lr_block < 16 || o.lr_block > dc_lowrank_max_block(true)) return 1;
    if (o.gemm_tile < 0 || o.gemm_tile >= DC_TILE_VARIANTS) return 1;
    return 0;
}

// Low-rank part of the workspace: for the block size and switch the caller
// fixed, or, for fields left automatic, the largest over the values the tuner
// may choose (so that a later tuning never outgrows a workspace sized now).
// The tables of the pair a solve would use now are uploaded (before any
// graph capture).
static hipError_t lr_workspace(Plan& P, const dc_opts* opt, const dc_opts& o, size_t* bytes) {
    *bytes = 0;
    if (!(o.lr_tol > 0.0)) return hipSuccess;
    std::vector<int> bs, ks;
    if (opt && opt->lr_block > 0) bs = {opt->lr_block};
    else bs = {128, 256, 512, o.lr_block};
    if (opt && opt->lr_min_k > 0) ks = {opt->lr_min_k};
    else ks = {1024, 2048, 4096, o.lr_min_k};
    for (int b : bs)
        for (int k : ks) {
            if (b > dc_lowrank_max_block(true)) continue;
            *bytes = std::max(*bytes, make_lr(P, b, k, nullptr)->bytes);
        }
    LrPlan* LP = nullptr;
    return get_lr_plan(P, o.lr_block, o.lr_min_k, &LP);
}

extern "C" size_t dc_stedc_workspace(int n, const dc_opts* opt) {
    if (n < 0) return 0;
    const dc_opts o = resolve_for(opt, {n});
    if (check_opts(o)) return 0;
    Plan* P = nullptr;
    if (get_plan({n}, o.leaf, o.gemm_tile, &P) != hipSuccess) return 0;
    size_t lrb = 0;
    if (lr_workspace(*P, opt, o, &lrb) != hipSuccess) return 0;
    return layout(*P).bytes + align256(lrb);
}

extern "C" int dc_stedc_ex(int n, double* d, double* e, double* Q, int ldq, void* work,
                           size_t lwork, int* info_dev, const dc_opts* opt,
                           hipStream_t stream) {
    if (n < 0) return -1;
    if (n > 0 && !d) return -2;
    if (n > 1 && !e) return -3;
    if (n > 0 && !Q) return -4;
    if (ldq < std::max(1, n)) return -5;
    const dc_opts o = resolve_for(opt, {n});
    if (check_opts(o)) return -9;
    if (!info_dev) return -8;
    Plan* P = nullptr;
    hipError_t err = get_plan({n}, o.leaf, o.gemm_tile, &P);
    if (err != hipSuccess) return (int)err;
    LrPlan* LP = nullptr;
    if (o.lr_tol > 0.0) {
        err = get_lr_plan(*P, o.lr_block, o.lr_min_k, &LP);
        if (err != hipSuccess) return (int)err;
    }
    const Layout L = layout(*P, LP);
    if (!work || lwork < L.bytes) return -7;
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return -6;
    err = (hipError_t)dc_fill_int(info_dev, 1, 0, stream);
    if (err != hipSuccess) return (int)err;
    if (n == 0) return 0;
    char* w = static_cast<char*>(work);
    Prob pr{};
    pr.d = d;
    pr.e = e;
    pr.Q = Q;
    pr.ldq = ldq;
    pr.B1 = reinterpret_cast<double*>(w + L.bufs);
    pr.ld1 = n;
    pr.B2 = reinterpret_cast<double*>(w + L.bufs) + (size_t)n * n;
    pr.ld2 = panel_ld(n);
    pr.n = n;
    pr.row0 = 0;
    pr.info = info_dev;
    err = run_plan(*P, LP, {pr}, w, o, stream);
    t_last_plan = P;
    t_last_lr = LP;
    t_last_work = w;
    return (int)err;
}

extern "C" size_t dc_stedc_batched_workspace(int count, const int* n_host, const dc_opts* opt) {
    if (count < 0 || (count > 0 && !n_host)) return 0;
    std::vector<int> sizes(n_host, n_host + count);
    for (int v : sizes)
        if (v < 0) return 0;
    const dc_opts o = resolve_for(opt, sizes);
    if (check_opts(o)) return 0;
    Plan* P = nullptr;
    if (get_plan(sizes, o.leaf, o.gemm_tile, &P) != hipSuccess) return 0;
    size_t lrb = 0;
    if (lr_workspace(*P, opt, o, &lrb) != hipSuccess) return 0;
    return layout(*P).bytes + align256(lrb);
}

// Per-problem pointers of a batch over the workspace `w` laid out as L.
static std::vector<Prob> batch_probs(const Plan& P, const Layout& L, char* w,
                                     double* const* d, double* const* e, double* const* Q,
                                     const int* ldq_host, int* info_dev) {
    const int count = (int)P.sizes.size();
    std::vector<Prob> probs(count);
    for (int p = 0; p < count; ++p) {
        Prob& pr = probs[p];
        pr.d = d[p];
        pr.e = e[p];
        pr.Q = Q[p];
        pr.ldq = ldq_host[p];
        pr.B1 = reinterpret_cast<double*>(w + L.bufs) + P.buf_off[p];
        pr.ld1 = std::max(1, P.sizes[p]);
        pr.B2 = reinterpret_cast<double*>(w + L.bufs) + P.buf_elems + P.pan_off[p];
        pr.ld2 = panel_ld(P.sizes[p]);
        pr.n = P.sizes[p];
        pr.row0 = (int)P.row0[p];
        pr.info = info_dev + p;
        pr.pad_ = 0;
    }
    return probs;
}

// Argument checks shared by the batched entry points (their error codes).
static int check_batch(int count, const int* n_host, double* const* d, double* const* e,
                       double* const* Q, const int* ldq_host, int* info_dev, const dc_opts& o) {
    if (count < 0) return -1;
    if (count > 0 && (!n_host || !d || !e || !Q || !ldq_host)) return -2;
    if (check_opts(o)) return -10;
    if (!info_dev) return -9;
    for (int p = 0; p < count; ++p) {
        if (n_host[p] < 0) return -2;
        if (n_host[p] > 0 && (!d[p] || !Q[p])) return -3;
        if (n_host[p] > 1 && !e[p]) return -4;
        if (ldq_host[p] < std::max(1, n_host[p])) return -6;
    }
    return 0;
}

// Batched solve; the captured graphs are cached below, per plan and pointers.
int dc_batched_impl(int count, const int* n_host, double* const* d, double* const* e,
                    double* const* Q, const int* ldq_host, void* work, size_t lwork,
                    int* info_dev, const dc_opts* opt, hipStream_t stream, bool use_graph);

namespace {
struct GraphEntry {
    std::vector<Prob> probs;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::map<std::vector<uintptr_t>, std::unique_ptr<GraphEntry>> g_graphs;
}  // namespace

int dc_batched_impl(int count, const int* n_host, double* const* d, double* const* e,
                    double* const* Q, const int* ldq_host, void* work, size_t lwork,
                    int* info_dev, const dc_opts* opt, hipStream_t stream, bool use_graph) {
    dc_opts o = dc_resolve_opts(opt);
    const int bad = check_batch(count, n_host, d, e, Q, ldq_host, info_dev, o);
    if (bad) return bad;
    std::vector<int> sizes(n_host, n_host + count);
    o = resolve_for(opt, sizes);
    Plan* P = nullptr;
    hipError_t err = get_plan(sizes, o.leaf, o.gemm_tile, &P);
    if (err != hipSuccess) return (int)err;
    LrPlan* LP = nullptr;
    if (o.lr_tol > 0.0) {
        err = get_lr_plan(*P, o.lr_block, o.lr_min_k, &LP);
        if (err != hipSuccess) return (int)err;
    }
    const Layout L = layout(*P, LP);
    if (!work || lwork < L.bytes) return -8;
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return -7;
    char* w = static_cast<char*>(work);
    const std::vector<Prob> probs = batch_probs(*P, L, w, d, e, Q, ldq_host, info_dev);
    t_last_plan = P;                     // for dc_last_stats
    t_last_lr = LP;
    t_last_work = w;
    if (!use_graph) {
        err = (hipError_t)dc_fill_int(info_dev, count, 0, stream);
        if (err != hipSuccess) return (int)err;
        return (int)run_plan(*P, LP, probs, w, o, stream);
    }
    // Graph path: capture the whole level schedule once per signature (the
    // low-rank tolerance, block size and switch are part of it).
    uint64_t tol_bits = 0;
    std::memcpy(&tol_bits, &o.lr_tol, sizeof(tol_bits));
    std::vector<uintptr_t> key{(uintptr_t)P,          (uintptr_t)LP,         (uintptr_t)work,
                               (uintptr_t)info_dev,   (uintptr_t)o.max_iter, (uintptr_t)tol_bits};
    for (int p = 0; p < count; ++p) {
        key.push_back((uintptr_t)d[p]);
        key.push_back((uintptr_t)e[p]);
        key.push_back((uintptr_t)Q[p]);
        key.push_back((uintptr_t)ldq_host[p]);
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        auto G = std::make_unique<GraphEntry>();
        G->probs = probs;
        hipStream_t cap;
        err = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (err != hipSuccess) return (int)err;
        err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) {
            const bool prof = g_prof;
            g_prof = false;                  // no event records inside the graph
            hipError_t e1 = dc_fill_int(info_dev, count, 0, cap);
            if (e1 == hipSuccess) e1 = run_plan(*P, LP, G->probs, w, o, cap);
            g_prof = prof;
            hipGraph_t graph = nullptr;
            err = hipStreamEndCapture(cap, &graph);
            if (e1 != hipSuccess) err = e1;
            if (err == hipSuccess) err = hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0);
            if (graph) hipGraphDestroy(graph);
        }
        hipStreamDestroy(cap);
        if (err != hipSuccess) return (int)err;
        it = g_graphs.emplace(key, std::move(G)).first;
    }
    return (int)hipGraphLaunch(it->second->exec, stream);
}

extern "C" int dc_stedc_batched(int count, const int* n_host, double* const* d,
                                double* const* e, double* const* Q, const int* ldq_host,
                                void* work, size_t lwork, int* info_dev, const dc_opts* opt,
                                hipStream_t stream) {
    return dc_batched_impl(count, n_host, d, e, Q, ldq_host, work, lwork, info_dev, opt,
                           stream, true);
}

extern "C" int dc_stedc_batched_eager(int count, const int* n_host, double* const* d,
                                      double* const* e, double* const* Q, const int* ldq_host,
                                      void* work, size_t lwork, int* info_dev,
                                      const dc_opts* opt, hipStream_t stream) {
    return dc_batched_impl(count, n_host, d, e, Q, ldq_host, work, lwork, info_dev, opt,
                           stream, false);
}

extern "C" int dc_last_stats(dc_merge_stat* out, int cap) {
    const Plan* P = t_last_plan;
    if (!P || !t_last_work) return 0;
    const LrPlan* LP = t_last_lr;
    const Layout L = layout(*P, LP);
    std::vector<MergeCnt> cnt(P->merges.size());
    if (!cnt.empty() &&
        hipMemcpy(cnt.data(), t_last_work + L.cnt, cnt.size() * sizeof(MergeCnt),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return 0;
    // low-rank records of the candidates (the job holds each record's place)
    std::vector<LrRec> rec(LP ? LP->cands.size() : 0);
    for (size_t c = 0; c < rec.size(); ++c) {
        const LrCand& C = LP->cands[c];
        const Node& N = P->merges[C.merge];
        LrJob J;
        std::memset(&J, 0, sizeof(J));
        J.pmax = C.pmax;
        dc_lowrank_carve(J, t_last_work + L.lr + LP->o_reg + C.reg, LP->b, N.n1 + N.n2);
        if (hipMemcpy(&rec[c], J.rec, sizeof(LrRec), hipMemcpyDeviceToHost) != hipSuccess)
            return 0;
    }
    const int nmr = (int)P->merges.size();
    for (int lv = 0; lv < (int)P->levels.size(); ++lv) {
        const Level& Lv = P->levels[lv];
        for (int i = 0; i < Lv.nm; ++i) {
            const int g = Lv.first + i;
            if (!out || g >= cap) continue;
            const Node& N = P->merges[g];
            dc_merge_stat& r = out[g];
            std::memset(&r, 0, sizeof(r));
            r.level = (int)P->levels.size() - 1 - lv;
            r.m = N.n1 + N.n2;
            r.K = cnt[g].K;
            r.nrot = cnt[g].nrot;
            r.n1 = N.n1;
            r.ntop = cnt[g].ntop;
            r.nbot = cnt[g].nbot;
            r.prob = N.prob;
            r.sec_iters_sum = cnt[g].sec_iters[0];
            r.sec_iters_max = cnt[g].sec_iters[1];
            const int c = LP ? LP->cand_of_merge[g] : -1;
            const bool lr = c >= 0 && rec[c].active == 1;
            r.path = lr ? 1 : 0;
            if (lr) {
                const LrRec& R = rec[c];
                r.lr_blocks = R.blocks;
                r.lr_rank_sum = R.rank_sum;
                r.lr_rank_max = R.rank_max;
                r.lr_dense = R.dense;
                r.lr_flops_skeleton = R.flops_skel;
                r.lr_flops_fused = R.flops_fused;
                r.flops = R.flops_skel + R.flops_fused;
            } else {
                r.flops = 2.0 * ((double)N.n1 * cnt[g].ntop + (double)N.n2 * cnt[g].nbot) *
                          cnt[g].K;
            }
        }
    }
    return nmr;
}

extern "C" int dc_profile_enable(int on) {
    g_prof = on != 0;
    return 0;
}

extern "C" int dc_profile_read(double* ms, int cap) {
    if (!g_prof) return 0;
    const int nl = g_ev_levels;
    // reported order: deflate, rotate (and gather), secular, assemble, product, copy
    static const int from[NPHASE] = {0, MARK_ROTATE, 1, 2, MARK_PRODUCT, MARK_COPY};
    static const int to[NPHASE] = {1, MARK_COPY, 2, MARK_ROTATE, NPHASE, MARK_PRODUCT};
    for (int li = 0; li < nl; ++li) {
        for (int ph = 0; ph < NPHASE; ++ph) {
            const int k = li * NPHASE + ph;
            if (!ms || k >= cap) continue;
            float t = 0.0f;
            const size_t a = (size_t)li * (NPHASE + 1);
            if (hipEventSynchronize(g_ev[a + to[ph]]) != hipSuccess ||
                hipEventElapsedTime(&t, g_ev[a + from[ph]], g_ev[a + to[ph]]) != hipSuccess)
                t = -1.0f;
            ms[k] = t;
        }
    }
    return nl;
}

extern "C" int dc_profile_read_lowrank(double* ms, int cap) {
    if (!g_prof) return 0;
    const int nl = g_ev_levels;
    for (int li = 0; li < nl; ++li) {
        const bool on = li < (int)g_lr_rec.size() && g_lr_rec[li];
        for (int ph = 0; ph < 3; ++ph) {
            const int k = li * 3 + ph;
            if (!ms || k >= cap) continue;
            float t = 0.0f;
            if (!on) {
                ms[k] = 0.0;
                continue;
            }
            const size_t a = (size_t)li * 4 + ph;
            if (hipEventSynchronize(g_lr_ev[a + 1]) != hipSuccess ||
                hipEventElapsedTime(&t, g_lr_ev[a], g_lr_ev[a + 1]) != hipSuccess)
                t = -1.0f;
            ms[k] = t;
        }
    }
    return nl;
}

// ---- Tile autotuner ----
namespace {

// The fastest variant, unless it beats the default rule's choice by less
// than 3 % (timing noise is not worth a different plan).
int pick_variant(const float* ms, int dflt) {
    int best = dflt;
    for (int v = 0; v < DC_TILE_VARIANTS; ++v)
        if (ms[v] < ms[best]) best = v;
    return ms[best] < 0.97f * ms[dflt] ? best : dflt;
}

__global__ void k_tune_fill(double* a, long long n, double scale) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = scale * (double)((i * 2654435761ll) % 1000003ll) / 1000003.0 - 0.5 * scale;
}

__global__ void k_tune_gens(double* D, int* org, double* tau, double* zhat, double* scale,
                            int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    D[i] = (double)i;
    org[i] = i;
    tau[i] = 0.5;
    zhat[i] = 1.0 / sqrt((double)n);
    scale[i] = 1.0;
}

}  // namespace

extern "C" int dc_autotune(int max_n, hipStream_t stream) {
    if (max_n < 0) return -1;
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return (int)err;
    if (max_n == 0) {                    // back to the default rule
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned.erase(dev);
        for (auto it = g_level_tuned.begin(); it != g_level_tuned.end();)
            it = it->first[0] == dev ? g_level_tuned.erase(it) : std::next(it);
        for (auto it = g_lr_tuned.begin(); it != g_lr_tuned.end();)
            it = it->first[0] == dev ? g_lr_tuned.erase(it) : std::next(it);
        ++g_tune_epoch;
        return 0;
    }
    const int cap = std::min(std::max(max_n, 64), 8192);
    const long long elems = (long long)cap * cap;
    double *A = nullptr, *C = nullptr, *g = nullptr;
    err = hipMalloc((void**)&A, elems * sizeof(double));
    if (err == hipSuccess) err = hipMalloc((void**)&C, elems * sizeof(double));
    if (err == hipSuccess) err = hipMalloc((void**)&g, 5 * (size_t)cap * sizeof(double));
    GemmTask* dtask = nullptr;
    int* dstart = nullptr;
    const int maxtasks = std::max(1, (cap / 64) * (cap / 64));
    if (err == hipSuccess) err = hipMalloc((void**)&dtask, maxtasks * sizeof(GemmTask));
    if (err == hipSuccess) err = hipMalloc((void**)&dstart, (maxtasks + 1) * sizeof(int));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    double* D = g;
    double* tau = g + cap;
    double* zhat = g + 2 * (size_t)cap;
    double* scl = g + 3 * (size_t)cap;
    int* org = reinterpret_cast<int*>(g + 4 * (size_t)cap);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0,
                           stream, A, elems, 2.0);
        hipLaunchKernelGGL(k_tune_gens, dim3((cap + 255) / 256), dim3(256), 0, stream, D, org,
                           tau, zhat, scl, cap);
        err = hipGetLastError();
    }
    std::vector<int> table(NBUCKET, -1);
    int last = -1;
    // A level of merges of size m: (cap / m)^2 merges, each an m x m
    // product, so that every bucket's level writes cap^2 outputs (a batch's
    // lower levels hold many small merges, not a few).
    for (int b = 6; err == hipSuccess && b < NBUCKET && (1 << (b - 1)) < cap; ++b) {
        const int m = std::min(1 << b, cap);
        const int nm = std::max(1, (cap / m) * (cap / m));
        float ms_v[DC_TILE_VARIANTS];
        for (int v = 0; v < DC_TILE_VARIANTS; ++v) {
            const int bm = dc_gemm_tile_m(v), bn = dc_gemm_tile_n(v);
            std::vector<GemmTask> tasks(nm);
            std::vector<int> start(nm + 1, 0);
            for (int t = 0; t < nm; ++t) {
                GemmTask& T = tasks[t];
                std::memset(&T, 0, sizeof(T));
                T.A = A + (size_t)t * m * m;
                T.lda = m;
                T.klen = m;
                T.rows = m;
                T.rD = D;
                T.rz = zhat;
                T.corg = org;
                T.coff = tau;
                T.cs = scl;
                T.ncol = m;
                T.C = C + (size_t)t * m * m;
                T.ldc = m;
                T.tiles_m = (m + bm - 1) / bm;
                T.tiles_n = (m + bn - 1) / bn;
                start[t + 1] = start[t] + T.tiles_m * T.tiles_n;
            }
            err = hipMemcpyAsync(dtask, tasks.data(), nm * sizeof(GemmTask),
                                 hipMemcpyHostToDevice, stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(dstart, start.data(), (nm + 1) * sizeof(int),
                                     hipMemcpyHostToDevice, stream);
            if (err == hipSuccess)
                err = dc_launch_cauchy_gemm(dtask, dstart, nm, start[nm], v, stream);
            const int reps = m >= 4096 ? 3 : 5;
            if (err == hipSuccess) err = hipEventRecord(e0, stream);
            for (int r = 0; r < reps && err == hipSuccess; ++r)
                err = dc_launch_cauchy_gemm(dtask, dstart, nm, start[nm], v, stream);
            if (err == hipSuccess) err = hipEventRecord(e1, stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess) break;
            ms_v[v] = ms;
        }
        if (err != hipSuccess) break;
        table[b] = pick_variant(ms_v, level_variant(0, m, nullptr));
        last = b;
    }
    for (int b = 0; b < 6 && last >= 0; ++b) table[b] = table[6];
    for (int b = last + 1; b < NBUCKET && last >= 0; ++b) table[b] = table[last];
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (dtask) (void)hipFree(dtask);
    if (dstart) (void)hipFree(dstart);
    if (g) (void)hipFree(g);
    if (C) (void)hipFree(C);
    if (A) (void)hipFree(A);
    if (err != hipSuccess) return (int)err;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[dev] = table;
    ++g_tune_epoch;
    return 0;
}

extern "C" int dc_autotune_batched(int count, const int* n_host, double* const* d,
                                   double* const* e, double* const* Q, const int* ldq_host,
                                   void* work, size_t lwork, int* info_dev, const dc_opts* opt,
                                   hipStream_t stream) {
    const dc_opts o = dc_resolve_opts(opt);
    const int bad = check_batch(count, n_host, d, e, Q, ldq_host, info_dev, o);
    if (bad) return bad;
    if (o.gemm_tile != 0) return -10;   // nothing to tune with a forced tile
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return (int)err;
    const std::vector<int> sizes(n_host, n_host + count);
    Plan* P0 = nullptr;
    err = get_plan(sizes, o.leaf, 0, &P0);
    if (err != hipSuccess) return (int)err;
    const Layout L = layout(*P0);
    if (!work || lwork < L.bytes) return -8;
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return -7;
    const int nl = (int)P0->levels.size();
    if (nl == 0) return 0;
    char* w = static_cast<char*>(work);
    const std::vector<Prob> probs = batch_probs(*P0, L, w, d, e, Q, ldq_host, info_dev);
    // Keep the diagonals: every timed solve starts from them, and the caller
    // gets them back.
    double* dsave = nullptr;
    err = hipMalloc((void**)&dsave, std::max<long long>(P0->rows, 1) * sizeof(double));
    for (int p = 0; p < count && err == hipSuccess; ++p)
        if (sizes[p] > 0)
            err = hipMemcpyAsync(dsave + P0->row0[p], d[p], sizes[p] * sizeof(double),
                                 hipMemcpyDeviceToDevice, stream);
    auto restore_d = [&]() {
        hipError_t r = hipSuccess;
        for (int p = 0; p < count && r == hipSuccess; ++p)
            if (sizes[p] > 0)
                r = hipMemcpyAsync(d[p], dsave + P0->row0[p], sizes[p] * sizeof(double),
                                   hipMemcpyDeviceToDevice, stream);
        return r;
    };
    // Product time of every level under every variant: the same tree with
    // all levels forced to one variant, solved twice, best of the two.
    std::vector<float> ms((size_t)nl * DC_TILE_VARIANTS, 1e30f);
    const bool prof = g_prof;
    g_prof = true;
    for (int v = 0; v < DC_TILE_VARIANTS && err == hipSuccess; ++v) {
        const std::vector<int> all_v(nl, v);
        auto Pv = make_plan(sizes, o.leaf, 0, nullptr, &all_v);
        err = upload(*Pv);
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
            err = restore_d();
            if (err == hipSuccess) err = dc_fill_int(info_dev, count, 0, stream);
            // levels that switch to the low-rank product keep it (the tile
            // variants are the plain product's, timed where it runs)
            LrPlan* LPv = nullptr;
            if (err == hipSuccess && o.lr_tol > 0.0)
                err = get_lr_plan(*Pv, o.lr_block, o.lr_min_k, &LPv);
            if (err == hipSuccess) err = run_plan(*Pv, LPv, probs, w, o, stream);
            for (int li = 0; li < nl && err == hipSuccess; ++li) {
                const size_t a = (size_t)li * (NPHASE + 1);
                float t = 0.0f;
                err = hipEventSynchronize(g_ev[a + NPHASE]);
                if (err == hipSuccess)
                    err = hipEventElapsedTime(&t, g_ev[a + MARK_PRODUCT], g_ev[a + NPHASE]);
                float& best = ms[(size_t)li * DC_TILE_VARIANTS + v];
                best = std::min(best, t);
            }
        }
        // Pv's node tables are freed at the end of this iteration.
        const hipError_t es = hipStreamSynchronize(stream);
        if (err == hipSuccess) err = es;
    }
    g_prof = prof;
    std::vector<int> per_level(nl);
    for (int li = 0; li < nl; ++li)
        per_level[li] = pick_variant(&ms[(size_t)li * DC_TILE_VARIANTS],
                                     level_variant(0, P0->levels[li].max_m, nullptr));
    std::vector<int> key{dev, o.leaf};
    key.insert(key.end(), sizes.begin(), sizes.end());
    if (err == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_level_tuned[key] = per_level;
        ++g_tune_epoch;
    }
    // Low-rank block size and switch (Algorithm 3's "large"): whole solves
    // over a small grid, for the fields the caller left to the library (0);
    // the default pair is kept unless another is at least 3 % faster.
    if (err == hipSuccess && o.lr_tol > 0.0 && (opt->lr_block <= 0 || opt->lr_min_k <= 0)) {
        Plan* PT = nullptr;
        err = get_plan(sizes, o.leaf, 0, &PT);           // with the tuned tiles
        std::vector<int> bs, ks;
        if (opt->lr_block > 0) bs = {o.lr_block};
        else for (int b : {128, 256, 512}) if (b <= dc_lowrank_max_block(true)) bs.push_back(b);
        if (opt->lr_min_k > 0) ks = {o.lr_min_k};
        else ks = {1024, 2048, 4096};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (err == hipSuccess) err = hipEventCreate(&e0);
        if (err == hipSuccess) err = hipEventCreate(&e1);
        float best = 1e30f, dflt = 1e30f;
        int bb = o.lr_block, bk = o.lr_min_k;
        for (int b : bs)
            for (int k : ks) {
                dc_opts oc = o;
                oc.lr_block = b;
                oc.lr_min_k = k;
                float t = 1e30f;
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
                    err = restore_d();
                    if (err == hipSuccess) err = dc_fill_int(info_dev, count, 0, stream);
                    if (err == hipSuccess) err = hipEventRecord(e0, stream);
                    LrPlan* LPT = nullptr;
                    if (err == hipSuccess) err = get_lr_plan(*PT, b, k, &LPT);
                    if (err == hipSuccess && lwork < layout(*PT, LPT).bytes)
                        err = hipErrorInvalidValue;
                    if (err == hipSuccess) err = run_plan(*PT, LPT, probs, w, oc, stream);
                    if (err == hipSuccess) err = hipEventRecord(e1, stream);
                    if (err == hipSuccess) err = hipEventSynchronize(e1);
                    float ms1 = 0.0f;
                    if (err == hipSuccess) err = hipEventElapsedTime(&ms1, e0, e1);
                    t = std::min(t, ms1);
                }
                if (b == o.lr_block && k == o.lr_min_k) dflt = t;
                if (t < best) { best = t; bb = b; bk = k; }
            }
        if (!(best < 0.97f * dflt)) { bb = o.lr_block; bk = o.lr_min_k; }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (err == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_lr_tuned[key] = {bb, bk};
        }
    }
    if (err == hipSuccess) err = restore_d();
    if (err == hipSuccess) err = hipStreamSynchronize(stream);
    if (dsave) (void)hipFree(dsave);
    return (int)err;
}

extern "C" int dc_autotune_lowrank(int count, const int* n_host, int leaf, int* block_out,
                                   int* min_k_out) {
    if (count < 0 || (count > 0 && !n_host) || !block_out || !min_k_out) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::vector<int> key{dev, leaf};
    key.insert(key.end(), n_host, n_host + count);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_lr_tuned.find(key);
    if (it == g_lr_tuned.end()) return 0;
    *block_out = it->second.first;
    *min_k_out = it->second.second;
    return 1;
}

extern "C" int dc_autotune_levels(int count, const int* n_host, int leaf, int* variant_out,
                                  int cap) {
    if (count < 0 || (count > 0 && !n_host)) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::vector<int> key{dev, leaf};
    key.insert(key.end(), n_host, n_host + count);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto t = g_level_tuned.find(key);
    if (t == g_level_tuned.end()) return 0;
    for (int li = 0; li < (int)t->second.size() && li < cap && variant_out; ++li)
        variant_out[li] = t->second[li];
    return (int)t->second.size();
}

extern "C" int dc_autotune_table(int* variant_out, int cap) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto t = g_tuned.find(dev);
    for (int b = 0; b < NBUCKET && b < cap && variant_out; ++b)
        variant_out[b] = t == g_tuned.end() ? -1 : t->second[b];
    return NBUCKET;
}
