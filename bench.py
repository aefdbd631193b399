"""Benchmark: the full divide-and-conquer eigensolve on one MI355X.

One step = one dc_stedc_ex solve (every leaf, every merge level: deflation,
secular roots, Loewner weights, scales, eigenvalue order, generated-Cauchy
merge product, deflated copy) of the n = 32768 Clement-type matrix
(d_i = 0, e_i = sqrt(i (n - i))), leaf 64, inputs resident in HBM.

Printed: one JSON line with the eigensolve seconds (the metric), the
roofline of the dominant kernel (the merge product of the root level, HIP
events on the solver's stream), per-level product rates, the optional
low-rank comparison, accuracy of the last solve and the CPU oracle baseline.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "n=32768 eigensolve sec; merge Q·U % FP64-MFMA peak; low-rank vs plain"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--family", default="clement", choices=["clement", "toeplitz"])
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--gemm-tile", type=int, default=0)
    ap.add_argument("--lowrank-tol", type=float, default=1e-10,
                    help="also time the low-rank path at this tolerance (0: skip)")
    ap.add_argument("--lowrank-block", type=int, default=256)
    ap.add_argument("--lowrank-min-k", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=0)
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched configuration (profiling)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint configuration (profiling)")
    ap.add_argument("--lowrank-only", action="store_true",
                    help="profiling: time only the low-rank solve (not the benchmark line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary configurations (n=1024, n=16384, batched, adjoint)")
    return ap.parse_args()


def inputs(family, n):
    from paper_2008_01990_amd import workloads as W
    return W.clement(n) if family == "clement" else W.toeplitz(n)


def closed_form(family, n):
    import numpy as np
    if family == "clement":
        return np.arange(-(n - 1), n, 2, dtype=np.float64)
    k = np.arange(1, n + 1)
    return 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))


def gpu_accuracy(d, e, lam, Qbuf, family, paper=True):
    """Eigenvalue error, residual and orthogonality of the last solve (GPU,
    plain torch ops independent of the solver's kernels), plus the paper's own
    measures: ||I - Q Q^T||_max (Example 2) and ||A - Q Lambda Q^T||_c /
    ||A||_2, the largest column 2-norm of the reconstruction error (Example 3),
    with ||A||_2 from the closed-form spectrum."""
    import torch
    n = d.numel()
    ref = torch.tensor(closed_form(family, n), device="cuda")
    tn = ref.abs().max()
    eig = float(((lam - ref).abs().max() / tn).item())
    Q = Qbuf.t()                                   # (n, n) view, Q[:, j] eigvec j
    TQ = d[:, None] * Q
    TQ[:-1] += e[:, None] * Q[1:]
    TQ[1:] += e[:, None] * Q[:-1]
    R = TQ - Q * lam[None, :]
    res = float((torch.linalg.norm(R) / (n * tn)).item())
    del TQ, R
    G = Qbuf @ Qbuf.t()                            # = Q^T Q
    G.diagonal().sub_(1.0)
    orth = float(G.abs().max().item())
    del G
    out = {"eig_err_rel": eig, "residual": res, "orthogonality": orth}
    if not paper:
        return out
    G = Qbuf.t() @ Qbuf                            # = Q Q^T (rows)
    G.diagonal().sub_(1.0)
    out["paper_orthogonality_rows"] = float(G.abs().max().item())
    del G
    # A - Q Lambda Q^T in column slabs: column j of A is tridiagonal
    QL = Q * lam[None, :]
    col_max = 0.0
    step = 8192
    for c0 in range(0, n, step):
        c1 = min(n, c0 + step)
        Rs = -(QL @ Qbuf[:, c0:c1])                 # -(Q Lambda Q^T)[:, c0:c1]
        j = torch.arange(c0, c1, device="cuda")
        Rs[j, j - c0] += d[c0:c1]
        jm = j[j > 0]
        Rs[jm - 1, jm - c0] += e[jm - 1]
        jp = j[j < n - 1]
        Rs[jp + 1, jp - c0] += e[jp]
        col_max = max(col_max, float(torch.linalg.norm(Rs, dim=0).max().item()))
        del Rs
    del QL
    out["paper_residual_colnorm"] = col_max / float(tn)
    return out


def cpu_baseline(family, n_full, n_sample, leaf):
    """The oracle on the host cores, timed on a bounded sample: full solves
    of the same family at growing orders n = 4000, ... (at most 1.5x per
    step, multiples of 250, never a power of two, capped at 16000) until one
    takes at least 10 s.  The time is carried to the benchmark's order with
    the growth exponent measured between the last samples.  That exponent
    rises toward 3 with n (the cubic merge product takes over from the
    quadratic steps), so the carried figure understates the oracle's time at
    n_full: it is a lower bound on the CPU time, i.e. it favours the CPU.  The
    cubic carry, (n_full / n)^3, is an upper bound and is reported beside it.
    Orders with a large power-of-two factor make the host BLAS thrash its
    caches, so none is used.  n_sample > 0: one solve at that order, cubic
    carry only."""
    import math
    from threadpoolctl import threadpool_info
    from oracle import dc
    visited = []
    if n_sample <= 0:
        d, e = inputs(family, 1000)             # untimed: the first solve pays start-up
        dc.eigh_tridiagonal(d, e, leaf=leaf)
        n = 4000
        while True:
            d, e = inputs(family, n)
            t0 = time.perf_counter()
            dc.eigh_tridiagonal(d, e, leaf=leaf)
            dt = time.perf_counter() - t0
            visited.append((n, dt))
            if dt >= 10.0 or n >= 16000:
                break
            grow = min(1.5, max(1.15, (15.0 / dt) ** 0.5))
            nxt = min(16000, int(n * grow) // 250 * 250)
            if nxt & (nxt - 1) == 0:
                nxt -= 250
            n = nxt
        n_sample = n
    else:
        d, e = inputs(family, n_sample)
        t0 = time.perf_counter()
        dc.eigh_tridiagonal(d, e, leaf=leaf)
        dt = time.perf_counter() - t0
        visited.append((n_sample, dt))
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    cubic = dt * (n_full / n_sample) ** 3
    if len(visited) >= 2:
        # least-squares slope of log t over log n on the last three samples
        pts = visited[-3:]
        xs = [math.log(m) for m, _ in pts]
        ys = [math.log(t) for _, t in pts]
        xm, ym = sum(xs) / len(xs), sum(ys) / len(ys)
        expo = sum((x - xm) * (y - ym) for x, y in zip(xs, ys)) / \
            sum((x - xm) ** 2 for x in xs)
        expo = min(3.0, max(1.0, expo))
    else:
        expo = 3.0
    value = dt * (n_full / n_sample) ** expo
    steps = ", ".join(f"n={m}: {t:.2f} s" for m, t in visited)
    return {"value": value, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"full oracle solves of the {family} matrix (leaf {leaf}): {steps}; "
                      f"carried from n={n_sample} to n={n_full} with the measured growth "
                      f"exponent {expo:.2f} (a lower bound on the oracle's time there: the "
                      f"exponent rises toward 3 with n); the cubic carry gives {cubic:.1f} s",
            "value_cubic_upper": cubic, "growth_exponent": expo,
            "sample_seconds": dt, "sample_n": n_sample}


def measured_traffic(workload):
    """HBM bytes per root-level product launch from the committed counter
    summary, or None if it was taken on another workload or on a different
    version of the kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_cauchy_gemm_reg_clement_n32768_traffic.md")
    src = os.path.join(ROOT, "paper_2008_01990_amd", "csrc", "cauchy_gemm.hip")
    if workload != "clement_n32768_leaf64_plain" or not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
    if rec is None:
        return None
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return rec["traffic_bytes"] if h == rec["source_sha256_16"] else None


def _time(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _events(fn, reps, torch):
    """Best of reps event-timed runs after one warm-up (seconds)."""
    fn()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    return best


def merge_traffic(r):
    """Algorithmic HBM bytes and flops of one merge (a dc_last_stats record)
    as the level's kernels move them.  Read once, over its child's rows (taken
    as m / 2, the mean of n1 and n2): every survivor's column and every column
    of a rotation chain (K + nrot columns) and, at a root merge, every other
    deflated column.  Written once: the survivor panel (n1 ntop + n2 nbot
    entries, read again by the product), each column deflated by a rotation
    (m rows), the product's m K entries and, at a root merge, the other
    deflated columns (m rows, zeros included).  Below the root the columns
    deflated without a rotation stay where they are and cost nothing."""
    m, n1, K, nrot = r["m"], r["n1"], r["K"], r["nrot"]
    n2 = m - n1
    root = r["level"] == 0
    panel = 8.0 * (n1 * r["ntop"] + n2 * r["nbot"])
    rest = m - K - nrot if root else 0
    move = (8.0 * 0.5 * m * (K + nrot + rest) + panel + 8.0 * m * nrot + 8.0 * m * rest)
    prod_b = panel + 8.0 * m * K
    prod_f = 2.0 * (n1 * r["ntop"] + n2 * r["nbot"]) * K
    return move, prod_b, prod_f


def level_traffic(stats, prof_levels, phases):
    """Per tree level (deepest first, as dc_profile_read orders them): the
    event-timed phases and the algorithmic bytes of the data-movement phases
    (rotations, gather and deflated copy) and of the product."""
    nlev = len(prof_levels)
    move = [0.0] * nlev
    pb = [0.0] * nlev
    pf = [0.0] * nlev
    for r in stats:
        li = nlev - 1 - r["level"]
        a, b, c = merge_traffic(r)
        move[li] += a
        pb[li] += b
        pf[li] += c
    out = []
    for li in range(nlev):
        ph = prof_levels[li]
        mv_ms = ph["rotate"] + ph["copy"]
        # the product is bound by the larger of its HBM and MFMA times
        floor_ms = max(pb[li] / (PEAK_HBM_GBS * 1e9), pf[li] / (PEAK_FP64_MFMA_TFLOPS * 1e12)) * 1e3
        out.append({"level_from_root": nlev - 1 - li,
                    "phase_ms": {k: ph[k] for k in phases},
                    "move_bytes": move[li],
                    "move_gbs": move[li] / (mv_ms * 1e-3) / 1e9 if mv_ms > 0 else 0.0,
                    "product_bytes": pb[li], "product_flops": pf[li],
                    "product_floor_ms": floor_ms})
    return out


def example1(L, torch, sizes=(8192, 16384, 32768), tol=1e-10, b=1024):
    """Example 1 on one GPU: C = A B with A random (N(0,1)) and B Example 0's
    Cauchy-like matrix B_ij = u_i v_j / (d_i - w_j) given by its generators.
      plain           generated-tile product, B never stored
      lowrank_block   SRRSC product on contiguous b x b blocks (block layout)
      lowrank_cyclic  the same on the block-cyclic storage order (block 64 over
                      n/b process rows), whose blocks lose the low rank
      dgemm           the library GEMM (torch.matmul) on the stored B
    Errors are against the library GEMM; the low-rank bound is
    tol * max_i sum_k |A_ik| (each U entry within tol)."""
    from paper_2008_01990_amd import workloads as W
    out = {}
    f64 = torch.float64
    for n in sizes:
        u, v, d, w = W.example_cauchy(n, seed=7)
        ud, vd, dd, wd = (torch.tensor(x, device="cuda") for x in (u, v, d, w))
        g = torch.Generator(device="cuda")
        g.manual_seed(n)
        At = torch.randn(n, n, generator=g, dtype=f64, device="cuda")   # column-major A
        BmT = (vd[:, None] * ud[None, :]) / (dd[None, :] - wd[:, None])  # column-major B
        Cref = torch.empty(n, n, dtype=f64, device="cuda")
        C = torch.empty(n, n, dtype=f64, device="cuda")
        reps = 2
        t_gemm = _events(lambda: torch.matmul(BmT, At, out=Cref), reps, torch)
        del BmT
        flops = 2.0 * n ** 3
        rowsum = float(At.abs().sum(dim=0).max())
        scale = float(Cref.abs().max())
        rec = {"dgemm": {"seconds": t_gemm, "tflops": flops / t_gemm / 1e12}}
        t = _events(lambda: L.merge_update(At, n, n, dd, None, wd, ud, vd, out=C), reps, torch)
        rec["plain"] = {"seconds": t, "tflops": flops / t / 1e12,
                        "max_rel_err_vs_dgemm": float((C - Cref).abs().max()) / scale}
        for name, perm in (("lowrank_block", None),
                           ("lowrank_cyclic", W.block_cyclic_order(n, n // b, 64))):
            if perm is None:
                A_, gens = At, (dd, wd, ud, vd)
            else:
                pt = torch.tensor(perm, device="cuda")
                A_ = At.index_select(0, pt)
                gens = tuple(x.index_select(0, pt) for x in (dd, wd, ud, vd))
            gd, gw, gu, gv = gens
            t = _events(lambda: L.merge_update(A_, n, n, gd, None, gw, gu, gv, lr_tol=tol,
                                               lr_block=b, out=C), reps, torch)
            ranks = L.merge_lowrank_ranks(gd, None, gw, gu, gv, tol, b)
            bs = [min(b, n - I * b) for I in range(ranks.shape[0])]
            ex = 0.0
            for I in range(ranks.shape[0]):
                ex += bs[I] ** 2
                for J in range(ranks.shape[0]):
                    if I != J:
                        r = bs[J] if ranks[I, J] == -2 else ranks[I, J]
                        ex += r * (bs[I] + bs[J])
            err = 0.0
            for c0 in range(0, n, 2048):
                rows = slice(c0, min(n, c0 + 2048))
                ref = Cref[rows] if perm is None else Cref.index_select(0, pt[rows])
                err = max(err, float((C[rows] - ref).abs().max()))
            off = ranks[ranks >= 0]
            rec[name] = {"seconds": t, "plain_equivalent_tflops": flops / t / 1e12,
                         "executed_flops": 2.0 * n * ex,
                         "ranks_mean": float(off.mean()) if off.size else None,
                         "ranks_max": int(off.max()) if off.size else None,
                         "blocks_dense": int((ranks == -2).sum()),
                         "max_abs_err_vs_dgemm": err,
                         "err_over_bound": err / (tol * rowsum)}
            del A_
        rec["speedup_plain_vs_dgemm"] = t_gemm / rec["plain"]["seconds"]
        rec["speedup_lowrank_block_vs_dgemm"] = t_gemm / rec["lowrank_block"]["seconds"]
        rec["speedup_lowrank_cyclic_vs_dgemm"] = t_gemm / rec["lowrank_cyclic"]["seconds"]
        out[f"n{n}"] = rec
        del At, Cref, C
        torch.cuda.empty_cache()
    return out


def table_rank(L, torch, n=16384, nprocs=4, tol=1e-12):
    """Table "rank": SRRSC ranks of B(2,1), B(3,1), B(4,1) of Example 1's B
    (n = 16384, 4096 x 4096 local blocks on 4 x 4 processes) for block-cyclic
    block sizes 64, 128, 256 and the block layout (4096)."""
    from paper_2008_01990_amd import workloads as W
    u, v, d, w = W.example_cauchy(n, seed=0)
    b = n // nprocs
    out = {"tol": tol, "n": n, "block": b, "printed": {"64": [1260, 892, 1252],
                                                       "128": [711, 445, 699],
                                                       "256": [401, 221, 390],
                                                       "4096": [34, 11, 9]}}
    for nb in (64, 128, 256, 4096):
        perm = W.block_cyclic_order(n, nprocs, nb)
        gens = [torch.tensor(x[perm], device="cuda") for x in (d, w, u, v)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ranks = L.merge_lowrank_ranks(gens[0], None, gens[1], gens[2], gens[3], tol, b,
                                      rank_cap=b)
        out[str(nb)] = {"ranks": [int(x) for x in ranks[1:, 0]],
                        "seconds": time.perf_counter() - t0}
    return out


BATCH_LEAF = 16   # leaf size of the batched configuration (8 / 12 / 16 / 32 measured)


def batched_config(L, torch):
    """Batched configuration: 256 problems, sizes log-uniform in [64, 4096],
    d, e ~ U(-1, 1), seed 3, leaf 16; default tile rule, bucket-tuned and
    batch-measured tiles, all replayed as graphs."""
    from paper_2008_01990_amd import workloads as W
    res = {}
    probs = W.batched_problems(256, 64, 4096, seed=3)
    sizes = [len(p[0]) for p in probs]
    B = L.BatchedSolver(sizes, leaf=BATCH_LEAF)
    B.load_inputs(probs)

    def step(graph):
        B.restore()  # the solve overwrites d; each timed step starts from the inputs
        B.solve(graph=graph)
    tg_rule = _time(lambda: step(True), 5, torch)
    t0 = time.perf_counter()
    table = L.autotune(4096)
    t_tune = time.perf_counter() - t0
    del B
    B = L.BatchedSolver(sizes, leaf=BATCH_LEAF)
    B.load_inputs(probs)
    tg_bucket = _time(lambda: step(True), 5, torch)
    L.autotune(0)
    # measured on this batch: every level's product timed under every variant
    del B
    B = L.BatchedSolver(sizes, leaf=BATCH_LEAF)
    B.load_inputs(probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    levels = B.autotune()
    t_meas = time.perf_counter() - t0
    tg = _time(lambda: step(True), 5, torch)
    te = _time(lambda: step(False), 5, torch)
    # One eager solve with phase events, for the bytes-moved accounting.
    L.profile_enable(True)
    B.restore()
    B.solve(graph=False)
    prof = L.profile_read()
    L.profile_enable(False)
    stats = L.last_stats()
    lv = level_traffic(stats, prof, L.PHASES)
    ph = {k: sum(x["phase_ms"][k] for x in lv) for k in L.PHASES}
    move_b = sum(x["move_bytes"] for x in lv)
    prod_b = sum(x["product_bytes"] for x in lv)
    prod_f = sum(x["product_flops"] for x in lv)
    prod_floor = sum(x["product_floor_ms"] for x in lv)
    # leaves: each writes its nb x nb block; the tree halves a problem until
    # its blocks hold at most `leaf` rows, so sum nb^2 ~ n * (n / 2^depth)
    leaf_b = 0.0
    for n in sizes:
        nb = float(n)
        while nb > BATCH_LEAF:
            nb /= 2.0
        leaf_b += 8.0 * n * nb
    total_b = move_b + prod_b + leaf_b
    move_ms = ph["rotate"] + ph["copy"]
    other_ms = te * 1e3 - sum(ph.values())
    res["batched_256_loguniform_64_4096"] = {
        "seconds_graph": tg, "seconds_eager": te, "seconds_graph_default_tiles": tg_rule,
        "seconds_graph_bucket_tuned": tg_bucket, "bucket_autotune_seconds": t_tune,
        "bucket_variant_by_size": {f"<={1 << b}": v for b, v in enumerate(table) if 6 <= b <= 12},
        "measured_autotune_seconds": t_meas, "measured_variant_by_level": levels,
        "problems": len(sizes), "sum_n": int(sum(sizes)), "leaf": BATCH_LEAF,
        "status_ok": all(v == 0 for v in B.status()),
        # whole batch against HBM: algorithmic bytes (merge_traffic per merge,
        # plus the leaf blocks) over the graph-replay time
        "roofline": {"bound": "hbm", "achieved": total_b / tg / 1e9, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": total_b / tg / 1e9 / PEAK_HBM_GBS,
                     "traffic": None, "bytes": total_b,
                     "floor_ms": total_b / (PEAK_HBM_GBS * 1e9) * 1e3},
        "phases": {
            "data_movement": {"ms": move_ms, "bytes": move_b,
                              "gbs": move_b / (move_ms * 1e-3) / 1e9 if move_ms > 0 else 0.0,
                              "frac": move_b / (move_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
                              if move_ms > 0 else 0.0,
                              "rotate_gather_ms": ph["rotate"], "copy_ms": ph["copy"]},
            "product": {"ms": ph["product"], "bytes": prod_b, "flops": prod_f,
                        "floor_ms": prod_floor,
                        "frac": prod_floor / ph["product"] if ph["product"] > 0 else 0.0},
            "secular_ms": ph["secular"], "deflate_ms": ph["deflate"],
            "assemble_ms": ph["assemble"],
            "leaves_and_setup": {"ms": other_ms, "leaf_bytes": leaf_b}},
        "levels": lv}
    del B
    L.autotune(0)
    torch.cuda.empty_cache()
    return res


def adjoint_config(L, torch):
    """Adjoint configuration: n = 4096, loss sum w lam + sum c (u^T q)^2;
    forward, rank-one and general backward."""
    from paper_2008_01990_amd import workloads as W
    res = {}
    P = W.adjoint_problem(n=4096, seed=4, n_coords=32)
    n = 4096
    dd, ee = torch.tensor(P["d"], device="cuda"), torch.tensor(P["e"], device="cuda")
    w, c, u = (torch.tensor(P[k], device="cuda") for k in ("w", "c", "u"))
    s = L.Solver(n, leaf=32)
    lam = dd.clone()
    Qb = torch.empty(n, n, dtype=torch.float64, device="cuda")

    def fwd():
        lam.copy_(dd)
        s.solve_into(lam, ee, Qb)
    tf = _time(fwd, 5, torch)
    Q = Qb.t()
    a = u @ Q
    g = 2 * c * a
    tb1 = _time(lambda: L.backward_rank1(lam, Qb, u, g, lam_bar=w), 5, torch)
    Qbar_cm = torch.outer(u, g).t().contiguous()
    tbg = _time(lambda: L.backward(lam, Qb, w, Qbar_cm), 5, torch)
    res["adjoint_n4096"] = {"forward_seconds": tf, "backward_rank1_seconds": tb1,
                            "backward_general_seconds": tbg,
                            "backward_general_tflops": 4.0 * n ** 3 / tbg / 1e12,
                            "backward_rank1_tflops": 2.0 * n ** 3 / tb1 / 1e12}
    return res


def extra_configs(L, torch):
    """Secondary configurations, each timed on the GPU after a warm-up."""
    import numpy as np
    from paper_2008_01990_amd import workloads as W
    res = {}
    # n=1024 1-2-1 Toeplitz, leaf 32 (latency-bound correctness config)
    d0, e0 = W.toeplitz(1024)
    d_in, e = torch.tensor(d0, device="cuda"), torch.tensor(e0, device="cuda")
    d = torch.empty_like(d_in)
    Qb = torch.empty(1024, 1024, dtype=torch.float64, device="cuda")
    s = L.Solver(1024, leaf=32)

    def c0():
        d.copy_(d_in)
        s.solve_into(d, e, Qb)
    t = _time(c0, 20, torch)
    res["toeplitz_n1024_leaf32"] = {"seconds": t, "accuracy": gpu_accuracy(d_in, e, d, Qb, "toeplitz")}
    # n=16384 Toeplitz, leaf 64: plain vs low rank at 1e-10
    n = 16384
    d0, e0 = W.toeplitz(n)
    d_in, e = torch.tensor(d0, device="cuda"), torch.tensor(e0, device="cuda")
    d = torch.empty_like(d_in)
    Qb = torch.empty(n, n, dtype=torch.float64, device="cuda")
    r = {}
    for name, kw in (("plain", {}), ("lowrank", dict(lr_tol=1e-10, lr_block=256, lr_min_k=2048))):
        s = L.Solver(n, leaf=64, **kw)

        def c1():
            d.copy_(d_in)
            s.solve_into(d, e, Qb)
        t = _time(c1, 3, torch)
        r[name] = {"seconds": t, "accuracy": gpu_accuracy(d_in, e, d, Qb, "toeplitz")}
        del s
    r["lowrank_speedup"] = r["plain"]["seconds"] / r["lowrank"]["seconds"]
    res["toeplitz_n16384_leaf64"] = r
    del Qb
    torch.cuda.empty_cache()
    res.update(batched_config(L, torch))
    # the paper's own sizes (Examples 2-3): n = 30000 Clement, Hermite-type,
    # 1-2-1 Toeplitz and SHT (m = n), plain and low-rank; residual on all
    # columns, orthogonality on 1024 sampled columns against all.
    n = 30000
    Qb = torch.empty(n, n, dtype=torch.float64, device="cuda")
    paper = {}
    for fam, gen in (("clement", W.clement), ("hermite", W.hermite),
                     ("toeplitz", W.toeplitz), ("sht", W.sht)):
        d0, e0 = gen(n)
        d_in, e = torch.tensor(d0, device="cuda"), torch.tensor(e0, device="cuda")
        d = torch.empty_like(d_in)
        rec = {}
        for name, kw in (("plain", {}), ("lowrank", dict(lr_tol=1e-10, lr_block=256,
                                                          lr_min_k=2048))):
            s = L.Solver(n, leaf=64, **kw)

            def c5():
                d.copy_(d_in)
                s.solve_into(d, e, Qb)
            t = _time(c5, 1, torch)
            Q = Qb.t()
            tn = float(d.abs().max())
            TQ = d_in[:, None] * Q
            TQ[:-1] += e[:, None] * Q[1:]
            TQ[1:] += e[:, None] * Q[:-1]
            resid = float(torch.linalg.norm(TQ - Q * d[None, :])) / (n * tn)
            del TQ
            idx = torch.randperm(n, device="cuda")[:1024]
            G = Qb[idx] @ Qb.t()
            G[torch.arange(1024, device="cuda"), idx] -= 1.0
            rec[name] = {"seconds": t, "residual": resid,
                         "orthogonality_sampled": float(G.abs().max()),
                         "status": s.status()}
            del G, s
        rec["lowrank_speedup"] = rec["plain"]["seconds"] / rec["lowrank"]["seconds"]
        paper[fam] = rec
    res["paper_sizes_n30000"] = paper
    del Qb
    torch.cuda.empty_cache()
    res["example1"] = example1(L, torch)
    res["table_rank"] = table_rank(L, torch)
    res.update(adjoint_config(L, torch))
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU row-sharded merge is a design, not a measured path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2008_01990_amd import dcstedc as L

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # A plain copy of known size: 2^27 doubles (1 GiB) read and written once.
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}), flush=True)
        return
    if args.batched_only or args.adjoint_only:
        out = batched_config(L, torch) if args.batched_only else adjoint_config(L, torch)
        print(json.dumps(out), flush=True)
        return
    n = args.n
    d0, e0 = inputs(args.family, n)
    d_in = torch.tensor(d0, device="cuda")
    e = torch.tensor(e0, device="cuda")
    d = torch.empty_like(d_in)
    Qbuf = torch.empty(n, n, dtype=torch.float64, device="cuda")
    if args.lowrank_only:
        lr = L.Solver(n, leaf=args.leaf, gemm_tile=args.gemm_tile, lr_tol=args.lowrank_tol,
                      lr_block=args.lowrank_block, lr_min_k=args.lowrank_min_k)

        def lr_only():
            d.copy_(d_in)
            lr.solve_into(d, e, Qbuf)
        for _ in range(args.warmup):
            lr_only()
        t = _time(lr_only, args.steps, torch) if args.steps > 0 else 0.0
        print(json.dumps({"lowrank_seconds": t, "tol": args.lowrank_tol,
                          "block": args.lowrank_block, "min_k": args.lowrank_min_k,
                          "status": lr.status()}), flush=True)
        return
    solver = L.Solver(n, leaf=args.leaf, gemm_tile=args.gemm_tile)

    def step():
        d.copy_(d_in)
        solver.solve_into(d, e, Qbuf)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if solver.status() != 0:
        raise RuntimeError(f"device status {solver.status()}")

    L.profile_enable(True)
    prof = []
    marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in marks:
        a.record()
        step()
        b.record()
        prof.append(L.profile_read())          # waits on this step's events
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    step_s = sorted(a.elapsed_time(b) / 1e3 for a, b in marks)
    stats = L.last_stats()

    # Per-level merge-product rates (algorithmic flops of the launch over its
    # event-timed duration, averaged over the timed steps).
    nlev = len(prof[0])
    flops_lvl = [0.0] * nlev
    for r in stats:
        flops_lvl[nlev - 1 - r["level"]] += r["flops"]
    levels = []
    for li in range(nlev):
        t_ms = sum(p[li]["product"] for p in prof) / len(prof)
        phase = {k: sum(p[li][k] for p in prof) / len(prof) for k in L.PHASES}
        levels.append({"level_from_root": nlev - 1 - li, "product_ms": t_ms,
                       "product_tflops": flops_lvl[li] / (t_ms * 1e-3) / 1e12 if t_ms > 0 else 0,
                       "phase_ms": phase})
    top = levels[-1]
    achieved = top["product_tflops"]
    total_prod_ms = sum(l["product_ms"] for l in levels)
    total_flops = sum(flops_lvl)
    sec_ms = sum(l["phase_ms"]["secular"] for l in levels)
    Ks = [r["K"] for r in stats]
    sec_bytes = sum(48.0 * k for k in Ks)
    # at least one reciprocal per (row, column) pair in each of the three
    # kernels (one secular evaluation, the Loewner products, the scales)
    sec_rcp = sum(3.0 * k * k for k in Ks)

    out = {
        "metric": METRIC,
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.family}_n{n}_leaf{args.leaf}_plain", "n": n,
                   "family": args.family, "leaf": args.leaf, "path": "plain"},
        "roofline": {"bound": "mfma", "achieved": achieved,
                     "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_MFMA_TFLOPS,
                     "traffic": measured_traffic(f"{args.family}_n{n}_leaf{args.leaf}_plain"),
                     "kernel": "k_cauchy_gemm_reg (root-level merge product)",
                     "flops_per_launch": flops_lvl[-1],
                     "launch_ms": top["product_ms"]},
        "merge_product": {"total_ms": total_prod_ms, "total_flops": total_flops,
                          "tflops": total_flops / (total_prod_ms * 1e-3) / 1e12,
                          "frac_peak": total_flops / (total_prod_ms * 1e-3) / 1e12
                          / PEAK_FP64_MFMA_TFLOPS},
        "step_seconds": {"best": step_s[0], "median": step_s[len(step_s) // 2],
                         "mean": ms / 1e3},
        "secular_phase": {"total_ms": sec_ms,
                          "hbm_gbs_algorithmic": sec_bytes / (sec_ms * 1e-3) / 1e9
                          if sec_ms > 0 else 0.0,
                          "reciprocals_min": sec_rcp,
                          "reciprocals_per_s_min": sec_rcp / (sec_ms * 1e-3)
                          if sec_ms > 0 else 0.0,
                          "fp64_valu_fma_per_s_peak": PEAK_FP64_MFMA_TFLOPS * 1e12 / 2},
        "levels": levels,
        "merges_top": [dict(m=r["m"], K=r["K"], nrot=r["nrot"],
                            secular_iters_mean=r["sec_iters_sum"] / max(r["K"], 1),
                            secular_iters_max=r["sec_iters_max"]) for r in stats
                       if r["level"] <= 1],
    }
    # HBM-bound phases of the root merge (rotations, gather and deflated
    # copy): the algorithmic bytes of merge_traffic over their event times.
    root = [r for r in stats if r["level"] == 0][0]
    mv_b = merge_traffic(root)[0]
    mv_ms = top["phase_ms"]["rotate"] + top["phase_ms"]["copy"]
    out["root_hbm_phases"] = {
        "data_movement": {"ms": mv_ms, "rotate_gather_ms": top["phase_ms"]["rotate"],
                          "copy_ms": top["phase_ms"]["copy"], "bytes": mv_b,
                          "gbs": mv_b / (mv_ms * 1e-3) / 1e9 if mv_ms > 0 else 0.0},
        "peak_gbs": PEAK_HBM_GBS}
    if not args.no_accuracy:
        out["accuracy"] = gpu_accuracy(d_in, e, d, Qbuf, args.family)
    if args.lowrank_tol > 0.0:
        lr = L.Solver(n, leaf=args.leaf, gemm_tile=args.gemm_tile, lr_tol=args.lowrank_tol,
                      lr_block=args.lowrank_block, lr_min_k=args.lowrank_min_k)
        del solver
        torch.cuda.empty_cache()

        def lr_step():
            d.copy_(d_in)
            lr.solve_into(d, e, Qbuf)

        for _ in range(args.warmup):
            lr_step()
        L.profile_enable(True)
        lprof, lrprof = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lr_step()
            lprof.append(L.profile_read())
            lrprof.append(L.profile_read_lowrank())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.profile_enable(False)
        lms = (t1 - t0) * 1e3 / args.steps
        lstats = L.last_stats()
        lr_top_ms = sum(p[-1]["product"] for p in lprof) / len(lprof)
        lnlev = len(lprof[0])
        lr_levels = [{"level_from_root": lnlev - 1 - li,
                      "phase_ms": {k: sum(p[li][k] for p in lprof) / len(lprof)
                                   for k in L.PHASES}} for li in range(lnlev)]
        out["lowrank"] = {
            "tol": args.lowrank_tol, "block": args.lowrank_block,
            "min_k": args.lowrank_min_k, "seconds": lms / 1e3,
            "levels": lr_levels,
            "speedup_vs_plain": ms / lms,
            "root_product_ms": lr_top_ms,
            "root_product_speedup_vs_plain": top["product_ms"] / lr_top_ms,
            "merges": [dict(m=r["m"], K=r["K"], path=r["path"], flops=r["flops"],
                            secular_iters_mean=r["sec_iters_sum"] / max(r["K"], 1),
                            secular_iters_max=r["sec_iters_max"],
                            flops_skeleton=r["lr_flops_skeleton"],
                            flops_fused=r["lr_flops_fused"],
                            blocks=r["lr_blocks"], dense=r["lr_dense"], rank_max=r["lr_rank_max"],
                            rank_mean=r["lr_rank_sum"] / max(r["lr_blocks"] - r["lr_dense"], 1))
                       for r in lstats if r["path"] == 1],
        }
        # Roofline of the two MFMA launches of the low-rank product, summed
        # over the levels that take it: executed flops (the skeleton columns
        # W = A(:, I) U(I, T); the diagonal blocks plus the interpolation
        # rows, 2 m (b^2 + b r) per block column) over their HIP-event times.
        fl = {"skeleton": sum(r["lr_flops_skeleton"] for r in lstats if r["path"] == 1),
              "fused": sum(r["lr_flops_fused"] for r in lstats if r["path"] == 1)}
        stages = {}
        for st in ("compress", "skeleton", "fused"):
            t_ms = sum(sum(lv[st] for lv in p) for p in lrprof) / len(lrprof)
            rec = {"ms": t_ms}
            if st in fl:
                tf = fl[st] / (t_ms * 1e-3) / 1e12 if t_ms > 0 else 0.0
                rec.update({"executed_flops": fl[st], "tflops": tf,
                            "frac": tf / PEAK_FP64_MFMA_TFLOPS, "bound": "mfma",
                            "peak": PEAK_FP64_MFMA_TFLOPS})
            stages[st] = rec
        out["lowrank"]["stages"] = stages
        if not args.no_accuracy:
            out["lowrank"]["accuracy"] = gpu_accuracy(d_in, e, d, Qbuf, args.family)
        if not args.no_extra:
            # block size and switch left to the library, tuned on this
            # problem by whole solves (then the tuning is cleared again)
            lt = L.Solver(n, leaf=args.leaf, lr_tol=args.lowrank_tol)
            d.copy_(d_in)
            t0 = time.perf_counter()
            lt.autotune_on(d, e, Qbuf)
            torch.cuda.synchronize()
            t_tune = time.perf_counter() - t0
            pair = lt.tuned_lowrank()

            def lt_step():
                d.copy_(d_in)
                lt.solve_into(d, e, Qbuf)

            t_lt = _time(lt_step, args.steps, torch)
            out["lowrank"]["tuned"] = {"block": pair[0], "min_k": pair[1], "seconds": t_lt,
                                       "tuning_seconds": t_tune}
            L.autotune(0)
    del Qbuf
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["extra_configs"] = extra_configs(L, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.family, n, args.cpu_n, args.leaf)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
