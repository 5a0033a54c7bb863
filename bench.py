#!/usr/bin/env python3
"""Benchmark of the FAS multigrid Poisson solve on one MI355X.

One step = one complete solve of the uniform 256^3 octree workload (8^3-cell
boxes, 37,449 boxes, 16,777,216 unknowns, Dirichlet values from two seeded
Gaussians): one FMG cycle, then V(2,2) cycles until the max-norm of the
composite residual has dropped by 1e-10.  Inputs are resident in HBM before
the timed region starts.

Prints one JSON line: throughput in unknowns/s, the roofline of the dominant
kernel (the finest-level red-black half sweep) measured with HIP events on
the solve's stream during the last timed step, and the FP64 CPU oracle timed on
the host cores on the same workload.  Further objects: the mixed-precision solve, the
256-tree batch, the adaptive octree (FP64 vs mixed) and the adjoint.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("afmg_kernels.hip", "afmg_kernels.h", "afmg_internal.h"):
        with open(os.path.join(ROOT, "paper_1701_04329_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel_tag):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if it is missing or was taken on
    other kernel sources."""
    path = os.path.join(PROFILES, f"{kernel_tag}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel source hash:\s*`?([0-9a-f]{16})", txt)
    m_bytes = re.search(r"HBM bytes per launch \(calibrated\):\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def make_workload(name):
    from paper_1701_04329_amd import workloads as W
    if name == "c2":
        return W.config2(), dict(cycle="FMG", tol=1e-10)
    if name == "c1":
        return W.config1(), dict(cycle="V", tol=1e-10)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, solve_kw):
    """Time the oracle on the host cores: the same workload and stop rule.
    Returns the baseline record and the oracle's solution (leaf order)."""
    from oracle import oracle as O
    t = O.Tree(w.dim, w.N, w.level, w.idx)
    kw = dict(solve_kw)
    t0 = time.perf_counter()
    u, st = t.solve(w.rho, w.bc, **kw)
    dt = time.perf_counter() - t0
    return u, {
        "value": w.n_unknowns / dt,
        "unit": "unknowns/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": f"one full solve of the benchmark workload ({w.n_unknowns} unknowns, "
                  f"{'FMG + ' if kw.get('cycle') == 'FMG' else ''}{st['cycles']} V-cycles to "
                  f"{kw.get('tol', 1e-10):g}), FP64, OpenMP over boxes, {dt:.1f} s",
    }


def batch_bench(args, A, torch, dev, stream):
    """The batch workload: independent trees of 64-8192 boxes, D alternating
    2/3, 1-3 Gaussian sources, zero Dirichlet values.  One step solves every
    tree (FMG, then V-cycles until each tree's own residual dropped by 1e-10):
    one batch per dimension, the two solved concurrently, each on its own
    stream driven by its own host thread; the sequential time (one batch
    after the other on one stream) is reported beside it."""
    from oracle import oracle as O
    from paper_1701_04329_amd import workloads as W

    workers = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    ws = W.config4(args.batch_trees, workers=workers)
    gen_s = time.perf_counter() - t0
    groups = []
    for dim in (2, 3):
        sub = [w for w in ws if w.dim == dim]
        if not sub:
            continue
        trees = [A.Tree(w.dim, w.level, w.idx) for w in sub]
        b = A.Batch(trees)
        rho = b.concat([t.leaf_to_boxes(torch.tensor(w.rho, device=dev)) for t, w in zip(trees, sub)])
        u = torch.zeros_like(rho)
        groups.append(dict(dim=dim, sub=sub, trees=trees, b=b, rho=rho, u=u, work={}))
    n_unk = sum(g["b"].n_unknowns for g in groups)

    import concurrent.futures as cf
    for g in groups:
        g["stream"] = torch.cuda.Stream(device=dev)  # default priority
    pool = cf.ThreadPoolExecutor(max_workers=max(1, len(groups)))

    def solve_group(g, precision, st):
        if precision not in g["work"]:
            nb = g["b"].workspace_bytes(A.make_opts(precision=precision))
            g["work"][precision] = torch.empty(nb, dtype=torch.uint8, device=dev)
        _, sts = A.solve_batch(g["b"], g["rho"], None, g["u"], cycle="FMG", tol=1e-10, precision=precision,
                               workspace=g["work"][precision], stream=st, use_guess=False, graph=True)
        return sts

    def step(precision, schedule="concurrent", only=None):
        """one step: every tree solved.  sequential: the batches one after the
        other on one stream; concurrent: each batch on its own stream, driven
        by its own host thread (the library calls release the GIL)"""
        gs = [g for g in groups if only is None or g["dim"] == only]
        if schedule == "sequential":
            return [solve_group(g, precision, stream) for g in gs]
        torch.cuda.synchronize()
        futs = [pool.submit(solve_group, g, precision, g["stream"]) for g in gs]
        return [f.result() for f in futs]

    def timed(precision, schedule="concurrent", only=None):
        for _ in range(args.warmup):
            step(precision, schedule, only)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sts = step(precision, schedule, only)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, sts

    untuned = None
    if not args.no_autotune:
        untuned = {f"{p}_ms_per_step": timed(p)[0] for p in ("fp64", "mixed")}
        t0 = time.perf_counter()
        for g in groups:
            g["b"].autotune(dev, stream)
        untuned["autotune_s"] = round(time.perf_counter() - t0, 3)

    res = {}
    sols = {}
    for precision in ("fp64", "mixed"):
        ms, sts = timed(precision)
        cyc = [s["cycles"] for st in sts for s in st]
        res[precision] = {"value": n_unk / (ms * 1e-3), "unit": "unknowns/s", "ms_per_step": ms,
                          "cycles_min": int(min(cyc)), "cycles_max": int(max(cyc)),
                          "cycles_median": float(np.median(cyc)),
                          "all_converged": bool(all(s["status"] == 0 for st in sts for s in st)),
                          "sequential_ms_per_step": timed(precision, "sequential")[0]}
        for g in groups:
            res[precision][f"{g['dim']}d_alone_ms_per_step"] = timed(precision, "sequential", g["dim"])[0]
        sols[precision] = [[t.boxes_to_leaf(x).cpu().numpy() for t, x in zip(g["trees"], g["b"].split(g["u"]))]
                           for g in groups]
    pool.shutdown()
    # per-tree error of the mixed solution against the FP64 one
    errs = [float(np.linalg.norm(m - f) / np.linalg.norm(f))
            for gm, gf in zip(sols["mixed"], sols["fp64"]) for m, f in zip(gm, gf)]
    # the same trees solved one at a time (one pass, mixed, graph replay)
    unbatched_ms = None
    if not args.skip_unbatched:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g in groups:
            for t, w in zip(g["trees"], g["sub"]):
                r = t.leaf_to_boxes(torch.tensor(w.rho, device=dev))
                A.solve(t, r, None, None, cycle="FMG", tol=1e-10, precision="mixed", stream=stream, graph=True)
        torch.cuda.synchronize()
        unbatched_ms = (time.perf_counter() - t0) * 1e3
    # oracle check of the smallest tree of each dimension
    oracle = {}
    for gi, g in enumerate(groups):
        q = int(np.argmin([w.n_unknowns for w in g["sub"]]))
        w = g["sub"][q]
        uo, _ = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="FMG", tol=1e-10)
        nrm = np.linalg.norm(uo)
        oracle[w.name] = {"fp64": float(np.linalg.norm(sols["fp64"][gi][q] - uo) / nrm),
                          "mixed": float(np.linalg.norm(sols["mixed"][gi][q] - uo) / nrm)}
    return {
        "workload": f"c4_batch_{args.batch_trees}_trees",
        "trees": len(ws),
        "unknowns": int(n_unk),
        "boxes": int(sum(g["b"].n_boxes for g in groups)),
        "per_dim": {f"{g['dim']}d": {"trees": len(g["sub"]), "unknowns": int(g["b"].n_unknowns),
                                     "boxes": int(g["b"].n_boxes), "lmax": g["b"].lmax} for g in groups},
        "fp64": res["fp64"],
        "mixed": res["mixed"],
        "mixed_vs_fp64_rel_l2_max": max(errs),
        "mixed_vs_fp64_rel_l2_median": float(np.median(errs)),
        "unbatched_mixed_ms": unbatched_ms,
        "untuned": untuned,
        "oracle_rel_l2_smallest_trees": oracle,
        "generation_s": round(gen_s, 1),
        "note": "one step = every tree solved (FMG, then V(2,2) until its own residual dropped by 1e-10); "
                "one batch per dimension, each on its own stream driven by its own host thread, cycles "
                "replayed from recorded HIP graphs; sequential = the two batches one after the other",
    }


def timed_loop(args, torch, fn):
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / args.steps, r


def adaptive_bench(args, A, torch, dev, stream):
    """The adaptive octree workload: about 2.3e7 unknowns on leaves of levels
    3-8 around four Gaussians, FMG then V(2,2) to a 1e-10 residual reduction,
    FP64 against FP32 V-cycles inside FP64 refinement; both against the
    oracle's FP64 solve of the same problem."""
    from oracle import oracle as O
    from paper_1701_04329_amd import workloads as W

    t0 = time.perf_counter()
    w = W.config3()
    gen_s = time.perf_counter() - t0
    tree = A.Tree(w.dim, w.level, w.idx)
    if not args.no_autotune:
        tree.autotune(dev, stream)
    rho = tree.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = tree.bc_rows(torch.tensor(w.bc, device=dev))
    u = torch.zeros_like(rho)
    work = torch.empty(tree.workspace_bytes(A.make_opts(precision="mixed")), dtype=torch.uint8, device=dev)
    out = {"workload": w.name, "unknowns": int(w.n_unknowns), "leaves": int(w.n_leaves), "boxes": int(tree.n_boxes),
           "leaf_levels": sorted(set(int(x) for x in w.level)), "generation_s": round(gen_s, 1)}
    sols = {}
    for precision in ("fp64", "mixed"):
        ms, (_, st) = timed_loop(args, torch, lambda: A.solve(
            tree, rho, bc, u, cycle="FMG", tol=1e-10, precision=precision, workspace=work, stream=stream,
            use_guess=False, graph=True))
        sols[precision] = tree.boxes_to_leaf(u).cpu().numpy()
        out[precision] = {"value": w.n_unknowns / (ms * 1e-3), "unit": "unknowns/s", "ms_per_step": ms,
                          "cycles": st["cycles"], "final_residual_ratio": st["r_max"] / st["r0_max"]}
    nrm = np.linalg.norm(sols["fp64"])
    out["mixed"]["rel_l2_vs_gpu_fp64"] = float(np.linalg.norm(sols["mixed"] - sols["fp64"]) / nrm)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        uo, so = O.Tree(w.dim, w.N, w.level, w.idx).solve(w.rho, w.bc, cycle="FMG", tol=1e-10)
        dt = time.perf_counter() - t0
        no = np.linalg.norm(uo)
        out["oracle"] = {"value": w.n_unknowns / dt, "unit": "unknowns/s", "cores": O.num_threads(),
                         "seconds": round(dt, 2), "cycles": so["cycles"]}
        out["fp64"]["rel_l2_vs_oracle"] = float(np.linalg.norm(sols["fp64"] - uo) / no)
        out["mixed"]["rel_l2_vs_oracle"] = float(np.linalg.norm(sols["mixed"] - uo) / no)
    return out


def adjoint_bench(args, A, torch, dev, stream):
    """The adjoint workload: 3D adaptive octree with about 4e6 unknowns, loss
    = sum over leaf cells of (u - u_t)^2.  Forward: FP64 FMG + V-cycles to
    1e-10; backward: afmg_adjoint (BiCGSTAB on L^T preconditioned by one
    V-cycle, to 1e-10).  Checked against central finite differences along
    seeded random directions of rho and of the Dirichlet values (exact for
    this quadratic loss up to the solve tolerance)."""
    from paper_1701_04329_amd import workloads as W

    t0 = time.perf_counter()
    w, u_t = W.config5()
    gen_s = time.perf_counter() - t0
    tree = A.Tree(w.dim, w.level, w.idx)
    if not args.no_autotune:
        tree.autotune(dev, stream)
    rho = tree.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = tree.bc_rows(torch.tensor(w.bc, device=dev))
    ut = tree.leaf_to_boxes(torch.tensor(u_t, device=dev))
    leaf = torch.zeros(tree.n_boxes, dtype=torch.bool, device=dev)
    leaf[torch.as_tensor(tree.leaf_boxes, device=dev).long()] = True
    work = torch.empty(max(tree.workspace_bytes(), tree.adjoint_workspace_bytes()), dtype=torch.uint8, device=dev)

    u_buf = torch.empty_like(rho)

    def loss_of(r, b, tol=1e-10):
        u, st = A.solve(tree, r, b, u_buf, cycle="FMG", tol=tol, workspace=work, stream=stream, use_guess=False,
                        graph=True)
        return float(((u - ut)[leaf] ** 2).sum()), u, st

    fwd_ms, (loss, u, st_f) = timed_loop(args, torch, lambda: loss_of(rho, bc))
    u_bar = torch.where(leaf[:, None], 2.0 * (u - ut), torch.zeros_like(u))
    bwd_ms, (rho_bar, bc_bar, st_b) = timed_loop(args, torch, lambda: A.adjoint(
        tree, u_bar, tol=1e-10, max_cycles=200, workspace=work, stream=stream))
    gen = torch.Generator(device="cpu").manual_seed(5002)
    checks = []
    t0 = time.perf_counter()
    for kind in ("rho", "bc", "rho"):
        if kind == "rho":
            d = torch.randn(rho.shape, generator=gen, dtype=torch.float64).to(dev) * leaf[:, None]
            d *= float(rho.abs().max()) / float(d.abs().max())
            lp = loss_of(rho + d, bc, 1e-12)[0]
            lm = loss_of(rho - d, bc, 1e-12)[0]
            g = float((rho_bar * d).sum())
        else:
            d = torch.randn(bc.shape, generator=gen, dtype=torch.float64).to(dev)
            d *= float(bc.abs().max()) / float(d.abs().max())
            lp = loss_of(rho, bc + d, 1e-12)[0]
            lm = loss_of(rho, bc - d, 1e-12)[0]
            g = float((bc_bar * d).sum())
        fd = (lp - lm) / 2.0
        checks.append({"wrt": kind, "adjoint": g, "finite_difference": fd, "rel_err": abs(g - fd) / abs(fd)})
    fd_ms = (time.perf_counter() - t0) * 1e3 / len(checks)
    return {
        "workload": w.name, "unknowns": int(w.n_unknowns), "leaves": int(w.n_leaves), "boxes": int(tree.n_boxes),
        "loss": loss, "forward_ms": fwd_ms, "forward_cycles": st_f["cycles"],
        "backward_ms": bwd_ms, "backward_iterations": st_b["cycles"],
        "backward_residual_ratio": st_b["r_max"] / st_b["r0_max"],
        "fd_ms_per_check": fd_ms, "fd_checks": checks, "generation_s": round(gen_s, 1),
        "note": "backward = BiCGSTAB on L^T right-preconditioned by a volume-scaled V-cycle (the operator is "
                "not symmetric at refinement boundaries); FD checks solve to 1e-12",
    }


def paper_ex_bench(args, A, torch, dev, stream):
    """The paper's scaling problem (§4.2): lap(phi) = 1 on the unit cube,
    phi = 0 on the boundary, uniform 512^3 grid of 8^3-cell boxes, one FMG
    cycle.  Time per FMG cycle in ns per unknown, beside the paper's figure
    for 8^3 boxes on a 16-core CPU (context, another machine)."""
    from paper_1701_04329_amd import workloads as W

    w = W.uniform_const_rhs(3, 8, 512)
    tree = A.Tree(w.dim, w.level, w.idx)
    rho = tree.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    del w
    u = torch.empty_like(rho)
    work = torch.empty(tree.workspace_bytes(A.make_opts(precision="mixed")), dtype=torch.uint8, device=dev)
    if not args.no_autotune:
        tree.autotune(dev, stream)
    out = {"workload": "ex4_3d_uniform_512", "unknowns": int(tree.n_unknowns), "boxes": int(tree.n_boxes),
           "paper_ns_per_unknown_8cube_16_cores": 22.0}
    for precision in ("fp64", "mixed"):
        # FP64: the FMG cycle alone; mixed: the first refinement step, whose
        # correction is one FP32 FMG cycle
        ms, (_, st) = timed_loop(args, torch, lambda: A.solve(
            tree, rho, None, u, cycle="FMG", max_cycles=0 if precision == "fp64" else 1, precision=precision,
            workspace=work, stream=stream, use_guess=False, check=False))
        out[precision] = {"ms_per_fmg_cycle": ms, "ns_per_unknown": ms * 1e6 / tree.n_unknowns,
                          "residual_ratio_after_fmg": st["r_max"] / st["r0_max"]}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c2", "c1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-tree batch workload")
    ap.add_argument("--batch-trees", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--skip-unbatched", action="store_true",
                    help="batch workload: skip the one-tree-at-a-time comparison pass")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the adaptive 3D workload (FP64 vs mixed)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-paper-ex", action="store_true",
                    help="skip the paper's scaling problem (512^3, one FMG cycle)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batch workload and print its record (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solve is not "
              "distributed across GPUs", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)

    if args.copy_calibration:
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return 0

    from paper_1701_04329_amd import afmg as A

    if args.batch_only:
        print(json.dumps(batch_bench(args, A, torch, dev, torch.cuda.current_stream(dev))), flush=True)
        return 0

    w, solve_kw = make_workload(args.workload)
    tree = A.Tree(w.dim, w.level, w.idx)
    rho = tree.leaf_to_boxes(torch.tensor(w.rho, device=dev))
    bc = tree.bc_rows(torch.tensor(w.bc, device=dev)) if tree.n_bfaces else None
    u = torch.zeros((tree.n_boxes, tree.cells_per_box), dtype=torch.float64, device=dev)
    opts = A.make_opts(**solve_kw)
    ws = torch.empty(tree.workspace_bytes(opts), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def timed_steps(precision, graph=False, profile=True):
        """warmup + exactly `steps` timed solves; returns ms/step, the
        summed event timings of the finest-level kernels, the last stats and
        the cycle counts.  With profile, the last timed solve carries the
        event pairs (one around each group of consecutive finest-level half
        sweeps and each other finest-level launch; a profiled solve launches
        eagerly): the pairs cost about 5% of a solve, so the other timed
        solves run without them."""
        kw = dict(solve_kw, precision=precision)
        ws_p = ws if tree.workspace_bytes(A.make_opts(**kw)) <= ws.numel() else torch.empty(
            tree.workspace_bytes(A.make_opts(**kw)), dtype=torch.uint8, device=dev)

        def one(prof):
            # every step starts from u = 0 (the library zeroes u itself)
            return A.solve(tree, rho, bc, u, workspace=ws_p, stream=stream, profile=prof,
                           use_guess=False, graph=graph, **kw)

        for _ in range(args.warmup):
            one(False)
        torch.cuda.synchronize()
        prof_ms = np.zeros(4)
        prof_n = np.zeros(4, dtype=np.int64)
        cycles = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            _, st = one(profile and i == args.steps - 1)
            prof_ms += np.array(st["prof_ms"])
            prof_n += np.array(st["prof_n"], dtype=np.int64)
            cycles.append(st["cycles"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / args.steps, prof_ms, prof_n, st, cycles

    # launch shapes: untuned time first, then the autotuner (setup, untimed)
    tune = None
    if not args.no_autotune:
        ms_untuned, _, _, _, _ = timed_steps("fp64", graph=True, profile=False)
        ms_untuned_m, _, _, _, _ = timed_steps("mixed", graph=True, profile=False)
        t0 = time.perf_counter()
        shapes = tree.autotune(dev, stream)
        tune = {"untuned_fp64_graph_ms_per_step": ms_untuned, "untuned_mixed_graph_ms_per_step": ms_untuned_m,
                "autotune_s": round(time.perf_counter() - t0, 3),
                "shapes": {f"{p}/{k}": [f"{wg}{'' if nr else 'x'}" for wg, nr in v] for (p, k), v in shapes.items()}}

    # FP64: the headline step
    ms, prof_ms, prof_n, st64, cycles = timed_steps("fp64")
    u64 = tree.boxes_to_leaf(u).cpu().numpy()
    value = w.n_unknowns / (ms * 1e-3)

    # dominant kernel: finest-level half sweep.  Algorithmic bytes per cell
    # of the level: read the other colour (s / 2), read rho of the updated
    # colour (s / 2), write the updated colour (s / 2) = 1.5 s, s = 8 B.
    n_fine = tree.n_leaves * tree.cells_per_box
    bytes_per_launch = 12.0 * n_fine
    avg_ms = prof_ms[0] / max(prof_n[0], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # the counters were taken on the default shape of the finest level
    fine_shape = tree.shape("fp64", "gsrb", tree.lmax)
    traffic = committed_traffic(f"k_gsrb_{w.name}") if fine_shape == (256, 0) else None
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "k_gsrb<3,8,double,256,false> (finest level, one half sweep; single-tree variant)",
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "avg_launch_ms": round(avg_ms, 5),
        "launches_timed": int(prof_n[0]),
    }

    # mixed: FP32 V-cycles inside FP64 refinement, same workload and stop rule
    ms_m, prof_m, prof_nm, stm, cycles_m = timed_steps("mixed")
    umx = tree.boxes_to_leaf(u).cpu().numpy()
    avg_m = prof_m[0] / max(prof_nm[0], 1)
    mixed = {
        "value": w.n_unknowns / (ms_m * 1e-3),
        "unit": "unknowns/s",
        "ms_per_step": ms_m,
        "outer_iterations": int(np.median(cycles_m)),
        "final_residual_ratio": stm["r_max"] / stm["r0_max"],
        "rel_l2_vs_gpu_fp64": float(np.linalg.norm(umx - u64) / np.linalg.norm(u64)),
        "dominant_kernel": "k_gsrb_cube<3,8,float,W> (finest level, one half sweep)",
        "dominant_achieved_GBs": round(6.0 * n_fine / (avg_m * 1e-3) / 1e9, 1) if prof_nm[0] else None,
        "dominant_avg_launch_ms": round(avg_m, 5),
    }

    # context: the repeated cycle replayed from a recorded HIP graph (no
    # event pairs)
    ms_g, _, _, _, _ = timed_steps("fp64", graph=True, profile=False)
    ms_gm, _, _, _, _ = timed_steps("mixed", graph=True, profile=False)
    graph = {"fp64_ms_per_step": ms_g, "mixed_ms_per_step": ms_gm,
             "fp64_value": w.n_unknowns / (ms_g * 1e-3), "mixed_value": w.n_unknowns / (ms_gm * 1e-3)}

    out = {
        "metric": "Poisson unknowns/s to 1e-10 residual reduction (FP64 vs mixed); HBM % of peak",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "dim": w.dim,
            "box": f"{w.N}^{w.dim}",
            "unknowns": int(w.n_unknowns),
            "boxes": int(tree.n_boxes),
            "cycle": "FMG + V(2,2)" if solve_kw["cycle"] == "FMG" else "V(2,2)",
            "tol": solve_kw["tol"],
            "v_cycles": int(np.median(cycles)),
            "final_residual_ratio": st64["r_max"] / st64["r0_max"],
            "precision": "fp64",
            "schedule": "eager launches, event pairs in the last timed solve; autotuned launch shapes",
        },
        "roofline": roofline,
        "mixed": mixed,
        "graph": graph,
        "autotune": tune,
    }
    if not args.no_batch:
        out["batch"] = batch_bench(args, A, torch, dev, stream)
    if not args.no_adaptive:
        out["adaptive"] = adaptive_bench(args, A, torch, dev, stream)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(args, A, torch, dev, stream)
    if not args.no_paper_ex:
        out["paper_ex"] = paper_ex_bench(args, A, torch, dev, stream)
    if not args.no_cpu_baseline:
        uo, out["cpu_baseline"] = cpu_baseline(w, solve_kw)
        nrm = np.linalg.norm(uo)
        out["config"]["rel_l2_vs_oracle"] = float(np.linalg.norm(u64 - uo) / nrm)
        out["mixed"]["rel_l2_vs_oracle"] = float(np.linalg.norm(umx - uo) / nrm)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
