"""Benchmark of the matrix-free SBM operator apply on one MI355X.

One step = one sbm_apply (cell term + surrogate-boundary faces) of the 3D CG Q4 operator
on 64^3 background cells over [-1,1]^3 clipped by the sphere r = 0.75 (3,443,241 DoFs),
with a seeded uniform[-1,1] input vector resident in HBM.  W warm-up applies, then K
timed applies replayed from captured HIP graphs, bracketed by device synchronisation.

Prints one JSON line: DoF/s of the FP64 apply (value), the FP32 apply, the roofline of the
dominant kernel (cell kernel, HIP-event timed on the launch stream), the surrogate-face
time share, and the CPU oracle timed on this host as a baseline.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--solve]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SBM apply DoF/s + % HBM roofline (FP64 vs FP32), 3D p=4; solves/s, p99 latency"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(op, s, part):
    """Bytes the method must move per launch (u read once, v written once, index and
    face data read once); s = bytes per scalar."""
    np_ = op.nq_face
    if part == "cells":
        idx = 4 * op.n_cells * np_ if op.disc == "cg" else 4 * op.n_cells * 2 * op.d
        return 2 * s * op.n_dofs + idx
    if part == "faces":
        # face records (cell id + code), shifted points (FP64), u_K read and w_K added
        return op.n_sbm_faces * (8 + np_ * op.d * 8) + 2 * s * op.n_sbm_faces * op.nb
    raise ValueError(part)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2507_17053_amd", "csrc", "kernels_apply.hip")
    with open(p, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def time_launches(torch, fn, k, graph_batch=20):
    """Average time per fn() call over k calls: captured into a HIP graph of graph_batch
    calls, replayed; timed with events recorded on the launch stream."""
    stream = torch.cuda.current_stream()
    g = None
    if graph_batch > 0:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(graph_batch):
                fn()
        torch.cuda.synchronize()
        reps = max(1, k // graph_batch)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n = reps * graph_batch
        return e0.elapsed_time(e1) / 1e3 / n, wall / n, n
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(k):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3 / k, wall / k, k


def cpu_baseline(w, budget_s=12.0):
    """The brute-force C oracle (OpenMP) on this host, on the same workload: as many full
    applies as fit in about budget_s seconds (at least one)."""
    from oracle import native
    from oracle import sbm_oracle as O
    from paper_2507_17053_amd import inputs

    native.build(force=False)
    prob = O.setup(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], disc=w["disc"])
    u = inputs.uniform_vector(prob.n_dofs, seed=0)
    ap = native.NativeApply(prob)
    threads = native.max_threads()
    ap(u)  # warm (page in)
    n = 0
    t0 = time.perf_counter()
    while True:
        ap(u)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or (n >= 1 and el * (n + 1) / n > 2.5 * budget_s):
            break
    return {"value": prob.n_dofs * n / el, "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full FP64 applies of the same workload ({prob.n_dofs} DoFs), brute-force "
                      f"dense local matrices in plain C + OpenMP, {el:.1f} s",
            "seconds": el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sphere3d_q4")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--solve", action="store_true", help="also time the FP64 and FP32+IR solves")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2507_17053_amd import inputs, sbm

    w = inputs.workload(args.workload)
    t_setup = time.perf_counter()
    op = sbm.Operator(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], disc=w["disc"])
    t_setup = time.perf_counter() - t_setup
    u64 = torch.from_numpy(inputs.uniform_vector(op.n_dofs, seed=0)).to("cuda")
    v64 = torch.empty_like(u64)
    u32 = u64.float()
    v32 = torch.empty_like(u32)
    gb = 0 if args.no_graph else 20

    for _ in range(args.warmup):
        op.apply(u64, v64)
        op.apply(u32, v32)
    torch.cuda.synchronize()

    res = {}
    for name, (u, v, s) in {"f64": (u64, v64, 8), "f32": (u32, v32, 4)}.items():
        t_apply, t_wall, n = time_launches(torch, lambda: op.apply(u, v), args.steps, gb)
        t_cell, _, _ = time_launches(torch, lambda: op.apply_parts(u, v, sbm.PART_CELLS), args.steps, gb)
        t_face, _, _ = time_launches(torch, lambda: op.apply_parts(u, v, sbm.PART_SBM_FACES), args.steps, gb)
        b_cell = algorithmic_bytes(op, s, "cells")
        b_face = algorithmic_bytes(op, s, "faces")
        res[name] = dict(t_apply=t_apply, t_wall=t_wall, n=n, t_cell=t_cell, t_face=t_face, b_cell=b_cell,
                         b_face=b_face)

    r = res["f64"]
    cell_gbs = r["b_cell"] / r["t_cell"] / 1e9
    apply_bytes = r["b_cell"] + op.n_sbm_faces * (8 + op.nq_face * op.d * 8)
    out = {
        "metric": METRIC,
        "value": op.n_dofs / r["t_apply"],
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": r["n"],
        "warmup": args.warmup,
        "ms_per_step": r["t_apply"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D CG Q4 SBM Poisson apply, 64^3 cells on [-1,1]^3, sphere r=0.75 at 0",
                   "name": args.workload, "n_dofs": op.n_dofs, "n_cells": op.n_cells,
                   "n_sbm_faces": op.n_sbm_faces, "p": op.p, "disc": op.disc, "timing": "hip-graph replay"
                   if gb else "eager"},
        "roofline": {"bound": "hbm", "kernel": "cell_kernel (FP64)", "achieved": cell_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": cell_gbs / HBM_PEAK_GBS,
                     "traffic": None, "kernel_ms": r["t_cell"] * 1e3,
                     "algorithmic_bytes_per_launch": r["b_cell"], "kernel_src": kernel_source_hash()},
        "apply_effective_GBs": apply_bytes / r["t_apply"] / 1e9,
        "apply_hbm_frac": apply_bytes / r["t_apply"] / 1e9 / HBM_PEAK_GBS,
        "sbm_face_time_share": r["t_face"] / (r["t_cell"] + r["t_face"]),
        "face_kernel_ms": r["t_face"] * 1e3,
        "wall_ms_per_step": r["t_wall"] * 1e3,
        "fp32": {"value": op.n_dofs / res["f32"]["t_apply"], "unit": "DoF/s",
                 "ms_per_step": res["f32"]["t_apply"] * 1e3,
                 "cell_kernel_GBs": res["f32"]["b_cell"] / res["f32"]["t_cell"] / 1e9,
                 "cell_kernel_frac": res["f32"]["b_cell"] / res["f32"]["t_cell"] / 1e9 / HBM_PEAK_GBS,
                 "face_kernel_ms": res["f32"]["t_face"] * 1e3},
        "setup_s": t_setup,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
