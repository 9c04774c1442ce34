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
VEC_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def algorithmic_bytes(op, s, what):
    """Bytes the method must move (each read once, each result written once); s = bytes per
    scalar.  'apply': u read, v written, the x-run index map of every cell, and per
    surrogate face its record (cell id + face code) and shifted points (FP64).  'brick':
    the brick kernel alone (CG), which does the cell term for every DoF and merges the
    surrogate-face results: u read, every DoF's value written once (inside a brick directly,
    on a brick boundary through its halo slot), the index map, and per face its record and
    its two result values per face node."""
    np_ = op.nq_face
    idx = 4 * op.n_cells * np_ if op.disc == "cg" else 4 * op.n_cells * 2 * op.d
    if what == "apply":
        return 2 * s * op.n_dofs + idx + op.n_sbm_faces * (8 + np_ * op.d * 8)
    if what == "brick":
        return 2 * s * op.n_dofs + idx + op.n_sbm_faces * (8 + 2 * np_ * s)
    raise ValueError(what)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2507_17053_amd", "csrc", "kernels_apply.hip")
    with open(p, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def _profile_record(name):
    """The machine-readable line of a committed counter summary, only if it was taken on the
    current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    for line in open(p):
        if line.startswith("machine-readable:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_src") == kernel_source_hash():
                return rec
    return None


def measured_traffic(key="traffic_bytes_per_launch"):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters) from
    the committed apply-kernel traffic summary: key names the brick kernel or the whole apply."""
    rec = _profile_record("apply_kernels_sphere3d_q4_traffic.md")
    return None if rec is None else rec.get(key)


def flop_rates(t_kernels, t_apply):
    """FP64/FP32 vector FLOP rates of the apply kernels: FLOPs per launch from the committed
    VALU counter summary over the kernel times measured in this run (t_kernels: name -> s)."""
    rec = _profile_record("apply_kernels_sphere3d_q4_valu.md")
    if rec is None:
        return None
    out = {}
    for name, t in t_kernels.items():
        fl = rec["flop_per_launch"].get(name)
        if fl is None or not t:
            continue
        peak = VEC_PEAK_TFLOPS["f64" if "double" in name else "f32"]
        rate = fl / t / 1e12
        out[name] = {"gflop_per_launch": fl / 1e9, "tflops": rate, "peak_tflops": peak, "frac": rate / peak}
    for prec, t in t_apply.items():
        tn = "double" if prec == "f64" else "float"
        fl = sum(v for k, v in rec["flop_per_launch"].items() if f"<{tn}," in k)
        rate = fl / t / 1e12
        out[f"apply_{prec}"] = {"gflop_per_apply": fl / 1e9, "tflops": rate, "peak_tflops": VEC_PEAK_TFLOPS[prec],
                                "frac": rate / VEC_PEAK_TFLOPS[prec]}
    return out


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


OTHER_CONFIGS = [
    # (label, workload, overrides)
    ("torus3d_dg_q3", "torus3d_dg", {}),
    ("torus3d_dg_q5", "torus3d_dg", {"p": 5}),
    # DG at a size that fills the device (about 0.36M cells)
    ("torus3d_dg_q3_n80", "torus3d_dg", {"n": 80}),
    ("spheres3d_q6", "spheres3d_q6", {}),
    # working set (vectors alone 229 MB in FP64) above the 256 MB last-level cache together
    ("sphere3d_q4_n128", "sphere3d_q4", {"n": 128}),
]


def configs_section(torch, sbm, inputs, steps, graph_batch):
    """FP64 and FP32 apply of the other workloads: DoF/s, effective bandwidth on the
    algorithmic bytes, and the FP32 result's relative deviation from the FP64 one."""
    out = []
    for label, name, over in OTHER_CONFIGS:
        w = inputs.workload(name, **over)
        t0 = time.perf_counter()
        op = sbm.Operator(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], disc=w["disc"])
        t_setup = time.perf_counter() - t0
        u64 = torch.from_numpy(inputs.uniform_vector(op.n_dofs, seed=0)).to("cuda")
        u32 = u64.float()
        v64, v32 = torch.empty_like(u64), torch.empty_like(u32)
        rec = {"config": label, "d": op.d, "p": op.p, "n": w["n"], "disc": op.disc, "n_dofs": op.n_dofs,
               "n_cells": op.n_cells, "n_sbm_faces": op.n_sbm_faces, "setup_s": t_setup}
        for prec, (u, v, s) in {"f64": (u64, v64, 8), "f32": (u32, v32, 4)}.items():
            for _ in range(5):
                op.apply(u, v)
            t, _, n = time_launches(torch, lambda: op.apply(u, v), steps, graph_batch)
            gbs = algorithmic_bytes(op, s, "apply") / t / 1e9
            rec[prec] = {"dofs_per_s": op.n_dofs / t, "ms_per_apply": t * 1e3, "applies": n,
                         "effective_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        op.apply(u64, v64)
        op.apply(u32, v32)
        torch.cuda.synchronize()
        rec["f32_rel_dev_from_f64"] = float((v32.double() - v64).norm() / v64.norm())
        out.append(rec)
        print(f"# config {label}: f64 {rec['f64']['ms_per_apply']:.4f} ms, f32 {rec['f32']['ms_per_apply']:.4f} ms",
              file=sys.stderr, flush=True)
        del op, u64, u32, v64, v32
        torch.cuda.empty_cache()
    return out


def taylor_section(torch, sbm, inputs, op, vecs, steps, graph_batch):
    """The truncated Taylor extension E_m (sbm_set_extension_order) on the headline operator:
    apply time for m = 1 and m = p against the default extension (FP64 and FP32); its solves
    are in the solve section."""
    out = {"workload": "sphere3d_q4", "apply": {}}
    for m in (None, 1, op.p):
        op.set_extension_order(m)
        rec = {}
        for prec, (u, v) in vecs.items():
            for _ in range(3):
                op.apply(u, v)
            t, _, n = time_launches(torch, lambda: op.apply(u, v), steps, graph_batch)
            rec[prec] = {"ms_per_apply": t * 1e3, "dofs_per_s": op.n_dofs / t, "applies": n}
        out["apply"]["default" if m is None else f"m{m}"] = rec
        print(f"# taylor apply m={m}: f64 {rec['f64']['ms_per_apply']:.4f} ms, f32 {rec['f32']['ms_per_apply']:.4f} ms",
              file=sys.stderr, flush=True)
    op.set_extension_order(None)
    return out


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
    # one apply on a single thread (then back to all threads: the OpenMP setting persists)
    t1 = time.perf_counter()
    ap(u, n_threads=1)
    el1 = time.perf_counter() - t1
    ap(u, n_threads=threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": prob.n_dofs * n / el, "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full FP64 applies of the same workload ({prob.n_dofs} DoFs), brute-force "
                      f"dense local matrices in plain C + OpenMP, {el:.1f} s",
            "seconds": el, "single_core_value": prob.n_dofs / el1, "cpu_model": model,
            "host_cpus": os.cpu_count()}


SOLVE_CASES = [
    # (name, workload, overrides, shift_scale, extension order, modes, max_it)
    # converging shifted cases (GMRES(64) in FP64 vs FP32 GMRES in FP64 refinement)
    ("disk2d_q2", "disk2d_q2", {}, 1.0, None, ("gmres", "gmres_ir"), 8000),
    ("sphere3d_q1_n64", "sphere3d_q4", {"p": 1}, 1.0, None, ("gmres", "gmres_ir"), 4000),
    # the 3D workloads with the method's extension: restarted GMRES stagnates (the operator is
    # near-singular and indefinite); the residual reached is reported
    ("sphere3d_q4", "sphere3d_q4", {}, 1.0, None, ("gmres", "gmres_ir"), 300),
    ("torus3d_dg_q3", "torus3d_dg", {}, 1.0, None, ("gmres", "gmres_ir"), 300),
    ("spheres3d_q6", "spheres3d_q6", {}, 1.0, None, ("gmres", "gmres_ir"), 300),
    # the same with the first-order extension E_1
    ("sphere3d_q2_n32_E1", "sphere3d_q4", {"p": 2, "n": 32}, 1.0, 1, ("gmres", "gmres_ir"), 1500),
    ("sphere3d_q4_E1", "sphere3d_q4", {}, 1.0, 1, ("gmres", "gmres_ir"), 600),
    ("torus3d_dg_q3_E1", "torus3d_dg", {}, 1.0, 1, ("gmres", "gmres_ir"), 600),
    ("spheres3d_q6_E1", "spheres3d_q6", {}, 1.0, 1, ("gmres", "gmres_ir"), 600),
    # the symmetric limit (shift 0) of the 3D CG workloads at full size: CG converges
    ("sphere3d_q4_unshifted", "sphere3d_q4", {}, 0.0, None, ("cg", "cg_ir", "cg_rr"), 4000),
    ("spheres3d_q6_unshifted", "spheres3d_q6", {}, 0.0, None, ("cg", "cg_ir", "cg_rr"), 4000),
]


def solve_section(torch, sbm, inputs):
    """FP64 Krylov vs FP64 refinement around the same Krylov method in FP32, to 1e-10 relative
    residual: GMRES(64) for the shifted (nonsymmetric) operators, CG for the symmetric limit.
    Per run: status, time, iterations, the FP64 residual reached and the L2 error of the
    solution against the manufactured solution (sbm_l2_error)."""
    out = []
    for name, wname, over, shift, order, modes, max_it in SOLVE_CASES:
        w = inputs.workload(wname, **over)
        op = sbm.Operator(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], disc=w["disc"],
                          shift_scale=shift, taylor_order=order)
        u_fn, f_fn = inputs.manufactured(w["d"])
        cq, bp = op.rhs_points()
        ustar = u_fn(cq.reshape(-1, w["d"]))
        b = torch.empty(op.n_dofs, dtype=torch.float64, device="cuda")
        op.rhs(f_fn(cq.reshape(-1, w["d"])), u_fn(bp.reshape(-1, w["d"])), b)
        rec = {"case": name, "n_dofs": op.n_dofs, "p": w["p"], "disc": w["disc"], "shift_scale": shift,
               "extension": "full" if order is None else f"E_{order}", "max_it": max_it}
        for mode in modes:
            x = torch.zeros_like(b)
            info = op.solve(b, x, rel_tol=1e-10, max_it=max_it, mode=mode, restart=64)
            rec[mode] = {"status": sbm.status_name(info["status"]), "seconds": info["seconds"],
                         "krylov_its": info["inner_its"], "refinements": info["outer_its"],
                         "applies_f64": info["applies_f64"], "applies_f32": info["applies_f32"],
                         "rel_residual_f64": info["rel_residual"], "l2_error": op.l2_error(x, ustar)}
            print(f"# solve {name} {mode}: {rec[mode]}", file=sys.stderr, flush=True)
        g = rec[modes[0]]
        for mode in modes[1:]:
            if g["status"] == "SBM_OK" and rec[mode]["status"] == "SBM_OK":
                rec[f"{mode}_speedup_vs_{modes[0]}"] = g["seconds"] / rec[mode]["seconds"]
        out.append(rec)
        op.close()
        del b
        torch.cuda.empty_cache()
    return out


def batch_section(torch, sbm, inputs, reps=20):
    """Applies of many operators at once (serving's launches): the operators of request streams
    (p in 2..6, ellipsoid or 8-ball union, CG or SIPG) applied one by one (eager, and captured
    into a graph) against the batched launches (one launch per stage per group of operators
    with the same discretisation and degree: the one-shot call on one stream, and prepared
    batches with the groups on one stream or forked over four, replayed from their graphs or
    launched directly).  FP64; times per pass over all operators, from events on the stream."""
    out = {}
    mixes = [("serving_stream_first_32", inputs.serving_requests(32, seed=2)),
             ("small_64_n16_24", inputs.serving_requests(64, seed=5, n_range=(16, 24)))]
    side = torch.cuda.Stream()
    for name, reqs in mixes:
        ops = [sbm.Operator(r["d"], r["n"], r["lo"], r["hi"], r["levelset"], r["p"], disc=r["disc"]) for r in reqs]
        us = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=i)).to("cuda") for i, o in enumerate(ops)]
        vs = [torch.empty_like(u) for u in us]
        ndofs = sum(o.n_dofs for o in ops)
        groups = len({(o.disc, o.p) for o in ops})

        def loop():
            for o, u, v in zip(ops, us, vs):
                o.apply(u, v)

        with torch.cuda.stream(side):
            for _ in range(3):
                loop()
                sbm.apply_batch(ops, us, vs)
            plan = sbm.Batch(ops, us, vs, graph=True, streams=4)
            plan1 = sbm.Batch(ops, us, vs, graph=True, streams=1)
            plan_e = sbm.Batch(ops, us, vs, graph=False, streams=4)
            for pl in (plan, plan1, plan_e):
                pl.run()
            torch.cuda.synchronize()
            t_loop, w_loop, _ = time_launches(torch, loop, reps, 0)
            t_loop_g, _, _ = time_launches(torch, loop, reps, 2)
            t_once, w_once, _ = time_launches(torch, lambda: sbm.apply_batch(ops, us, vs), reps, 0)
            t_plan, w_plan, _ = time_launches(torch, plan.run, reps, 0)
            t_plan1, _, _ = time_launches(torch, plan1.run, reps, 0)
            t_plan_e, _, _ = time_launches(torch, plan_e.run, reps, 0)
            for pl in (plan, plan1, plan_e):
                pl.close()
        out[name] = {"operators": len(ops), "groups": groups, "total_dofs": int(ndofs),
                     "loop_eager_ms": t_loop * 1e3, "loop_eager_wall_ms": w_loop * 1e3,
                     "loop_graph_ms": t_loop_g * 1e3, "apply_batch_ms": t_once * 1e3,
                     "apply_batch_wall_ms": w_once * 1e3, "batch_graph_ms": t_plan * 1e3,
                     "batch_graph_wall_ms": w_plan * 1e3, "batch_graph_one_stream_ms": t_plan1 * 1e3,
                     "batch_eager_4_streams_ms": t_plan_e * 1e3,
                     "batch_graph_dofs_per_s": ndofs / t_plan, "loop_graph_dofs_per_s": ndofs / t_loop_g,
                     "speedup_batch_graph_vs_loop_graph": t_loop_g / t_plan,
                     "speedup_batch_graph_vs_loop_eager": t_loop / t_plan}
        # the solve phase of serving: the same systems solved one after another (sbm_solve)
        # against one lockstep batch (sbm_solve_batch), FP32 GMRES(32) inside FP64 refinement
        # with the serving iteration cap; the results are identical, so are the iteration counts
        bs = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=700 + i)).to("cuda") for i, o in enumerate(ops)]
        xs = [torch.zeros_like(b) for b in bs]
        for o, b, x in zip(ops, bs, xs):  # workspaces allocated outside the timing
            o.solve(b, x, rel_tol=1e-10, max_it=4, mode="gmres_ir", restart=32)
        torch.cuda.synchronize()
        for x in xs:
            x.zero_()
        t0 = time.perf_counter()
        single = [o.solve(b, x, rel_tol=1e-10, max_it=100, mode="gmres_ir", restart=32) for o, b, x in zip(ops, bs, xs)]
        torch.cuda.synchronize()
        t_single = time.perf_counter() - t0
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = sbm.solve_batch(ops, bs, xs, rel_tol=1e-10, max_it=100, mode="gmres_ir", restart=32)
        t_batch = time.perf_counter() - t0
        out[name]["solves"] = {
            "mode": "gmres_ir", "restart": 32, "max_it": 100,
            "one_by_one_s": t_single, "lockstep_batch_s": t_batch, "speedup": t_single / t_batch,
            "same_iterations": all(a["inner_its"] == b["inner_its"] for a, b in zip(single, infos)),
            "krylov_its_total": int(sum(i["inner_its"] for i in infos))}
        print(f"# batched applies {name}: {out[name]}", file=sys.stderr, flush=True)
        for o in ops:
            o.close()
        del bs, xs
        del us, vs
        torch.cuda.empty_cache()
    return out


def serve_section(n_req, max_it, rate, slots, budget_gb, deadline_s):
    """Request stream (p in 2..6, 16^3..64^3 cells, ellipsoid or 8-ball union, CG or SIPG,
    FP32 GMRES inside FP64 refinement to 1e-10 with an iteration cap).  First closed loop (all
    requests queued at t = 0) for the capacity mu in solves/s, then open loop with Poisson
    arrivals at 0.7 mu (rate > 0 overrides the open-loop rate); then the same requests in closed
    loop with the first-order extension E_1 and a 10x iteration cap; then closed loop again in
    lockstep batches (every admitted request of a set solved together by sbm_solve_batch, the
    applies of each Krylov step batched).  Each run admits requests for at most deadline_s
    seconds (the prefix served is reported)."""
    from paper_2507_17053_amd import inputs
    from paper_2507_17053_amd.serving import Server, run_batched

    def one(reqs, time_scale, cap=max_it, batched_slots=0, prefetch=False):
        srv = Server(budget_bytes=int(budget_gb * (1 << 30)), slots=(2 if prefetch else 1) * batched_slots or slots,
                     mode="gmres_ir", rel_tol=1e-10, max_it=cap, restart=32)
        if batched_slots:
            s = run_batched(srv, reqs, time_scale=time_scale, deadline_s=deadline_s, set_size=batched_slots,
                            prefetch=prefetch)
        else:
            s = srv.run(reqs, time_scale=time_scale, deadline_s=deadline_s)
        res = list(s["results"].values())
        rr = sorted(r["info"].get("rel_residual", float("nan")) for r in res)
        conv = [r for r in res if r["error"] is None and r["info"].get("status") == 0]
        return {"requests": s["requests"], "served": s["served"], "converged_to_1e-10": s["converged"],
                "errors": s["errors"], "solves_per_s": s["solves_per_s"],
                "converged_solves_per_s": s["converged_solves_per_s"],
                "latency_p50_s": s["latency_p50_s"], "latency_p99_s": s["latency_p99_s"],
                "converged_latency_p50_s": s["converged_latency_p50_s"],
                "converged_latency_p99_s": s["converged_latency_p99_s"],
                "median_rel_residual": rr[len(rr) // 2] if rr else None,
                "converged_by_kind": {k: sum(1 for r in conv if f"{r['info'].get('disc', '')}" == k) for k in ("cg", "dg")},
                "total_dofs": int(sum(r["info"].get("n_dofs", 0) for r in res)), "wall_s": s["wall_s"],
                **{k: s[k] for k in ("sets", "setup_and_rhs_s", "lockstep_solve_s") if k in s}}

    closed = one(inputs.serving_requests(n_req, seed=2, rate=1.0), 0.0)
    mu = closed["solves_per_s"]
    lam = rate if rate > 0 else 0.7 * mu
    opened = one(inputs.serving_requests(n_req, seed=2, rate=lam), 1.0)
    # the same requests with the first-order extension E_1, closed loop, 10x iteration cap
    first = one([dict(r, taylor_order=1) for r in inputs.serving_requests(n_req, seed=2, rate=1.0)], 0.0,
                cap=10 * max_it)
    # lockstep sets of up to 32 admitted requests (sbm_solve_batch), closed loop; then with the
    # next set prepared on a host thread while the current one solves
    batched = one(inputs.serving_requests(n_req, seed=2, rate=1.0), 0.0, batched_slots=32)
    piped = one(inputs.serving_requests(n_req, seed=2, rate=1.0), 0.0, batched_slots=32, prefetch=True)
    return {"closed_loop": closed, "open_loop": dict(opened, arrival_rate_per_s=lam),
            "closed_loop_lockstep_batches": dict(batched, batch_slots=32),
            "closed_loop_lockstep_batches_prefetch": dict(piped, batch_slots=32), "slots": slots,
            "hbm_budget_GB": budget_gb, "krylov_cap": max_it, "admission_deadline_s": deadline_s,
            "closed_loop_first_order_extension": dict(first, krylov_cap=10 * max_it)}


def serve_in_child(args):
    """The serving section in a child process (its worker threads, allocations and teardowns are
    isolated from the measurement above: whatever happens there, this run still prints its
    line); returns the child's JSON, or the child's exit status and the tail of its output."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serve-only", "--serve", str(args.serve),
           "--serve-max-it", str(args.serve_max_it), "--serve-rate", str(args.serve_rate),
           "--serve-deadline", str(args.serve_deadline), "--serve-slots", str(args.serve_slots)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=max(120.0, 8 * args.serve_deadline + 120.0))
    lines = [ln for ln in r.stdout.strip().splitlines() if ln.startswith("{")]
    if r.returncode == 0 and lines:
        return json.loads(lines[-1])
    return {"error": f"serving process exited with status {r.returncode}",
            "stderr_tail": r.stderr[-2000:], "stdout_tail": r.stdout[-500:]}


def profile_run(torch, sbm, inputs, n=5, order=None, prec="f64", workload="sphere3d_q4"):
    """A few eager applies and plain device copies of the vector, for counter runs (order:
    extension order set on the operator first; None keeps the full extension; prec: f64 or
    f32)."""
    w = inputs.workload(workload)
    op = sbm.Operator(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], disc=w["disc"], taylor_order=order)
    u = torch.from_numpy(inputs.uniform_vector(op.n_dofs, seed=0)).to("cuda")
    if prec == "f32":
        u = u.float()
    v = torch.empty_like(u)
    for _ in range(n):
        op.apply(u, v)
    for _ in range(n):
        v.copy_(u)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": True, "workload": workload, "n_dofs": op.n_dofs, "prec": prec,
                      "copy_bytes_each_way": u.element_size() * op.n_dofs, "taylor_order": order}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sphere3d_q4")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads' applies")
    ap.add_argument("--no-solve", action="store_true", help="skip the FP64 vs FP32+refinement solves")
    ap.add_argument("--no-taylor", action="store_true", help="skip the truncated-Taylor extension section")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-applies section")
    ap.add_argument("--batch-only", action="store_true", help="only the batched-applies section")
    ap.add_argument("--profile-run", action="store_true", help="few eager applies + copies (counter runs)")
    ap.add_argument("--profile-order", type=int, default=None,
                    help="with --profile-run: extension order of the operator (default: full extension)")
    ap.add_argument("--profile-prec", default="f64", choices=("f64", "f32"), help="with --profile-run")
    ap.add_argument("--serve", type=int, default=512, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-deadline", type=float, default=20.0,
                    help="seconds during which each serving run admits requests")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving section and print its JSON (used by the main run, which "
                         "runs the serving section in a child process)")
    ap.add_argument("--serve-max-it", type=int, default=100)
    ap.add_argument("--serve-slots", type=int, default=1,
                    help="requests solved at once (each on its own thread and stream); the default runs one "
                         "at a time: a 12-slot run of this section aborted inside the process (glibc "
                         "'free(): invalid pointer') without a cause found in the library")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="open-loop arrival rate (default: 0.7 of the closed-loop capacity)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the library has no multi-GPU path; use --gpus 1"}))
        sys.exit(2)

    if args.serve_only:
        import torch  # noqa: F401  (the library runs on torch's HIP runtime)
        print(json.dumps(serve_section(args.serve, args.serve_max_it, args.serve_rate, slots=args.serve_slots,
                                       budget_gb=96.0, deadline_s=args.serve_deadline)), flush=True)
        return

    import torch

    from paper_2507_17053_amd import inputs, sbm

    if args.profile_run:
        profile_run(torch, sbm, inputs, order=args.profile_order, prec=args.profile_prec, workload=args.workload)
        return
    if args.batch_only:
        print(json.dumps({"batched_apply": batch_section(torch, sbm, inputs)}), flush=True)
        return

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
    NA = sbm.PART_NO_ASSEMBLY
    for name, (u, v, s) in {"f64": (u64, v64, 8), "f32": (u32, v32, 4)}.items():
        t_apply, t_wall, n = time_launches(torch, lambda: op.apply(u, v), args.steps, gb)
        # the brick kernel alone: cells + merge of the surrogate-face results the applies
        # above left on the handle (no face evaluation, no assembly pass)
        RF = sbm.PART_REUSE_FACES
        t_brick, _, _ = time_launches(torch, lambda: op.apply_parts(u, v, sbm.PART_ALL | NA | RF), args.steps, gb)
        # the apply without surrogate faces (for the share of time spent in them)
        t_cell, _, _ = time_launches(torch, lambda: op.apply_parts(u, v, sbm.PART_CELLS), args.steps, gb)
        res[name] = dict(t_apply=t_apply, t_wall=t_wall, n=n, t_brick=t_brick, t_cell=t_cell,
                         b_brick=algorithmic_bytes(op, s, "brick"), b_apply=algorithmic_bytes(op, s, "apply"))

    r = res["f64"]
    brick_gbs = r["b_brick"] / r["t_brick"] / 1e9
    apply_gbs = r["b_apply"] / r["t_apply"] / 1e9
    n_bricks, n_bdofs, n_bslots = op.layout_stats()
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
        "roofline": {"bound": "hbm", "kernel": "brick_kernel (FP64: cells + merge of surrogate-face results)",
                     "achieved": brick_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": brick_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel_ms": r["t_brick"] * 1e3,
                     "algorithmic_bytes_per_launch": r["b_brick"], "kernel_src": kernel_source_hash(),
                     # the whole apply (surrogate faces, bricks, boundary sums) against the same peak
                     "apply_achieved": apply_gbs, "apply_frac": apply_gbs / HBM_PEAK_GBS,
                     "apply_traffic": measured_traffic("apply_traffic_bytes_f64")},
        "apply_roofline": {"bound": "hbm", "achieved": apply_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": apply_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("apply_traffic_bytes_f64"),
                           "algorithmic_bytes_per_apply": r["b_apply"], "ms": r["t_apply"] * 1e3,
                           "fp32": {"achieved": res["f32"]["b_apply"] / res["f32"]["t_apply"] / 1e9,
                                    "frac": res["f32"]["b_apply"] / res["f32"]["t_apply"] / 1e9 / HBM_PEAK_GBS,
                                    "traffic": measured_traffic("apply_traffic_bytes_f32"),
                                    "algorithmic_bytes_per_apply": res["f32"]["b_apply"]}},
        "flop_rates": flop_rates({"brick_kernel<double, 3, 5>": r["t_brick"],
                                  "brick_kernel<float, 3, 5>": res["f32"]["t_brick"]},
                                 {"f64": r["t_apply"], "f32": res["f32"]["t_apply"]})
        if (op.d, op.p, op.disc) == (3, 4, "cg") else None,
        "apply_effective_GBs": apply_gbs,
        "apply_hbm_frac": apply_gbs / HBM_PEAK_GBS,
        "apply_algorithmic_bytes": r["b_apply"],
        "face_and_assembly_ms": (r["t_apply"] - r["t_brick"]) * 1e3,
        "sbm_face_time_share": 1.0 - r["t_cell"] / r["t_apply"],
        "layout": {"bricks": n_bricks, "boundary_dofs": n_bdofs, "boundary_slots": n_bslots},
        "wall_ms_per_step": r["t_wall"] * 1e3,
        "fp32": {"value": op.n_dofs / res["f32"]["t_apply"], "unit": "DoF/s",
                 "ms_per_step": res["f32"]["t_apply"] * 1e3,
                 "apply_effective_GBs": res["f32"]["b_apply"] / res["f32"]["t_apply"] / 1e9,
                 "apply_hbm_frac": res["f32"]["b_apply"] / res["f32"]["t_apply"] / 1e9 / HBM_PEAK_GBS,
                 "brick_kernel_ms": res["f32"]["t_brick"] * 1e3,
                 "brick_kernel_frac": res["f32"]["b_brick"] / res["f32"]["t_brick"] / 1e9 / HBM_PEAK_GBS},
        "setup_s": t_setup,
    }
    # setup again on a warm process (the first one also loads the library's kernels)
    t0 = time.perf_counter()
    sbm.Operator(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], disc=w["disc"]).close()
    out["setup_warm_s"] = time.perf_counter() - t0
    if not args.no_taylor:
        out["taylor_extension"] = taylor_section(torch, sbm, inputs, op, {"f64": (u64, v64), "f32": (u32, v32)},
                                                 min(args.steps, 200), gb)
    if not args.no_configs:
        out["other_configs"] = configs_section(torch, sbm, inputs, min(args.steps, 200), gb)
    if not args.no_batch:
        out["batched_apply"] = batch_section(torch, sbm, inputs)
    if not args.no_solve:
        out["solve"] = solve_section(torch, sbm, inputs)
    if args.serve > 0:
        out["serving"] = serve_in_child(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
