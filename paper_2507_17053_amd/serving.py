"""Continuous-batching request loop for SBM Poisson solves.

Requests (mesh, level set, degree, CG|DG) arrive over time.  The scheduler admits an
arrived request when a slot is free and its device footprint fits in the remaining HBM
budget; each slot owns a HIP stream and a host worker that runs setup -> right-hand side ->
solve for its request through the C ABI, so the device work of all admitted requests
overlaps.  When a solve completes, its operator and vectors are released and the next
arrived request is admitted.  Latency = completion - arrival.

The admission and ordering logic (Scheduler) is plain host code and is tested on the CPU
with fake footprints; Server binds it to the library.
"""

from __future__ import annotations

import heapq
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass(order=True)
class _Pending:
    arrival: float
    rid: int
    footprint: int = field(compare=False)
    payload: object = field(compare=False, default=None)


class Scheduler:
    """First-come-first-served admission by arrival time, bounded by slots and a byte budget.

    A request whose footprint exceeds the whole budget is rejected (never admitted).
    Head-of-line: a request that does not fit yet blocks later ones (keeps FCFS order)."""

    def __init__(self, budget_bytes: int, slots: int):
        if budget_bytes <= 0 or slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.used = 0
        self.active = {}
        self.pending = []
        self.rejected = []

    def submit(self, rid, arrival, footprint, payload=None):
        if footprint > self.budget:
            self.rejected.append(rid)
            return False
        heapq.heappush(self.pending, _Pending(float(arrival), int(rid), int(footprint), payload))
        return True

    def admit(self, now, limit=None):
        """Pop every request that has arrived by `now` and fits (at most `limit` of them);
        returns [(rid, payload)]."""
        out = []
        while (self.pending and self.pending[0].arrival <= now and len(self.active) < self.slots
               and (limit is None or len(out) < limit)):
            head = self.pending[0]
            if self.used + head.footprint > self.budget:
                break
            heapq.heappop(self.pending)
            self.used += head.footprint
            self.active[head.rid] = head.footprint
            out.append((head.rid, head.payload))
        return out

    def release(self, rid):
        self.used -= self.active.pop(rid)

    def idle(self):
        return not self.pending and not self.active


def _up(b: int) -> int:
    return (int(b) + 255) // 256 * 256


def workspace_bytes(n_dofs: int, restart: int, mixed: bool, jacobi: bool = False) -> int:
    """Device bytes of the solver workspace sbm_solve allocates for GMRES(restart) on n_dofs
    unknowns, piece by piece as the library carves it (every piece on a 256-byte boundary):
    FP64 basis of restart + 1 row-tiled columns, five FP64 work vectors, the block partials of
    the reductions (1024 blocks) and the small Hessenberg state; in the mixed mode the FP32
    basis and five FP32 work vectors; with Jacobi the FP64 (and FP32) inverse diagonal."""
    n = max(1, int(n_dofs))
    m = int(restart)
    npad = (n + 127) // 128 * 128
    b = _up(8 * npad * (m + 1)) + 5 * _up(8 * n) + _up(8 * 1024 * (m + 2)) + _up(8 * 3 * (m + 2))
    b += _up(8 * (m + 2)) + _up(8 * ((m + 1) * m + 4 * m + 2)) + _up(4)
    if mixed:
        b += _up(4 * npad * (m + 1)) + 5 * _up(4 * n)
    if jacobi:
        b += 8 * n + (4 * n if mixed else 0)
    return b


def footprint_bytes(n_dofs: int, device_bytes: int, restart: int, mixed: bool, jacobi: bool = False) -> int:
    """Device bytes a solve holds: operator data and scratch + b, x + the solver workspace."""
    return int(device_bytes + 16 * n_dofs + workspace_bytes(n_dofs, restart, mixed, jacobi))


def _phi_sign(ls, x):
    """Level-set value for the admission estimate (sign only matters)."""
    d = x.shape[1]
    k = ls["kind"]
    if k == "sphere":
        return np.linalg.norm(x - np.asarray(ls["centre"][:d]), axis=1) - ls["radius"]
    if k == "ellipsoid":
        return np.sum(((x - np.asarray(ls["centre"][:d])) / np.asarray(ls["semi_axes"][:d])) ** 2, axis=1) - 1.0
    if k == "torus":
        y = x - np.asarray(ls["centre"])
        return np.hypot(np.hypot(y[:, 0], y[:, 1]) - ls["R"], y[:, 2]) - ls["r"]
    if k == "halfspace":
        return x @ np.asarray(ls["normal"][:d]) - ls["offset"]
    if k == "sphere_union":
        cs = np.asarray(ls["centres"])[:, :d]
        return np.min(np.linalg.norm(x[:, None, :] - cs[None], axis=2) - np.asarray(ls["radii"])[None], axis=1)
    raise KeyError(k)


def count_inside_cells(req) -> int:
    """Background cells with all vertices strictly inside the domain."""
    d, n = req["d"], int(req["n"])
    lo, hi = float(req["lo"]), float(req["hi"])
    g = lo + (hi - lo) / n * np.arange(n + 1)
    pts = np.stack(np.meshgrid(*([g] * d), indexing="ij"), -1).reshape(-1, d)
    inside = (_phi_sign(req["levelset"], pts) < 0).reshape([n + 1] * d)
    act = np.ones([n] * d, dtype=bool)
    for off in np.ndindex(*([2] * d)):
        act &= inside[tuple(slice(o, o + n) for o in off)]
    return int(act.sum())


def problem_data(op, req):
    """The request's problem data for sbm_rhs: f of the manufactured solution at the cells'
    Gauss points (from the cells' corners by its product structure) and g = u* at the
    true-boundary points of the surrogate faces."""
    from . import inputs
    d = req["d"]
    u_fn, _ = inputs.manufactured(d)
    _, bp = op.rhs_points(cells=False)
    f_qp = inputs.manufactured_cell_f(d, op.export_cells(), req["lo"], (req["hi"] - req["lo"]) / req["n"], req["p"])
    return f_qp, u_fn(bp.reshape(-1, d))


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else float("nan")


class Server:
    """Runs a request stream on the GPU through the library (see module docstring)."""

    def __init__(self, budget_bytes, slots=4, mode="gmres_ir", rel_tol=1e-10, max_it=400, restart=32,
                 taylor_order=None, jacobi=False, solver_graphs=False):
        """taylor_order: extension of the surrogate-face term for requests that do not name one
        (None: the full extension; m >= 0: the Taylor expansion kept to order m)."""
        self.sched = Scheduler(budget_bytes, slots)
        self.mode, self.rel_tol, self.max_it, self.restart = mode, rel_tol, max_it, restart
        self.jacobi = bool(jacobi)
        # the solver's graph capture stays off in the slots (see the serving notes of the design)
        self.solver_graphs = bool(solver_graphs)
        self.taylor_order = taylor_order
        self.lock = threading.Lock()
        self.done = threading.Condition(self.lock)
        self.results = {}

    def _estimate(self, req):
        """Upper-bound footprint from the number of background cells whose vertices are all
        inside the domain (vectorised vertex test; no setup): the library's bound of the
        operator's device data (at most 2d surrogate faces per cell) plus b, x and the exact
        workspace layout of the solve for at most n_cells (p+1)^d unknowns."""
        from . import sbm
        n_cells = count_inside_cells(req)
        nb = (req["p"] + 1) ** req["d"]
        n_dofs = n_cells * nb  # bound for CG, exact for DG
        dev = sbm.footprint_estimate(req["d"], req["n"], req["lo"], req["hi"], req["p"], req["disc"], n_cells,
                                     2 * req["d"] * n_cells)
        return footprint_bytes(n_dofs, dev, self.restart, self.mode == "gmres_ir", self.jacobi), n_dofs

    def solve_one(self, req, stream=None):
        """Setup, right-hand side and solve of one request on `stream`; returns (x, info)."""
        import torch

        from . import sbm
        op = sbm.Operator(req["d"], req["n"], req["lo"], req["hi"], req["levelset"], req["p"], disc=req["disc"],
                          taylor_order=req.get("taylor_order", self.taylor_order), solver_graphs=self.solver_graphs)
        try:
            f_qp, g_bp = problem_data(op, req)
            with torch.cuda.stream(stream) if stream is not None else _null():
                b = torch.empty(op.n_dofs, dtype=torch.float64, device="cuda")
                op.rhs(f_qp, g_bp, b, stream=stream)
                x = torch.zeros_like(b)
                info = op.solve(b, x, rel_tol=self.rel_tol, max_it=self.max_it, mode=self.mode,
                                restart=self.restart, jacobi=self.jacobi, stream=stream)
                info["device_bytes"] = op.device_bytes
                xh = x.cpu().numpy() if stream is None else _to_host(x, stream)
            info["n_dofs"] = op.n_dofs
            info["disc"], info["p"] = req["disc"], req["p"]
            return xh, info
        finally:
            op.close()

    def run(self, requests, time_scale=1.0, keep_solutions=False, deadline_s=None):
        """Serve `requests` (dicts with 'id' and 'arrival' seconds).  Arrival times are
        scaled by time_scale (0 = all present at t=0, closed loop).  deadline_s: no request is
        admitted after this many seconds (the ones admitted finish; the rest are reported as
        not served).  Returns a summary."""
        import torch

        reqs = {r["id"]: r for r in requests}
        for r in requests:
            fp, nd = self._estimate(r)
            r["_footprint"], r["_n_dofs"] = fp, nd
            self.sched.submit(r["id"], r["arrival"] * time_scale, fp, r)
        streams = [torch.cuda.Stream() for _ in range(self.sched.slots)]
        free_streams = list(range(self.sched.slots))
        t0 = time.perf_counter()
        threads = []

        def worker(rid, req, si):
            t_start = time.perf_counter() - t0
            try:
                x, info = self.solve_one(req, streams[si])
                err = None
            except Exception as exc:  # a failed request is reported, the server keeps running
                x, info, err = None, {}, repr(exc)
            t_end = time.perf_counter() - t0
            with self.lock:
                self.results[rid] = dict(id=rid, arrival=req["arrival"] * time_scale, start=t_start, end=t_end,
                                         latency=t_end - req["arrival"] * time_scale, error=err,
                                         info=info, x=x if keep_solutions else None)
                self.sched.release(rid)
                free_streams.append(si)
                self.done.notify_all()

        with self.lock:
            while not self.sched.idle():
                now = time.perf_counter() - t0
                if deadline_s is not None and now > deadline_s:
                    self.sched.pending.clear()  # stop admitting; wait for the admitted ones
                    if self.sched.idle():
                        break
                    self.done.wait(timeout=0.05)
                    continue
                for rid, req in self.sched.admit(now):
                    si = free_streams.pop()
                    th = threading.Thread(target=worker, args=(rid, req, si), daemon=True)
                    threads.append(th)
                    th.start()
                if self.sched.idle():
                    break
                nxt = self.sched.pending[0].arrival - now if self.sched.pending else None
                self.done.wait(timeout=max(1e-3, nxt) if nxt is not None and nxt > 0 else 0.05)
        for th in threads:
            th.join()
        wall = time.perf_counter() - t0
        lat = [r["latency"] for r in self.results.values() if r["error"] is None]
        ok = [r for r in self.results.values() if r["error"] is None and r["info"].get("status") == 0]
        lat_ok = [r["latency"] for r in ok]
        first_arrival = min((r["arrival"] for r in self.results.values()), default=0.0)
        last_end = max((r["end"] for r in self.results.values()), default=0.0)
        span = max(1e-9, last_end - first_arrival)
        return {
            "requests": len(requests), "served": len(self.results), "rejected": list(self.sched.rejected),
            "converged": len(ok), "errors": sum(1 for r in self.results.values() if r["error"]),
            "solves_per_s": len(self.results) / span, "converged_solves_per_s": len(ok) / span,
            "latency_p50_s": percentile(lat, 50), "latency_p99_s": percentile(lat, 99),
            "converged_latency_p50_s": percentile(lat_ok, 50), "converged_latency_p99_s": percentile(lat_ok, 99),
            "wall_s": wall, "results": self.results,
        }


def _prepare_set(server, batch):
    """Operators, right-hand sides and zero initial guesses of an admitted set; returns the
    prepared items [(rid, req, op, b, x)] and the setup failures [(rid, req, error)]."""
    import torch

    from . import sbm
    items, failed = [], []
    for rid, req in batch:
        try:
            op = sbm.Operator(req["d"], req["n"], req["lo"], req["hi"], req["levelset"], req["p"], disc=req["disc"],
                              taylor_order=req.get("taylor_order", server.taylor_order), solver_graphs=False)
        except Exception as exc:  # a failed setup is reported; the others go on
            failed.append((rid, req, repr(exc)))
            continue
        try:
            f_qp, g_bp = problem_data(op, req)
            b = torch.empty(op.n_dofs, dtype=torch.float64, device="cuda")
            op.rhs(f_qp, g_bp, b)  # synchronous
        except Exception as exc:
            op.close()
            failed.append((rid, req, repr(exc)))
            continue
        items.append((rid, req, op, b, torch.zeros_like(b)))
    return items, failed


def run_batched(server, requests, time_scale=1.0, deadline_s=None, keep_solutions=False, set_size=None,
                prefetch=False):
    """Serve `requests` in lockstep sets: the scheduler admits up to set_size arrived requests
    that fit (the server's slots and HBM budget), their operators and right-hand sides are set
    up, and the whole set is solved together by sbm_solve_batch (each Krylov step's applies of
    all of them in one batch of launches).  prefetch: while a set is solving, one host thread
    admits and sets up the next one (both sets then hold slots and HBM: give the server twice
    set_size slots), so the host's setup overlaps the device's solves.  Requests that arrive
    while a set is solving wait for a later set.  Same summary as Server.run, plus the time
    spent preparing sets and solving them."""
    from concurrent.futures import ThreadPoolExecutor

    from . import sbm
    sched = server.sched
    set_size = set_size or sched.slots
    for r in requests:
        fp, nd = server._estimate(r)
        r["_footprint"], r["_n_dofs"] = fp, nd
        sched.submit(r["id"], r["arrival"] * time_scale, fp, r)
    t0 = time.perf_counter()
    results = {}
    t_setup = t_solve = 0.0
    sets = 0
    pool = ThreadPoolExecutor(max_workers=1) if prefetch else None

    def prepare(batch):
        t = time.perf_counter()
        items, failed = _prepare_set(server, batch)
        return items, failed, t - t0, time.perf_counter() - t

    def record_failures(failed, starts):
        for rid, req, err in failed:
            end = time.perf_counter() - t0
            results[rid] = dict(id=rid, arrival=req["arrival"] * time_scale, start=starts, end=end, error=err,
                                latency=end - req["arrival"] * time_scale, info={}, x=None)
            sched.release(rid)

    def admit_next(block):
        """Admit the next set (waiting for arrivals if block); None when nothing is left."""
        while not sched.idle():
            now = time.perf_counter() - t0
            if deadline_s is not None and now > deadline_s:
                sched.pending.clear()
                return None
            batch = sched.admit(now, limit=set_size)
            if batch or not block:
                return batch or None
            nxt = sched.pending[0].arrival - now if sched.pending else 0.0
            time.sleep(min(0.05, max(1e-3, nxt)))
        return None

    try:
        current = None
        while True:
            if current is None:
                batch = admit_next(block=True)
                if batch is None:
                    break
                current = prepare(batch)
            items, failed, starts, prep_s = current
            t_setup += prep_s
            record_failures(failed, starts)
            fut = None
            if pool is not None:
                nxt = admit_next(block=False)
                if nxt:
                    fut = pool.submit(prepare, nxt)
            sets += 1
            t_solve0 = time.perf_counter()
            err = None
            try:
                infos = sbm.solve_batch([it[2] for it in items], [it[3] for it in items], [it[4] for it in items],
                                        rel_tol=server.rel_tol, max_it=server.max_it, mode=server.mode,
                                        restart=server.restart) if items else []
            except Exception as exc:  # reported for every request of the set; the server goes on
                infos, err = [{} for _ in items], repr(exc)
            end = time.perf_counter() - t0
            t_solve += time.perf_counter() - t_solve0
            try:
                for (rid, req, op, b, x), info in zip(items, infos):
                    info = dict(info, n_dofs=op.n_dofs, disc=req["disc"], p=req["p"], device_bytes=op.device_bytes)
                    results[rid] = dict(id=rid, arrival=req["arrival"] * time_scale, start=starts, end=end,
                                        error=err, latency=end - req["arrival"] * time_scale, info=info,
                                        x=x.cpu().numpy() if keep_solutions and err is None else None)
            finally:
                for rid, req, op, b, x in items:
                    op.close()
                    sched.release(rid)
            current = fut.result() if fut is not None else None
    finally:
        if pool is not None:
            pool.shutdown(wait=True)
    wall = time.perf_counter() - t0
    lat = [r["latency"] for r in results.values() if r["error"] is None]
    ok = [r for r in results.values() if r["error"] is None and r["info"].get("status") == 0]
    first_arrival = min((r["arrival"] for r in results.values()), default=0.0)
    last_end = max((r["end"] for r in results.values()), default=0.0)
    span = max(1e-9, last_end - first_arrival)
    return {
        "requests": len(requests), "served": len(results), "rejected": list(sched.rejected),
        "converged": len(ok), "errors": sum(1 for r in results.values() if r["error"]),
        "solves_per_s": len(results) / span, "converged_solves_per_s": len(ok) / span,
        "latency_p50_s": percentile(lat, 50), "latency_p99_s": percentile(lat, 99),
        "converged_latency_p50_s": percentile([r["latency"] for r in ok], 50),
        "converged_latency_p99_s": percentile([r["latency"] for r in ok], 99),
        "wall_s": wall, "sets": sets, "setup_and_rhs_s": t_setup, "lockstep_solve_s": t_solve,
        "results": results,
    }


class _null:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def _to_host(x, stream):
    stream.synchronize()
    return x.cpu().numpy()
