"""Serving: host-side admission logic (CPU) and the alone-vs-in-the-mix property (GPU)."""

import numpy as np
import pytest

from paper_2507_17053_amd import inputs
from paper_2507_17053_amd.serving import Scheduler, count_inside_cells, footprint_bytes


def test_scheduler_respects_budget_slots_and_order():
    s = Scheduler(budget_bytes=100, slots=2)
    assert s.submit(0, 0.0, 60)
    assert s.submit(1, 0.5, 30)
    assert s.submit(2, 0.7, 30)
    assert not s.submit(3, 0.1, 200)          # larger than the whole budget: rejected
    assert s.rejected == [3]
    assert s.admit(0.0) == [(0, None)]         # 1 has not arrived yet
    assert s.admit(1.0) == [(1, None)]         # 2 would exceed slots
    assert s.used == 90 and len(s.active) == 2
    s.release(0)
    assert s.admit(1.0) == [(2, None)]
    assert s.used == 60
    s.release(1)
    s.release(2)
    assert s.idle() and s.used == 0


def test_scheduler_head_of_line_keeps_fcfs():
    s = Scheduler(budget_bytes=100, slots=4)
    s.submit(0, 0.0, 80)
    s.submit(1, 0.1, 50)   # does not fit while 0 runs
    s.submit(2, 0.2, 10)   # would fit, but must wait behind 1 (first come, first served)
    assert [r for r, _ in s.admit(1.0)] == [0]
    assert s.admit(1.0) == []
    s.release(0)
    assert [r for r, _ in s.admit(1.0)] == [1, 2]


def test_scheduler_limit_caps_a_set_and_keeps_order():
    """admit(limit=k) takes at most k of the arrived requests, in arrival order, the rest stay
    queued for the next set (the lockstep sets of the serving loop)."""
    s = Scheduler(budget_bytes=1000, slots=8)
    for i in range(7):
        s.submit(i, 0.1 * i, 10)
    assert [r for r, _ in s.admit(10.0, limit=3)] == [0, 1, 2]
    assert [r for r, _ in s.admit(10.0, limit=3)] == [3, 4, 5]   # a second set while the first holds slots
    assert [r for r, _ in s.admit(10.0, limit=3)] == [6]
    assert s.admit(10.0, limit=3) == []
    for i in range(7):
        s.release(i)
    assert s.idle() and s.used == 0
    s2 = Scheduler(budget_bytes=1000, slots=2)
    for i in range(4):
        s2.submit(i, 0.0, 10)
    assert [r for r, _ in s2.admit(1.0, limit=3)] == [0, 1]        # slots bind before the limit


def test_problem_data_by_product_structure_equals_pointwise():
    """The serving loop's f at the cell Gauss points, formed per cell from one-dimensional
    factors, equals f evaluated point by point at the library's Gauss points, bit for bit."""
    from paper_2507_17053_amd import sbm
    from paper_2507_17053_amd.serving import problem_data
    for d, n, ls, p in [(3, 8, inputs.ellipsoid((0, 0, 0), (0.7, 0.6, 0.5)), 4),
                        (2, 12, inputs.sphere((0.05, -0.03), 0.7), 3),
                        (3, 16, inputs.sphere_union(1003), 6)]:
        op = sbm.Operator(d, n, -1.0, 1.0, ls, p, host_only=True)
        try:
            cq, bp = op.rhs_points()
            u_fn, f_fn = inputs.manufactured(d)
            f_qp, g_bp = problem_data(op, dict(d=d, n=n, lo=-1.0, hi=1.0, p=p))
            assert f_qp.shape == (op.n_cells, (p + 1) ** d)
            assert np.array_equal(f_qp, f_fn(cq.reshape(-1, d)).reshape(op.n_cells, -1))
            assert np.array_equal(g_bp, u_fn(bp.reshape(-1, d)))
        finally:
            op.close()


def test_footprint_counts_workspace():
    from paper_2507_17053_amd.serving import workspace_bytes
    # the FP64 basis alone is (m + 1) row-tiled columns; the mixed mode adds the FP32 copies
    assert workspace_bytes(1000, 32, False) >= 8 * 1024 * 33 + 5 * 8 * 1000
    assert footprint_bytes(1000, 0, 32, False) == 16 * 1000 + workspace_bytes(1000, 32, False)
    assert footprint_bytes(1000, 0, 32, True) > footprint_bytes(1000, 0, 32, False)
    assert footprint_bytes(1000, 0, 32, True, jacobi=True) == footprint_bytes(1000, 0, 32, True) + 12 * 1000


def test_inside_cell_count_matches_setup():
    sbm = pytest.importorskip("paper_2507_17053_amd.sbm")
    for w in (inputs.workload("disk2d_q2"), inputs.workload("spheres3d_q6", n=24)):
        op = sbm.Operator(w["d"], w["n"], w["lo"], w["hi"], w["levelset"], w["p"], host_only=True)
        assert count_inside_cells(w) == op.n_cells


def test_request_stream_is_seeded():
    a = inputs.serving_requests(20, seed=3)
    b = inputs.serving_requests(20, seed=3)
    assert [r["p"] for r in a] == [r["p"] for r in b]
    assert all(2 <= r["p"] <= 6 and 16 <= r["n"] <= 64 for r in a)
    assert np.all(np.diff([r["arrival"] for r in a]) > 0)


SOLVABLE = [
    dict(d=2, n=16, lo=-1.0, hi=1.0, p=2, disc="cg", levelset=inputs.sphere((0.05, -0.03), 0.7)),
    dict(d=2, n=16, lo=-1.0, hi=1.0, p=1, disc="cg", levelset=inputs.sphere((0.05, -0.03), 0.7)),
    dict(d=2, n=8, lo=-1.0, hi=1.0, p=2, disc="dg", levelset=inputs.sphere((0.05, -0.03), 0.7)),
    dict(d=3, n=8, lo=-1.0, hi=1.0, p=1, disc="cg", levelset=inputs.sphere((0, 0, 0), 0.75)),
    dict(d=3, n=6, lo=-1.0, hi=1.0, p=2, disc="dg", levelset=inputs.sphere((0, 0, 0), 0.75)),
    dict(d=2, n=12, lo=-1.0, hi=1.0, p=1, disc="dg", levelset=inputs.ellipsoid((0, 0), (0.8, 0.6))),
]


@pytest.mark.gpu
def test_each_result_same_alone_and_in_the_mix():
    torch = pytest.importorskip("torch")
    from paper_2507_17053_amd.serving import Server

    reqs = [dict(r, id=i, arrival=0.01 * i) for i, r in enumerate(SOLVABLE)]
    srv = Server(budget_bytes=8 << 30, slots=3, mode="gmres_ir", rel_tol=1e-10, max_it=8000, restart=64)
    summary = srv.run(reqs, time_scale=1.0, keep_solutions=True)
    errs = {rid: r["error"] for rid, r in summary["results"].items() if r["error"]}
    assert summary["served"] == len(reqs) and summary["errors"] == 0, errs
    assert summary["converged"] == len(reqs)
    # overlap happened: some request started before another finished
    res = sorted(summary["results"].values(), key=lambda r: r["start"])
    assert any(res[i + 1]["start"] < res[i]["end"] for i in range(len(res) - 1))
    alone = Server(budget_bytes=8 << 30, slots=1, mode="gmres_ir", rel_tol=1e-10, max_it=8000, restart=64)
    for r in reqs:
        x_alone, info = alone.solve_one(r)
        x_mix = summary["results"][r["id"]]["x"]
        rr_alone, rr_mix = info["rel_residual"], summary["results"][r["id"]]["info"]["rel_residual"]
        assert info["status"] == 0 and rr_alone <= 1e-10 and rr_mix <= 1e-10
        # The applies take every sum in a fixed order and the solver's reductions are block
        # partials added in a fixed order, so a request's solve does not depend on what else
        # runs on the device: the result is the same bit for bit.
        rel = np.linalg.norm(x_mix - x_alone) / np.linalg.norm(x_alone)
        print(f"  request {r['id']}: |x_mix - x_alone| / |x_alone| = {rel:.3e}", flush=True)
        assert np.array_equal(x_mix, x_alone), (r["id"], rel)
    torch.cuda.synchronize()


@pytest.mark.gpu
@pytest.mark.parametrize("prefetch", [False, True], ids=["sequential", "prefetch"])
def test_batched_serving_same_alone_and_in_the_mix(prefetch):
    """Lockstep batched serving (all admitted requests solved together, each Krylov step's
    applies in one batch of launches), with the next set prepared on a host thread during the
    solve or not: every request converges and its solution equals the one it gets alone, bit
    for bit; each set holds at most set_size requests."""
    torch = pytest.importorskip("torch")
    from paper_2507_17053_amd.serving import Server, run_batched

    reqs = [dict(r, id=i, arrival=0.0) for i, r in enumerate(SOLVABLE)]
    srv = Server(budget_bytes=8 << 30, slots=8, mode="gmres_ir", rel_tol=1e-10, max_it=8000, restart=64)
    summary = run_batched(srv, reqs, time_scale=0.0, keep_solutions=True, set_size=4, prefetch=prefetch)
    errs = {rid: r["error"] for rid, r in summary["results"].items() if r["error"]}
    assert summary["served"] == len(reqs) and summary["errors"] == 0, errs
    assert summary["converged"] == len(reqs)
    starts = sorted({r["start"] for r in summary["results"].values()})
    assert len(starts) == 2  # 6 requests, 4 slots: two sets
    alone = Server(budget_bytes=8 << 30, slots=1, mode="gmres_ir", rel_tol=1e-10, max_it=8000, restart=64)
    for r in reqs:
        x_alone, info = alone.solve_one(r)
        got = summary["results"][r["id"]]
        for k in ("status", "outer_its", "inner_its", "applies_f64", "applies_f32", "rel_residual"):
            assert got["info"][k] == info[k], (r["id"], k)
        assert np.array_equal(got["x"], x_alone), r["id"]
    torch.cuda.synchronize()


@pytest.mark.gpu
@pytest.mark.parametrize("mode,jacobi", [("gmres", False), ("gmres_ir", True)])
def test_admission_estimate_bounds_what_a_solve_holds(mode, jacobi):
    """The server's admission estimate is at least the device bytes the request's handle holds
    after its solve (operator data and scratch + solver workspace, from sbm_info) plus b and x."""
    pytest.importorskip("torch")
    from paper_2507_17053_amd.serving import Server

    srv = Server(budget_bytes=8 << 30, slots=1, mode=mode, rel_tol=1e-10, max_it=50, restart=32, jacobi=jacobi)
    for i, r in enumerate(SOLVABLE + [dict(d=3, n=16, lo=-1.0, hi=1.0, p=4, disc="cg",
                                           levelset=inputs.sphere_union(1))]):
        req = dict(r, id=i, arrival=0.0)
        est, n_dofs_bound = srv._estimate(req)
        _, info = srv.solve_one(req)
        held = info["device_bytes"] + 16 * info["n_dofs"]
        assert info["n_dofs"] <= n_dofs_bound
        assert est >= held, (i, est, held)


@pytest.mark.gpu
def test_request_extension_order_reaches_the_operator():
    """A request naming taylor_order = 1 is solved with the first-order extension: its
    solution solves the oracle's E_1 system (and not the full-extension one)."""
    pytest.importorskip("torch")
    from paper_2507_17053_amd.serving import Server
    from oracle import sbm_oracle as O

    r = dict(SOLVABLE[0], id=0, arrival=0.0, taylor_order=1)
    srv = Server(budget_bytes=8 << 30, slots=1, mode="gmres", rel_tol=1e-10, max_it=8000, restart=64)
    x, info = srv.solve_one(r)
    assert info["status"] == 0, info
    u_fn, f_fn = inputs.manufactured(r["d"])
    for m, ok in ((1, True), (None, False)):
        ref = O.setup(r["d"], r["n"], r["lo"], r["hi"], r["levelset"], r["p"], disc=r["disc"], taylor_order=m)
        b = O.rhs(ref, f_fn, u_fn)
        res = np.linalg.norm(b - O.assemble(ref) @ x) / np.linalg.norm(b)
        assert (res <= 2e-10) == ok, (m, res)
