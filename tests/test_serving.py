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


def test_footprint_counts_workspace():
    assert footprint_bytes(1000, 0, 32, False) == 16 * 1000 + 8 * 1000 * 37
    assert footprint_bytes(1000, 0, 32, True) > footprint_bytes(1000, 0, 32, False)


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
    from oracle import sbm_oracle as O

    for r in reqs:
        x_alone, info = alone.solve_one(r)
        x_mix = summary["results"][r["id"]]["x"]
        rr_alone, rr_mix = info["rel_residual"], summary["results"][r["id"]]["info"]["rel_residual"]
        assert info["status"] == 0 and rr_alone <= 1e-10 and rr_mix <= 1e-10
        # Both are solutions of the same system to the same residual; the applies sum with
        # atomics, so the iterates differ at rounding level and the solutions within the
        # perturbation bound |x1 - x2| / |x| <= cond(A) (r1 + r2) (relative residuals).
        ref = O.setup(r["d"], r["n"], r["lo"], r["hi"], r["levelset"], r["p"], disc=r["disc"])
        sv = np.linalg.svd(O.assemble(ref).toarray(), compute_uv=False)
        bound = sv[0] / sv[-1] * (rr_alone + rr_mix)
        rel = np.linalg.norm(x_mix - x_alone) / np.linalg.norm(x_alone)
        assert rel <= bound, (r["id"], rel, bound)
    torch.cuda.synchronize()


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
