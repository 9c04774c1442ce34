"""Batched applies across operators (sbm_apply_batch, sbm_batch_create / run / destroy).

Operators that share a kernel instantiation run in one launch per stage; every result must be
bitwise the operator's own sbm_apply (the single apply is held to the FP64 oracle by the apply
parity tests).  The mix covers CG and DG, 2D and 3D, several degrees, groups with several
operators of different mesh sizes, the two DG cell-kernel forms (parallel faces at p <= 3,
face by face above), the 2D and 3D DG face kernels, a truncated extension inside a group and a
high-degree brick."""

import pytest

from paper_2507_17053_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sbm = pytest.importorskip("paper_2507_17053_amd.sbm")

MIX = [
    dict(d=3, n=10, ls=inputs.sphere((0, 0, 0), 0.75), p=4, disc="cg"),
    dict(d=3, n=12, ls=inputs.ellipsoid((0.0, 0.02, -0.01), (0.8, 0.6, 0.7)), p=4, disc="cg"),
    dict(d=3, n=8, ls=inputs.torus(0.55, 0.4), p=4, disc="cg", taylor=1),
    dict(d=2, n=16, ls=inputs.sphere((0.05, -0.03), 0.7), p=2, disc="cg"),
    dict(d=2, n=20, ls=inputs.ellipsoid((0.02, 0.01), (0.8, 0.45)), p=2, disc="cg"),
    dict(d=3, n=6, ls=inputs.sphere((0, 0, 0), 0.75), p=2, disc="dg"),
    dict(d=3, n=8, ls=inputs.torus(0.55, 0.4), p=2, disc="dg"),
    dict(d=3, n=6, ls=inputs.sphere((0, 0, 0), 0.75), p=3, disc="dg"),
    dict(d=3, n=5, ls=inputs.sphere((0, 0, 0), 0.75), p=5, disc="dg"),
    dict(d=2, n=9, ls=inputs.sphere((0.05, -0.03), 0.7), p=3, disc="dg"),
    dict(d=3, n=5, ls=inputs.sphere((0, 0, 0), 0.75), p=7, disc="cg"),
]


def _ops(cases):
    ops = []
    for c in cases:
        ops.append(sbm.Operator(c["d"], c["n"], -1.0, 1.0, c["ls"], c["p"], disc=c["disc"],
                                taylor_order=c.get("taylor")))
    return ops


def _vectors(ops, dtype, seed0):
    us = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=seed0 + i)).to("cuda", dtype)
          for i, o in enumerate(ops)]
    vs = [torch.full_like(u, 7.0) for u in us]
    return us, vs


def _singles(ops, us):
    refs = []
    for o, u in zip(ops, us):
        r = torch.empty_like(u)
        o.apply(u, r)
        refs.append(r)
    torch.cuda.synchronize()
    return refs


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batch_mix_is_bitwise_single_applies(dtype):
    print(f"batch mix {dtype}", flush=True)
    ops = _ops(MIX)
    try:
        us, vs = _vectors(ops, dtype, 100)
        refs = _singles(ops, us)
        sbm.apply_batch(ops, us, vs)
        torch.cuda.synchronize()
        for c, v, r in zip(MIX, vs, refs):
            assert torch.equal(v, r), c
        # the caller's order does not matter: reversed, and a second one-shot batch right after
        vs2 = [torch.full_like(u, -3.0) for u in us]
        sbm.apply_batch(ops[::-1], us[::-1], vs2[::-1])
        sbm.apply_batch(ops[:3], us[:3], vs[:3])
        torch.cuda.synchronize()
        for c, v, v2, r in zip(MIX, vs, vs2, refs):
            assert torch.equal(v2, r), c
            assert torch.equal(v, r), c
    finally:
        for o in ops:
            o.close()


@pytest.mark.parametrize("dtype,graph,streams", [(torch.float64, True, 4), (torch.float32, True, 4),
                                                  (torch.float64, False, 4), (torch.float64, True, 1)],
                         ids=["f64-graph-4streams", "f32-graph-4streams", "f64-eager-4streams", "f64-graph-1stream"])
def test_batch_plan_replays(dtype, graph, streams):
    """A prepared batch (groups forked over the batch's streams, or all on the run's stream;
    captured into a graph on a side stream, or launched directly): three runs with new inputs
    written into the same vectors between them (and eager work in between), each run equal bit
    for bit to the single applies of that input."""
    print(f"batch plan {dtype} graph={graph} streams={streams}", flush=True)
    ops = _ops(MIX)
    s = torch.cuda.Stream()
    try:
        us, vs = _vectors(ops, dtype, 200)
        with sbm.Batch(ops, us, vs, graph=graph, streams=streams) as b:
            for rep in range(3):
                for i, u in enumerate(us):
                    u.copy_(torch.from_numpy(inputs.uniform_vector(u.numel(), seed=300 + 17 * rep + i)).to(dtype))
                torch.cuda.synchronize()
                b.run(s)
                s.synchronize()
                refs = _singles(ops, us)
                for c, v, r in zip(MIX, vs, refs):
                    assert torch.equal(v, r), (rep, c)
                for v in vs:
                    v.fill_(5.0)  # eager work between replays; the next replay rewrites every entry
                torch.cuda.synchronize()
    finally:
        for o in ops:
            o.close()


def test_batch_rejects_overlapping_arguments():
    ops = _ops(MIX[:1] + MIX[:1] + MIX[5:6])  # the first two alike (same sizes)
    try:
        us, vs = _vectors(ops, torch.float64, 400)
        with pytest.raises(sbm.SbmError):
            sbm.apply_batch([ops[0], ops[0]], [us[0], us[1]], [vs[0], vs[1]])  # one handle twice
        with pytest.raises(sbm.SbmError):
            sbm.Batch([ops[0], ops[1]], [us[0], vs[0]], [vs[0], vs[1]])  # an input is another's output
        with pytest.raises(sbm.SbmError):
            sbm.apply_batch([ops[0], ops[1]], [us[0], us[1]], [vs[0], vs[0]])  # one output twice
        with pytest.raises(ValueError):
            sbm.apply_batch(ops, us, vs[:2])
        with pytest.raises(ValueError):
            sbm.apply_batch(ops[1:], [us[2], us[1]], vs[1:])  # sizes do not match the operators
        sbm.apply_batch([], [], [])  # empty batch: no-op
        b = sbm.Batch(ops, us, vs, graph=False)
        b.run()
        b.close()
        b.close()
        with pytest.raises(sbm.SbmError):
            b.run()
        torch.cuda.synchronize()
    finally:
        for o in ops:
            o.close()


SOLVE_MIX = [
    dict(d=2, n=16, ls=inputs.sphere((0.05, -0.03), 0.7), p=2, disc="cg"),
    dict(d=2, n=13, ls=inputs.ellipsoid((0.02, 0.01), (0.8, 0.45)), p=1, disc="cg"),
    dict(d=2, n=9, ls=inputs.sphere((0.05, -0.03), 0.7), p=3, disc="dg"),
    dict(d=3, n=8, ls=inputs.sphere((0, 0, 0), 0.75), p=1, disc="cg"),
    dict(d=3, n=8, ls=inputs.sphere((0, 0, 0), 0.75), p=4, disc="cg"),
    dict(d=3, n=6, ls=inputs.sphere((0, 0, 0), 0.75), p=2, disc="dg"),
    dict(d=3, n=8, ls=inputs.torus(0.55, 0.4), p=2, disc="cg", taylor=1),
]
INFO_KEYS = ("status", "outer_its", "inner_its", "applies_f64", "applies_f32", "rel_residual")


@pytest.mark.parametrize("mode", ["gmres", "gmres_ir"])
def test_solve_batch_is_bitwise_single_solves(mode):
    """Lockstep batched GMRES (FP64, and FP32 inside FP64 refinement) over operators of
    different kinds: every solution and every solve report equals the operator's own sbm_solve,
    bit for bit, whether the system converges within the iteration bound or not."""
    print(f"solve batch {mode}", flush=True)
    ops = _ops(SOLVE_MIX)
    try:
        bs = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=500 + i)).to("cuda") for i, o in enumerate(ops)]
        x0 = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=600 + i, lo=-0.1, hi=0.1)).to("cuda")
              for i, o in enumerate(ops)]
        xs_single = [x.clone() for x in x0]
        ref = [o.solve(b, x, rel_tol=1e-10, max_it=150, mode=mode, restart=20) for o, b, x in zip(ops, bs, xs_single)]
        xs = [x.clone() for x in x0]
        infos = sbm.solve_batch(ops, bs, xs, rel_tol=1e-10, max_it=150, mode=mode, restart=20)
        torch.cuda.synchronize()
        assert any(r["status"] == sbm.SBM_OK for r in ref)  # the mix has converging systems
        for c, r, inf, x, xr in zip(SOLVE_MIX, ref, infos, xs, xs_single):
            for k in INFO_KEYS:
                assert inf[k] == r[k], (c, k, inf[k], r[k])
            assert torch.equal(x, xr), c
    finally:
        for o in ops:
            o.close()


def test_solve_batch_arguments():
    ops = _ops(SOLVE_MIX[:2])
    try:
        bs = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=i)).to("cuda") for i, o in enumerate(ops)]
        xs = [torch.zeros_like(b) for b in bs]
        with pytest.raises(sbm.SbmError):
            sbm.solve_batch([ops[0], ops[0]], [bs[0], bs[0].clone()], [xs[0], xs[0].clone()])
        with pytest.raises(sbm.SbmError):
            sbm.solve_batch(ops, bs, xs, mode="cg")
        with pytest.raises(ValueError):
            sbm.solve_batch(ops, bs[::-1], xs)
        assert sbm.solve_batch([], [], []) == []
    finally:
        for o in ops:
            o.close()


def test_batch_with_an_empty_operator_and_single_item():
    """An operator without unknowns (no cell inside the domain) is allowed in a batch and
    skipped; a batch of one operator is its own apply; a lockstep solve with an empty system
    reports success for it and solves the others as alone."""
    cases = [dict(d=3, n=8, ls=inputs.sphere((0, 0, 0), 0.05), p=3, disc="cg"), SOLVE_MIX[0], SOLVE_MIX[5]]
    ops = _ops(cases)
    try:
        assert ops[0].n_dofs == 0
        us = [torch.from_numpy(inputs.uniform_vector(max(o.n_dofs, 1), seed=900 + i)).to("cuda")[:o.n_dofs]
              for i, o in enumerate(ops)]
        vs = [torch.full_like(u, 3.0) for u in us]
        refs = _singles(ops[1:], us[1:])
        sbm.apply_batch(ops, us, vs)
        v1 = torch.full_like(us[2], 3.0)
        with sbm.Batch(ops[2:], us[2:], [v1], graph=True) as b1:
            b1.run(torch.cuda.Stream())
            torch.cuda.synchronize()
        for v, r in zip(vs[1:], refs):
            assert torch.equal(v, r)
        assert torch.equal(v1, refs[1])
        bs = [u.clone() for u in us]
        xs = [torch.zeros_like(u) for u in us]
        x_single = torch.zeros_like(us[1])
        ref = ops[1].solve(bs[1], x_single, rel_tol=1e-10, max_it=60, mode="gmres", restart=20)
        infos = sbm.solve_batch(ops, bs, xs, rel_tol=1e-10, max_it=60, mode="gmres", restart=20)
        assert infos[0]["status"] == sbm.SBM_OK and infos[0]["inner_its"] == 0
        for k in INFO_KEYS:
            assert infos[1][k] == ref[k], k
        assert torch.equal(xs[1], x_single)
    finally:
        for o in ops:
            o.close()


def test_solve_batch_long_restart_falls_back_bitwise():
    """Restart 80: past 64 columns the lockstep solver orthogonalises system by system (the wide
    Gram-Schmidt kernels); solutions and reports still equal the single solves bit for bit."""
    print("solve batch restart 80", flush=True)
    cases = [SOLVE_MIX[0], SOLVE_MIX[3], SOLVE_MIX[5]]
    ops = _ops(cases)
    try:
        bs = [torch.from_numpy(inputs.uniform_vector(o.n_dofs, seed=800 + i)).to("cuda") for i, o in enumerate(ops)]
        xs_single = [torch.zeros_like(b) for b in bs]
        ref = [o.solve(b, x, rel_tol=1e-12, max_it=150, mode="gmres", restart=80) for o, b, x in zip(ops, bs, xs_single)]
        xs = [torch.zeros_like(b) for b in bs]
        infos = sbm.solve_batch(ops, bs, xs, rel_tol=1e-12, max_it=150, mode="gmres", restart=80)
        torch.cuda.synchronize()
        assert any(r["inner_its"] > 64 for r in ref)  # the wide path was taken
        for c, r, inf, x, xr in zip(cases, ref, infos, xs, xs_single):
            for k in INFO_KEYS:
                assert inf[k] == r[k], (c, k, inf[k], r[k])
            assert torch.equal(x, xr), c
    finally:
        for o in ops:
            o.close()
