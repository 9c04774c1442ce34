"""GPU solver tests: matrix-free diagonal, right-hand side, FP64 GMRES, FP32-inner GMRES with
FP64 iterative refinement, and CG on the symmetric (unshifted) limit.  Every solution is
checked with the oracle's own assembled matrix and right-hand side."""

import numpy as np
import pytest

from oracle import sbm_oracle as O
from paper_2507_17053_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sbm = pytest.importorskip("paper_2507_17053_amd.sbm")

DISK = inputs.sphere((0.05, -0.03), 0.7)


def _problem(d, n, ls, p, disc, shift=1.0):
    ref = O.setup(d, n, -1.0, 1.0, ls, p, disc=disc, shift_scale=shift)
    op = sbm.Operator(d, n, -1.0, 1.0, ls, p, disc=disc, shift_scale=shift)
    return ref, op


def _rhs(ref, op):
    u_fn, f_fn = inputs.manufactured(ref.d)
    cq, bp = op.rhs_points()
    b = torch.empty(op.n_dofs, dtype=torch.float64, device="cuda")
    op.rhs(f_fn(cq.reshape(-1, ref.d)), u_fn(bp.reshape(-1, ref.d)), b)
    return b, O.rhs(ref, f_fn, u_fn)


@pytest.mark.parametrize("d,n,ls,p,disc", [
    (2, 16, DISK, 2, "cg"), (2, 10, DISK, 3, "dg"),
    (3, 8, inputs.sphere((0, 0, 0), 0.75), 4, "cg"), (3, 7, inputs.torus(0.55, 0.4), 3, "dg"),
    (3, 16, inputs.sphere_union(1), 2, "cg"),
])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_diagonal_matches_assembled(d, n, ls, p, disc, dtype):
    ref, op = _problem(d, n, ls, p, disc)
    dg = torch.empty(op.n_dofs, dtype=dtype, device="cuda")
    op.diagonal(dg)
    torch.cuda.synchronize()
    dref = O.assemble(ref).diagonal()
    err = np.linalg.norm(dg.double().cpu().numpy() - dref) / np.linalg.norm(dref)
    assert err <= (1e-12 if dtype == torch.float64 else 1e-6), err


@pytest.mark.parametrize("d,n,ls,p,disc", [(2, 16, DISK, 2, "cg"), (3, 6, inputs.sphere((0, 0, 0), 0.75), 3, "dg")])
def test_rhs_matches_oracle(d, n, ls, p, disc):
    ref, op = _problem(d, n, ls, p, disc)
    b, bref = _rhs(ref, op)
    err = np.linalg.norm(b.cpu().numpy() - bref) / np.linalg.norm(bref)
    assert err <= 1e-12, err


SOLVABLE = [
    (2, 16, DISK, 2, "cg", 64),        # the 2D disk workload
    (2, 16, DISK, 1, "cg", 64),
    (2, 8, DISK, 2, "dg", 64),
    (3, 8, inputs.sphere((0, 0, 0), 0.75), 1, "cg", 64),
    (3, 6, inputs.sphere((0, 0, 0), 0.75), 2, "dg", 64),
]


@pytest.mark.parametrize("mode", ["gmres", "gmres_ir"])
@pytest.mark.parametrize("d,n,ls,p,disc,m", SOLVABLE,
                         ids=[f"{c[0]}d-n{c[1]}-p{c[3]}-{c[4]}" for c in SOLVABLE])
def test_gmres_reaches_1e10_against_oracle(d, n, ls, p, disc, m, mode):
    ref, op = _problem(d, n, ls, p, disc)
    b, bref = _rhs(ref, op)
    x = torch.zeros_like(b)
    info = op.solve(b, x, rel_tol=1e-10, max_it=8000, mode=mode, restart=m)
    print(mode, info, flush=True)
    assert info["status"] == sbm.SBM_OK and info["rel_residual"] <= 1e-10
    if mode == "gmres_ir":
        assert info["applies_f32"] > info["applies_f64"]
    A = O.assemble(ref)
    xs = x.cpu().numpy()
    res = np.linalg.norm(bref - A @ xs) / np.linalg.norm(bref)
    assert res <= 2e-10, res
    xd = O.solve_direct(A, bref)
    u_fn, _ = inputs.manufactured(d)
    e_gpu, e_ref = O.l2_error(ref, xs, u_fn), O.l2_error(ref, xd, u_fn)
    assert abs(e_gpu - e_ref) <= 1e-6 * e_ref + 1e-12, (e_gpu, e_ref)


@pytest.mark.parametrize("mode", ["cg", "cg_ir"])
def test_cg_on_unshifted_symmetric_limit(mode):
    """CG in FP64, and FP64 refinement around FP32 CG, on the symmetric limit (shift 0)."""
    ls = inputs.sphere((0, 0, 0), 0.75)
    ref, op = _problem(3, 8, ls, 2, "cg", shift=0.0)
    b, bref = _rhs(ref, op)
    x = torch.zeros_like(b)
    info = op.solve(b, x, rel_tol=1e-10, max_it=4000, mode=mode)
    assert info["status"] == sbm.SBM_OK and info["rel_residual"] <= 1e-10, info
    if mode == "cg_ir":
        assert info["applies_f32"] > info["applies_f64"] and info["outer_its"] >= 1
    A = O.assemble(ref)
    res = np.linalg.norm(bref - A @ x.cpu().numpy()) / np.linalg.norm(bref)
    assert res <= 2e-10


def test_jacobi_preconditioned_gmres():
    ref, op = _problem(2, 16, DISK, 1, "cg")
    b, bref = _rhs(ref, op)
    x = torch.zeros_like(b)
    info = op.solve(b, x, rel_tol=1e-10, max_it=2000, mode="gmres", restart=64, jacobi=True)
    assert info["status"] == sbm.SBM_OK, info
    res = np.linalg.norm(bref - O.assemble(ref) @ x.cpu().numpy()) / np.linalg.norm(bref)
    assert res <= 2e-10


def test_not_converged_is_reported():
    """max_it = 1 cannot reach 1e-10: status ENOCONV with the residual actually reached."""
    ref, op = _problem(2, 16, DISK, 2, "cg")
    b, _ = _rhs(ref, op)
    x = torch.zeros_like(b)
    info = op.solve(b, x, rel_tol=1e-10, max_it=1, mode="gmres")
    assert info["status"] == sbm.SBM_ENOCONV
    assert 0 < info["rel_residual"] < 1.0
