"""sbm_apply_noalloc (the apply for callers that cannot allocate) against sbm_apply, through
the C ABI: the same operator with the scratch taken from the library's static device array.
Every sum of the apply (default or truncated extension) is taken in an order fixed by the
setup, so the two agree bit for bit.  Two calls in a row on the shared array, the second with a
smaller operator and input."""

import numpy as np
import pytest

from paper_2507_17053_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sbm = pytest.importorskip("paper_2507_17053_amd.sbm")


def _pair(op, seed, dtype):
    u = torch.from_numpy(inputs.uniform_vector(op.n_dofs, seed=seed)).to("cuda", dtype)
    ref = torch.full_like(u, float("nan"))
    out = torch.full_like(u, float("nan"))
    op.apply(u, ref)
    op.apply_noalloc(u, out)
    torch.cuda.synchronize()
    return out, ref


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_equals_apply_twice_second_smaller(dtype):
    big = sbm.Operator(3, 32, -1.0, 1.0, inputs.sphere((0, 0, 0), 0.75), 4)          # CG Q4
    small = sbm.Operator(3, 12, -1.0, 1.0, inputs.ellipsoid((0, 0, 0), (0.8, 0.6, 0.7)), 2, disc="dg")
    assert small.n_dofs < big.n_dofs
    print(f"noalloc: big n_dofs={big.n_dofs}, small n_dofs={small.n_dofs}, dtype={dtype}", flush=True)
    for op, seed in ((big, 0), (small, 1), (big, 2)):
        out, ref = _pair(op, seed, dtype)
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), (op.n_dofs, (out - ref).abs().max().item())
    big.close()
    small.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_truncated_extension_matches_apply(dtype):
    op = sbm.Operator(3, 16, -1.0, 1.0, inputs.sphere((0, 0, 0), 0.75), 3, taylor_order=1)
    small = sbm.Operator(2, 16, -1.0, 1.0, inputs.sphere((0.05, -0.03), 0.7), 2, taylor_order=1)
    for o, seed in ((op, 0), (small, 1)):
        out, ref = _pair(o, seed, dtype)
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), (o.n_dofs, (out - ref).abs().max().item())
    op.close()
    small.close()


def test_noalloc_rejects_operators_beyond_the_static_scratch():
    """The 128^3 Q4 sphere needs about 0.27 GB of brick-boundary scratch in FP64: refused with
    EINVAL and a message naming the size, before any launch."""
    op = sbm.Operator(3, 128, -1.0, 1.0, inputs.sphere((0, 0, 0), 0.75), 4)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(u)
    with pytest.raises(sbm.SbmError) as e:
        op.apply_noalloc(u, v)
    assert e.value.status == sbm.SBM_EINVAL
    assert "static device scratch" in str(e.value)
    op.close()


def test_noalloc_rejects_bad_arguments():
    op = sbm.Operator(2, 8, -1.0, 1.0, inputs.sphere((0, 0), 0.7), 2)
    u = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(sbm.SbmError):
        op.apply_noalloc(u, u)
    op.close()
