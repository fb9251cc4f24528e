"""dcg_apply_noalloc (the entry point that allocates nothing: its work buffers
live in one static device array) against dcg_apply on the same handle and
input.  Both run the same kernels in the same order, so the outputs agree to
rounding of the order of the FP64 operators' bar (1e-13; observed equal).
Each case makes two calls in a row on the shared array, the second with a
smaller mesh, so that it also runs over the first call's leftovers."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2606_13429_amd._binding")
import paper_2606_13429_amd as dcg  # noqa: E402


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _run(solver, n, op, seed):
    m = (4 if op == lib.DCG_OP_INNER else 16) * n * n
    inp = torch.from_numpy(np.random.default_rng(seed).standard_normal(m)).cuda()
    ref = torch.empty_like(inp)
    got = torch.full_like(inp, np.nan)
    solver.apply(op, inp, ref)
    lib.dcg_apply_noalloc(solver.handle, op, inp, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("sizes", [((64, 0), (32, 0)), ((128, 3), (64, 2))],
                         ids=["full-hierarchy", "shortened-hierarchy"])
def test_noalloc_matches_apply_on_two_calls(prec, sizes):
    for call, (n, levels) in enumerate(sizes):
        s = dcg.Solver(n, 1e-3, prec=prec, levels=levels)
        for op in (lib.DCG_OP_INNER, lib.DCG_OP_DEFLATED):
            got, ref = _run(s, n, op, 10 * call + op)
            assert np.isfinite(got).all()
            assert _rel(got, ref) <= 1e-13, (n, levels, op, _rel(got, ref))
        s.close()


def test_noalloc_rejects_other_ops_and_meshes_above_its_array():
    assert lib.dcg_noalloc_bytes() == 48 << 20
    n = 32
    s = dcg.Solver(n, 1e-3)
    x = torch.zeros(16 * n * n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(lib.DCGError) as ei:
        lib.dcg_apply_noalloc(s.handle, lib.DCG_OP_ASTAR, x, y)
    assert ei.value.status == lib.DCG_EINVAL
    s.close()
    s = dcg.Solver(32, 1e-3, inner="exact")
    with pytest.raises(lib.DCGError) as ei:
        lib.dcg_apply_noalloc(s.handle, lib.DCG_OP_DEFLATED, x, y)
    assert ei.value.status == lib.DCG_EINVAL
    s.close()
    n = 512
    s = dcg.Solver(n, 1e-3, prec="fp64")
    x = torch.zeros(16 * n * n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(lib.DCGError) as ei:
        lib.dcg_apply_noalloc(s.handle, lib.DCG_OP_DEFLATED, x, y)
    assert ei.value.status == lib.DCG_EINVAL and "bytes of scratch" in str(ei.value)
    s.close()
