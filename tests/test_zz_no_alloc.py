"""skelfmm_apply_noalloc: the apply with its workspace in the library's static
device array, through the C ABI, against skelfmm_apply / skelfmm_apply_adjoint
(the same kernels, so the same bits) and the oracle."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2310_16668_amd as sk  # noqa: E402


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dtype)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matches_apply_on_two_calls():
    big = workloads.uniform_points(40000, 3, 701)
    small = workloads.ellipsoid_points(12000, 702)
    op_big = sk.build(big, "laplace", tol=1e-7, leaf_size=64)
    op_small = sk.build(small, "laplace", tol=1e-6, leaf_size=64)
    for op in (op_big, op_small):
        op.prepare(0, torch.float64)          # upload only: no workspace of its own
        op.prepare(0, torch.float32)
    assert sk._lib.skelfmm_noalloc_scratch_bytes() == 64 << 20
    # first call: the larger operator, one float64 RHS, forward and adjoint
    q = workloads.charges(big.shape[0], 1, 703)
    qd = _dev(q, torch.float64)
    for adjoint in (False, True):
        out = torch.empty_like(qd)
        op_big.apply_noalloc(qd, out, adjoint=adjoint)
        ref = op_big.apply_adjoint(qd) if adjoint else op_big.apply(qd)
        assert torch.equal(out, ref)
        P = op_big.export()
        assert _relerr(out.cpu().numpy(), oracle.apply(P, q, adjoint=adjoint)) <= 1e-12
    # second call: the smaller operator (a smaller input), float32 with 8 RHS
    # (matrix-core path) and with one RHS (pair kernel), then float64 again
    for dt, nrhs in ((torch.float32, 8), (torch.float32, 1), (torch.float64, 1)):
        Q = workloads.charges(small.shape[0], nrhs, 704)
        Qd = _dev(Q, dt)
        out = torch.empty_like(Qd)
        op_small.apply_noalloc(Qd, out)
        assert torch.equal(out, op_small.apply(Qd)), (dt, nrhs)
        outa = torch.empty_like(Qd)
        op_small.apply_noalloc(Qd, outa, adjoint=True)
        assert torch.equal(outa, op_small.apply_adjoint(Qd)), (dt, nrhs)
    torch.cuda.synchronize()


def test_noalloc_rejects_what_it_cannot_serve():
    x = workloads.uniform_points(65536, 3, 705)
    op = sk.build(x, "laplace", tol=1e-7, leaf_size=128)
    q = _dev(workloads.charges(x.shape[0], 1, 706), torch.float64)
    out = torch.zeros_like(q)
    # not uploaded yet
    with pytest.raises(sk.SkelfmmError) as e:
        op.apply_noalloc(q, out)
    assert e.value.status == -1
    op.prepare(0, torch.float32)
    # 64 float32 columns of this operator need more than the static array holds
    Q = _dev(workloads.charges(x.shape[0], 64, 707), torch.float32)
    O = torch.zeros_like(Q)
    with pytest.raises(sk.SkelfmmError) as e:
        op.apply_noalloc(Q, O)
    assert e.value.status == -1 and "bytes of workspace" in str(e.value)
    assert not torch.any(O)                   # left untouched
