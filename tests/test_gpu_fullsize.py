"""GPU parity at the workloads' full sizes, on sampled outputs.

At these sizes the oracle computes selected outputs only: the dense sum O1 on
2,048 random targets, and O2 restricted to the ancestor chains of a few sampled
leaves (exact there).  Launch configuration = the one bench.py times.

Bars: float64 vs O2 <= 1e-12 at the sampled leaves; every path vs O1 <= 10 x
the ID tolerance (the 1M cube's float32 path must also meet 1e-6, the accuracy
its benchmark line is quoted at).
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2310_16668_amd as sk  # noqa: E402


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def say(*a):
    print(*a, flush=True)


def sampled_o2(op, q, n_leaves=6, seed=0):
    P = op.export()
    leaves = np.nonzero(P["is_leaf"])[0]
    pick = np.random.default_rng(seed).choice(leaves, size=min(n_leaves, len(leaves)), replace=False)
    u = oracle.apply(P, q, box_mask=oracle.ancestors_mask(P, pick))
    pts = np.concatenate([P["idx"][P["idx_ptr"][b]:P["idx_ptr"][b + 1]] for b in pick])
    return pts, u[pts]


@pytest.fixture(scope="module")
def cube_1m():
    w = workloads.LAPLACE3D_1M
    say("build", w.name)
    x = w.points()
    op = sk.build(x, "laplace", tol=w.tol, leaf_size=w.leaf_size)
    return w, x, op


def test_cube_1m_f64_and_f32(cube_1m):
    w, x, op = cube_1m
    q = w.charges()
    tg = w.targets()
    u1 = oracle.direct(x, q, targets=tg)
    pts, u2 = sampled_o2(op, q)
    for dt in (torch.float64, torch.float32):
        u = op.apply(torch.from_numpy(q).to("cuda:0", dt)).double().cpu().numpy()
        e1 = relerr(u[tg], u1)
        e2 = relerr(u[pts], u2)
        say(w.name, dt, "vs O1", e1, "vs O2 (sampled leaves)", e2)
        assert e1 <= 1e-6
        if dt == torch.float64:
            assert e2 <= 1e-12
    # the adjoint (Laplace: Atilde^T = Atilde) on the benchmark's second input
    v = w.weights()
    wv = op.apply_adjoint(torch.from_numpy(v).to("cuda:0", torch.float32)).double().cpu().numpy()
    e = relerr(wv[tg], oracle.direct(x, v, targets=tg))
    say(w.name, "f32 adjoint vs O1", e)
    assert e <= 1e-6


def test_ellipsoid_4m_f32():
    w = workloads.LAPLACE3D_ELLIPSOID_4M
    say("build", w.name)
    x = w.points()
    op = sk.build(x, "laplace", tol=w.tol, leaf_size=w.leaf_size)
    st = op.stats()
    say(w.name, "levels", st["max_level"], "k_max", st["k_max"], "pairs", st["pairs_near"])
    assert st["max_level"] >= 9
    q = w.charges()
    tg = w.targets()
    u1 = oracle.direct(x, q, targets=tg)
    u = op.apply(torch.from_numpy(q).to("cuda:0", torch.float32)).double().cpu().numpy()
    e1 = relerr(u[tg], u1)
    say(w.name, "f32 vs O1", e1)
    assert e1 <= 10 * w.tol
    ud = op.apply(torch.from_numpy(q).to("cuda:0", torch.float64)).cpu().numpy()
    pts, u2 = sampled_o2(op, q, n_leaves=4)
    e2 = relerr(ud[pts], u2)
    say(w.name, "f64 vs O2 (sampled leaves)", e2)
    assert e2 <= 1e-12


def test_helmholtz_1m_c64_f64_leaf():
    w = workloads.HELMHOLTZ3D_1M
    say("build", w.name)
    x = w.points()
    op = sk.build(x, "helmholtz", tol=w.tol, leaf_size=w.leaf_size, kappa=w.kappa, f64_leaf=True)
    q = w.charges()
    tg = w.targets()
    u1 = oracle.direct(x, q.astype(np.complex64).astype(np.complex128), "helmholtz", w.kappa, targets=tg)
    qd = torch.from_numpy(q).to("cuda:0", torch.complex64)
    u = op.apply(qd).cpu().numpy().astype(np.complex128)
    e1 = relerr(u[tg], u1)
    say(w.name, "c64 + f64 leaf vs O1", e1)
    assert e1 <= 10 * w.tol
    # conjugated adjoint: Atilde^H v = conj(Atilde conj v)
    wa = op.apply_adjoint(qd).cpu().numpy()
    wb = np.conj(op.apply(torch.conj(qd).resolve_conj()).cpu().numpy())
    assert relerr(wa, wb) <= 1e-5
