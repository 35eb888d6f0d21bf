"""GPU parity: the HIP sweep against the oracle on the same seeded inputs.

Bars (written per test):
  * float64 / complex128 apply vs O2 on the same skeleton operators: relative
    l2 <= 1e-12 (results differ only by summation order and by the exactly
    cancelling uncompressed pairs the GPU skips);
  * any apply vs O1, the dense sum: <= 10 x the ID tolerance;
  * float32 / complex64 applies: vs O2 on the same float32-rounded charges
    <= F32_VS_O2 (16 float32 units, derived in tests/_record.py); vs O1
    <= 10 x tol + F32_VS_O2 (the ID truncation plus the float32 arithmetic).
    Every measured error is recorded (tests/_record.py).
Every GPU call goes through the C ABI (the binding only marshals arguments).
"""
import numpy as np
import pytest

import oracle
import workloads
from _record import F32_VS_O2, maxrel, record

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2310_16668_amd as sk  # noqa: E402


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dtype)


def host(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)


CASES = {
    # name: (points, kind, kappa, tol, leaf)
    "lap2d_16k": (lambda: workloads.LAPLACE2D_16K.points(), "laplace", 0.0, 1e-8, 64),
    "lap3d_uniform_64k": (lambda: workloads.uniform_points(65536, 3, 501), "laplace", 0.0, 1e-7, 128),
    "lap3d_ellipsoid_60k": (lambda: workloads.ellipsoid_points(60000, 502), "laplace", 0.0, 1e-6, 64),
    "helm3d_uniform_32k": (lambda: workloads.uniform_points(32768, 3, 503), "helmholtz", 20.0, 1e-6, 64),
    # 2D Helmholtz (i/4) H0^(1)(kappa r) at the paper's kappa = 100
    "helm2d_k100_16k": (lambda: workloads.HELMHOLTZ2D_16K.points(), "helmholtz", 100.0, 1e-8, 64),
}
# layout-only cases (parity with O2, no accuracy bar against O1)
EXTRA_CASES = {
    # tight tolerance: tree boxes of up to ~2200 entries (several symmetric items per pair)
    "lap3d_bigbox_40k": (lambda: workloads.uniform_points(40000, 3, 504), "laplace", 0.0, 1e-10, 256),
}
_built = {}


def _op(name, **kw):
    key = (name, tuple(sorted(kw.items())))
    if key not in _built:
        mk, kind, kappa, tol, b = {**CASES, **EXTRA_CASES}[name]
        x = mk()
        op = sk.build(x, kind, tol=tol, leaf_size=b, kappa=kappa, **kw)
        _built[key] = (x, op, op.export())
    return _built[key]


def _charges(name, n, seed):
    kind = {**CASES, **EXTRA_CASES}[name][1]
    return workloads.charges(n, 1, seed, complex_=(kind == "helmholtz"))


@pytest.mark.parametrize("name", list(CASES))
def test_f64_forward_and_adjoint_match_o2(name):
    _say("case", name)
    x, op, P = _op(name)
    kind, kappa, tol = CASES[name][1], CASES[name][2], CASES[name][3]
    q = _charges(name, x.shape[0], 7)
    dt = torch.complex128 if kind == "helmholtz" else torch.float64
    u = host(op.apply(dev(q, dt)))
    u2 = oracle.apply(P, q)
    e2 = relerr(u, u2)
    _say(name, "fwd vs O2", e2, "max", maxrel(u, u2))
    assert e2 <= 1e-12
    # a wrong leaf would stand out in the max norm
    assert maxrel(u, u2) <= 1e-11
    w = host(op.apply_adjoint(dev(q, dt)))
    w2 = oracle.apply(P, q, adjoint=True)
    ew = relerr(w, w2)
    _say(name, "adj vs O2T", ew)
    assert ew <= 1e-12
    tg = workloads.target_subset(x.shape[0], 2048, 11)
    u1 = oracle.direct(x, q, kind, kappa, targets=tg)
    e1 = relerr(u[tg], u1)
    _say(name, "fwd vs O1", e1, "tol", tol)
    assert e1 <= 10 * tol


@pytest.mark.parametrize("name", ["lap3d_uniform_64k", "lap3d_ellipsoid_60k"])
def test_keep_transparent_matches_o2(name):
    x, op, P = _op(name, keep_transparent=True)
    q = _charges(name, x.shape[0], 8)
    u = host(op.apply(dev(q, torch.float64)))
    assert relerr(u, oracle.apply(P, q)) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_single_precision_error_stated(name):
    x, op, P = _op(name)
    kind, kappa, tol = CASES[name][1], CASES[name][2], CASES[name][3]
    q = _charges(name, x.shape[0], 9)
    cplx = kind == "helmholtz"
    dt = torch.complex64 if cplx else torch.float32
    qr = q.astype(np.complex64 if cplx else np.float32).astype(q.dtype)
    up = np.complex128 if cplx else np.float64
    u = host(op.apply(dev(q, dt))).astype(up)
    w = host(op.apply_adjoint(dev(q, dt))).astype(up)
    tg = workloads.target_subset(x.shape[0], 2048, 12)
    u1 = oracle.direct(x, qr, kind, kappa, targets=tg)
    e1 = relerr(u[tg], u1)
    u2 = oracle.apply(P, qr)
    e2 = relerr(u, u2)
    ew = relerr(w, oracle.apply(P, qr, adjoint=True))
    # the adjoint against the dense sum: A^H v = conj(A conj v) (A = A^T)
    ew1 = relerr(w[tg], np.conj(oracle.direct(x, np.conj(qr), kind, kappa, targets=tg)))
    record(f"{name} {dt}", vs_o1=e1, vs_o2=e2, max_vs_o2=maxrel(u, u2), adjoint_vs_o2t=ew, adjoint_vs_o1=ew1)
    assert e2 <= F32_VS_O2 and ew <= F32_VS_O2
    assert e1 <= 10 * tol + F32_VS_O2 and ew1 <= 10 * tol + F32_VS_O2


def test_f64_leaf_single_precision_helmholtz():
    name = "helm3d_uniform_32k"
    x, op, P = _op(name, f64_leaf=True)
    q = _charges(name, x.shape[0], 10)
    qr = q.astype(np.complex64).astype(np.complex128)
    u = host(op.apply(dev(q, torch.complex64))).astype(np.complex128)
    w = host(op.apply_adjoint(dev(q, torch.complex64))).astype(np.complex128)
    tg = workloads.target_subset(x.shape[0], 2048, 13)
    e1 = relerr(u[tg], oracle.direct(x, qr, "helmholtz", 20.0, targets=tg))
    ew1 = relerr(w[tg], np.conj(oracle.direct(x, np.conj(qr), "helmholtz", 20.0, targets=tg)))
    e2 = relerr(u, oracle.apply(P, qr))
    ew = relerr(w, oracle.apply(P, qr, adjoint=True))
    record(f"{name} c64 + f64 leaf", vs_o1=e1, vs_o2=e2, adjoint_vs_o2t=ew, adjoint_vs_o1=ew1)
    assert e1 <= 10 * CASES[name][3] and ew1 <= 10 * CASES[name][3]
    assert e2 <= F32_VS_O2 and ew <= F32_VS_O2


def test_deterministic_and_linear():
    x, op, P = _op("lap3d_ellipsoid_60k")
    q1 = _charges("lap3d_ellipsoid_60k", x.shape[0], 1)
    q2 = _charges("lap3d_ellipsoid_60k", x.shape[0], 2)
    a = host(op.apply(dev(q1, torch.float64)))
    b = host(op.apply(dev(q1, torch.float64)))
    assert np.array_equal(a, b)
    c = host(op.apply(dev(0.5 * q1 - 2.0 * q2, torch.float64)))
    d = 0.5 * a - 2.0 * host(op.apply(dev(q2, torch.float64)))
    assert relerr(c, d) <= 1e-14


def test_edge_cases():
    rng = np.random.default_rng(0)
    # a single point: nothing acts on it
    op = sk.build(np.array([[0.3, 0.4, 0.5]]), "laplace", tol=1e-6, leaf_size=8)
    u = host(op.apply(dev(np.array([2.0]), torch.float64)))
    assert u[0] == 0.0
    # root is a leaf: the direct sum
    x = rng.random((100, 3))
    q = rng.uniform(-1, 1, 100)
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=128)
    assert relerr(host(op.apply(dev(q, torch.float64))), oracle.direct(x, q)) <= 1e-14
    # leaves on level 1
    x = rng.random((500, 3))
    q = rng.uniform(-1, 1, 500)
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=100)
    assert op.export()["max_level"] == 1
    assert relerr(host(op.apply(dev(q, torch.float64))), oracle.direct(x, q)) <= 1e-14
    # coincident points contribute zero, in every level of the tree
    x = np.vstack([rng.random((3000, 3)), np.repeat(rng.random((5, 3)), 40, axis=0)])
    q = rng.uniform(-1, 1, x.shape[0])
    op = sk.build(x, "laplace", tol=1e-8, leaf_size=32)
    P = op.export()
    u = host(op.apply(dev(q, torch.float64)))
    assert np.all(np.isfinite(u))
    assert relerr(u, oracle.apply(P, q)) <= 1e-12
    assert relerr(u, oracle.direct(x, q)) <= 1e-7
    # float32: the zero distances of coincident points are masked in every
    # targets-per-lane variant (boxes paired with themselves included)
    ur = oracle.apply(P, q.astype(np.float32).astype(np.float64))
    for t in (1, 2, 3, 4):
        op.set_targets_per_lane(t)
        us = host(op.apply(dev(q, torch.float32))).astype(np.float64)
        assert np.all(np.isfinite(us))
        record(f"coincident points f32 tpl{t}", vs_o2=relerr(us, ur))
        assert relerr(us, ur) <= F32_VS_O2
    # no compression: the GPU sweep is the dense sum
    x = rng.random((4000, 2))
    q = rng.uniform(-1, 1, 4000)
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=16, no_compression=True, keep_transparent=True)
    assert relerr(host(op.apply(dev(q, torch.float64))), oracle.direct(x, q)) <= 1e-13


def test_autograd_backward_is_adjoint():
    name = "helm3d_uniform_32k"
    x, op, P = _op(name)
    q = _charges(name, x.shape[0], 3)
    w = workloads.charges(x.shape[0], 1, 4, complex_=True)
    qt = dev(q, torch.complex128).requires_grad_(True)
    wt = dev(w, torch.complex128)
    u = sk.fmm_apply(op, qt)
    loss = torch.real(torch.sum(torch.conj(wt) * u))
    loss.backward()
    # L = Re <w, A q>  =>  dL/dq (PyTorch convention, conj-Wirtinger) = A^H w
    g = host(qt.grad)
    assert relerr(g, oracle.apply(P, w, adjoint=True)) <= 1e-12


def test_argument_errors_leave_output_untouched():
    x, op, P = _op("lap3d_ellipsoid_60k")
    q = torch.zeros(x.shape[0], dtype=torch.complex128, device="cuda:0")
    with pytest.raises(sk.SkelfmmError) as e:
        op.apply(q)
    assert e.value.status == -1


@pytest.mark.parametrize("name,nrhs", [("lap3d_ellipsoid_60k", 3), ("lap3d_uniform_64k", 8),
                                       ("lap2d_16k", 17), ("helm3d_uniform_32k", 5), ("helm2d_k100_16k", 6)])
def test_many_rhs_match_single_and_o2(name, nrhs):
    x, op, P = _op(name)
    kind = CASES[name][1]
    n = x.shape[0]
    Q = workloads.charges(n, nrhs, 20, complex_=(kind == "helmholtz"))
    dt = torch.complex128 if kind == "helmholtz" else torch.float64
    U = host(op.apply(dev(Q, dt)))
    assert U.shape == (n, nrhs)
    for c in (0, nrhs - 1):
        assert relerr(U[:, c], host(op.apply(dev(np.ascontiguousarray(Q[:, c]), dt)))) <= 1e-13
    assert relerr(U, oracle.apply(P, Q)) <= 1e-12
    W = host(op.apply_adjoint(dev(Q, dt)))
    assert relerr(W, oracle.apply(P, Q, adjoint=True)) <= 1e-12


@pytest.mark.parametrize("name", ["lap3d_uniform_64k", "helm3d_uniform_32k"])
def test_many_rhs_single_precision(name):
    x, op, P = _op(name)
    kind, kappa, tol = CASES[name][1], CASES[name][2], CASES[name][3]
    n = x.shape[0]
    Q = workloads.charges(n, 16, 21, complex_=(kind == "helmholtz"))
    dt = torch.complex64 if kind == "helmholtz" else torch.float32
    U = host(op.apply(dev(Q, dt))).astype(np.complex128 if kind == "helmholtz" else np.float64)
    Qr = Q.astype(np.complex64 if kind == "helmholtz" else np.float32).astype(Q.dtype)
    tg = workloads.target_subset(n, 512, 22)
    e1 = relerr(U[tg], oracle.direct(x, Qr, kind, kappa, targets=tg))
    _say(name, "16 rhs single vs O1", e1)
    assert e1 <= max(10 * tol, 1e-5)


@pytest.mark.parametrize("nrhs", [40, 70])
def test_many_rhs_single_precision_column_tiles(nrhs):
    """float32 with many RHS runs on the matrix cores in 32-column tiles, two
    tiles per wave where a work item has no uhat rows: 40 RHS pad to two tiles
    (one pair), 70 to three (the last pair holds one tile).  Every column must
    match O2 on the rounded charges and the one-column apply of the same column."""
    x, op, P = _op("lap3d_uniform_64k")
    n = x.shape[0]
    Q = workloads.charges(n, nrhs, 23)
    Qr = Q.astype(np.float32).astype(np.float64)
    U = host(op.apply(dev(Q, torch.float32))).astype(np.float64)
    W = host(op.apply_adjoint(dev(Q, torch.float32))).astype(np.float64)
    e_u = relerr(U, oracle.apply(P, Qr))
    e_w = relerr(W, oracle.apply(P, Qr, adjoint=True))
    _say("lap3d_uniform_64k", f"{nrhs} rhs float32 vs O2", e_u, "adjoint", e_w)
    assert e_u <= 2e-6 and e_w <= 2e-6
    for c in sorted(c for c in {0, 31, 32, 33, 63, 64, nrhs - 1} if c < nrhs):
        one = host(op.apply(dev(np.ascontiguousarray(Q[:, c]), torch.float32))).astype(np.float64)
        assert relerr(U[:, c], one) <= 2e-6, c


def _batch_ops(f64_leaf=False):
    geo = [workloads.uniform_points(20000, 3, 601), workloads.ellipsoid_points(30000, 602),
           workloads.uniform_points(15000, 3, 603)]
    return geo, [sk.build(x, "laplace", tol=1e-6, leaf_size=64, f64_leaf=f64_leaf) for x in geo]


@pytest.mark.parametrize("nrhs", [1, 8])
def test_batch_equals_separate_applies(nrhs):
    geo, ops = _batch_ops()
    batch = sk.Batch(ops)
    qs = [dev(workloads.charges(x.shape[0], nrhs, 30 + i), torch.float64) for i, x in enumerate(geo)]
    outs = batch.apply(qs)
    adj = batch.apply(qs, adjoint=True)
    for i, op in enumerate(ops):
        ref = op.apply(qs[i])
        assert torch.equal(outs[i].reshape(ref.shape), ref)
        assert torch.equal(adj[i].reshape(ref.shape), op.apply_adjoint(qs[i]))
    P = ops[1].export()
    assert relerr(host(outs[1]), oracle.apply(P, host(qs[1]))) <= 1e-12


def test_batch_graph_capture_replays():
    geo, ops = _batch_ops()
    batch = sk.Batch(ops)
    qs = [dev(workloads.charges(x.shape[0], 4, 40 + i), torch.float32) for i, x in enumerate(geo)]
    ref = [o.clone() for o in batch.apply(qs)]        # eager; also sizes the workspace
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.apply(qs)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = batch.apply(qs)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
        batch.apply(qs, adjoint=True)      # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["lap2d_16k", "lap3d_uniform_64k", "lap3d_ellipsoid_60k", "lap3d_bigbox_40k"])
def test_symmetric_pairing_matches_unpaired_and_o2(name):
    """One kernel evaluation per colleague pair (both orders) against the unpaired
    sweep and O2, for every targets-per-lane variant."""
    _say("case", name)
    x, op, P = _op(name)
    _, op_ns, _ = _op(name, symmetric=False)
    assert op.stats()["n_sym_tasks"] > 0
    assert op_ns.stats()["n_sym_tasks"] == 0
    q = _charges(name, x.shape[0], 11)
    u2 = oracle.apply(P, q)
    un = host(op_ns.apply(dev(q, torch.float64)))
    for t in (1, 2, 3, 4):
        op.set_targets_per_lane(t)
        u = host(op.apply(dev(q, torch.float64)))
        e2, en = relerr(u, u2), relerr(u, un)
        _say(name, "tpl", t, "paired vs O2", e2, "vs unpaired", en)
        assert e2 <= 1e-12 and en <= 1e-12
        w = host(op.apply_adjoint(dev(q, torch.float64)))
        assert relerr(w, oracle.apply(P, q, adjoint=True)) <= 1e-12
    # float32: every targets-per-lane variant, paired and unpaired, against O2 on
    # the rounded charges
    qr = q.astype(np.float32).astype(np.float64)
    u2r = oracle.apply(P, qr)
    w2r = oracle.apply(P, qr, adjoint=True)
    ens = relerr(host(op_ns.apply(dev(q, torch.float32))).astype(np.float64), u2r)
    for t in (1, 2, 3, 4):
        op.set_targets_per_lane(t)
        us = host(op.apply(dev(q, torch.float32))).astype(np.float64)
        ws = host(op.apply_adjoint(dev(q, torch.float32))).astype(np.float64)
        es, ew = relerr(us, u2r), relerr(ws, w2r)
        record(f"{name} f32 paired tpl{t}", vs_o2=es, adjoint_vs_o2t=ew, unpaired_vs_o2=ens)
        assert es <= F32_VS_O2 and ew <= F32_VS_O2
    assert ens <= F32_VS_O2
    op.set_targets_per_lane(2)
    # compensated leaf sums: float32 partials of at most four products, column
    # sums in float64
    _, op_c, _ = _op(name, compensated_leaf=True)
    for t in (1, 2, 3, 4):
        op_c.set_targets_per_lane(t)
        uc = host(op_c.apply(dev(q, torch.float32))).astype(np.float64)
        wc = host(op_c.apply_adjoint(dev(q, torch.float32))).astype(np.float64)
        ec, ewc = relerr(uc, u2r), relerr(wc, w2r)
        record(f"{name} f32 paired compensated tpl{t}", vs_o2=ec, adjoint_vs_o2t=ewc, unpaired_vs_o2=ens)
        assert ec <= F32_VS_O2 and ewc <= F32_VS_O2


@pytest.mark.parametrize("name,nrhs", [("lap3d_uniform_64k", 70), ("lap3d_ellipsoid_60k", 40), ("lap2d_16k", 33)])
def test_matrix_core_transfers_every_shape(name, nrhs):
    """Float32 applies with 8 or more RHS run the transfers as one GEMM per box
    on the matrix cores.  Every launch shape gives the same bits (no shape changes
    the arithmetic of an output tile), the autotuner picks one of them, and the
    result matches O2 on the rounded charges."""
    x, op, P = _op(name)
    n = x.shape[0]
    Q = workloads.charges(n, nrhs, 24)
    Qr = Q.astype(np.float32).astype(np.float64)
    qd = dev(Q, torch.float32)
    ref_u = ref_w = None
    for shape in range(sk.NXFER):
        op.set_transfer_shape(shape)
        u, w = op.apply(qd), op.apply_adjoint(qd)
        if ref_u is None:
            ref_u, ref_w = u, w
        assert torch.equal(u, ref_u) and torch.equal(w, ref_w), shape
    tuned = op.autotune_transfers(nrhs)
    assert 0 <= tuned["shape"] < sk.NXFER and all(t > 0 for t in tuned["ms"])
    assert torch.equal(op.apply(qd), ref_u)
    U, W = host(ref_u).astype(np.float64), host(ref_w).astype(np.float64)
    e_u, e_w = relerr(U, oracle.apply(P, Qr)), relerr(W, oracle.apply(P, Qr, adjoint=True))
    record(f"{name} {nrhs} rhs float32 matrix-core transfers", vs_o2=e_u, adjoint_vs_o2t=e_w,
           tuned_shape=tuned["shape"])
    assert e_u <= F32_VS_O2 and e_w <= F32_VS_O2


@pytest.mark.parametrize("name", ["helm3d_uniform_32k", "helm2d_k100_16k"])
def test_helmholtz_symmetric_pairing(name):
    """The complex-symmetric Helmholtz kernels share one evaluation per pair of
    distinct colleagues between both directions (complex products, conjugated
    in the adjoint): complex128 against O2 and the unpaired sweep at every
    targets-per-lane setting, complex64 (float64 leaf sums) against O2."""
    x, op, P = _op(name)
    _, op_ns, _ = _op(name, symmetric=False)
    assert op.stats()["n_sym_tasks"] > 0 and op_ns.stats()["n_sym_tasks"] == 0
    q = _charges(name, x.shape[0], 12)
    u2 = oracle.apply(P, q)
    w2 = oracle.apply(P, q, adjoint=True)
    un = host(op_ns.apply(dev(q, torch.complex128)))
    for t in (1, 2, 3, 4):
        op.set_targets_per_lane(t)
        u = host(op.apply(dev(q, torch.complex128)))
        w = host(op.apply_adjoint(dev(q, torch.complex128)))
        e2, en, ew = relerr(u, u2), relerr(u, un), relerr(w, w2)
        record(f"{name} c128 paired tpl{t}", vs_o2=e2, vs_unpaired=en, adjoint_vs_o2t=ew)
        assert e2 <= 1e-12 and en <= 1e-12 and ew <= 1e-12
    _, op_l, _ = _op(name, f64_leaf=True)
    qr = q.astype(np.complex64).astype(np.complex128)
    u2r, w2r = oracle.apply(P, qr), oracle.apply(P, qr, adjoint=True)
    for t in (1, 2):
        op_l.set_targets_per_lane(t)
        uc = host(op_l.apply(dev(q, torch.complex64))).astype(np.complex128)
        wc = host(op_l.apply_adjoint(dev(q, torch.complex64))).astype(np.complex128)
        ec, ewc = relerr(uc, u2r), relerr(wc, w2r)
        record(f"{name} c64 f64-leaf paired tpl{t}", vs_o2=ec, adjoint_vs_o2t=ewc)
        assert ec <= F32_VS_O2 and ewc <= F32_VS_O2


@pytest.mark.parametrize("name", ["lap3d_uniform_64k", "lap2d_16k", "lap3d_ellipsoid_60k", "helm3d_uniform_32k"])
def test_fused_forward_adjoint(name):
    """skelfmm_apply_fwd_adj: (A q, A^H v) in one call.  Real kernels in float32
    share one sweep (two interleaved columns) at every targets-per-lane setting;
    each column equals its own single apply bit for bit (the same products
    summed in the same order) and matches O2 to the float32 bar.  Complex kernels
    run the two sweeps in turn (same results as the separate calls, bit for bit)."""
    x, op, P = _op(name)
    kind = CASES[name][1]
    cplx = kind == "helmholtz"
    dt = torch.complex64 if cplx else torch.float32
    q = _charges(name, x.shape[0], 21)
    v = _charges(name, x.shape[0], 22)
    qd, vd = dev(q, dt), dev(v, dt)
    u1, w1 = host(op.apply(qd)), host(op.apply_adjoint(vd))
    up = np.complex128 if cplx else np.float64
    qr = q.astype(np.complex64 if cplx else np.float32).astype(q.dtype)
    vr = v.astype(np.complex64 if cplx else np.float32).astype(v.dtype)
    u2 = oracle.apply(P, qr)
    w2 = oracle.apply(P, vr, adjoint=True)
    if cplx:
        u, w = op.apply_fwd_adj(qd, vd)
        assert np.array_equal(host(u), u1) and np.array_equal(host(w), w1)
        return
    for tpl in (1, 2, 3, 4, 0):
        if tpl:
            op.set_targets_per_lane(tpl)
            u1, w1 = host(op.apply(qd)), host(op.apply_adjoint(vd))
        else:
            # the autotuned two-column shape, against separate applies at that shape
            tpl = op.autotune_fwd_adj()["targets_per_lane"]
            assert tpl in (1, 2, 3, 4)
            op.set_targets_per_lane(tpl)
            u1, w1 = host(op.apply(qd)), host(op.apply_adjoint(vd))
        u, w = op.apply_fwd_adj(qd, vd)
        u, w = host(u).astype(up), host(w).astype(up)
        e_single = max(relerr(u, u1.astype(up)), relerr(w, w1.astype(up)))
        e_u, e_w = relerr(u, u2), relerr(w, w2)
        record(f"{name} fwd_adj tpl={tpl}", vs_single=e_single, vs_o2=e_u, adjoint_vs_o2t=e_w)
        # each column runs the separate apply's arithmetic in the same order
        assert np.array_equal(u, u1.astype(up)) and np.array_equal(w, w1.astype(up))
        assert e_u <= F32_VS_O2 and e_w <= F32_VS_O2


@pytest.mark.parametrize("name", ["lap3d_uniform_64k", "lap2d_16k", "lap3d_ellipsoid_60k"])
def test_f32_differences(name):
    """f32_differences: pair items whose reach is at most 1024 x their smallest
    spacing form |d|^2 from float32 coordinate differences about the source box's
    first entry.  Every targets-per-lane variant, forward and adjoint, against O2
    on the rounded charges (F32_VS_O2) and O1 (10 tol + F32_VS_O2); the fused
    forward + adjoint equals the separate applies bit for bit."""
    _say("case", name)
    x, op, P = _op(name, f32_differences=True)
    _, op_e, _ = _op(name)
    st = op.stats()
    record(f"{name} f32 differences layout", items=st["n_sym_tasks"], f32diff_items=st["n_sym_f32diff"],
           expanded_items=st["n_sym_expanded"])
    assert st["n_sym_f32diff"] > 0
    assert op_e.stats()["n_sym_f32diff"] == 0
    tol = CASES[name][3]
    q = _charges(name, x.shape[0], 31)
    v = _charges(name, x.shape[0], 32)
    qr = q.astype(np.float32).astype(np.float64)
    vr = v.astype(np.float32).astype(np.float64)
    u2, w2 = oracle.apply(P, qr), oracle.apply(P, vr, adjoint=True)
    tg = np.random.default_rng(33).choice(x.shape[0], size=512, replace=False)
    u1 = oracle.direct(x, qr, targets=tg)
    qd, vd = dev(q, torch.float32), dev(v, torch.float32)
    for t in (1, 2, 3, 4):
        op.set_targets_per_lane(t)
        op_e.set_targets_per_lane(t)
        u = host(op.apply(qd)).astype(np.float64)
        w = host(op.apply_adjoint(vd)).astype(np.float64)
        ue = host(op_e.apply(qd)).astype(np.float64)
        e2, ew, e1 = relerr(u, u2), relerr(w, w2), relerr(u[tg], u1)
        record(f"{name} f32 differences tpl{t}", vs_o2=e2, adjoint_vs_o2t=ew, vs_o1=e1,
               default_vs_o2=relerr(ue, u2), default_vs_o1=relerr(ue[tg], u1))
        assert e2 <= F32_VS_O2 and ew <= F32_VS_O2
        assert e1 <= 10 * tol + F32_VS_O2
        uf, wf = op.apply_fwd_adj(qd, vd)
        assert np.array_equal(host(uf).astype(np.float64), u) and np.array_equal(host(wf).astype(np.float64), w)
