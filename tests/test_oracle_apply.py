"""Pins for O2, the CPU float64 apply of given skeleton operators (section 3,
"FMM apply"), and for its literal transpose.

* no compression (every box keeps all its points): every ifo / ifs / tfo pair
  cancels exactly and the top-level direct sum is the whole answer, so O2 must
  equal the dense sum O1 to rounding;
* the dense matrix form of the recursive factorization (section 2.3, equation
  (13)) assembled on tiny trees must equal O2 column by column;
* symmetry: for Laplace E_B = F_B^T and the neighbor relations are symmetric,
  so Atilde = Atilde^T; for Helmholtz (complex symmetric kernel, real T)
  Atilde = Atilde^T as well, hence Atilde^H v = conj(Atilde conj v);
* the error against O1 falls with the ID tolerance and stays within 10 tol;
* a planted mistake (a dropped colleague) breaks that bound.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2310_16668_amd as sk


def relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


CASES = {
    "lap2d_uniform": (lambda: workloads.uniform_points(3000, 2, 21), "laplace", 0.0, 24),
    "lap3d_uniform": (lambda: workloads.uniform_points(4000, 3, 22), "laplace", 0.0, 32),
    "lap3d_ellipsoid": (lambda: workloads.ellipsoid_points(5000, 23), "laplace", 0.0, 24),
    "helm3d_uniform": (lambda: workloads.uniform_points(4000, 3, 24), "helmholtz", 15.0, 32),
    "helm2d_uniform": (lambda: workloads.uniform_points(3000, 2, 25), "helmholtz", 100.0, 24),
}


def _charges(n, kind, seed, nrhs=1):
    q = workloads.charges(n, nrhs, seed, complex_=(kind == "helmholtz"))
    return q


@pytest.mark.parametrize("case", list(CASES))
def test_no_compression_equals_direct(case):
    mk, kind, kappa, b = CASES[case]
    x = mk()
    op = sk.build(x, kind, tol=1e-6, leaf_size=b, kappa=kappa, no_compression=True)
    P = op.export()
    assert P["max_level"] >= 3
    q = _charges(x.shape[0], kind, 1)
    u2 = oracle.apply(P, q)
    u1 = oracle.direct(x, q, kind, kappa)
    assert relerr(u2, u1) <= 1e-13
    w2 = oracle.apply(P, q, adjoint=True)
    w1 = np.conj(oracle.direct(x, np.conj(q), kind, kappa))
    assert relerr(w2, w1) <= 1e-13


@pytest.mark.parametrize("dim,kind,kappa,geom", [(2, "laplace", 0.0, "uniform"), (3, "laplace", 0.0, "uniform"),
                                                 (3, "laplace", 0.0, "ellipsoid"), (3, "helmholtz", 10.0, "uniform"),
                                                 (2, "helmholtz", 40.0, "uniform")])
def test_matrix_form_equals_o2(dim, kind, kappa, geom):
    x = workloads.uniform_points(700, dim, 31) if geom == "uniform" else workloads.ellipsoid_points(900, 32)
    op = sk.build(x, kind, tol=1e-4, leaf_size=12, kappa=kappa)
    P = op.export()
    assert P["max_level"] >= 3
    A = oracle.matrix_form(P)
    n = x.shape[0]
    rng = np.random.default_rng(1)
    Q = rng.uniform(-1, 1, (n, 4))
    if kind == "helmholtz":
        Q = Q + 1j * rng.uniform(-1, 1, (n, 4))
    U = oracle.apply(P, Q)
    assert relerr(U, A @ Q) <= 1e-13
    W = oracle.apply(P, Q, adjoint=True)
    assert relerr(W, A.conj().T @ Q) <= 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_symmetry_and_adjoint(case):
    mk, kind, kappa, b = CASES[case]
    x = mk()
    op = sk.build(x, kind, tol=1e-5, leaf_size=b, kappa=kappa)
    P = op.export()
    n = x.shape[0]
    q = _charges(n, kind, 2)
    v = _charges(n, kind, 3)
    Aq, Av = oracle.apply(P, q), oracle.apply(P, v)
    lhs, rhs = v @ Aq, q @ Av   # no conjugation: Atilde = Atilde^T
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    w = oracle.apply(P, v, adjoint=True)
    assert relerr(w, np.conj(oracle.apply(P, np.conj(v)))) <= 1e-13
    # <v, A q> = <A^H v, q>
    assert abs(np.vdot(v, Aq) - np.vdot(w, q)) <= 1e-13 * abs(np.vdot(v, Aq))


@pytest.mark.parametrize("case", list(CASES))
def test_error_falls_with_tolerance(case):
    mk, kind, kappa, b = CASES[case]
    x = mk()
    q = _charges(x.shape[0], kind, 4)
    u1 = oracle.direct(x, q, kind, kappa)
    errs = []
    for tol in (1e-3, 1e-5, 1e-7, 1e-9):
        op = sk.build(x, kind, tol=tol, leaf_size=b, kappa=kappa)
        e = relerr(oracle.apply(op.export(), q), u1)
        assert e <= 10 * tol, (tol, e)
        errs.append(e)
    # strictly falling until the operator is exact to rounding
    for a, b in zip(errs, errs[1:]):
        assert b < a or max(a, b) <= 1e-13, errs
    assert errs[0] > 1e-10


def test_linearity():
    mk, kind, kappa, b = CASES["lap3d_ellipsoid"]
    x = mk()
    P = sk.build(x, kind, tol=1e-6, leaf_size=b).export()
    n = x.shape[0]
    q1, q2 = _charges(n, kind, 5), _charges(n, kind, 6)
    lhs = oracle.apply(P, 0.3 * q1 - 1.7 * q2)
    rhs = 0.3 * oracle.apply(P, q1) - 1.7 * oracle.apply(P, q2)
    assert relerr(lhs, rhs) <= 1e-14
    both = oracle.apply(P, np.stack([q1, q2], axis=1))
    assert relerr(both[:, 0], oracle.apply(P, q1)) <= 1e-15


def test_masked_apply_matches_full_at_flagged_leaves():
    mk, kind, kappa, b = CASES["lap3d_ellipsoid"]
    x = mk()
    P = sk.build(x, kind, tol=1e-6, leaf_size=b).export()
    q = _charges(x.shape[0], kind, 7)
    full = oracle.apply(P, q)
    leaves = np.nonzero(P["is_leaf"])[0][::9]
    part = oracle.apply(P, q, box_mask=oracle.ancestors_mask(P, leaves))
    pts = np.concatenate([P["idx"][P["idx_ptr"][l]:P["idx_ptr"][l + 1]] for l in leaves])
    np.testing.assert_allclose(part[pts], full[pts], rtol=1e-13, atol=1e-14 * np.abs(full).max())


def test_planted_mistake_is_caught():
    """Drop one colleague pair between two compressed boxes: the bound against O1
    must break.  (A pair of two uncompressed boxes cancels exactly, so dropping it
    is harmless by construction.)"""
    x, kind, b = workloads.uniform_points(20000, 3, 25), "laplace", 64
    q = _charges(x.shape[0], kind, 8)
    tol = 1e-8
    P = sk.build(x, kind, tol=tol, leaf_size=b).export()
    u1 = oracle.direct(x, q)
    good = relerr(oracle.apply(P, q), u1)
    assert good <= 10 * tol
    n = np.diff(P["idx_ptr"])
    comp = (P["rank"] >= 0) & (P["rank"] < n)
    b0 = next(i for i in range(P["n_boxes"]) if comp[i] and any(
        comp[c] and c != i for c in P["coll_idx"][P["coll_ptr"][i]:P["coll_ptr"][i + 1]]))
    s, e = P["coll_ptr"][b0], P["coll_ptr"][b0 + 1]
    drop = s + int(next(j for j in range(e - s) if P["coll_idx"][s + j] != b0 and comp[P["coll_idx"][s + j]]))
    bad = dict(P)
    bad["coll_idx"] = np.delete(P["coll_idx"], drop)
    bad["coll_ptr"] = P["coll_ptr"].copy()
    bad["coll_ptr"][b0 + 1:] -= 1
    bad_err = relerr(oracle.apply(bad, q), u1)
    assert bad_err > 10 * tol and bad_err > 100 * good


def test_one_level_and_root_leaf_are_exact():
    x = workloads.uniform_points(300, 3, 41)
    q = _charges(300, "laplace", 9)
    u1 = oracle.direct(x, q)
    P = sk.build(x, "laplace", tol=1e-6, leaf_size=400).export()   # root is a leaf
    assert P["top_level"] == 0 and P["n_boxes"] == 1
    assert relerr(oracle.apply(P, q), u1) <= 1e-14
    P = sk.build(x, "laplace", tol=1e-6, leaf_size=100).export()   # leaves on level 1
    assert P["max_level"] == 1
    assert relerr(oracle.apply(P, q), u1) <= 1e-14
