"""Pins for O1, the dense direct sum (section 1: u_i = sum_{j != i} G(x_i, x_j) q_j).

Each pin reaches the definition another way: exact distances of integer point
sets, brute force as an explicit numpy matrix, geometric closed forms
(equidistant charges), and the invariances the kernels must satisfy.
"""
import cmath
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "direct_sum_small.txt")


def _read_golden():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    pts = np.array([[float(v) for v in r] for r in rows[:4]])
    q = np.array([float(v) for v in rows[4]])
    return pts, q


def test_golden_closed_form():
    pts, q = _read_golden()
    # exact 3D distances of the integer point set (Pythagorean triples 3-4-5, 5-12-13)
    r3 = {(0, 1): 5, (0, 2): 12, (0, 3): 13, (1, 2): 13, (1, 3): 12, (2, 3): 5}
    r2 = {(0, 1): 5, (0, 2): 0, (0, 3): 5, (1, 2): 5, (1, 3): 0, (2, 3): 5}

    def dist(tab, i, j):
        return tab[(min(i, j), max(i, j))]

    kappa = 0.7
    for i in range(4):
        lap3 = sum(q[j] / dist(r3, i, j) for j in range(4) if j != i) / (4 * math.pi)
        lap2 = sum(-math.log(dist(r2, i, j)) * q[j] for j in range(4) if j != i and dist(r2, i, j) > 0) / (2 * math.pi)
        helm = sum(cmath.exp(1j * kappa * dist(r3, i, j)) / dist(r3, i, j) * q[j] for j in range(4) if j != i) / (4 * math.pi)
        assert oracle.direct(pts, q)[i] == pytest.approx(lap3, rel=1e-15, abs=1e-16)
        assert oracle.direct(pts[:, :2], q)[i] == pytest.approx(lap2, rel=1e-14, abs=1e-16)
        assert oracle.direct(pts, q.astype(complex), "helmholtz", kappa)[i] == pytest.approx(helm, rel=1e-14)


@pytest.mark.parametrize("dim,kind", [(2, "laplace"), (3, "laplace"), (3, "helmholtz"), (2, "helmholtz")])
def test_brute_force_matrix(dim, kind):
    rng = np.random.default_rng(5)
    n = 300
    x = rng.random((n, dim))
    kappa = 9.0
    q = rng.uniform(-1, 1, (n, 3))
    if kind == "helmholtz":
        q = q + 1j * rng.uniform(-1, 1, (n, 3))
    A = oracle.dense_matrix(x, kind, kappa)
    ref = A @ q
    got = oracle.direct(x, q, kind, kappa)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
    # the diagonal is excluded: a single charge does not act on itself
    e = np.zeros(n, dtype=q.dtype)
    e[17] = 1.0
    col = oracle.direct(x, e, kind, kappa)
    assert col[17] == 0.0
    assert np.max(np.abs(col - A[:, 17])) <= 1e-15 * np.max(np.abs(A[:, 17]))


@pytest.mark.parametrize("dim,kind", [(2, "laplace"), (3, "laplace"), (3, "helmholtz"), (2, "helmholtz")])
def test_equidistant_charges(dim, kind):
    """A target at the centre of M charges on a circle / sphere of radius R."""
    rng = np.random.default_rng(11)
    M, R, kappa = 257, 0.37, 6.0
    d = rng.standard_normal((M, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c = np.full(dim, 0.25)
    x = np.vstack([c, c + R * d])
    q = np.concatenate([[0.0], rng.uniform(-1, 1, M)])
    if kind == "helmholtz":
        q = q.astype(complex)
    u0 = oracle.direct(x, q, kind, kappa, targets=np.array([0]))[0]
    s = q[1:].sum()
    if kind == "helmholtz" and dim == 2:
        from scipy.special import hankel1   # an independent evaluation of H0^(1)
        ref = 0.25j * hankel1(0, kappa * R) * s
    elif kind == "helmholtz":
        ref = cmath.exp(1j * kappa * R) / (4 * math.pi * R) * s
    elif dim == 3:
        ref = s / (4 * math.pi * R)
    else:
        ref = -math.log(R) / (2 * math.pi) * s
    assert abs(u0 - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("dim,kind", [(2, "laplace"), (3, "laplace"), (3, "helmholtz"), (2, "helmholtz")])
def test_symmetric_not_hermitian(dim, kind):
    rng = np.random.default_rng(3)
    n = 500
    x = rng.random((n, dim))
    q, v = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    if kind == "helmholtz":
        q = q + 1j * rng.uniform(-1, 1, n)
        v = v + 1j * rng.uniform(-1, 1, n)
    a = v @ oracle.direct(x, q, kind, 8.0)    # v^T A q, no conjugation
    b = q @ oracle.direct(x, v, kind, 8.0)
    assert abs(a - b) <= 1e-13 * abs(a)
    if kind == "helmholtz":   # A is symmetric, so it is not Hermitian
        ah = np.conj(v) @ oracle.direct(x, q, kind, 8.0)
        bh = np.conj(oracle.direct(x, v, kind, 8.0)) @ q
        assert abs(ah - bh) > 1e-3 * abs(ah)


def test_scaling_laws():
    rng = np.random.default_rng(4)
    n, s = 400, 3.5
    x3, x2 = rng.random((n, 3)), rng.random((n, 2))
    q = rng.uniform(-1, 1, n)
    # 3D Laplace is homogeneous of degree -1
    np.testing.assert_allclose(oracle.direct(s * x3, q), oracle.direct(x3, q) / s, rtol=1e-13)
    # 2D Laplace: -log(s r) = -log r - log s, summed over j != i
    ref = oracle.direct(x2, q) - math.log(s) / (2 * math.pi) * (q.sum() - q)
    np.testing.assert_allclose(oracle.direct(s * x2, q), ref, rtol=1e-12, atol=1e-13)
    # Helmholtz: G(s r; kappa / s) = G(r; kappa) / s
    qc = q + 1j * rng.uniform(-1, 1, n)
    np.testing.assert_allclose(oracle.direct(s * x3, qc, "helmholtz", 4.0 / s),
                               oracle.direct(x3, qc, "helmholtz", 4.0) / s, rtol=1e-12)


def test_rigid_motion_invariance():
    rng = np.random.default_rng(8)
    n = 400
    x = rng.random((n, 3))
    q = rng.uniform(-1, 1, n)
    Qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    y = x @ Qm.T + np.array([0.3, -2.0, 5.0])
    np.testing.assert_allclose(oracle.direct(y, q), oracle.direct(x, q), rtol=1e-11)


def test_coincident_points_contribute_zero():
    x = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [0.6, 0.2, 0.3]])
    q = np.array([1.0, 2.0, 4.0])
    u = oracle.direct(x, q)
    # points 0 and 1 coincide: only point 2 acts on them, at r = 0.5
    assert u[0] == pytest.approx(4.0 / (4 * math.pi * 0.5), rel=1e-15)
    assert u[1] == pytest.approx(4.0 / (4 * math.pi * 0.5), rel=1e-15)
    assert u[2] == pytest.approx(3.0 / (4 * math.pi * 0.5), rel=1e-15)


def test_subset_targets_match_full():
    rng = np.random.default_rng(2)
    x = rng.random((1000, 3))
    q = rng.uniform(-1, 1, (1000, 2))
    t = np.array([0, 5, 999, 400])
    np.testing.assert_array_equal(oracle.direct(x, q, targets=t), oracle.direct(x, q)[t])
