"""Host build: tree invariants, neighbor relations by brute force, and ID quality.

The tree, its 2:1 balance and the neighbor lists follow section 3 ("Adaptive
tree data structure"); the skeletons follow section 2.1 (equation (5), proxy
surface) and the build stage of section 3.
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads
import paper_2310_16668_amd as sk


def _cases():
    return {
        "uniform3d": (workloads.uniform_points(6000, 3, 1), 3, 40),
        "ellipsoid3d": (workloads.ellipsoid_points(8000, 2), 3, 32),
        "uniform2d": (workloads.uniform_points(5000, 2, 3), 2, 30),
        "clustered2d": (np.vstack([workloads.uniform_points(3000, 2, 4) * 0.01 + 0.3,
                                   workloads.uniform_points(1000, 2, 5)]), 2, 16),
    }


@pytest.fixture(scope="module", params=list(_cases().keys()))
def built(request):
    x, dim, b = _cases()[request.param]
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=b)
    return x, b, op.export(), op.stats()


def _touch(la, ca, lb, cb, dim, D=20):
    """Closed cubes (level, integer coords) intersect."""
    sa, sb = 1 << (D - la), 1 << (D - lb)
    for d in range(dim):
        lo = max(ca[d] * sa, cb[d] * sb)
        hi = min((ca[d] + 1) * sa, (cb[d] + 1) * sb)
        if lo > hi:
            return False
    return True


def _interior_overlap(la, ca, lb, cb, dim, D=20):
    sa, sb = 1 << (D - la), 1 << (D - lb)
    for d in range(dim):
        if min((ca[d] + 1) * sa, (cb[d] + 1) * sb) <= max(ca[d] * sa, cb[d] * sb):
            return False
    return True


def test_partition_and_leaf_size(built):
    x, b, P, _ = built
    n = x.shape[0]
    seen = np.zeros(n, dtype=int)
    for bx in np.nonzero(P["is_leaf"])[0]:
        ids = P["idx"][P["idx_ptr"][bx]:P["idx_ptr"][bx + 1]]
        seen[ids] += 1
        assert len(ids) <= b or P["level"][bx] == 20
        # the leaf's points lie in its cube
        a = P["root_side"] / 2 ** P["level"][bx]
        lo = P["root_lo"][:P["dim"]] + P["coord"][bx, :P["dim"]] * a
        assert np.all(x[ids] >= lo - 1e-12) and np.all(x[ids] <= lo + a + 1e-12)
    assert np.all(seen == 1)


def test_parent_child_and_concat(built):
    _, _, P, _ = built
    top = P["top_level"]
    for bx in range(P["n_boxes"]):
        kids = P["child_idx"][P["child_ptr"][bx]:P["child_ptr"][bx + 1]]
        assert len(kids) <= 2 ** P["dim"]
        assert (len(kids) == 0) == bool(P["is_leaf"][bx])
        for c in kids:
            assert P["parent"][c] == bx and P["level"][c] == P["level"][bx] + 1
            assert np.all(P["coord"][c] // 2 == P["coord"][bx])
        if P["level"][bx] >= top and not P["is_leaf"][bx]:
            cat = []
            for c in kids:
                ic = P["idx"][P["idx_ptr"][c]:P["idx_ptr"][c + 1]]
                pc = P["pos"][P["idx_ptr"][c]:P["idx_ptr"][c] + P["rank"][c]]
                cat.extend(ic[pc])
            assert np.array_equal(P["idx"][P["idx_ptr"][bx]:P["idx_ptr"][bx + 1]], cat)


def test_strong_balance_and_neighbors_brute_force(built):
    _, _, P, _ = built
    dim, nb = P["dim"], P["n_boxes"]
    lev, crd, leaf = P["level"], P["coord"], P["is_leaf"]
    for i in range(nb):
        for j in range(nb):
            if leaf[i] and lev[j] >= lev[i] + 2:
                assert not _touch(lev[i], crd[i], lev[j], crd[j], dim), "strong 2:1 balance violated"
    for i in range(nb):
        coll = set(P["coll_idx"][P["coll_ptr"][i]:P["coll_ptr"][i + 1]].tolist())
        brute = {j for j in range(nb) if lev[j] == lev[i] and _touch(lev[i], crd[i], lev[j], crd[j], dim)}
        assert coll == brute and i in coll and len(coll) <= 3 ** dim
        coarse = set(P["coarse_idx"][P["coarse_ptr"][i]:P["coarse_ptr"][i + 1]].tolist())
        brute_c = {j for j in range(nb) if lev[j] == lev[i] - 1 and leaf[j]
                   and _touch(lev[i], crd[i], lev[j], crd[j], dim)
                   and not _interior_overlap(lev[i], crd[i], lev[j], crd[j], dim)}
        assert coarse == brute_c
        fine = set(P["fine_idx"][P["fine_ptr"][i]:P["fine_ptr"][i + 1]].tolist())
        assert fine == {j for j in range(nb) if i in
                        set(P["coarse_idx"][P["coarse_ptr"][j]:P["coarse_ptr"][j + 1]].tolist())}
        if fine:
            assert leaf[i]


def test_adaptive_lists_present():
    x, dim, b = _cases()["ellipsoid3d"]
    P = sk.build(x, "laplace", tol=1e-6, leaf_size=b).export()
    assert len(P["coarse_idx"]) > 0 and len(P["fine_idx"]) > 0
    assert len(np.unique(P["level"][P["is_leaf"] == 1])) >= 3


def test_identical_points_hit_depth_cap():
    x = np.vstack([np.full((50, 3), 0.5), workloads.uniform_points(200, 3, 9)])
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=8)
    P = op.export()
    assert P["max_level"] == 20
    big = [b for b in np.nonzero(P["is_leaf"])[0] if P["idx_ptr"][b + 1] - P["idx_ptr"][b] > 8]
    assert big and all(P["level"][b] == 20 for b in big)


def _proxy_matrix(P, b, kind, kappa, p):
    """Proxy matrix of box b by its definition (first-kind Chebyshev nodes on the
    faces of a cube of side 2.95 a around the box)."""
    a = P["root_side"] / 2 ** P["level"][b]
    c = P["root_lo"] + (P["coord"][b] + 0.5) * a
    t = np.cos((2 * np.arange(p) + 1) * np.pi / (2 * p)) * 1.475 * a
    Y = []
    for ax in range(3):
        for sgn in (-1, 1):
            for i, j in itertools.product(range(p), range(p)):
                y = np.zeros(3)
                y[ax] = sgn * 1.475 * a
                y[(ax + 1) % 3], y[(ax + 2) % 3] = t[i], t[j]
                Y.append(c + y)
    ids = P["idx"][P["idx_ptr"][b]:P["idx_ptr"][b + 1]]
    return oracle.kernel(np.array(Y), P["points"][ids], kind, kappa), ids


@pytest.mark.parametrize("kind,kappa,tol", [("laplace", 0.0, 1e-6), ("laplace", 0.0, 1e-9), ("helmholtz", 12.0, 1e-6)])
def test_interpolative_decomposition_quality(kind, kappa, tol):
    x = workloads.uniform_points(20000, 3, 12)
    op = sk.build(x, kind, tol=tol, leaf_size=64, kappa=kappa, proxy_points=10)
    P = op.export()
    rng = np.random.default_rng(0)
    boxes = [b for b in range(P["n_boxes"]) if P["rank"][b] > 0 and P["rank"][b] < P["idx_ptr"][b + 1] - P["idx_ptr"][b]]
    for b in rng.choice(boxes, 6, replace=False):
        n = P["idx_ptr"][b + 1] - P["idx_ptr"][b]
        k = P["rank"][b]
        pos = P["pos"][P["idx_ptr"][b]:P["idx_ptr"][b + 1]]
        T = P["T"][P["T_ptr"][b]:P["T_ptr"][b + 1]].reshape(n - k, k).T
        M, ids = _proxy_matrix(P, b, kind, kappa, 10)
        res = np.linalg.norm(M[:, pos[k:]] - M[:, pos[:k]] @ T) / np.linalg.norm(M)
        assert res <= 10 * tol, res
        # true far field: points outside the 3a box around the box
        a = P["root_side"] / 2 ** P["level"][b]
        c = P["root_lo"] + (P["coord"][b] + 0.5) * a
        far = x[np.max(np.abs(x - c), axis=1) > 1.5 * a]
        F = oracle.kernel(far, P["points"][ids], kind, kappa)
        res_f = np.linalg.norm(F[:, pos[k:]] - F[:, pos[:k]] @ T) / np.linalg.norm(F)
        assert res_f <= 10 * tol, res_f
