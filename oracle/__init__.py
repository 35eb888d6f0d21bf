"""ORACLE -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library never does, and this package never imports
the library: skeleton operators reach it as plain numpy arrays.

* ``direct``      O1, the dense direct sum that defines the problem (section 1,
                  u_i = sum_{j != i} G(x_i, x_j) q_j), compiled C with OpenMP and
                  Neumaier-compensated accumulation.
* ``dense_matrix`` the same definition as an explicit numpy matrix, for tiny N.
* ``apply``       O2, a float64 CPU apply of given skeleton operators following
                  the FMM apply of section 3 step by step; ``adjoint=True`` runs
                  its literal transpose.
* ``matrix_form`` the approximate operator assembled densely from the recursive
                  factorization of section 2.3 (equation (13)), for tiny trees.

Pins for each of these live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "direct.c"), os.path.join(_HERE, "apply.c"), os.path.join(_HERE, "hankel.c")]

KIND = {"laplace": 0, "helmholtz": 1}


def build(force: bool = True) -> str:
    """Compile the oracle's C sources with gcc + OpenMP into oracle/liboracle.so."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", tmp, *_SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.oracle_direct.restype = ctypes.c_int
        _lib.oracle_apply.restype = ctypes.c_int
        _lib.oracle_num_threads.restype = ctypes.c_int
        _lib.oracle_h0_many.restype = None
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a: np.ndarray, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_values(q: np.ndarray, kind: str):
    """(n,) or (n, nrhs) real/complex -> contiguous float64 (n, W) and nrhs."""
    q = np.asarray(q)
    squeeze = q.ndim == 1
    q2 = q.reshape(q.shape[0], -1)
    nrhs = q2.shape[1]
    if kind == "helmholtz":
        q2 = np.ascontiguousarray(q2.astype(np.complex128)).view(np.float64)
    else:
        if np.iscomplexobj(q2):
            raise ValueError("Laplace takes real charges")
        q2 = np.ascontiguousarray(q2, dtype=np.float64)
    return q2, nrhs, squeeze


def _from_values(out: np.ndarray, kind: str, squeeze: bool):
    if kind == "helmholtz":
        out = out.view(np.complex128)
    return out[:, 0] if squeeze else out


def direct(points, q, kind="laplace", kappa=0.0, targets=None):
    """O1: u[t] = sum_{j != targets[t]} G(x_targets[t], x_j) q_j, float64 / complex128."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = pts.shape
    q2, nrhs, squeeze = _as_values(q, kind)
    targ = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    out = np.zeros((targ.shape[0], q2.shape[1]), dtype=np.float64)
    rc = _load().oracle_direct(
        ctypes.c_int(dim), ctypes.c_int(KIND[kind]), ctypes.c_double(kappa), ctypes.c_int64(n),
        _ptr(pts), ctypes.c_int(nrhs), _ptr(q2), ctypes.c_int64(targ.shape[0]),
        _ptr(targ, ctypes.c_int64), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_direct: unsupported dim/kind")
    return _from_values(out, kind, squeeze)


def h0(x) -> np.ndarray:
    """H0^(1)(x) = J0(x) + i Y0(x) for x > 0, as the oracle's C code evaluates it
    (the 2D Helmholtz kernel is (i/4) H0^(1)(kappa r))."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    j = np.zeros_like(x)
    y = np.zeros_like(x)
    _load().oracle_h0_many(ctypes.c_int64(x.size), _ptr(x), _ptr(j), _ptr(y))
    return j + 1j * y


def kernel(points_t, points_s, kind="laplace", kappa=0.0, same=None):
    """Dense kernel block G(x_t, x_s) by its definition (section 2), numpy.

    ``same`` is a boolean mask of (t, s) pairs that are the same point (the
    excluded diagonal); pairs at distance zero are zero as well.
    """
    xt = np.asarray(points_t, dtype=np.float64)
    xs = np.asarray(points_s, dtype=np.float64)
    dim = xt.shape[1]
    d = xt[:, None, :] - xs[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    zero = r == 0.0
    if same is not None:
        zero = zero | same
    rs = np.where(zero, 1.0, r)
    if kind == "laplace":
        g = -np.log(rs) / (2 * np.pi) if dim == 2 else 1.0 / (4 * np.pi * rs)
    elif dim == 2:
        from scipy.special import hankel1   # an independent evaluation of H0^(1)
        g = 0.25j * hankel1(0, kappa * rs)
    else:
        g = np.exp(1j * kappa * rs) / (4 * np.pi * rs)
    return np.where(zero, 0.0, g)


def dense_matrix(points, kind="laplace", kappa=0.0):
    """The N x N matrix A of the problem statement, zero diagonal (tiny N only)."""
    n = points.shape[0]
    return kernel(points, points, kind, kappa, same=np.eye(n, dtype=bool))


class _O2Plan(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("kind", ctypes.c_int32), ("kappa", ctypes.c_double),
        ("n_points", ctypes.c_int64), ("pts", ctypes.POINTER(ctypes.c_double)),
        ("n_boxes", ctypes.c_int32), ("top_level", ctypes.c_int32), ("max_level", ctypes.c_int32),
        ("level", ctypes.POINTER(ctypes.c_int32)), ("parent", ctypes.POINTER(ctypes.c_int32)),
        ("is_leaf", ctypes.POINTER(ctypes.c_int32)), ("child_ptr", ctypes.POINTER(ctypes.c_int32)),
        ("child_idx", ctypes.POINTER(ctypes.c_int32)),
        ("idx_ptr", ctypes.POINTER(ctypes.c_int64)), ("idx", ctypes.POINTER(ctypes.c_int64)),
        ("pos", ctypes.POINTER(ctypes.c_int64)),
        ("rank", ctypes.POINTER(ctypes.c_int32)),
        ("T_ptr", ctypes.POINTER(ctypes.c_int64)), ("T", ctypes.POINTER(ctypes.c_double)),
        ("coll_ptr", ctypes.POINTER(ctypes.c_int32)), ("coll_idx", ctypes.POINTER(ctypes.c_int32)),
        ("coarse_ptr", ctypes.POINTER(ctypes.c_int32)), ("coarse_idx", ctypes.POINTER(ctypes.c_int32)),
        ("fine_ptr", ctypes.POINTER(ctypes.c_int32)), ("fine_idx", ctypes.POINTER(ctypes.c_int32)),
    ]


_I32 = ("level", "parent", "is_leaf", "child_ptr", "child_idx", "rank",
        "coll_ptr", "coll_idx", "coarse_ptr", "coarse_idx", "fine_ptr", "fine_idx")
_I64 = ("idx_ptr", "idx", "pos", "T_ptr")


def _make_plan(plan: dict):
    """Keep contiguous copies alive and fill the C struct from a plan dict."""
    keep = {}
    for k in _I32:
        keep[k] = np.ascontiguousarray(plan[k], dtype=np.int32)
        if keep[k].size == 0:
            keep[k] = np.zeros(1, dtype=np.int32)
    for k in _I64:
        keep[k] = np.ascontiguousarray(plan[k], dtype=np.int64)
        if keep[k].size == 0:
            keep[k] = np.zeros(1, dtype=np.int64)
    keep["T"] = np.ascontiguousarray(plan["T"], dtype=np.float64)
    if keep["T"].size == 0:
        keep["T"] = np.zeros(1)
    keep["pts"] = np.ascontiguousarray(plan["points"], dtype=np.float64)
    s = _O2Plan()
    s.dim = int(plan["dim"])
    s.kind = KIND[plan["kind"]]
    s.kappa = float(plan.get("kappa", 0.0))
    s.n_points = keep["pts"].shape[0]
    s.pts = _ptr(keep["pts"])
    s.n_boxes = int(plan["n_boxes"])
    s.top_level = int(plan["top_level"])
    s.max_level = int(plan["max_level"])
    for k in _I32:
        setattr(s, k, _ptr(keep[k], ctypes.c_int32))
    for k in _I64:
        setattr(s, k, _ptr(keep[k], ctypes.c_int64))
    s.T = _ptr(keep["T"])
    return s, keep


def apply(plan: dict, q, adjoint: bool = False, box_mask=None):
    """O2 (or its transpose): the approximate operator of the given plan times q.

    ``plan`` holds the skeleton operators as numpy arrays (see ``_O2Plan``).
    ``box_mask`` (forward only) restricts the translations to flagged target
    boxes; results are then valid only at leaves whose ancestors are all flagged.
    """
    kind = plan["kind"]
    q2, nrhs, squeeze = _as_values(q, kind)
    s, keep = _make_plan(plan)
    out = np.zeros_like(q2)
    mask_p = None
    if box_mask is not None:
        if adjoint:
            raise ValueError("box_mask is forward-only")
        keep["mask"] = np.ascontiguousarray(box_mask, dtype=np.uint8)
        mask_p = _ptr(keep["mask"], ctypes.c_uint8)
    rc = _load().oracle_apply(ctypes.byref(s), ctypes.c_int(nrhs), _ptr(q2), _ptr(out),
                              ctypes.c_int(1 if adjoint else 0), mask_p)
    if rc == -2:
        raise ValueError("plan: a tree box's index set is not its children's skeletons")
    if rc != 0:
        raise MemoryError("oracle_apply failed")
    return _from_values(out, kind, squeeze)


def ancestors_mask(plan: dict, leaves) -> np.ndarray:
    """Per-box flags for the given leaves and all their ancestors."""
    m = np.zeros(int(plan["n_boxes"]), dtype=np.uint8)
    parent = plan["parent"]
    for b in leaves:
        b = int(b)
        while b >= 0 and not m[b]:
            m[b] = 1
            b = int(parent[b])
    return m


def matrix_form(plan: dict) -> np.ndarray:
    """Dense approximate operator from the recursive factorization (section 2.3).

    For tiny trees only.  Level by level, from the top level down:
        A^(top)  = kernel matrix on the top level's index sets (all pairs)
        A^(l)    = N_l - E_l N^S_l F_l + E_l A^(l-1) F_l + (adaptive terms)
    written here as the sum over the paper's translations, each as an explicit
    dense block placed into an N x N matrix through the E / F operators of every
    level (E_B = [I; T^*], F_B = [I T] in skeleton/redundant positions).
    """
    n = plan["points"].shape[0]
    pts = plan["points"]
    kind, kappa = plan["kind"], float(plan.get("kappa", 0.0))
    nb = int(plan["n_boxes"])
    level, parent, is_leaf = plan["level"], plan["parent"], plan["is_leaf"]
    idx_ptr, idx, pos, rank = plan["idx_ptr"], plan["idx"], plan["pos"], plan["rank"]
    T_ptr, Tall = plan["T_ptr"], plan["T"]
    top = int(plan["top_level"])

    def bidx(b):
        return idx[idx_ptr[b]:idx_ptr[b + 1]]

    def skel(b):
        k = int(rank[b])
        return bidx(b)[pos[idx_ptr[b]:idx_ptr[b] + k]]

    def Fmat(b):
        """F_B as a k x n matrix acting on B's natural order."""
        nbb = idx_ptr[b + 1] - idx_ptr[b]
        k = int(rank[b])
        p = pos[idx_ptr[b]:idx_ptr[b + 1]]
        T = Tall[T_ptr[b]:T_ptr[b] + k * (nbb - k)].reshape(nbb - k, k).T  # column-major k x (n-k)
        F = np.zeros((k, nbb))
        F[np.arange(k), p[:k]] = 1.0
        F[:, p[k:]] = T
        return F

    # Z_B: maps the N-vector of charges to box B's natural-order vector q_B
    # (leaf: selection; tree box: stacked F_c Z_c of its children).
    Z = {}
    order = np.argsort(-np.asarray(level), kind="stable")
    for b in order:
        b = int(b)
        if level[b] < top:
            continue
        if is_leaf[b]:
            M = np.zeros((idx_ptr[b + 1] - idx_ptr[b], n))
            M[np.arange(M.shape[0]), bidx(b)] = 1.0
        else:
            kids = plan["child_idx"][plan["child_ptr"][b]:plan["child_ptr"][b + 1]]
            M = np.vstack([Fmat(int(c)) @ Z[int(c)] for c in kids])
        Z[b] = M

    def Fz(b):
        return Fmat(b) @ Z[b]      # N -> k_B : qhat_B as a function of q

    def Ez(b):
        return Fz(b).T            # k_B -> N, real T: E_B = F_B^T

    def G(ti, si):
        return kernel(pts[ti], pts[si], kind, kappa, same=(ti[:, None] == si[None, :]))

    dt = np.complex128 if kind == "helmholtz" else np.float64
    A = np.zeros((n, n), dtype=dt)
    coll_ptr, coll_idx = plan["coll_ptr"], plan["coll_idx"]
    co_ptr, co_idx = plan["coarse_ptr"], plan["coarse_idx"]
    fi_ptr, fi_idx = plan["fine_ptr"], plan["fine_idx"]
    for b in range(nb):
        lb = int(level[b])
        if lb < top:
            continue
        if lb == top:
            for c in range(nb):
                if level[c] == top:
                    A += Z[b].T @ G(bidx(b), bidx(c)) @ Z[c]
        else:
            for c in coll_idx[coll_ptr[b]:coll_ptr[b + 1]]:
                c = int(c)
                A += Z[b].T @ G(bidx(b), bidx(c)) @ Z[c]
                A -= Ez(b) @ G(skel(b), skel(c)) @ Fz(c)
            for c in co_idx[co_ptr[b]:co_ptr[b + 1]]:
                c = int(c)
                A += Z[b].T @ G(bidx(b), bidx(c)) @ Z[c]
                A -= Ez(b) @ G(skel(b), bidx(c)) @ Z[c]
        if is_leaf[b]:
            for c in fi_idx[fi_ptr[b]:fi_ptr[b + 1]]:
                c = int(c)
                A += Z[b].T @ G(bidx(b), bidx(c)) @ Z[c]
                A -= Z[b].T @ G(bidx(b), skel(c)) @ Fz(c)
    return A
