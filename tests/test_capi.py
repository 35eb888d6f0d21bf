"""C ABI checks that need no GPU: every declared entry point is exported, and
argument errors come back as status codes with a message, before any GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2310_16668_amd as sk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skelfmm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(skelfmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(sk.library_path())
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sk.EXPORTED)


def _build_raw(points, n, dim=3, kind=0, kappa=0.0, tol=1e-6, leaf=16, opt=None, out=True):
    lib = sk._lib
    h = ctypes.c_void_p()
    ptr = points.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if points is not None else None
    st = lib.skelfmm_build(ptr, n, sk.Kernel(kind, dim, kappa), tol, leaf, opt,
                           ctypes.byref(h) if out else None)
    return st, h


@pytest.mark.parametrize("case,expect", [
    ("null_points", -1), ("n_zero", -1), ("bad_dim", -1), ("tol_zero", -1), ("tol_one", -1),
    ("leaf_zero", -1), ("neg_kappa", -1), ("nan_point", -1), ("helm_2d_neg_kappa", -1), ("bad_kind", -1),
    ("null_out", -1), ("bad_proxy", -1),
])
def test_build_argument_errors(case, expect):
    x = np.random.default_rng(0).random((100, 3))
    kw = {}
    if case == "null_points":
        st, _ = _build_raw(None, 100)
    elif case == "n_zero":
        st, _ = _build_raw(x, 0)
    elif case == "bad_dim":
        st, _ = _build_raw(x, 100, dim=4)
    elif case == "tol_zero":
        st, _ = _build_raw(x, 100, tol=0.0)
    elif case == "tol_one":
        st, _ = _build_raw(x, 100, tol=1.0)
    elif case == "leaf_zero":
        st, _ = _build_raw(x, 100, leaf=0)
    elif case == "neg_kappa":
        st, _ = _build_raw(x, 100, kind=1, kappa=-1.0)
    elif case == "nan_point":
        y = x.copy()
        y[5, 1] = np.nan
        st, _ = _build_raw(y, 100)
    elif case == "helm_2d_neg_kappa":
        st, _ = _build_raw(np.ascontiguousarray(x[:, :2]), 100, dim=2, kind=1, kappa=-1.0)
    elif case == "bad_kind":
        st, _ = _build_raw(x, 100, kind=7)
    elif case == "null_out":
        st, _ = _build_raw(x, 100, out=False)
    else:
        o = sk.Options()
        o.proxy_shape = 2      # the proxy circle is 2D only
        st, _ = _build_raw(x, 100, opt=ctypes.byref(o))
    assert st == expect, (case, st)
    assert len(sk._lib.skelfmm_last_error()) > 0


def test_apply_argument_errors_before_gpu_work():
    x = np.random.default_rng(1).random((300, 3))
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=32)
    lib = sk._lib
    buf = ctypes.c_void_p(0x1000)
    # NULL vectors, aliasing, bad nrhs, dtype / kernel mismatch: all EINVAL, no device touched
    assert lib.skelfmm_apply(op.handle, None, buf, 1, sk.F64, None) == -1
    assert lib.skelfmm_apply(op.handle, buf, buf, 1, sk.F64, None) == -1
    assert lib.skelfmm_apply(op.handle, buf, ctypes.c_void_p(0x2000), 0, sk.F64, None) == -1
    assert lib.skelfmm_apply(op.handle, buf, ctypes.c_void_p(0x2000), 1, sk.C128, None) == -1
    assert lib.skelfmm_apply(op.handle, buf, ctypes.c_void_p(0x2000), 1, 9, None) == -1
    assert lib.skelfmm_apply(None, buf, ctypes.c_void_p(0x2000), 1, sk.F64, None) == -1
    b2, b3, b4 = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000)
    assert lib.skelfmm_apply_fwd_adj(op.handle, None, b2, b3, b4, sk.F32, None) == -1
    assert lib.skelfmm_apply_fwd_adj(op.handle, buf, b2, b3, b3, sk.F32, None) == -1
    assert lib.skelfmm_apply_fwd_adj(op.handle, buf, b2, buf, b4, sk.F32, None) == -1
    assert lib.skelfmm_apply_fwd_adj(op.handle, buf, b2, b3, b4, sk.C64, None) == -1
    assert lib.skelfmm_apply_fwd_adj(None, buf, b2, b3, b4, sk.F32, None) == -1
    assert lib.skelfmm_autotune_fwd_adj(op.handle, None, None, None) == -1
    assert lib.skelfmm_set_targets_per_lane(op.handle, 5) == -1
    assert lib.skelfmm_set_targets_per_lane(op.handle, 0) == -1
    assert lib.skelfmm_set_targets_per_lane(op.handle, 3) == 0
    assert lib.skelfmm_set_targets_per_lane(op.handle, 4) == 0
    assert b"complex" in lib.skelfmm_last_error() or lib.skelfmm_last_error() != b""


def test_stats_and_export_consistent():
    x = np.random.default_rng(2).random((3000, 3))
    op = sk.build(x, "laplace", tol=1e-6, leaf_size=32)
    st = op.stats()
    P = op.export()
    assert st["n_points"] == 3000 and st["n_boxes"] == P["n_boxes"]
    assert st["n_leaves"] == int(P["is_leaf"].sum())
    assert st["m_proj_elems"] == P["T"].size
    assert st["k_max"] == int(P["rank"].max())
    assert st["pairs_near"] > 0 and st["t_skel"] >= 0


def test_destroy_and_batch_null_safe():
    sk._lib.skelfmm_destroy(None)
    sk._lib.skelfmm_batch_destroy(None)
    assert sk._lib.skelfmm_batch_create(None, 0, ctypes.byref(ctypes.c_void_p())) == -1


def test_batch_rejects_mixed_kernels():
    x = np.random.default_rng(3).random((500, 3))
    a = sk.build(x, "laplace", tol=1e-6, leaf_size=32)
    b = sk.build(x, "helmholtz", tol=1e-6, leaf_size=32, kappa=2.0)
    with pytest.raises(sk.SkelfmmError) as e:
        sk.Batch([a, b])
    assert e.value.status == -1


def test_f32_differences_gate_is_the_tighter_reach_bound():
    """An item takes float32 differences only where its reach is at most 1024 x its
    smallest spacing, a subset of the items whose reach allows the expanded form
    (4096 x): with the option, expanded + float32-difference items equal the
    expanded items without it.  Batches must agree on the option."""
    x = np.random.default_rng(5).random((20000, 3))
    a = sk.build(x, "laplace", tol=1e-7, leaf_size=64)
    b = sk.build(x, "laplace", tol=1e-7, leaf_size=64, f32_differences=True)
    sa, sb = a.stats(), b.stats()
    assert sa["n_sym_f32diff"] == 0
    assert 0 < sb["n_sym_f32diff"] <= sa["n_sym_expanded"]
    assert sb["n_sym_f32diff"] + sb["n_sym_expanded"] == sa["n_sym_expanded"]
    assert sb["n_sym_tasks"] == sa["n_sym_tasks"]
    c = sk.build(x, "laplace", tol=1e-7, leaf_size=64, expansion=False, f32_differences=True)
    assert c.stats()["n_sym_expanded"] == 0 and c.stats()["n_sym_f32diff"] == sb["n_sym_f32diff"]
    with pytest.raises(sk.SkelfmmError) as e:
        sk.Batch([a, b])
    assert e.value.status == -1 and b"pairing options" in sk._lib.skelfmm_last_error()
