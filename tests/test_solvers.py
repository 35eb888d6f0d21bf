"""GMRES over the apply (iterative use that amortizes one build).

CPU tests drive the solver with a dense stand-in operator (its logic only);
the GPU test solves a second-kind system with the GPU apply and checks the
solution against a right-hand side formed by the dense O1 sum."""
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from paper_2310_16668_amd.solvers import gmres  # noqa: E402


class _Dense:
    """Stand-in operator: a dense matrix (test of the solver logic only)."""

    def __init__(self, A):
        self.A = A

    def apply(self, q):
        return self.A @ q

    def apply_adjoint(self, v):
        return self.A.conj().T @ v


@pytest.mark.parametrize("cplx,adjoint,nrhs", [(False, False, 1), (False, True, 5), (True, False, 3)])
def test_gmres_dense_second_kind(cplx, adjoint, nrhs):
    rng = np.random.default_rng(7)
    n = 300
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    if cplx:
        A = A + 1j * rng.standard_normal((n, n)) / np.sqrt(n)
    X = rng.standard_normal((n, nrhs)) + (1j * rng.standard_normal((n, nrhs)) if cplx else 0)
    M = 2.0 * np.eye(n) + 0.5 * (A.conj().T if adjoint else A)
    B = M @ X
    At, Bt = torch.from_numpy(A), torch.from_numpy(B)
    x, info = gmres(_Dense(At), Bt[:, 0] if nrhs == 1 else Bt, shift=2.0, scale=0.5, adjoint=adjoint, tol=1e-12,
                    restart=20, maxiter=400)
    x = x.numpy().reshape(n, -1)
    assert np.linalg.norm(x - X) / np.linalg.norm(X) <= 1e-10
    assert float(info["relres"].max()) <= 1e-11


def test_gmres_restarts_and_stops_at_maxiter():
    rng = np.random.default_rng(8)
    n = 200
    A = torch.from_numpy(rng.standard_normal((n, n)) / np.sqrt(n))
    b = torch.from_numpy(rng.standard_normal(n))
    # restarts of 5 cannot reach 1e-14 within 12 products: the cap must hold
    _, info = gmres(_Dense(A), b, shift=1.0, scale=1.0, tol=1e-14, restart=5, maxiter=12)
    assert info["iterations"] <= 12 + 2


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,nrhs,bar", [(torch.float64, 4, 1e-8), (torch.float32, 16, 2e-5)])
def test_gmres_gpu_second_kind_laplace(dtype, nrhs, bar):
    """(1/2) x + (1/n) A x = b on 16,384 uniform points; b from the dense O1
    sum of a known x; every product is one GPU apply of all columns."""
    import paper_2310_16668_amd as sk

    n = 16384
    x_pts = workloads.uniform_points(n, 3, 811)
    X = workloads.charges(n, nrhs, 812)
    Xr = X.astype(np.float32).astype(np.float64) if dtype == torch.float32 else X
    B = 0.5 * Xr + oracle.direct(x_pts, Xr, "laplace", 0.0) / n
    op = sk.build(x_pts, "laplace", tol=1e-10, leaf_size=64)
    Bd = torch.from_numpy(B).to("cuda:0", dtype)
    x, info = gmres(op, Bd, shift=0.5, scale=1.0 / n, tol=1e-11 if dtype == torch.float64 else 1e-6,
                    restart=30, maxiter=200)
    e = np.linalg.norm(x.cpu().numpy().astype(np.float64) - Xr) / np.linalg.norm(Xr)
    print(f"gmres {dtype} nrhs={nrhs}: {info['iterations']} products, relres {float(info['relres'].max()):.2e}, "
          f"error vs x {e:.2e}", flush=True)
    assert e <= bar
