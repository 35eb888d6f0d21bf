"""Iterative solves that reuse one skeletonized operator for many applies.

The FMM apply is cheap next to the build, so a built operator is meant to be
applied many times, for example inside a Krylov solver for a second-kind
integral equation  (shift I + scale A) x = b  (section 1 of the paper names
iterative use of the fast apply as the setting; section 5 the amortization of
the build over many right-hand sides).  `gmres` solves every column of b at
once: each matrix-vector product is one many-RHS apply of all columns (the
GPU sweep), and only the small Hessenberg least-squares problems and the
Gram-Schmidt bookkeeping run outside the library, as tensor operations on the
columns' device.
"""
from __future__ import annotations


def gmres(op, b, shift: float = 0.0, scale: float = 1.0, adjoint: bool = False, tol: float = 1e-8,
          restart: int = 30, maxiter: int = 300):
    """Restarted GMRES (modified Gram-Schmidt Arnoldi) for (shift I + scale A) x = b.

    op: an object with apply / apply_adjoint taking [n, nrhs] tensors (an
        Operator); A is op's matrix, or its adjoint when `adjoint` is set.
    b:  [n] or [n, nrhs] tensor (real or complex) on the operator's device.
    Stops when every column's residual estimate is <= tol ||b_col||, or after
    `maxiter` products.  Returns (x, info) with info = {"iterations": products
    used, "relres": true relative residual per column (one extra product)}.
    """
    import torch

    squeeze = b.dim() == 1
    B = b.reshape(b.shape[0], -1)
    nrhs = B.shape[1]
    cplx = B.is_complex()
    hdt = torch.complex128 if cplx else torch.float64

    def mv(v):
        av = op.apply_adjoint(v) if adjoint else op.apply(v)
        return shift * v + scale * av

    def dot(u, w):   # column-wise <u, w>, accumulated in double precision
        return (u.conj().to(hdt) * w.to(hdt)).sum(0) if cplx else (u.to(hdt) * w.to(hdt)).sum(0)

    def norm(u):
        return dot(u, u).real.sqrt()

    bnorm = norm(B)
    bnorm = torch.where(bnorm > 0, bnorm, torch.ones_like(bnorm))
    x = torch.zeros_like(B)
    used = 0
    while used < maxiter:
        r = B - mv(x)
        used += 1
        beta = norm(r)
        if bool((beta <= tol * bnorm).all()):
            break
        safe_beta = torch.where(beta > 0, beta, torch.ones_like(beta))
        V = [r / safe_beta.to(B.dtype)]
        H = torch.zeros(nrhs, restart + 1, restart, dtype=hdt, device=B.device)
        y = None
        for j in range(restart):
            w = mv(V[j])
            used += 1
            for i in range(j + 1):
                h = dot(V[i], w)
                H[:, i, j] = h
                w = w - V[i] * h.to(B.dtype)
            hn = norm(w)
            H[:, j + 1, j] = hn
            V.append(w / torch.where(hn > 0, hn, torch.ones_like(hn)).to(B.dtype))
            # least squares min || H[:j+2, :j+1] y - beta e1 || per column (small, on the host)
            Hj = H[:, : j + 2, : j + 1].cpu()
            e1 = torch.zeros(nrhs, j + 2, 1, dtype=hdt)
            e1[:, 0, 0] = beta.cpu()
            y = torch.linalg.lstsq(Hj, e1).solution
            res = torch.linalg.vector_norm(Hj @ y - e1, dim=(1, 2))
            if bool((res <= tol * bnorm.cpu()).all()) or used >= maxiter:
                break
        yd = y.to(B.device)
        for i in range(yd.shape[1]):
            x = x + V[i] * yd[:, i, 0].to(B.dtype)
    relres = norm(B - mv(x)) / bnorm
    used += 1
    out = x[:, 0] if squeeze else x
    return out, {"iterations": used, "relres": relres.cpu()}
