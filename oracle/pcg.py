"""Oracle: preconditioned conjugate gradients and the Lanczos condition estimate.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

Section 5 runs PCG with the multilevel BDDC preconditioner; Table 1 states
the stopping tolerance 1e-8 and reports a condition-number estimate.
Readings: stop when ||r_k||_2 <= rtol ||b||_2 on the recursively updated
residual; the estimate is the ratio of the extreme eigenvalues of the Lanczos
tridiagonal matrix built from the CG coefficients.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pcg(apply_A, apply_M, b, x0=None, rtol=1e-8, maxit=1000, keep_iterates=False):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x)
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    alphas, betas, iterates = [], [], []
    if hist[-1] <= rtol:
        return dict(x=x, iters=0, relres=hist, alphas=alphas, betas=betas, iterates=iterates)
    z = apply_M(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = apply_A(p)
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        alphas.append(alpha)
        hist.append(np.linalg.norm(r) / bnorm)
        if keep_iterates:
            iterates.append(x.copy())
        if hist[-1] <= rtol:
            break
        z = apply_M(r)
        rz_new = r @ z
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    return dict(x=x, iters=it, relres=hist, alphas=alphas, betas=betas, iterates=iterates)


def lanczos_tridiagonal(alphas, betas):
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i]
        if i > 0:
            T[i, i] += betas[i - 1] / alphas[i - 1]
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return T


def condition_estimate(alphas, betas):
    k = len(alphas)
    if k == 0:
        return 1.0
    T = lanczos_tridiagonal(alphas, betas[:k - 1])
    ev = sla.eigvalsh(T)
    return float(ev[-1] / ev[0])


def solve(bddc, b, rtol=1e-8, maxit=1000, interface_reduced=True, keep_iterates=False):
    """PCG on A x = b with the BDDC preconditioner; start from the condensed
    x0 (interface reduction) or from zero."""
    A = bddc.A
    x0 = bddc.condensed_x0(b) if interface_reduced else None
    out = pcg(lambda v: A @ v, bddc.apply, b, x0=x0, rtol=rtol, maxit=maxit,
              keep_iterates=keep_iterates)
    out["kappa"] = condition_estimate(out["alphas"], out["betas"])
    return out


def energy_error(A, x, xref):
    e = x - xref
    return float(np.sqrt(e @ (A @ e)) / np.sqrt(xref @ (A @ xref)))
