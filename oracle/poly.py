"""Oracle: the GMRES-polynomial right preconditioner (§III-D).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The preconditioner is M = p(A) where p comes from the GMRES residual
polynomial pi of a (d+1)-step Arnoldi run: pi(z) = prod_i (1 - z/theta_i)
over the harmonic Ritz values theta_i, and p(z) = (1 - pi(z)) / z has degree
d.  The paper writes p in the monomial basis; this oracle uses the product
(roots) form with Leja ordering from the cited polynomial-preconditioning
work, which is the same polynomial in exact arithmetic.
"""
from __future__ import annotations

import numpy as np

from .krylov import arnoldi, spmv


def harmonic_ritz_values(H: np.ndarray, k: int) -> np.ndarray:
    """Eigenvalues of H_k + h_{k+1,k}^2 f e_k^T with H_k^T f = e_k.

    ``H`` is the (k+1) x k Hessenberg matrix of k Arnoldi steps.  These are
    the roots of the k-step GMRES residual polynomial.
    """
    Hk = H[:k, :k].copy()
    hk1 = H[k, k - 1]
    ek = np.zeros(k)
    ek[-1] = 1.0
    f = np.linalg.solve(Hk.T, ek)
    Hk[:, k - 1] += hk1 * hk1 * f
    return np.linalg.eigvals(Hk)


def leja_order(theta: np.ndarray) -> np.ndarray:
    """Modified Leja ordering keeping complex-conjugate pairs adjacent.

    First the value of largest modulus, then repeatedly the remaining value
    that maximises sum(log|theta - chosen|).  A complex value is taken with
    its positive-imaginary member first, immediately followed by its
    conjugate.
    """
    rest = [complex(t) for t in theta]
    out = []

    def take(i):
        t0 = rest.pop(i)
        if t0.imag != 0.0:
            # remove the matching conjugate of the value taken
            j = min(range(len(rest)), key=lambda q: abs(rest[q] - t0.conjugate()))
            rest.pop(j)
            t = complex(t0.real, abs(t0.imag))
            out.append(t)
            out.append(t.conjugate())
        else:
            out.append(t0)

    i0 = max(range(len(rest)), key=lambda q: (abs(rest[q]), rest[q].imag))
    take(i0)
    while rest:
        def score(q):
            with np.errstate(divide="ignore"):
                return float(np.sum(np.log(np.abs(rest[q] - np.array(out)))))
        best = max(range(len(rest)), key=lambda q: (score(q), rest[q].imag))
        take(best)
    return np.array(out)


def poly_roots(A, degree: int, v0: np.ndarray, dt=np.float64) -> np.ndarray:
    """Leja-ordered harmonic Ritz values of a (degree+1)-step Arnoldi run in
    precision ``dt`` from v0.  On a lucky breakdown after s < degree+1 steps
    the s Ritz values are exact and the polynomial degree drops to s-1."""
    k = degree + 1
    V, H, steps = arnoldi(A, v0, k, dt)
    if steps < k:
        theta = np.linalg.eigvals(H[:steps, :steps])
    else:
        theta = harmonic_ritz_values(H, k)
    return leja_order(theta)


def poly_apply(A, roots: np.ndarray, x: np.ndarray, dt=np.float64) -> np.ndarray:
    """y = p(A) x from the roots, using exactly len(roots) - 1 products with A.

    Real root theta: y += prod/theta, then (unless last) prod -= A prod/theta.
    Pair a +- ib with |theta|^2 = a^2 + b^2: t = A prod,
    y += (2a prod - t)/|theta|^2, then (unless last) prod -= (2a t - A t)/|theta|^2.
    """
    dt = np.dtype(dt)
    prod = np.asarray(x).astype(dt).copy()
    y = np.zeros_like(prod)
    k = len(roots)
    i = 0
    while i < k:
        th = complex(roots[i])
        if th.imag == 0.0:
            t_re = dt.type(th.real)
            y = y + prod / t_re
            if i < k - 1:
                prod = prod - spmv(A, prod, dt) / t_re
            i += 1
        else:
            a = dt.type(th.real)
            mod2 = dt.type(th.real * th.real + th.imag * th.imag)
            two_a = dt.type(2.0) * a
            t = spmv(A, prod, dt)
            y = y + (two_a * prod - t) / mod2
            if i < k - 2:
                prod = prod - (two_a * t - spmv(A, t, dt)) / mod2
            i += 2
    return y
