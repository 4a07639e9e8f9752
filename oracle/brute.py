"""Brute-force solve of one time step on a tiny grid (TEST INFRASTRUCTURE ONLY).

An independent formulation of the step used to pin the oracle's FAS solver:
eliminate mu and kappa to get one scalar equation per cell in phi^{k+1}, build
the periodic five-point Laplacian as an explicit dense (mn x mn) matrix, and
run Newton's method with a dense LU solve (numpy) to machine precision.

Scheme 1 (Sec. 3.1, eqs. scheme1_3, scheme1_4, discrete_1_a):
    kappa = L phi,  mu = phi^3 + alpha phi + 2 L phi^k + L kappa,
    R(phi) = phi - phi^k - c1 L mu - d1 psi^k = 0.
Scheme 2 (Sec. 3.2, eqs. mpfc_scheme2_3, mpfc_scheme2_4, discrete_2_a):
    kappa = L (phi + phi^k)/2,
    mu = chi(phi, phi^k)(phi + phi^k)/2 + alpha (phi + phi^k)/2 + 2 L phi~ + L kappa,
    R(phi) = phi - phi^k - c2 L mu - d2 psi^k = 0,
with chi(a, b) = (a^2 + b^2)/2 and phi~ = (3 phi^k - phi^{k-1})/2.
Pinning (Sec. 4.6, scheme 2): mu is replaced by
    mu~ = mu + 2 ((phi + phi^k)/2 - phi_hat) W
in R, with the weight W and the prescribed configuration phi_hat.

This module shares nothing with the FAS code in mpfc_oracle.c: different
unknowns (phi only), a matrix Laplacian, and a library LU solve.
"""
from __future__ import annotations

import numpy as np


def laplacian_matrix(m: int, n: int, h: float) -> np.ndarray:
    """Dense periodic five-point Laplacian on an m x n cell grid, x fastest."""
    N = m * n
    L = np.zeros((N, N))
    for j in range(n):
        for i in range(m):
            q = j * m + i
            L[q, q] -= 4.0 / h**2
            for (ii, jj) in (((i + 1) % m, j), ((i - 1) % m, j), (i, (j + 1) % n), (i, (j - 1) % n)):
                L[q, jj * m + ii] += 1.0 / h**2
    return L


def laplacian_matrix3(m: int, n: int, l: int, h: float) -> np.ndarray:
    """Dense periodic seven-point Laplacian on an m x n x l cell grid, x fastest."""
    N = m * n * l
    L = np.zeros((N, N))
    for k in range(l):
        for j in range(n):
            for i in range(m):
                q = (k * n + j) * m + i
                L[q, q] -= 6.0 / h**2
                for (ii, jj, kk) in (((i + 1) % m, j, k), ((i - 1) % m, j, k),
                                     (i, (j + 1) % n, k), (i, (j - 1) % n, k),
                                     (i, j, (k + 1) % l), (i, j, (k - 1) % l)):
                    L[q, (kk * n + jj) * m + ii] += 1.0 / h**2
    return L


def solve_step(scheme, eps, beta, M, h, s, phik, phikm1=None, psik=None, tol=1e-15, maxit=60,
               pin=None, phihat=None):
    """Return (phi, mu, kappa, iterations) of one step by dense Newton (with
    pinning weight `pin` and configuration `phihat`: scheme 2 only; mu is then
    the pinned mu~).  A 3-D array (l, n, m) is a three-dimensional grid (the
    seven-point Laplacian); the reduced equation is the same."""
    if phik.ndim == 3:
        L = laplacian_matrix3(phik.shape[2], phik.shape[1], phik.shape[0], h)
    else:
        L = laplacian_matrix(phik.shape[1], phik.shape[0], h)
    pk = phik.reshape(-1).astype(np.float64)
    pkm1 = (phikm1 if phikm1 is not None else phik).reshape(-1).astype(np.float64)
    ps = (psik if psik is not None else np.zeros_like(phik)).reshape(-1).astype(np.float64)
    alpha = 1.0 - eps
    I = np.eye(pk.size)
    if scheme == 1:
        c = s * M / (beta + 1.0 / s)
        d = 1.0 / (beta + 1.0 / s)
        rhs_const = pk + d * ps + 2.0 * c * (L @ (L @ pk))

        def R(x):
            return x - c * (L @ (x**3 + alpha * x + L @ (L @ x))) - rhs_const

        def J(x):
            return I - c * (L @ (np.diag(3.0 * x**2) + alpha * I + L @ L))
    else:
        c = s * M / (beta + 2.0 / s)
        d = 2.0 / (beta + 2.0 / s)
        tilde = 0.5 * (3.0 * pk - pkm1)

        W = np.zeros_like(pk) if pin is None else np.asarray(pin, dtype=np.float64).reshape(-1)
        hat = np.zeros_like(pk) if phihat is None else np.asarray(phihat, dtype=np.float64).reshape(-1)

        def mu_of(x):
            g = 0.25 * (x**2 + pk**2) * (x + pk)
            mu = g + 0.5 * alpha * (x + pk) + 2.0 * (L @ tilde) + 0.5 * (L @ (L @ (x + pk)))
            return mu + 2.0 * (0.5 * (x + pk) - hat) * W

        def R(x):
            return x - pk - c * (L @ mu_of(x)) - d * ps

        def J(x):
            gp = 0.25 * (3.0 * x**2 + 2.0 * x * pk + pk**2)
            return I - c * (L @ (np.diag(gp + W) + 0.5 * alpha * I + 0.5 * (L @ L)))
    x = pk.copy()
    it = 0
    for it in range(1, maxit + 1):
        dx = np.linalg.solve(J(x), -R(x))
        x = x + dx
        if np.max(np.abs(dx)) <= tol * (1.0 + np.max(np.abs(x))):
            break
    if scheme == 1:
        kappa = L @ x
        mu = x**3 + alpha * x + 2.0 * (L @ pk) + L @ kappa
    else:
        kappa = 0.5 * (L @ (x + pk))
        mu = mu_of(x)
    shp = phik.shape
    return x.reshape(shp), mu.reshape(shp), kappa.reshape(shp), it
