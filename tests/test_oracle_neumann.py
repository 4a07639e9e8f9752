"""Pins of the oracle's homogeneous Neumann and mixed periodic-Neumann
boundary conditions (App. A, eqs. h-n-bcs; Sec. 4.5 uses periodic in x and
Neumann in y).

Two references that do not go through the Neumann code path:
  * closed forms: the cosine modes cos(pi p (i + 1/2) / m) are the
    eigenvectors of the cell-centred Neumann Laplacian, eigenvalue
    -(4/h^2) sin^2(pi p / (2 m));
  * the even reflection: a grid function with Neumann ghosts on an axis of m
    cells is the restriction of the periodic function on 2m cells that is
    mirrored about the boundary edge.  Every operator without an ordering
    (Laplacian, N(u), source, prolongation, energies, Poisson solve) and the
    converged solution of a step therefore equal the periodic oracle's on the
    mirrored grid.  (The red-black smoother is the exception: reflection
    swaps the two colours, so its single sweeps are pinned by their fixed
    point instead.)
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1208_2643_amd import inputs as I

BCS = [(1, 0), (0, 1), (1, 1)]


def P(scheme, bc, h=0.5, dt=0.1, eps=0.025, beta=0.9, M=1.0):
    return O.Params(eps=eps, beta=beta, M=M, h=h, dt=dt, scheme=scheme, bc=bc)


def mirror(f, bc):
    """Even extension of the (n, m) array f across every Neumann axis."""
    f = np.asarray(f)
    if bc[0]:
        f = np.concatenate([f, f[:, ::-1]], axis=1)
    if bc[1]:
        f = np.concatenate([f, f[::-1, :]], axis=0)
    return np.ascontiguousarray(f)


def corner(f, shape):
    n, m = shape
    return f[:n, :m]


def field(m, n, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return 0.2 + scale * rng.standard_normal((n, m))


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("m,n,h", [(8, 8, 0.5), (16, 8, 0.3)])
def test_neumann_laplacian_cosine_eigenvalues(m, n, h):
    """Delta_h cos-mode = -(4/h^2)(sin^2(pi p/2m) + sin^2(pi q/2n)) cos-mode with
    Neumann ghosts on both axes (App. A, eqs. h-n-bcs)."""
    i = np.arange(m) + 0.5
    j = np.arange(n) + 0.5
    for p in range(m):
        for q in (0, 1, n // 2, n - 1):
            v = np.outer(np.cos(math.pi * q * j / n), np.cos(math.pi * p * i / m))
            lam = 4.0 / h**2 * (math.sin(math.pi * p / (2 * m)) ** 2 + math.sin(math.pi * q / (2 * n)) ** 2)
            np.testing.assert_allclose(O.laplacian(v, h, bc=(1, 1)), -lam * v, atol=1e-12 * (1 + lam))


def test_mixed_laplacian_modes():
    """Periodic in x (Fourier modes), Neumann in y (cosine modes)."""
    m, n, h = 16, 8, 0.7
    i = np.arange(m) + 0.5
    j = np.arange(n) + 0.5
    for p in (0, 1, 3, 8):
        for q in (0, 2, 7):
            v = np.outer(np.cos(math.pi * q * j / n), np.cos(2 * math.pi * p * i / m + 0.4))
            lam = 4.0 / h**2 * (math.sin(math.pi * p / m) ** 2 + math.sin(math.pi * q / (2 * n)) ** 2)
            np.testing.assert_allclose(O.laplacian(v, h, bc=(0, 1)), -lam * v, atol=1e-12 * (1 + lam))


def test_neumann_gradient_has_no_boundary_edge():
    """||grad_h f||^2 sums interior edges only on a Neumann axis: a function
    that varies only in y has zero gradient energy along x for any bc in x, and
    its y-edges are the n - 1 interior ones."""
    m, n = 8, 6
    y = np.arange(n, dtype=float) ** 2
    f = np.tile(y[:, None], (1, m))
    expect = m * np.sum(np.diff(y) ** 2)
    assert O.grad_sq(f, bc=(1, 1)) == pytest.approx(expect, rel=1e-14)
    # periodic in y adds the wrap edge (y[0] - y[n-1])^2 on every column
    assert O.grad_sq(f, bc=(1, 0)) == pytest.approx(expect + m * (y[0] - y[-1]) ** 2, rel=1e-14)


# ------------------------------------------------------------------ even reflection
@pytest.mark.parametrize("bc", BCS)
def test_operators_equal_mirrored_periodic(bc):
    m, n, h = 8, 8, 0.6
    phi, mu, ka, xk, xkm1, psi = (field(m, n, s) for s in range(6))
    for scheme in (1, 2):
        pn, pp = P(scheme, bc, h=h), P(scheme, (0, 0), h=h)
        np.testing.assert_allclose(O.laplacian(phi, h, bc=bc),
                                   corner(O.laplacian(mirror(phi, bc), h), phi.shape), atol=1e-13)
        Sn = O.source(pn, xk, xkm1, psi)
        Sp = O.source(pp, mirror(xk, bc), mirror(xkm1, bc), mirror(psi, bc))
        for a, b in zip(Sn, Sp):
            np.testing.assert_allclose(a, corner(b, a.shape), atol=1e-12)
        Nn = O.operator(pn, [phi, mu, ka], phik=xk)
        Np = O.operator(pp, [mirror(x, bc) for x in (phi, mu, ka)], phik=mirror(xk, bc))
        for a, b in zip(Nn, Np):
            np.testing.assert_allclose(a, corner(b, a.shape), atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_prolongation_equals_mirrored_periodic(bc):
    m, n = 8, 8
    coarse = field(m // 2, n // 2, 7)
    fine = field(m, n, 8)
    a = O.prolong_add(coarse, fine, bc=bc)
    b = O.prolong_add(mirror(coarse, bc), mirror(fine, bc))
    np.testing.assert_allclose(a, corner(b, a.shape), atol=1e-14)


@pytest.mark.parametrize("bc", BCS)
def test_poisson_and_energies_equal_mirrored_periodic(bc):
    m, n, h = 16, 8, 0.5
    b = field(m, n, 9)
    w, it = O.poisson(b, h, bc=bc)
    assert it > 0
    # -Lap_h w = b - mean(b) with the Neumann Laplacian, w mean-free
    np.testing.assert_allclose(-O.laplacian(w, h, bc=bc), b - b.mean(), atol=1e-10)
    assert abs(w.mean()) < 1e-12
    wp, _ = O.poisson(mirror(b, bc), h)
    np.testing.assert_allclose(w, corner(wp, w.shape), atol=1e-10)
    # the mirrored grid holds 2 (one Neumann axis) or 4 copies: every energy
    # sum and the mass scale by that factor
    k = 2 ** (bc[0] + bc[1])
    p = P(2, bc, h=h)
    phi, prev, psi = field(m, n, 10), field(m, n, 11), field(m, n, 12, 0.05)
    e = O.energies(p, phi, prev, psi)
    ep = O.energies(P(2, (0, 0), h=h), mirror(phi, bc), mirror(prev, bc), mirror(psi, bc))
    np.testing.assert_allclose(k * e, ep, rtol=1e-10)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", [1, 2])
def test_dense_newton_equals_mirrored_periodic(bc, scheme):
    """The coarsest-grid Newton solve (exact Neumann Jacobian) gives the
    restriction of the mirrored periodic solution."""
    m, n = 4, 4
    p, pp = P(scheme, bc, h=0.5, dt=0.05), P(scheme, (0, 0), h=0.5, dt=0.05)
    xk = field(m, n, 13)
    S = O.source(p, xk, xk, field(m, n, 14, 0.01))
    u0 = O.complete_guess(p, xk, S, phik=xk)
    un, it = O.dense_newton(p, u0, S, phik=xk)
    assert 0 < it < 50
    up, it2 = O.dense_newton(pp, [mirror(x, bc) for x in u0], [mirror(x, bc) for x in S],
                             phik=mirror(xk, bc))
    assert 0 < it2 < 50
    for a, b in zip(un, up):
        np.testing.assert_allclose(a, corner(b, a.shape), atol=1e-11)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", [1, 2])
def test_step_equals_mirrored_periodic(bc, scheme):
    """A whole step (FAS to 1e-12) on the Neumann grid reaches the restriction
    of the mirrored periodic step's solution (the step's solution is unique,
    Sec. 3), although the iterates differ (reflection swaps the colours)."""
    m, n, h = 16, 16, math.pi / 4
    p = P(scheme, bc, h=h, dt=0.05)
    pp = P(scheme, (0, 0), h=h, dt=0.05)
    phi = I.crystallites(m, n, h, count=1, radius_cells=4, seed=3)
    prev = phi + 0.01 * field(m, n, 15, 1.0)
    psi = 0.02 * field(m, n, 16, 1.0)
    r = O.step(p, phi, prev, psi, guess=1, tol=1e-12)
    assert r.cycles > 0
    rp = O.step(pp, mirror(phi, bc), mirror(prev, bc), mirror(psi, bc), guess=1, tol=1e-12)
    assert rp.cycles > 0
    for a, b in ((r.phi, rp.phi), (r.mu, rp.mu), (r.kappa, rp.kappa), (r.psi, rp.psi)):
        np.testing.assert_allclose(a, corner(b, a.shape), atol=1e-9)
    k = 2 ** (bc[0] + bc[1])
    np.testing.assert_allclose(k * r.energies, rp.energies, rtol=1e-9)


# ------------------------------------------------------------------ smoother and invariants
@pytest.mark.parametrize("bc", BCS)
def test_smoother_fixed_point_is_the_neumann_solution(bc):
    """Red-black sweeps (lagged ghosts) and lexicographic sweeps converge to
    the Newton solution with the exact Neumann Jacobian on a small grid with a
    small time step (where the collective smoother contracts)."""
    m, n = 4, 4
    p = P(2, bc, h=1.0, dt=0.01)
    xk = field(m, n, 17, 0.1)
    S = O.source(p, xk, xk, field(m, n, 18, 0.01))
    u0 = O.complete_guess(p, xk, S, phik=xk)
    ref, _ = O.dense_newton(p, u0, S, phik=xk)
    for order in ("rb", "lex"):
        u = O.smooth(p, u0, S, phik=xk, sweeps=400, order=order)
        for a, b in zip(u, ref):
            np.testing.assert_allclose(a, b, atol=1e-11)


@pytest.mark.parametrize("bc", BCS)
def test_neumann_steps_conserve_mass_and_dissipate_energy(bc):
    """Both schemes conserve the mass h^2 sum phi and (scheme 2) do not
    increase the modified energy (Sec. 3, energy stability), with Neumann
    conditions as with periodic ones."""
    m, n, h = 32, 32, math.pi / 4
    for scheme in (1, 2):
        p = P(scheme, bc, h=h, dt=0.05)
        phi0 = I.crystallites(m, n, h, count=2, radius_cells=5, seed=4)
        phi, prev, psi, res = O.run(p, phi0, 6, guess=1, tol=1e-11)
        mass0 = h * h * phi0.sum()
        for r in res:
            assert r.cycles > 0
            assert r.energies[3] == pytest.approx(mass0, abs=1e-9)
        mod = [r.energies[2] for r in res]
        assert all(b <= a + 1e-9 for a, b in zip(mod, mod[1:]))
