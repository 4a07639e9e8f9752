"""Pins of the oracle on grids whose sides are not powers of two (Sec. 4.6
runs on 512 x 400).  Such a grid is coarsened while both sides of the next
level stay even, and its coarsest level is either solved by dense Newton or
relaxed by a fixed number of red-black sweeps (coarse_sweeps).

References that do not go through the FAS code:
  * closed forms: Fourier and cosine modes are eigenvectors of the five-point
    Laplacian for any number of cells per axis;
  * the brute-force dense Newton solve of the reduced scalar equation
    (oracle.brute), for both schemes and with the pinning term;
  * invariants: translation by an even shift (the red-black colouring is
    unchanged) maps one V-cycle's iterate to the shifted iterate; mass is
    conserved and the modified energy does not increase over steps.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import brute
from paper_1208_2643_amd import inputs as I


def P(scheme=2, h=0.5, dt=0.1, eps=0.025, beta=0.9, M=1.0, bc=(0, 0)):
    return O.Params(eps=eps, beta=beta, M=M, h=h, dt=dt, scheme=scheme, bc=bc)


@pytest.mark.parametrize("m,n,bc", [(12, 20, (0, 0)), (12, 10, (1, 1)), (20, 12, (0, 1))])
def test_laplacian_modes_on_general_grids(m, n, bc):
    h = 0.7
    i = np.arange(m) + 0.5
    j = np.arange(n) + 0.5
    for p in (0, 1, 3, m // 2):
        for q in (0, 1, n // 2 - 1):
            if bc[0]:
                vx, lx = np.cos(math.pi * p * i / m), math.sin(math.pi * p / (2 * m)) ** 2
            else:
                vx, lx = np.cos(2 * math.pi * p * i / m + 0.3), math.sin(math.pi * p / m) ** 2
            if bc[1]:
                vy, ly = np.cos(math.pi * q * j / n), math.sin(math.pi * q / (2 * n)) ** 2
            else:
                vy, ly = np.cos(2 * math.pi * q * j / n - 0.2), math.sin(math.pi * q / n) ** 2
            v = np.outer(vy, vx)
            lam = 4.0 / h**2 * (lx + ly)
            np.testing.assert_allclose(O.laplacian(v, h, bc=bc), -lam * v, atol=1e-12 * (1 + lam))


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("m,n", [(12, 8), (8, 20)])
@pytest.mark.parametrize("coarse_sweeps", [0, 4])
def test_fas_matches_brute_force_on_general_grids(scheme, m, n, coarse_sweeps):
    """12 x 8 coarsens to 6 x 4, 8 x 20 to 4 x 10; the FAS solution (coarsest
    by dense Newton or by sweeps) equals the reduced-equation Newton solve.
    (Relaxing the coarsest level by sweeps only works where the smoother
    converges on it, i.e. a coarse spacing that is large for the time step,
    as on every level of 8 cells or more of a real grid; h = 1 here.)"""
    p = P(scheme, h=1.0, dt=0.1, M=1.3)
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=51)
    phikm1 = I.noise(m, n, mean=0.1, amp=0.1, seed=52)
    psik = I.noise(m, n, mean=0.0, amp=0.05, seed=53)
    psik -= psik.mean()
    r = O.step(p, phik, phikm1, psik, tol=1e-13, max_cycles=400, energy=False,
               coarse_sweeps=coarse_sweeps)
    assert r.cycles > 0
    x, mu, ka, _ = brute.solve_step(scheme, p.eps, p.beta, p.M, p.h, p.dt, phik, phikm1, psik)
    for a, b in ((r.phi, x), (r.mu, mu), (r.kappa, ka)):
        assert np.max(np.abs(a - b)) <= 1e-11 * max(1.0, np.max(np.abs(b)))


def test_pinned_fas_matches_brute_force_on_a_general_grid():
    p = P(2, h=1.0, dt=0.1)
    m, n = 12, 20
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=54)
    psik = I.noise(m, n, mean=0.0, amp=0.05, seed=55)
    psik -= psik.mean()
    rng = np.random.default_rng(56)
    W = 2.0 * rng.random((n, m))
    hat = I.noise(m, n, mean=0.2, amp=0.2, seed=57)
    r = O.step(p, phik, phik, psik, tol=1e-13, max_cycles=400, energy=False, pin=W, phihat=hat,
               coarse_sweeps=4)
    assert r.cycles > 0
    x, mu, ka, _ = brute.solve_step(2, p.eps, p.beta, p.M, p.h, p.dt, phik, phik, psik,
                                    pin=W, phihat=hat)
    for a, b in ((r.phi, x), (r.mu, mu), (r.kappa, ka)):
        assert np.max(np.abs(a - b)) <= 1e-11 * max(1.0, np.max(np.abs(b)))


def test_coarse_sweeps_change_the_iterate_but_not_the_solution():
    """One V-cycle depends on how the coarsest level is treated; the solution
    of the step does not (it is unique, Sec. 3)."""
    p = P(2, h=math.pi / 4, dt=0.05)
    m, n = 48, 40   # levels 48x40, 24x20, 12x10 (coarsest)
    phik = I.crystallites(m, n, p.h, count=1, radius_cells=8, seed=58)
    S = O.source(p, phik, phik, np.zeros_like(phik))
    u0 = O.complete_guess(p, phik, S, phik=phik)
    one = [O.fas_solve(p, u0, S, phik=phik, tol=1e-30, max_cycles=1, coarse_sweeps=k)[0][0]
           for k in (0, 1, 8)]
    assert np.max(np.abs(one[1] - one[2])) > 0
    full = [O.step(p, phik, phik, np.zeros_like(phik), tol=1e-12, max_cycles=100,
                   coarse_sweeps=k) for k in (0, 1, 8)]
    for r in full:
        assert r.cycles > 0
        np.testing.assert_allclose(r.phi, full[0].phi, atol=1e-11)


@pytest.mark.parametrize("bc", [(0, 0), (1, 0)])
def test_even_translation_equivariance_of_one_cycle(bc):
    """Shifting the data by an even number of cells along a periodic axis
    shifts one V-cycle's iterate by the same amount (the colouring, the 2x2
    restriction blocks and the bilinear stencils are all preserved)."""
    p = P(2, h=math.pi / 4, dt=0.05, bc=bc)
    m, n = 24, 40
    phik = I.crystallites(m, n, p.h, count=1, radius_cells=6, seed=59)
    prev = phik + 0.01 * I.noise(m, n, mean=0.0, amp=1.0, seed=60)
    psi = 0.01 * I.noise(m, n, mean=0.0, amp=1.0, seed=61)
    sy = 4  # along y (periodic in both cases); levels 24x40, 12x20, 6x10

    def cycle(a, b, c):
        S = O.source(p, a, b, c)
        u0 = O.complete_guess(p, 2 * a - b, S, phik=a)
        return O.fas_solve(p, u0, S, phik=a, tol=1e-30, max_cycles=1, coarse_sweeps=3)[0]

    base = cycle(phik, prev, psi)
    moved = cycle(*(np.roll(x, sy, axis=0) for x in (phik, prev, psi)))
    for a, b in zip(moved, base):
        np.testing.assert_allclose(a, np.roll(b, sy, axis=0), atol=1e-13)


@pytest.mark.parametrize("bc", [(0, 0), (0, 1)])
def test_general_grid_steps_conserve_mass_and_dissipate_energy(bc):
    m, n, h = 48, 40, math.pi / 4
    p = P(2, h=h, dt=0.05, bc=bc)
    phi0 = I.crystallites(m, n, h, count=2, radius_cells=5, seed=62)
    phi, prev, psi, res = O.run(p, phi0, 6, guess=1, tol=1e-11, coarse_sweeps=4)
    mass0 = h * h * phi0.sum()
    for r in res:
        assert r.cycles > 0
        assert r.energies[3] == pytest.approx(mass0, abs=1e-9)
    mod = [r.energies[2] for r in res]
    assert all(b <= a + 1e-9 for a, b in zip(mod, mod[1:]))


def test_sheared_crystal_input_recipe():
    """The Sec. 4.6 set-up: band of 20 rows of atoms, pinning strips of
    weight 2 and height pi at its bottom and top rows, phi_hat shifted by 4 %
    of 2 pi at the bottom only."""
    phi, W, hat = I.strained_crystal()
    h = 4 * math.pi / (16 * math.sqrt(3))
    assert phi.shape == W.shape == hat.shape == (400, 512)
    rows = np.nonzero(W[:, 0])[0]
    assert set(np.unique(W)) == {0.0, 2.0}
    # two strips, each about pi high
    gaps = np.nonzero(np.diff(rows) > 1)[0]
    assert len(gaps) == 1
    for strip in (rows[: gaps[0] + 1], rows[gaps[0] + 1:]):
        assert abs(len(strip) * h - math.pi) <= 2 * h
    # liquid far from the band, crystal inside
    assert abs(phi[0].mean() - 0.57) < 2e-3 and abs(phi[-1].mean() - 0.57) < 2e-3
    assert min(np.ptp(phi[j - 8:j + 8]) for j in range(120, 290, 16)) > 0.5
    # phi_hat equals phi away from the bottom strip (up to the perturbation)
    top = rows[gaps[0] + 1:]
    assert np.max(np.abs(hat[top] - phi[top])) < 2e-3
    bottom = rows[: gaps[0] + 1]
    assert np.max(np.abs(hat[bottom] - phi[bottom])) > 0.05
