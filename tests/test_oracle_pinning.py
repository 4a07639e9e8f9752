"""Pins of the oracle's pinning term (Sec. 4.6): in the second-order scheme
mu is replaced by mu~ = mu + 2 (phi^{k+1/2} - phi_hat) W, phi^{k+1/2} =
(phi^{k+1} + phi^k)/2, with a weight W >= 0 and a prescribed configuration
phi_hat.  The oracle carries mu~ as its unknown (an extra -W phi in N^(2) and
W (phi^k - 2 phi_hat) in S^(2)); the references here do not:
  * a brute-force dense Newton solve of the reduced scalar equation written
    with mu~ exactly as the paper states it;
  * the closed-form linear amplification factor of a small Fourier mode;
  * invariants: W = 0 is the unpinned step, mass is conserved (mu~ enters only
    under the Laplacian), and the modified energy with the added term
    h^2 sum W (phi - phi_hat)^2 does not increase.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import brute
from paper_1208_2643_amd import inputs as I


def P(h=0.5, dt=0.1, eps=0.025, beta=0.9, M=1.0, scheme=2, bc=(0, 0)):
    return O.Params(eps=eps, beta=beta, M=M, h=h, dt=dt, scheme=scheme, bc=bc)


def strips(m, n, width, value):
    """W = value in horizontal strips of `width` rows at the top and bottom."""
    W = np.zeros((n, m))
    W[:width] = value
    W[-width:] = value
    return W


def test_zero_weight_is_the_unpinned_step():
    p = P(h=math.pi / 4, dt=0.05)
    phi = I.crystallites(32, 32, p.h, count=2, radius_cells=6, seed=3)
    prev = phi + 0.01 * I.noise(32, 32, mean=0.0, amp=1.0, seed=4)
    psi = 0.01 * I.noise(32, 32, mean=0.0, amp=1.0, seed=5)
    a = O.step(p, phi, prev, psi, guess=1, tol=1e-12)
    b = O.step(p, phi, prev, psi, guess=1, tol=1e-12, pin=np.zeros_like(phi),
               phihat=np.ones_like(phi))
    for x, y in ((a.phi, b.phi), (a.mu, b.mu), (a.kappa, b.kappa), (a.psi, b.psi)):
        assert np.array_equal(x, y)
    assert np.array_equal(a.energies, b.energies)


@pytest.mark.parametrize("dt", [0.1, 10.0])
def test_fas_matches_brute_force_with_pinning(dt):
    """FAS V-cycles on the mu~ form and a dense Newton solve of the paper's
    reduced equation agree to 1e-12 on an 8 x 8 grid."""
    p = P(h=0.5, dt=dt, M=1.3)
    m = n = 8
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=41)
    phikm1 = I.noise(m, n, mean=0.1, amp=0.1, seed=42)
    psik = I.noise(m, n, mean=0.0, amp=0.05, seed=43)
    psik -= psik.mean()
    rng = np.random.default_rng(44)
    W = 2.0 * rng.random((n, m))
    hat = I.noise(m, n, mean=0.2, amp=0.2, seed=45)
    r = O.step(p, phik, phikm1, psik, tol=1e-13, max_cycles=400, energy=False, pin=W, phihat=hat)
    assert r.cycles > 0
    x, mu, ka, _ = brute.solve_step(2, p.eps, p.beta, p.M, p.h, p.dt, phik, phikm1, psik,
                                    pin=W, phihat=hat)
    for a, b in ((r.phi, x), (r.mu, mu), (r.kappa, ka)):
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))


def test_linear_amplification_with_uniform_weight():
    """Small single Fourier mode, phi_hat = 0, uniform W: the pinning term adds
    W to (alpha + lam^2)/2 in the scheme-2 linear factor
    [(1 - c lam ((alpha+lam^2)/2 + W) + 3 c lam^2) a^k - c lam^2 a^{k-1} + d b^k]
    / [1 + c lam ((alpha + lam^2)/2 + W)]."""
    m, n, h = 16, 16, 0.5
    p = P(h=h, dt=0.3, M=1.2, beta=0.7)
    Wc = 1.7
    X, Y = I.cell_centres(m, n, h)
    v = np.cos(2 * math.pi * 2 * X / (m * h) + 0.3) * np.cos(2 * math.pi * Y / (n * h) - 0.7)
    delta = 1e-5
    a_k, a_km1, b_k = 1.0, 0.8, 0.6
    r = O.step(p, a_k * delta * v, a_km1 * delta * v, b_k * delta * v, tol=1e-17,
               max_cycles=200, energy=False, pin=np.full((n, m), Wc), phihat=np.zeros((n, m)))
    lam = 4.0 / h**2 * (math.sin(math.pi * 2 / m) ** 2 + math.sin(math.pi * 1 / n) ** 2)
    c, d = O.coefficients(p)
    q = 0.5 * (p.alpha + lam**2) + Wc
    factor = ((1 - c * lam * q + 3 * c * lam**2) * a_k - c * lam**2 * a_km1 + d * b_k) / (1 + c * lam * q)
    got = float(np.sum(r.phi * v) / np.sum(v * v)) / delta
    assert got == pytest.approx(factor, rel=1e-8)


@pytest.mark.parametrize("bc", [(0, 0), (0, 1)])
def test_pinned_steps_conserve_mass_and_dissipate_energy(bc):
    m, n, h = 32, 32, math.pi / 4
    p = P(h=h, dt=0.05, bc=bc)
    phi0 = I.crystallites(m, n, h, count=2, radius_cells=6, seed=6)
    W = strips(m, n, 3, 2.0)
    hat = np.roll(phi0, 2, axis=1)
    phi, prev, psi, res = O.run(p, phi0, 8, guess=1, tol=1e-11, pin=W, phihat=hat)
    mass0 = h * h * phi0.sum()
    for r in res:
        assert r.cycles > 0
        assert r.energies[3] == pytest.approx(mass0, abs=1e-9)
    mod = [r.energies[2] for r in res]
    assert all(b <= a + 1e-9 for a, b in zip(mod, mod[1:]))
    # the pinned rows move towards phi_hat relative to the unpinned run
    _, _, _, free = O.run(p, phi0, 8, guess=1, tol=1e-11)
    d_pin = np.abs(res[-1].phi - hat)[:3].mean()
    d_free = np.abs(free[-1].phi - hat)[:3].mean()
    assert d_pin < d_free


def test_first_order_scheme_rejects_pinning():
    p = P(scheme=1)
    phi = I.noise(8, 8, seed=7)
    with pytest.raises(ValueError):
        O.step(p, phi, phi, np.zeros_like(phi), pin=np.ones_like(phi), phihat=phi)
