"""Pins of the three-dimensional oracle (the paper states that the schemes
extend to three dimensions in a straightforward way; seven-point Laplacian,
2 x 2 x 2 restriction, trilinear prolongation, h^3 grid sums).

References that do not go through the 3-D FAS code:
  * closed forms: products of Fourier modes are eigenvectors of the
    seven-point Laplacian; the linear amplification factors of both schemes
    with the three-dimensional eigenvalue;
  * the brute-force dense Newton solve of the reduced scalar equation with an
    explicit seven-point Laplacian matrix (oracle.brute);
  * the two-dimensional oracle (pinned on its own): data constant along one
    axis give the 2-D step's solution on every slice, and every energy scales
    by (cells along that axis) x h;
  * invariants: mass conservation, non-increasing modified energy, and
    equivariance under a permutation of the axes.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import brute
from paper_1208_2643_amd import inputs as I


def P(scheme=2, h=0.5, dt=0.1, eps=0.025, beta=0.9, M=1.0):
    return O.Params(eps=eps, beta=beta, M=M, h=h, dt=dt, scheme=scheme)


def field3(m, n, l, seed, mean=0.1, amp=0.1):
    rng = np.random.default_rng(seed)
    return mean + amp * rng.standard_normal((l, n, m))


def test_laplacian_modes_3d():
    m, n, l, h = 8, 4, 6, 0.7
    x = np.arange(m) + 0.5
    y = np.arange(n) + 0.5
    z = np.arange(l) + 0.5
    for a in (0, 1, 3):
        for b in (0, 1, 2):
            for c in (0, 2, 3):
                v = (np.cos(2 * math.pi * c * z / l + 0.1)[:, None, None]
                     * np.cos(2 * math.pi * b * y / n - 0.4)[None, :, None]
                     * np.cos(2 * math.pi * a * x / m + 0.3)[None, None, :])
                lam = 4.0 / h**2 * (math.sin(math.pi * a / m) ** 2 + math.sin(math.pi * b / n) ** 2
                                    + math.sin(math.pi * c / l) ** 2)
                np.testing.assert_allclose(O.laplacian3(v, h), -lam * v, atol=1e-12 * (1 + lam))


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 4, 4)])
@pytest.mark.parametrize("coarse_sweeps", [0, 4])
def test_fas_matches_brute_force_3d(scheme, shape, coarse_sweeps):
    l, n, m = shape
    p = P(scheme, h=1.0, dt=0.1, M=1.3)
    pk = field3(m, n, l, 1)
    pkm1 = field3(m, n, l, 2)
    ps = field3(m, n, l, 3, mean=0.0, amp=0.05)
    ps -= ps.mean()
    r = O.step3(p, pk, pkm1, ps, tol=1e-13, max_cycles=400, energy=False,
                coarse_sweeps=coarse_sweeps)
    assert r.cycles > 0
    x, mu, ka, _ = brute.solve_step(scheme, p.eps, p.beta, p.M, p.h, p.dt, pk, pkm1, ps)
    for a, b in ((r.phi, x), (r.mu, mu), (r.kappa, ka)):
        assert np.max(np.abs(a - b)) <= 1e-11 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme", [1, 2])
def test_constant_along_an_axis_is_the_2d_step(axis, scheme):
    """A field constant along one axis: the 3-D step's solution is the 2-D
    step's on every slice, and F, the pseudo and modified energies and the
    mass are (cells along that axis) x h times the 2-D ones."""
    h = 1.0                # (in 3-D the collective smoother is slower for larger c / h^6)
    p = P(scheme, h=h, dt=0.05)
    a, b = 16, 8           # 2-D slice (rows, columns)
    phi2 = I.crystallites(b, a, h, count=1, radius_cells=4, seed=4)
    prev2 = phi2 + 0.01 * I.noise(b, a, mean=0.0, amp=1.0, seed=5)
    psi2 = 0.01 * I.noise(b, a, mean=0.0, amp=1.0, seed=6)
    r2 = O.step(p, phi2, prev2, psi2, guess=1, tol=1e-12)
    reps = 4

    def lift(f):
        return np.ascontiguousarray(np.stack([f] * reps, axis=axis))

    r3 = O.step3(p, lift(phi2), lift(prev2), lift(psi2), guess=1, tol=1e-12)
    assert r2.cycles > 0 and r3.cycles > 0
    for x3, x2 in ((r3.phi, r2.phi), (r3.mu, r2.mu), (r3.kappa, r2.kappa), (r3.psi, r2.psi)):
        np.testing.assert_allclose(x3, lift(x2), atol=1e-10)
    np.testing.assert_allclose(r3.energies, reps * h * r2.energies, rtol=1e-9)


@pytest.mark.parametrize("scheme", [1, 2])
def test_linear_amplification_3d(scheme):
    """Zero background, one small Fourier mode: the step multiplies it by the
    linear factor of the scheme with lam = (4/h^2) sum of sin^2 over the axes
    (the same formulas as in two dimensions)."""
    m = n = l = 8
    h = 0.6
    p = P(scheme, h=h, dt=0.3, M=1.2, beta=0.7)
    x = (np.arange(m) + 0.5) * h
    v = (np.cos(2 * math.pi * 1 * x / (l * h))[:, None, None]
         * np.cos(2 * math.pi * 2 * x / (n * h) + 0.3)[None, :, None]
         * np.cos(2 * math.pi * 1 * x / (m * h) - 0.2)[None, None, :])
    lam = 4.0 / h**2 * (math.sin(math.pi / l) ** 2 + math.sin(2 * math.pi / n) ** 2
                        + math.sin(math.pi / m) ** 2)
    delta = 1e-5
    a_k, a_km1, b_k = 1.0, 0.8, 0.6
    r = O.step3(p, a_k * delta * v, a_km1 * delta * v, b_k * delta * v, tol=1e-17,
                max_cycles=300, energy=False)
    c, d = O.coefficients(p)
    if scheme == 1:
        factor = ((1 + 2 * c * lam**2) * a_k + d * b_k) / (1 + c * lam * (p.alpha + lam**2))
    else:
        q = 0.5 * (p.alpha + lam**2)
        factor = ((1 - c * lam * q + 3 * c * lam**2) * a_k - c * lam**2 * a_km1 + d * b_k) / \
            (1 + c * lam * q)
    got = float(np.sum(r.phi * v) / np.sum(v * v)) / delta
    assert got == pytest.approx(factor, rel=1e-8)


@pytest.mark.parametrize("scheme", [1, 2])
def test_mass_and_energy_3d(scheme):
    m = n = l = 16
    h = 1.0
    p = P(scheme, h=h, dt=0.05)
    phi0 = 0.07 + 0.05 * field3(m, n, l, 7, mean=0.0, amp=1.0)
    phi, prev, psi, res = O.run3(p, phi0, 5, guess=1, tol=1e-11)
    mass0 = h**3 * phi0.sum()
    for r in res:
        assert r.cycles > 0
        assert r.energies[3] == pytest.approx(mass0, abs=1e-9)
    k = 1 if scheme == 1 else 2    # pseudo energy (scheme 1) / modified energy (scheme 2)
    e = [r.energies[k] for r in res]
    assert all(b <= a + 1e-9 for a, b in zip(e, e[1:]))


def test_axis_permutation_equivariance_3d():
    m, n, l = 16, 8, 8
    h = math.pi / 4
    p = P(2, h=h, dt=0.05)
    phi = 0.07 + 0.05 * field3(m, n, l, 8, mean=0.0, amp=1.0)
    prev = phi + 0.01 * field3(m, n, l, 9, mean=0.0, amp=1.0)
    psi = 0.01 * field3(m, n, l, 10, mean=0.0, amp=1.0)
    r = O.step3(p, phi, prev, psi, guess=1, tol=1e-12)
    perm = (2, 0, 1)   # (l, n, m) -> (m, l, n): x becomes the slowest axis
    t = [np.ascontiguousarray(np.transpose(a, perm)) for a in (phi, prev, psi)]
    rt = O.step3(p, *t, guess=1, tol=1e-12)
    assert r.cycles > 0 and rt.cycles > 0
    for a, b in ((rt.phi, r.phi), (rt.mu, r.mu), (rt.kappa, r.kappa)):
        np.testing.assert_allclose(a, np.transpose(b, perm), atol=1e-10)
    np.testing.assert_allclose(rt.energies, r.energies, rtol=1e-10)
