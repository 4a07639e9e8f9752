"""Parity of the HIP library with the CPU oracle on grids whose sides are not
powers of two (Sec. 4.6 runs on 512 x 400).

Both sides coarsen while both sides of the next level stay even and relax
the coarsest level by the same number of red-black sweeps, so single
V-cycles agree element by element; whole steps (phi, mu, psi and the
energies, whose -1 norm uses the coarsest level's separable Poisson solve)
agree at convergence.  Grids: several tiles per level with ragged tile
counts, tile sides that are divisors of the level sides, periodic and
Neumann axes, both schemes, both linearisations and the pinning term.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1208_2643_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1208_2643_amd import api  # noqa: E402
from paper_1208_2643_amd import _lib as L  # noqa: E402

DEV = torch.device("cuda:0")
K = 4  # coarse_sweeps on both sides


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def both(bc=0, **kw):
    d = dict(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=2)
    d.update(kw)
    return O.Params(**d, bc=(bc & 1, (bc >> 1) & 1)), api.Params(**d, bc=bc)


def one_cycle(m, n, bc=0, scheme=2, newton=True, pin=False, seed=70, nu=(2, 2), **kw):
    po, pg = both(bc, scheme=scheme, **kw)
    phik = I.crystallites(m, n, pg.h, count=2, radius_cells=min(m, n) / 8, seed=seed)
    prev = phik + 0.002 * I.noise(m, n, mean=0.0, amp=1.0, seed=seed + 1)
    psi0 = 0.002 * I.noise(m, n, mean=0.0, amp=1.0, seed=seed + 2)
    W = hat = None
    lin = L.MPFC_NEWTON if newton else L.MPFC_PICARD
    st = api.Stepper(m, n, pg, tol=1e-30, max_cycles=1, energy=0, coarse_sweeps=K,
                     linearization=lin, nu1=nu[0], nu2=nu[1])
    if pin:
        W = np.zeros((n, m))
        W[:4] = 2.0
        W[n // 2:n // 2 + 6] = 1.5
        hat = np.roll(phik, 2, axis=1)
        st.set_pinning(dev(W), dev(hat))
    psi = dev(psi0)
    mu = torch.empty_like(psi)
    ka = torch.empty_like(psi)
    phi_g, info = st.step(dev(phik), dev(prev), psi, mu=mu, kappa=ka, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED and info.n_cycles == 1
    S = O.source(po, phik, prev, psi0, pin=W, phihat=hat)
    u0 = O.complete_guess(po, 2 * phik - prev, S, phik=phik, pin=W)
    u, hist, _ = O.fas_solve(po, u0, S, phik=phik, tol=1e-30, max_cycles=1, newton=newton,
                             pin=W, coarse_sweeps=K, nu1=nu[0], nu2=nu[1])
    out = (host(phi_g), host(mu), host(ka))
    st.close()
    return out, u, info, hist


@pytest.mark.parametrize("m,n", [(96, 80), (160, 96), (200, 120), (64, 100), (12, 4)])
@pytest.mark.parametrize("scheme", [1, 2])
def test_one_cycle_matches_oracle(m, n, scheme):
    """96 x 80 -> 48 x 40 -> 24 x 20 -> 12 x 10; 160 x 96 -> ... -> 10 x 6;
    200 x 120 -> 100 x 60 -> 50 x 30 (tile sides 40 x 24 / 50 x 30 ...);
    64 x 100 -> 32 x 50; 12 x 4 -> 6 x 2 (one tile larger than the level)."""
    got, ref, info, hist = one_cycle(m, n, scheme=scheme)
    for a, b in zip(got, ref):
        assert relmax(a, b) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)


@pytest.mark.parametrize("bc", [L.MPFC_BC_NEUMANN_Y, L.MPFC_BC_NEUMANN_X,
                                L.MPFC_BC_NEUMANN_X | L.MPFC_BC_NEUMANN_Y])
@pytest.mark.parametrize("m,n", [(96, 80), (200, 120)])
def test_one_cycle_neumann_matches_oracle(bc, m, n):
    got, ref, info, hist = one_cycle(m, n, bc=bc)
    for a, b in zip(got, ref):
        assert relmax(a, b) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)


def test_one_cycle_picard_and_pinning_match_oracle():
    for kw in (dict(newton=False), dict(pin=True), dict(pin=True, bc=L.MPFC_BC_NEUMANN_Y)):
        got, ref, info, hist = one_cycle(160, 96, **kw)
        for a, b in zip(got, ref):
            assert relmax(a, b) <= 1e-12, kw
        np.testing.assert_allclose(info.history, hist, rtol=1e-9)


@pytest.mark.parametrize("nu", [(1, 0), (0, 1), (1, 1), (2, 1)])
def test_other_cycles_match_oracle(nu):
    """V(nu1, nu2) with fewer smoothing passes (the fastest cycles for the
    Sec. 4.6 parameters), pinned as in that workload."""
    got, ref, info, hist = one_cycle(200, 120, nu=nu, pin=True)
    for a, b in zip(got, ref):
        assert relmax(a, b) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)


@pytest.mark.parametrize("shape", ["0", "2"])
def test_both_general_tile_shapes_give_the_same_cycle(shape, monkeypatch):
    monkeypatch.setenv("MPFC_TILE_SHAPE", shape)
    got, ref, _, _ = one_cycle(192, 160, seed=80)
    for a, b in zip(got, ref):
        assert relmax(a, b) <= 1e-12


@pytest.mark.parametrize("bc,scheme", [(0, 2), (0, 1), (L.MPFC_BC_NEUMANN_Y, 2)])
def test_steps_with_energies_match_oracle(bc, scheme):
    m, n = 192, 160
    po, pg = both(bc, scheme=scheme)
    phi0 = I.crystallites(m, n, pg.h, radius_cells=14, seed=81)
    st = api.Stepper(m, n, pg, tol=1e-10, coarse_sweeps=K)
    phi = dev(phi0)
    prev = phi.clone()
    psi = torch.zeros_like(phi)
    nxt = torch.empty_like(phi)
    mu = torch.empty_like(phi)
    infos = []
    for _ in range(4):
        _, info = st.step(phi, prev, psi, nxt, mu=mu)
        infos.append(info)
        prev, phi, nxt = phi, nxt, prev
    phi_o, _, psi_o, res = O.run(po, phi0, 4, tol=1e-12, max_cycles=300, guess=1,
                                 coarse_sweeps=K)
    assert all(i.status == 0 for i in infos) and all(r.cycles > 0 for r in res)
    assert rel_l2(host(phi), phi_o) <= 1e-10
    assert rel_l2(host(psi), psi_o) <= 1e-8
    assert rel_l2(host(mu), res[-1].mu) <= 1e-8
    for i, r in zip(infos, res):
        assert abs(i.energy_F - r.energies[0]) <= 1e-9 * abs(r.energies[0])
        assert abs(i.energy_pseudo - r.energies[1]) <= 1e-9 * abs(r.energies[1])
        assert abs(i.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])
        assert abs(i.mass - r.energies[3]) <= 1e-12 * abs(r.energies[3])
    st.close()


def test_energies_of_a_state_match_oracle():
    """mpfc_energies starts its -1 norm solve cold (no warm start), so the
    Poisson cycles and the coarsest-level eigenbasis solve do all the work."""
    for bc in (0, L.MPFC_BC_NEUMANN_X | L.MPFC_BC_NEUMANN_Y):
        m, n = 96, 80
        po, pg = both(bc)
        phi = I.crystallites(m, n, pg.h, radius_cells=10, seed=82)
        prev = phi + 0.01 * I.noise(m, n, mean=0.0, amp=1.0, seed=83)
        psi = 0.05 * I.noise(m, n, mean=0.0, amp=1.0, seed=84)
        st = api.Stepper(m, n, pg, coarse_sweeps=K)
        e = st.energies(dev(phi), dev(prev), dev(psi))
        ref = O.energies(po, phi, prev, psi)
        np.testing.assert_allclose(e, ref, rtol=1e-10)
        st.close()


def test_full_size_512x400_step():
    """Sec. 4.6's grid at the cycle test's parameters: one step from the
    crystallites workload, to 1e-10, against the oracle at 1e-12."""
    m, n = 512, 400
    po, pg = both()
    phi0 = I.crystallites(m, n, pg.h, radius_cells=20, seed=2)
    st = api.Stepper(m, n, pg, tol=1e-10, coarse_sweeps=K)
    psi = torch.zeros(n, m, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=100, coarse_sweeps=K)
    assert r.cycles > 0 and info.status == 0
    assert rel_l2(host(phi_g), r.phi) <= 1e-10
    assert abs(info.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])
    st.close()


def test_sheared_crystal_sec44_one_cycle_full_size():
    """The Sec. 4.6 workload itself (eps 0.6, M = 15^2, h = 4 pi / (16 sqrt 3),
    s = 0.025 h^2, beta 0.2, pinning strips, 512 x 400): one V-cycle element
    by element."""
    m, n = 512, 400
    h = 4 * math.pi / (16 * math.sqrt(3))
    d = dict(eps=0.6, beta=0.2, M=225.0, h=h, dt=0.025 * h * h, scheme=2)
    po, pg = O.Params(**d), api.Params(**d)
    phi0, W, hat = I.strained_crystal()
    st = api.Stepper(m, n, pg, tol=1e-30, max_cycles=1, energy=0, coarse_sweeps=K)
    st.set_pinning(dev(W), dev(hat))
    psi = torch.zeros(n, m, dtype=torch.float64, device=DEV)
    mu = torch.empty_like(psi)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi, mu=mu, allow_fail=True)
    S = O.source(po, phi0, phi0, np.zeros_like(phi0), pin=W, phihat=hat)
    u0 = O.complete_guess(po, phi0, S, phik=phi0, pin=W)
    u, hist, _ = O.fas_solve(po, u0, S, phik=phi0, tol=1e-30, max_cycles=1, pin=W,
                             coarse_sweeps=K)
    assert relmax(host(phi_g), u[0]) <= 1e-12
    assert relmax(host(mu), u[1]) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)
    st.close()


def test_tile_sides_divide_the_levels():
    st = api.Stepper(200, 120, both()[1], coarse_sweeps=K)
    for level, (m, n) in enumerate([(200, 120), (100, 60)]):
        for which in (0, 1):
            tx, ty, halo = st.tile_shape(level, which)
            assert m % tx == 0 and n % ty == 0 and tx % 2 == 0 and ty % 2 == 0
            assert tx <= 64 and ty <= 32
    st.close()


def test_diverged_status():
    """A solve whose residual grows stops with MPFC_EDIVERGED.  On a 12 x 12
    grid the coarsest level (6 x 6) is relaxed by two red-black sweeps, not
    solved, and at h = 0.5, dt = 0.3 the collective smoother is unstable there:
    the oracle's residual rises above its initial value by a clear margin (the
    first cycle above 1.01 x the initial norm is at least 5 % above it).  With a
    divergence factor of 1.01 the GPU stops at that cycle with the same history."""
    po, pg = both(scheme=2, h=0.5, dt=0.3)
    phi = I.noise(12, 12, mean=0.1, amp=0.05, seed=91)
    r = O.step(po, phi, phi, np.zeros_like(phi), tol=1e-12, max_cycles=10, energy=False,
               coarse_sweeps=2)
    hs = np.asarray(r.history)
    k = int(np.argmax(hs > 1.01 * hs[0]))
    assert k > 0 and hs[k] > 1.05 * hs[0] and np.all(hs[1:k] < 0.95 * hs[0])
    st = api.Stepper(12, 12, pg, tol=1e-12, max_cycles=50, energy=0, coarse_sweeps=2,
                     diverge=1.01)
    psi = torch.zeros(12, 12, dtype=torch.float64, device=DEV)
    _, info = st.step(dev(phi), dev(phi), psi, allow_fail=True)
    assert info.status == L.MPFC_EDIVERGED and info.n_cycles == k
    np.testing.assert_allclose(info.history, hs[:k + 1], rtol=1e-6)
    st.close()


@pytest.mark.parametrize("m,n,bc", [(192, 160, 0), (192, 160, L.MPFC_BC_NEUMANN_Y), (512, 400, 0)])
def test_axis_exchange_general(m, n, bc):
    """Sides that are not powers of two: the transposed input, on the n x m
    grid with the two axes' boundary conditions exchanged, gives the
    transposed step, its psi and mu, and the same energies."""
    swapped = ((bc & 1) << 1) | ((bc >> 1) & 1)
    phik = I.crystallites(m, n, math.pi / 4, radius_cells=14, seed=151)
    phikm1 = phik + 0.002 * I.noise(m, n, mean=0.0, amp=1.0, seed=152)
    out = []
    for b, t, (mm, nn) in ((bc, lambda a: a, (m, n)),
                           (swapped, lambda a: np.ascontiguousarray(a.T), (n, m))):
        _, pg = both(b)
        st = api.Stepper(mm, nn, pg, tol=1e-11, max_cycles=200, coarse_sweeps=K)
        psi = torch.zeros(nn, mm, dtype=torch.float64, device=DEV)
        mu = torch.empty_like(psi)
        phi, info = st.step(dev(t(phik)), dev(t(phikm1)), psi, mu=mu)
        assert info.status == 0 and info.n_cycles > 0
        out.append((t(host(phi)), t(host(psi)), t(host(mu)), info))
        st.close()
    (pa, sa, ma, ia), (pb, sb, mb, ib) = out
    assert pa.shape == pb.shape == (n, m)
    assert np.max(np.abs(pa - pb)) <= 1e-10
    assert np.max(np.abs(sa - sb)) <= 1e-8
    assert np.max(np.abs(ma - mb)) <= 1e-8
    for key in ("energy_F", "energy_mod", "mass"):
        a, b = getattr(ia, key), getattr(ib, key)
        assert abs(a - b) <= 1e-10 * max(1.0, abs(a)), key
