"""Parity of the three-dimensional HIP step (mpfc3d_*) with the 3-D CPU oracle
(seven-point Laplacian, 2x2x2 restriction, trilinear prolongation, coarsest
level relaxed by the same number of red-black sweeps on both sides).

Single V-cycles agree element by element (several levels, non-cubic boxes,
both schemes, both linearisations); whole steps with energies agree at
convergence; mass and the modified energy behave at the benchmark size.
"""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1208_2643_amd import api  # noqa: E402
from paper_1208_2643_amd import _lib as L  # noqa: E402

DEV = torch.device("cuda:0")
K = 2


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def both(**kw):
    d = dict(eps=0.025, beta=0.9, M=1.0, h=1.0, dt=0.05, scheme=2)
    d.update(kw)
    return O.Params(**d), api.Params(**d)


def field3(m, n, l, seed, mean=0.07, amp=0.05):
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=(l, n, m))


@pytest.mark.parametrize("shape", [(8, 8, 8), (16, 8, 8), (8, 16, 32), (32, 32, 32)])
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("newton", [True, False])
def test_one_cycle_matches_oracle_3d(shape, scheme, newton):
    l, n, m = shape
    po, pg = both(scheme=scheme)
    phik = field3(m, n, l, 11)
    prev = phik + 0.002 * field3(m, n, l, 12, mean=0.0, amp=1.0)
    psi0 = 0.002 * field3(m, n, l, 13, mean=0.0, amp=1.0)
    st = api.Stepper3(m, n, l, pg, tol=1e-30, max_cycles=1, energy=0, coarse_sweeps=K,
                      linearization=L.MPFC_NEWTON if newton else L.MPFC_PICARD)
    psi = dev(psi0)
    mu = torch.empty_like(psi)
    ka = torch.empty_like(psi)
    phi_g, info = st.step(dev(phik), dev(prev), psi, mu=mu, kappa=ka, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED and info.n_cycles == 1
    S = O.source3(po, phik, prev, psi0)
    u0 = O.complete_guess3(po, 2 * phik - prev, S, phik=phik)
    u, hist, _ = O.fas_solve3(po, u0, S, phik=phik, tol=1e-30, max_cycles=1, newton=newton,
                              coarse_sweeps=K)
    for a, b in zip((host(phi_g), host(mu), host(ka)), u):
        assert relmax(a, b) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)
    st.close()


@pytest.mark.parametrize("scheme", [1, 2])
def test_steps_with_energies_match_oracle_3d(scheme):
    m = n = l = 32
    po, pg = both(scheme=scheme)
    phi0 = field3(m, n, l, 14)
    st = api.Stepper3(m, n, l, pg, tol=1e-10, coarse_sweeps=K)
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
    phi_o, _, psi_o, res = O.run3(po, phi0, 4, tol=1e-12, max_cycles=300, guess=1,
                                  coarse_sweeps=K)
    assert all(i.status == 0 for i in infos) and all(r.cycles > 0 for r in res)
    assert rel_l2(host(phi), phi_o) <= 1e-10
    assert rel_l2(host(psi), psi_o) <= 1e-8
    assert rel_l2(host(mu), res[-1].mu) <= 1e-8
    for i, r in zip(infos, res):
        for k, v in enumerate((i.energy_F, i.energy_pseudo, i.energy_mod)):
            assert abs(v - r.energies[k]) <= 1e-9 * abs(r.energies[k])
        assert abs(i.mass - r.energies[3]) <= 1e-12 * abs(r.energies[3])
    st.close()


def test_64_cubed_step_matches_oracle():
    """The benchmark's parameters (h = pi/4, dt = 0.05, scheme 2) on 64^3."""
    m = n = l = 64
    po, pg = both(h=math.pi / 4)
    phi0 = field3(m, n, l, 15)
    st = api.Stepper3(m, n, l, pg, tol=1e-10, coarse_sweeps=K)
    psi = torch.zeros(l, n, m, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step3(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=200, coarse_sweeps=K)
    assert r.cycles > 0 and info.status == 0
    assert rel_l2(host(phi_g), r.phi) <= 1e-10
    assert abs(info.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])
    st.close()


def test_128_cubed_mass_and_energy():
    """Benchmark size: mass is conserved and the modified energy does not
    increase (Sec. 3's properties, which hold in any dimension)."""
    m = n = l = 128
    _, pg = both(h=math.pi / 4)
    phi0 = field3(m, n, l, 7)
    st = api.Stepper3(m, n, l, pg, tol=1e-10)
    phi = dev(phi0)
    prev = phi.clone()
    psi = torch.zeros_like(phi)
    nxt = torch.empty_like(phi)
    mass0 = (math.pi / 4) ** 3 * float(phi0.sum())
    mods = []
    for _ in range(5):
        _, info = st.step(phi, prev, psi, nxt)
        assert info.status == 0
        assert info.mass == pytest.approx(mass0, rel=1e-12)
        mods.append(info.energy_mod)
        prev, phi, nxt = phi, nxt, prev
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(mods, mods[1:]))
    st.close()


@pytest.mark.timeout(300)
def test_128_cubed_step_matches_oracle():
    """The benchmark's configuration at its full size (128^3, h = pi/4, dt =
    0.05, scheme 2, the bench's seeded initial data): one step, element by
    element against the oracle solved to 1e-12 (about a minute on one CPU
    thread; the energies are checked against the oracle on 32^3 and 64^3).
    Bars as in two dimensions: phi 1e-10; mu 1e-9; psi = (2/s)(phi^{k+1} -
    phi^k) - psi^k scales the error of phi by 2/s = 40 against a much smaller
    field, 1e-8."""
    m = n = l = 128
    po, pg = both(h=math.pi / 4)
    phi0 = field3(m, n, l, 7)
    st = api.Stepper3(m, n, l, pg, tol=1e-10)
    psi = torch.zeros(l, n, m, dtype=torch.float64, device=DEV)
    mu = torch.empty_like(psi)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi, mu=mu)
    r = O.step3(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=200, coarse_sweeps=2,
                energy=False)
    assert r.cycles > 0 and info.status == 0
    e_phi, e_mu, e_psi = (rel_l2(host(phi_g), r.phi), rel_l2(host(mu), r.mu),
                          rel_l2(host(psi), r.psi))
    print(f"\n128^3 step: rel L2 phi {e_phi:.2e}, mu {e_mu:.2e}, psi {e_psi:.2e}")
    assert e_phi <= 1e-10
    assert e_mu <= 1e-9
    assert e_psi <= 1e-8
    h3 = (math.pi / 4) ** 3
    assert info.mass == pytest.approx(h3 * float(r.phi.sum()), rel=1e-12)
    st.close()


@pytest.mark.parametrize("mnl,perm", [((64, 64, 64), (1, 2, 0)), ((64, 64, 64), (0, 2, 1)),
                                      ((64, 32, 16), (1, 2, 0)), ((16, 64, 32), (2, 0, 1))])
@pytest.mark.parametrize("scheme", [1, 2])
def test_axis_permutation_3d(mnl, perm, scheme):
    """The seven-point scheme treats x, y and z alike: permuting the axes of
    the input permutes those of phi^{k+1}, psi^{k+1} and mu and keeps the
    energies and the mass.  The relaxation blocks are not cubes, so an index
    slip along one axis breaks the symmetry."""
    m, n, l = mnl
    _, pg = both(scheme=scheme, h=math.pi / 4)
    phik = field3(m, n, l, 141, mean=0.1, amp=0.1)
    phikm1 = field3(m, n, l, 142, mean=0.1, amp=0.1)
    out = []
    for t in (lambda a: a, lambda a: np.ascontiguousarray(a.transpose(perm))):
        pk = t(phik)
        ll, nn, mm = pk.shape
        st = api.Stepper3(mm, nn, ll, pg, tol=1e-11, max_cycles=200, coarse_sweeps=K)
        psi = torch.zeros(pk.shape, dtype=torch.float64, device=DEV)
        mu = torch.empty_like(psi)
        phi, info = st.step(dev(pk), dev(t(phikm1)), psi, mu=mu)
        assert info.status == 0 and info.n_cycles > 0
        out.append((host(phi), host(psi), host(mu), info))
        st.close()
    (pa, sa, ma, ia), (pb, sb, mb, ib) = out
    for a, b in ((pa, pb), (sa, sb), (ma, mb)):
        assert b.shape == a.transpose(perm).shape
    assert np.max(np.abs(pa.transpose(perm) - pb)) <= 1e-10
    assert np.max(np.abs(sa.transpose(perm) - sb)) <= 1e-8
    assert np.max(np.abs(ma.transpose(perm) - mb)) <= 1e-8
    for key in ("energy_F", "energy_mod", "mass"):
        a, b = getattr(ia, key), getattr(ib, key)
        assert abs(a - b) <= 1e-10 * max(1.0, abs(a)), key
