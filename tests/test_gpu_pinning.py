"""Parity of the HIP library with the CPU oracle for the pinning term of
Sec. 4.6 (second-order scheme): mu~ = mu + 2 (phi^{k+1/2} - phi_hat) W.

Whole steps (phi, mu~, psi and the energies, whose F includes the pinning
energy) and one V-cycle element by element, on periodic and mixed
periodic-Neumann grids; W = 0 reproduces the unpinned step; switching the
term off restores the unpinned iterates; unsupported configurations are
rejected.
"""
import math

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


def pinning(m, n, seed, phi0):
    """Weight 2 in strips of 4 rows at the top and bottom (as Sec. 4.6's
    horizontal strips) plus a random interior patch; phi_hat a shifted copy of
    the initial field."""
    W = np.zeros((n, m))
    W[:4] = 2.0
    W[-4:] = 2.0
    rng = np.random.default_rng(seed)
    W[n // 2 - 3:n // 2 + 3, m // 3:m // 3 + 8] = 3.0 * rng.random((6, 8))
    hat = np.roll(phi0, 3, axis=1)
    return W, hat


@pytest.mark.parametrize("bc", [0, L.MPFC_BC_NEUMANN_Y])
def test_pinned_steps_match_oracle(bc):
    po, pg = both(bc)
    m, n = 128, 64
    phi0 = I.crystallites(m, n, pg.h, radius_cells=10, seed=21)
    W, hat = pinning(m, n, 22, phi0)
    st = api.Stepper(m, n, pg, tol=1e-10)
    st.set_pinning(dev(W), dev(hat))
    mu = torch.empty(n, m, dtype=torch.float64, device=DEV)
    phi = dev(phi0)
    prev = phi.clone()
    psi = torch.zeros_like(phi)
    nxt = torch.empty_like(phi)
    infos = []
    for _ in range(5):
        _, info = st.step(phi, prev, psi, nxt, mu=mu)
        infos.append(info)
        prev, phi, nxt = phi, nxt, prev
    phi_o, prev_o, psi_o, res = O.run(po, phi0, 5, tol=1e-12, max_cycles=300, guess=1,
                                      pin=W, phihat=hat)
    assert all(i.status == 0 for i in infos) and all(r.cycles >= 0 for r in res)
    assert rel_l2(host(phi), phi_o) <= 1e-10
    assert rel_l2(host(psi), psi_o) <= 1e-8
    assert rel_l2(host(mu), res[-1].mu) <= 1e-8
    for i, r in zip(infos, res):
        assert abs(i.energy_F - r.energies[0]) <= 1e-9 * abs(r.energies[0])
        assert abs(i.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])
        assert abs(i.mass - r.energies[3]) <= 1e-12 * abs(r.energies[3])


@pytest.mark.parametrize("N", [64, 256])
def test_pinned_one_cycle_iterate_matches_oracle(N):
    po, pg = both()
    phik = I.crystallites(N, N, pg.h, radius_cells=N / 10, seed=23)
    prev = phik + 0.002 * I.noise(N, N, mean=0.0, amp=1.0, seed=24)
    W, hat = pinning(N, N, 25, phik)
    st = api.Stepper(N, N, pg, tol=1e-30, max_cycles=1, energy=0)
    st.set_pinning(dev(W), dev(hat))
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    mu = torch.empty_like(psi)
    ka = torch.empty_like(psi)
    phi_g, info = st.step(dev(phik), dev(prev), psi, mu=mu, kappa=ka, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED and info.n_cycles == 1
    S = O.source(po, phik, prev, np.zeros_like(phik), pin=W, phihat=hat)
    u0 = O.complete_guess(po, 2 * phik - prev, S, phik, pin=W)
    u, hist, _ = O.fas_solve(po, u0, S, phik=phik, tol=1e-30, max_cycles=1, pin=W)
    for a, b in zip((host(phi_g), host(mu), host(ka)), u):
        assert relmax(a, b) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)


def test_zero_weight_and_switching_off():
    _, pg = both()
    N = 128
    phi0 = dev(I.crystallites(N, N, pg.h, radius_cells=12, seed=26))

    def one(setup):
        st = api.Stepper(N, N, pg, tol=1e-10, energy=1)
        setup(st)
        phi, _, _, infos = api.run(st, phi0, 3)
        st.close()
        return host(phi), infos[-1]

    ref, ir = one(lambda st: None)
    zero, iz = one(lambda st: st.set_pinning(torch.zeros_like(phi0), phi0.clone()))
    assert relmax(zero, ref) <= 1e-12
    assert iz.energy_mod == pytest.approx(ir.energy_mod, rel=1e-12)

    def on_off(st):
        st.set_pinning(torch.full_like(phi0, 5.0), torch.zeros_like(phi0))
        st.set_pinning(None)
    off, _ = one(on_off)
    assert relmax(off, ref) <= 1e-12


def test_full_size_1024_pinned_step():
    N = 1024
    po, pg = both()
    phi0 = I.crystallites(N, N, pg.h, seed=2)
    W, hat = pinning(N, N, 27, phi0)
    st = api.Stepper(N, N, pg, tol=1e-10)
    st.set_pinning(dev(W), dev(hat))
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=100, pin=W, phihat=hat)
    assert r.cycles > 0 and info.status == 0
    assert rel_l2(host(phi_g), r.phi) <= 1e-10
    assert abs(info.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])


@pytest.mark.parametrize("kw", [dict(scheme=1), dict(precision=L.MPFC_MIXED),
                                dict(linearization=L.MPFC_PICARD)])
def test_unsupported_configurations_rejected(kw):
    scheme = kw.pop("scheme", 2)
    _, pg = both(scheme=scheme)
    st = api.Stepper(64, 64, pg, energy=0, **kw)
    w = torch.ones(64, 64, dtype=torch.float64, device=DEV)
    with pytest.raises(L.MpfcError):
        st.set_pinning(w, w.clone())
    st.close()


@pytest.mark.parametrize("bc", [0, L.MPFC_BC_NEUMANN_Y])
def test_pinned_axis_exchange(bc):
    """With the weight, phi_hat, the input and the two axes' boundary
    conditions all transposed (horizontal strips become vertical ones), the
    pinned step is the transposed step, with the same energies."""
    m, n = 128, 64
    swapped = ((bc & 1) << 1) | ((bc >> 1) & 1)
    phi0 = I.crystallites(m, n, math.pi / 4, radius_cells=10, seed=171)
    W, hat = pinning(m, n, 172, phi0)
    out = []
    for b, t, (mm, nn) in ((bc, lambda a: a, (m, n)),
                           (swapped, lambda a: np.ascontiguousarray(a.T), (n, m))):
        _, pg = both(b)
        st = api.Stepper(mm, nn, pg, tol=1e-12, max_cycles=200)
        st.set_pinning(dev(t(W)), dev(t(hat)))
        phi, prev, psi, infos = api.run(st, dev(t(phi0)), 3)
        assert all(i.status == 0 for i in infos)
        out.append((t(host(phi)), t(host(psi)), infos))
        st.close()
    (pa, sa, ia), (pb, sb, ib) = out
    assert pa.shape == pb.shape == (n, m)
    assert np.max(np.abs(pa - pb)) <= 1e-10
    assert np.max(np.abs(sa - sb)) <= 1e-8
    for a, b in zip(ia, ib):
        for key in ("energy_F", "energy_mod", "mass"):
            x, y = getattr(a, key), getattr(b, key)
            assert abs(x - y) <= 1e-10 * max(1.0, abs(x)), key
