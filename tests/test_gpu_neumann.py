"""Parity of the HIP library with the CPU oracle under homogeneous Neumann and
mixed periodic-Neumann boundary conditions (App. A, eqs. h-n-bcs; Sec. 4.5
runs periodic in x and Neumann in y).

Operator level on the same seeded inputs, element by element; one whole
V-cycle element by element (tiled levels restore their mirrored halo after
every pass, the coarse levels and the coarsest Newton solve use the ghost
rule); whole steps to the FP64 bar of the periodic tests (relative L2 1e-10);
and the even-reflection property: a Neumann run equals the periodic run on
the mirrored grid.
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
BCS = [1, 2, 3]   # MPFC_BC_NEUMANN_X, _Y, both


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def both(scheme, bc, **kw):
    d = dict(eps=0.025, beta=0.9, M=1.0, h=0.5, dt=0.1, scheme=scheme)
    d.update(kw)
    return O.Params(**d, bc=(bc & 1, (bc >> 1) & 1)), api.Params(**d, bc=bc)


def mirror(f, bc):
    if bc & 1:
        f = np.concatenate([f, f[:, ::-1]], axis=1)
    if bc & 2:
        f = np.concatenate([f, f[::-1, :]], axis=0)
    return np.ascontiguousarray(f)


SIZES = [(8, 8), (64, 32), (128, 256), (32, 512)]


def state(m, n, seed):
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=seed)
    phikm1 = I.noise(m, n, mean=0.1, amp=0.1, seed=seed + 1)
    psik = I.noise(m, n, mean=0.0, amp=0.05, seed=seed + 2)
    u = [I.noise(m, n, mean=0.1, amp=0.1, seed=seed + 3),
         I.noise(m, n, mean=0.0, amp=0.2, seed=seed + 4),
         I.noise(m, n, mean=0.0, amp=0.2, seed=seed + 5)]
    return phik, phikm1, psik, u


# ------------------------------------------------------------ operator level
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("m,n", SIZES)
def test_source_and_residual(bc, scheme, m, n):
    po, pg = both(scheme, bc, h=0.37, dt=0.3)
    phik, phikm1, psik, u = state(m, n, 500)
    ref = O.source(po, phik, phikm1, psik)
    got = api.op_source(pg, dev(phik), dev(phikm1), dev(psik))
    for a, b in zip(got, ref):
        if np.max(np.abs(b)) == 0:
            assert np.max(np.abs(host(a))) == 0
        else:
            assert relmax(host(a), b) <= 1e-14
    ref = O.residual(po, u, ref, phik)
    got = api.op_residual(pg, [dev(x) for x in u], [dev(x) for x in O.source(po, phik, phikm1, psik)],
                          dev(phik))
    for a, b in zip(got, ref):
        assert relmax(host(a), b) <= 1e-13


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("m,n", SIZES)
def test_smooth(bc, scheme, sweeps, m, n):
    """Red-black passes of the fused tile kernel (mirrored halo restored after
    every pass) against the oracle's sweeps with Neumann ghosts."""
    po, pg = both(scheme, bc, h=0.5, dt=0.1)
    phik, phikm1, psik, u = state(m, n, 600)
    f = O.source(po, phik, phikm1, psik)
    ref = O.smooth(po, u, f, phik=phik, sweeps=sweeps)
    ud = [dev(x) for x in u]
    api.op_smooth(pg, ud, [dev(x) for x in f], dev(phik), sweeps=sweeps)
    for a, b in zip(ud, ref):
        assert relmax(host(a), b) <= 1e-12


# ------------------------------------------------------------ one V-cycle
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("N", [64, 256])
def test_one_cycle_iterate_matches_oracle(bc, N):
    """After exactly one FAS V(2,2) cycle the GPU iterate equals the oracle's
    element by element: tiled levels, the persistent coarse kernel and the
    coarsest Newton solve all follow the Neumann ghost rule."""
    po, pg = both(2, bc, h=math.pi / 4, dt=0.05)
    phik = I.crystallites(N, N, math.pi / 4, radius_cells=N / 10, seed=11)
    prev = phik + 0.002 * I.noise(N, N, mean=0.0, amp=1.0, seed=12)
    st = api.Stepper(N, N, pg, tol=1e-30, max_cycles=1, energy=0)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    mu = torch.empty_like(psi)
    ka = torch.empty_like(psi)
    phi_g, info = st.step(dev(phik), dev(prev), psi, mu=mu, kappa=ka, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED and info.n_cycles == 1
    S = O.source(po, phik, prev, np.zeros_like(phik))
    u0 = O.complete_guess(po, 2 * phik - prev, S, phik)
    u, hist, _ = O.fas_solve(po, u0, S, phik=phik, tol=1e-30, max_cycles=1)
    for a, b in zip((host(phi_g), host(mu), host(ka)), u):
        assert relmax(a, b) <= 1e-12
    np.testing.assert_allclose(info.history, hist, rtol=1e-9)


@pytest.mark.parametrize("bc", [1, 2])
@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_tile_shape_invariance(bc, shape, monkeypatch):
    """Every tile shape (different tiles touch the boundary) gives the oracle's
    iterate after two V-cycles."""
    N = 128
    po, pg = both(1, bc, h=0.5, dt=0.1)
    phik = I.noise(N, N, mean=0.1, amp=0.1, seed=13)
    monkeypatch.setenv("MPFC_TILE_SHAPE", str(shape))
    st = api.Stepper(N, N, pg, tol=1e-30, max_cycles=2, energy=0)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    phi, info = st.step(dev(phik), dev(phik), psi, allow_fail=True)
    assert info.n_cycles == 2
    S = O.source(po, phik, phik, np.zeros_like(phik))
    u0 = O.complete_guess(po, phik.copy(), S)
    u, _, _ = O.fas_solve(po, u0, S, tol=1e-30, max_cycles=2)
    assert relmax(host(phi), u[0]) <= 1e-12


# ---------------------------------------------------------------- step level
def run_both(po, pg, phi0, steps, **opts):
    st = api.Stepper(phi0.shape[1], phi0.shape[0], pg, tol=1e-10, **opts)
    phi_g, prev_g, psi_g, infos = api.run(st, dev(phi0), steps)
    phi_o, prev_o, psi_o, res = O.run(po, phi0, steps, tol=1e-12, max_cycles=300)
    assert all(r.cycles >= 0 for r in res)
    assert all(i.status == 0 for i in infos)
    return (host(phi_g), host(psi_g), infos), (phi_o, psi_o, res)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", [1, 2])
def test_steps_match_oracle(bc, scheme):
    """Six steps on a 128 x 64 grid (crystallites touching the boundaries),
    h = pi/4, dt = 0.05: phi, psi and the energies against the oracle."""
    po, pg = both(scheme, bc, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(128, 64, math.pi / 4, radius_cells=12, seed=14)
    (pg_, sg, infos), (po_, so, res) = run_both(po, pg, phi0, 6)
    assert rel_l2(pg_, po_) <= 1e-10
    assert rel_l2(sg, so) <= 1e-8
    for i, r in zip(infos, res):
        assert abs(i.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])
        assert abs(i.energy_pseudo - r.energies[1]) <= 1e-9 * abs(r.energies[1])
        assert abs(i.mass - r.energies[3]) <= 1e-12 * abs(r.energies[3])


@pytest.mark.parametrize("bc", BCS)
def test_cycle_history_matches_oracle(bc):
    po, pg = both(2, bc, h=math.pi / 4, dt=0.05)
    phi0 = I.noise(64, 64, mean=0.1, amp=0.1, seed=15)
    prev = I.noise(64, 64, mean=0.1, amp=0.1, seed=16)
    st = api.Stepper(64, 64, pg, tol=1e-11, guess=L.MPFC_GUESS_EXTRAP, energy=0)
    psi = torch.zeros(64, 64, dtype=torch.float64, device=DEV)
    _, info = st.step(dev(phi0), dev(prev), psi)
    r = O.step(po, phi0, prev, np.zeros_like(phi0), guess=1, tol=1e-11, energy=False)
    assert info.n_cycles == r.cycles
    np.testing.assert_allclose(info.history, r.history, rtol=1e-6, atol=1e-13)


@pytest.mark.parametrize("bc", BCS)
def test_neumann_equals_mirrored_periodic_gpu(bc):
    """The Neumann step equals the periodic step on the mirror-extended grid
    (both converged to 1e-11; the iterates differ, the solution does not)."""
    _, pg = both(2, bc, h=math.pi / 4, dt=0.05)
    _, pp = both(2, 0, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(64, 64, math.pi / 4, radius_cells=8, seed=17)
    prev = phi0 + 0.001 * I.noise(64, 64, mean=0.0, amp=1.0, seed=18)
    sn = api.Stepper(64, 64, pg, tol=1e-11, energy=1)
    psi_n = torch.zeros(64, 64, dtype=torch.float64, device=DEV)
    a, ia = sn.step(dev(phi0), dev(prev), psi_n)
    M0 = mirror(phi0, bc)
    sp = api.Stepper(M0.shape[1], M0.shape[0], pp, tol=1e-11, energy=1)
    psi_p = torch.zeros(M0.shape, dtype=torch.float64, device=DEV)
    b, ib = sp.step(dev(M0), dev(mirror(prev, bc)), psi_p)
    assert ia.status == 0 and ib.status == 0
    np.testing.assert_allclose(host(a), host(b)[:64, :64], atol=1e-10)
    k = 2 ** ((bc & 1) + ((bc >> 1) & 1))
    assert k * ia.energy_mod == pytest.approx(ib.energy_mod, rel=1e-9)
    assert k * ia.mass == pytest.approx(ib.mass, rel=1e-12)


@pytest.mark.parametrize("bc,nuc", [(2, 0), (3, 0), (2, 1), (3, 1)])
def test_mixed_precision_matches_fp64_oracle(bc, nuc):
    """Mixed precision with Neumann axes (nuc: smoothing passes of the FP32
    cycles below the finest level, 0 = nu1, nu2) reaches the FP64 fixed point."""
    po, pg = both(2, bc, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(128, 128, math.pi / 4, radius_cells=14, seed=19)
    st = api.Stepper(128, 128, pg, tol=1e-10, precision=L.MPFC_MIXED, energy=0,
                     inner_cycles_next=2 if nuc else 0, inner_nu_coarse=nuc)
    phi_g, _, _, infos = api.run(st, dev(phi0), 4)
    phi_o, _, _, res = O.run(po, phi0, 4, tol=1e-12, max_cycles=300, energy=False)
    assert all(i.status == 0 for i in infos)
    assert rel_l2(host(phi_g), phi_o) <= 1e-9


def test_full_size_1024_periodic_x_neumann_y():
    """One step of the 1024^2 workload with Sec. 4.5's boundary conditions
    (periodic in x, Neumann in y), in the benchmark's launch configuration,
    against the oracle."""
    N = 1024
    po, pg = both(2, 2, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, seed=2)
    st = api.Stepper(N, N, pg, tol=1e-10)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=100)
    assert r.cycles > 0 and info.status == 0
    assert rel_l2(host(phi_g), r.phi) <= 1e-10
    assert abs(info.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])


def test_batch_with_neumann_members():
    """Batched simulations with different boundary conditions: each member's
    iterates equal its own single-grid context's."""
    sims = []
    for k, (bc, N) in enumerate([(0, 64), (1, 64), (2, 128), (3, 64)]):
        p = api.Params(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=2, bc=bc)
        sims.append((N, N, p))
    b = api.Batch(sims, tol=1e-10, precision=0)
    states = []
    for k, (m, n, p) in enumerate(sims):
        phi = dev(I.crystallites(m, n, p.h, radius_cells=m / 8, seed=20 + k))
        states.append([phi, phi.clone(), torch.zeros_like(phi)])
    for _ in range(3):
        outs = [torch.empty_like(s[0]) for s in states]
        psis = [s[2].clone() for s in states]
        infos = b.step([s[0] for s in states], [s[1] for s in states], psis, outs, history=False)
        assert all(i.status == 0 for i in infos)
        for s, o, ps in zip(states, outs, psis):
            s[1], s[0], s[2] = s[0], o, ps
    b.close()
    for k, (m, n, p) in enumerate(sims):
        st = api.Stepper(m, n, p, tol=1e-10, energy=0)
        phi0 = dev(I.crystallites(m, n, p.h, radius_cells=m / 8, seed=20 + k))
        phi, _, _, _ = api.run(st, phi0, 3)
        assert rel_l2(host(states[k][0]), host(phi)) <= 1e-12


@pytest.mark.parametrize("bc,m,n", [(0, 256, 128), (1, 256, 128), (2, 128, 256), (3, 256, 128),
                                    (1, 256, 256)])
@pytest.mark.parametrize("scheme", [1, 2])
def test_axis_exchange(bc, m, n, scheme):
    """The scheme treats x and y alike, so the step on the transposed input
    with the boundary conditions of the two axes exchanged is the transposed
    step.  Each axis's Neumann path is then checked against the other's, on
    grids that are not square and tiles that are not square."""
    swapped = ((bc & 1) << 1) | ((bc >> 1) & 1)
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=131)
    phikm1 = I.noise(m, n, mean=0.1, amp=0.1, seed=132)
    out = []
    for b, t, (mm, nn) in ((bc, lambda a: a, (m, n)),
                           (swapped, lambda a: np.ascontiguousarray(a.T), (n, m))):
        _, pg = both(scheme, b, h=math.pi / 4, dt=0.05)
        st = api.Stepper(mm, nn, pg, tol=1e-12, max_cycles=100)
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
