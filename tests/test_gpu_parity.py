"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Operator level: each V-cycle operation on the same seeded inputs, element by
element.  Step level: whole time steps of both schemes against the oracle
solved to a tighter tolerance; the bar is a relative L2 difference of 1e-10
(FP64).  Sizes span several workgroups with ragged tails, plus the full
1024^2 grid of the benchmark workload.
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


def both(scheme, **kw):
    d = dict(eps=0.025, beta=0.9, M=1.0, h=0.5, dt=0.1, scheme=scheme)
    d.update(kw)
    return O.Params(**d), api.Params(**d)


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
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("m,n", SIZES)
def test_source(scheme, m, n):
    po, pg = both(scheme, h=0.37, dt=0.3)
    phik, phikm1, psik, _ = state(m, n, 100)
    ref = O.source(po, phik, phikm1, psik)
    got = api.op_source(pg, dev(phik), dev(phikm1), dev(psik))
    for a, b in zip(got, ref):
        if np.max(np.abs(b)) == 0:
            assert np.max(np.abs(host(a))) == 0
        else:
            assert relmax(host(a), b) <= 1e-14


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("m,n", SIZES)
def test_residual(scheme, m, n):
    po, pg = both(scheme, h=0.37, dt=0.3)
    phik, phikm1, psik, u = state(m, n, 200)
    f = O.source(po, phik, phikm1, psik)
    ref = O.residual(po, u, f, phik)
    got = api.op_residual(pg, [dev(x) for x in u], [dev(x) for x in f], dev(phik))
    for a, b in zip(got, ref):
        assert relmax(host(a), b) <= 1e-13


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("newton", [True, False])
@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("m,n", SIZES)
def test_smooth(scheme, newton, sweeps, m, n):
    """Red-black sweeps: GPU and oracle visit cells in the same colour order,
    so iterates agree up to rounding."""
    po, pg = both(scheme, h=0.5, dt=0.1)
    phik, phikm1, psik, u = state(m, n, 300)
    f = O.source(po, phik, phikm1, psik)
    ref = O.smooth(po, u, f, phik=phik, sweeps=sweeps, newton=newton)
    ud = [dev(x) for x in u]
    api.op_smooth(pg, ud, [dev(x) for x in f], dev(phik), sweeps=sweeps, newton=newton)
    for a, b in zip(ud, ref):
        assert relmax(host(a), b) <= 1e-12


@pytest.mark.parametrize("m,n", [(4, 4), (64, 32), (128, 256)])
def test_restrict(m, n):
    f = I.noise(m, n, mean=0.0, amp=1.0, seed=400)
    assert relmax(host(api.op_restrict(dev(f))), O.restrict(f)) <= 1e-15


# ---------------------------------------------------------------- step level
def run_both(po, pg, phi0, steps, tol_gpu=1e-10, tol_orc=1e-12, **opts):
    st = api.Stepper(phi0.shape[1], phi0.shape[0], pg, tol=tol_gpu, **opts)
    phi_g, prev_g, psi_g, infos = api.run(st, dev(phi0), steps)
    phi_o, prev_o, psi_o, res = O.run(po, phi0, steps, tol=tol_orc, max_cycles=300)
    assert all(r.cycles >= 0 for r in res)
    assert all(i.status == 0 for i in infos)
    return (host(phi_g), host(psi_g), infos), (phi_o, psi_o, res)


def test_scheme1_64_ten_steps():
    """First-order scheme, 64^2, h = 0.5, eps = 0.025, beta = 0.9, M = 1,
    dt = 0.1, noise initial data, 10 steps of V(2,2) to 1e-10."""
    po, pg = both(1, h=0.5, dt=0.1)
    phi0 = I.noise(64, 64, mean=0.07, amp=0.05, seed=1)
    (pg_, sg, infos), (po_, so, res) = run_both(po, pg, phi0, 10)
    assert rel_l2(pg_, po_) <= 1e-10
    assert rel_l2(sg, so) <= 1e-8   # psi = (phi^{k+1} - phi^k)/s amplifies by 1/s
    for i, r in zip(infos, res):
        assert i.energy_status == 0  # the -1 norm's Poisson solve converged
        assert abs(i.energy_pseudo - r.energies[1]) <= 1e-9 * abs(r.energies[1])
        assert abs(i.mass - r.energies[3]) <= 1e-12 * abs(r.energies[3])


@pytest.mark.parametrize("N", [32, 128])
def test_scheme2_crystallites(N):
    """Second-order scheme with the parameters of the 1024^2 workload
    (h = pi/4, dt = 0.05) on smaller grids, crystallite initial data."""
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, radius_cells=N / 8, seed=2)
    (pg_, sg, infos), (po_, so, res) = run_both(po, pg, phi0, 6)
    assert rel_l2(pg_, po_) <= 1e-10
    assert rel_l2(sg, so) <= 1e-8
    for i, r in zip(infos, res):
        assert i.energy_status == 0
        assert abs(i.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])


@pytest.mark.parametrize("scheme", [1, 2])
def test_cycle_history_matches_oracle(scheme):
    """Same guess and same V-cycle components: the GPU's residual history
    follows the oracle's cycle by cycle."""
    po, pg = both(scheme, h=math.pi / 4, dt=0.05)
    phi0 = I.noise(64, 64, mean=0.1, amp=0.1, seed=7)
    prev = I.noise(64, 64, mean=0.1, amp=0.1, seed=8)
    st = api.Stepper(64, 64, pg, tol=1e-11, guess=L.MPFC_GUESS_EXTRAP, energy=0)
    psi = torch.zeros(64, 64, dtype=torch.float64, device=DEV)
    _, info = st.step(dev(phi0), dev(prev), psi)
    r = O.step(po, phi0, prev, np.zeros_like(phi0), guess=1, tol=1e-11, energy=False)
    assert info.n_cycles == r.cycles
    # relative agreement above the FP64 rounding floor of the residual (~1e-14 here)
    np.testing.assert_allclose(info.history, r.history, rtol=1e-6, atol=1e-13)


def test_full_size_single_step_1024():
    """One step of the 1024^2 workload (scheme 2, h = pi/4, dt = 0.05,
    crystallites) in the benchmark's configuration, against the oracle."""
    N = 1024
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, seed=2)
    st = api.Stepper(N, N, pg, tol=1e-10)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=100)
    assert r.cycles > 0 and info.status == 0 and info.energy_status == 0
    assert rel_l2(host(phi_g), r.phi) <= 1e-10
    assert abs(info.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])


@pytest.mark.parametrize("scheme", [1, 2])
def test_guess_independence_gpu(scheme):
    """Unique solvability: previous-step and extrapolated guesses give the
    same phi^{k+1}."""
    _, pg = both(scheme, h=0.5, dt=2.0)
    phik = dev(I.noise(64, 64, mean=0.1, amp=0.05, seed=61))
    phikm1 = dev(I.noise(64, 64, mean=0.1, amp=0.05, seed=62))
    outs = []
    for g in (L.MPFC_GUESS_PREV, L.MPFC_GUESS_EXTRAP):
        st = api.Stepper(64, 64, pg, tol=1e-12, guess=g, max_cycles=300, energy=0)
        psi = torch.zeros_like(phik)
        phi, info = st.step(phik, phikm1, psi)
        assert info.status == 0
        outs.append(host(phi))
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-10


@pytest.mark.parametrize("scheme", [1, 2])
def test_mass_and_energy_invariants_gpu(scheme):
    """Mass conservation and the monotone energy (pseudo energy for scheme 1,
    modified energy for scheme 2) over a run at a large time step."""
    _, pg = both(scheme, h=0.5, dt=2.0)
    phi0 = I.noise(64, 64, mean=0.1, amp=0.05, seed=71)
    st = api.Stepper(64, 64, pg, tol=1e-11, max_cycles=300)
    phi, prev, psi, infos = api.run(st, dev(phi0), 8)
    mass0 = 0.25 * phi0.sum()
    key = "energy_pseudo" if scheme == 1 else "energy_mod"
    e = [getattr(i, key) for i in infos]
    for i in infos:
        assert i.energy_status == 0
        assert abs(i.mass - mass0) <= 1e-10 * abs(mass0)
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(e, e[1:]))
    assert abs(host(psi).mean()) <= 1e-10


def test_status_codes():
    _, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.noise(64, 64, mean=0.1, amp=0.1, seed=81)
    st = api.Stepper(64, 64, pg, tol=1e-14, max_cycles=1, energy=0)
    psi = torch.zeros(64, 64, dtype=torch.float64, device=DEV)
    _, info = st.step(dev(phi0), dev(phi0), psi, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED and info.n_cycles == 1
    bad = phi0.copy()
    bad[3, 5] = np.nan
    st2 = api.Stepper(64, 64, pg, energy=0)
    psi = torch.zeros(64, 64, dtype=torch.float64, device=DEV)
    _, info = st2.step(dev(bad), dev(bad), psi, allow_fail=True)
    assert info.status == L.MPFC_ENONFINITE and info.n_cycles == 0


def test_constant_state_gpu():
    _, pg = both(2, h=0.5, dt=0.7)
    f = dev(np.full((32, 32), 0.23))
    st = api.Stepper(32, 32, pg, energy=0)
    psi = torch.zeros_like(f)
    phi, info = st.step(f, f, psi)
    assert info.n_cycles == 0
    assert np.max(np.abs(host(phi) - 0.23)) == 0.0


def test_translation_equivariance():
    """A periodic shift of the input by a non-tile-multiple offset shifts the
    result (checks the index wrap of every kernel)."""
    _, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.noise(128, 64, mean=0.1, amp=0.1, seed=91)
    st = api.Stepper(128, 64, pg, tol=1e-12, energy=0)
    a, _ = st.step(dev(phi0), dev(phi0), torch.zeros(64, 128, dtype=torch.float64, device=DEV))
    sh = np.roll(phi0, (13, 37), axis=(0, 1))
    b, _ = st.step(dev(sh), dev(sh), torch.zeros(64, 128, dtype=torch.float64, device=DEV))
    assert np.max(np.abs(np.roll(host(a), (13, 37), axis=(0, 1)) - host(b))) <= 1e-10


@pytest.mark.parametrize("scheme,precision,N", [
    (1, L.MPFC_FP64, 256), (2, L.MPFC_FP64, 256), (2, L.MPFC_MIXED, 256), (2, L.MPFC_FP64, 1024)])
def test_transposition_equivariance(scheme, precision, N):
    """On a square periodic grid the scheme treats x and y alike, so
    exchanging the axes of the input exchanges them in phi^{k+1}, psi^{k+1}
    and mu and leaves the energies and the mass unchanged.  The tiles are not
    square (64 x 32, 32 x 16 ...), so an index or halo mistake along one axis
    breaks the symmetry."""
    _, pg = both(scheme, h=math.pi / 4, dt=0.05)
    phik = I.noise(N, N, mean=0.1, amp=0.1, seed=95)
    phikm1 = I.noise(N, N, mean=0.1, amp=0.1, seed=96)
    psik = I.noise(N, N, mean=0.0, amp=0.05, seed=97)
    tol = 1e-12 if N <= 256 else 1e-11
    out = []
    for t in (lambda a: a, lambda a: np.ascontiguousarray(a.T)):
        st = api.Stepper(N, N, pg, tol=tol, precision=precision, max_cycles=100)
        psi = dev(t(psik))
        mu = torch.empty_like(psi)
        phi, info = st.step(dev(t(phik)), dev(t(phikm1)), psi, mu=mu)
        assert info.status == 0 and info.n_cycles > 0
        out.append((t(host(phi)), t(host(psi)), t(host(mu)), info))
        st.close()
    (pa, sa, ma, ia), (pb, sb, mb, ib) = out
    assert np.max(np.abs(pa - pb)) <= 1e-10
    assert np.max(np.abs(sa - sb)) <= 1e-8   # psi scales the phi difference by 1/s or 2/s
    assert np.max(np.abs(ma - mb)) <= 1e-8
    for key in ("energy_F", "energy_pseudo", "energy_mod", "mass"):
        a, b = getattr(ia, key), getattr(ib, key)
        assert abs(a - b) <= 1e-10 * max(1.0, abs(a)), key


@pytest.mark.parametrize("dims,scheme,precision,sched", [
    (2, 1, L.MPFC_FP64, None), (2, 2, L.MPFC_FP64, None), (2, 2, L.MPFC_MIXED, None),
    (2, 2, L.MPFC_MIXED, (3, 1, 1)), (3, 2, L.MPFC_FP64, None)])
def test_graph_replay_equals_eager_launches(dims, scheme, precision, sched):
    """Steps replay captured HIP graphs; with launch timing switched on the
    same kernels are launched one by one.  Six steps of each, with the
    program's own eager work and a synchronisation between the steps, give
    the same states and energies (every replay after the first is checked).
    sched: FP32 cycles of a step's first and later outer iterations and the
    passes below the finest level (runs holding a step's first outer
    iteration are graphs of their own)."""
    _, pg = both(scheme, h=math.pi / 4, dt=0.05)
    if dims == 2:
        phi0 = I.crystallites(256, 256, math.pi / 4, radius_cells=20, seed=2)
    else:
        phi0 = np.random.default_rng(161).uniform(0.02, 0.12, size=(32, 32, 32))

    def touch(phi, nxt, psi, info):
        assert info.status == 0
        float((nxt - phi).abs().sum())   # eager torch kernels, then a sync

    runs = []
    for eager in (False, True):
        if dims == 2:
            kw = {} if sched is None else dict(inner_cycles=sched[0], inner_cycles_next=sched[1],
                                               inner_nu_coarse=sched[2])
            st = api.Stepper(256, 256, pg, tol=1e-10, precision=precision, **kw)
        else:
            st = api.Stepper3(32, 32, 32, pg, tol=1e-10, coarse_sweeps=2)
        if eager:
            st.profile(True)
        phi, _, psi, infos = api.run(st, dev(phi0), 6, record=touch)
        runs.append((host(phi), host(psi), infos))
        st.close()
    (pa, sa, ia), (pb, sb, ib) = runs
    assert np.max(np.abs(pa - pb)) <= 1e-12
    assert np.max(np.abs(sa - sb)) <= 1e-10
    for a, b in zip(ia, ib):
        assert abs(a.energy_mod - b.energy_mod) <= 1e-12 * abs(a.energy_mod)
        assert abs(a.mass - b.mass) <= 1e-12 * abs(a.mass)


# ------------------------------------------------------------ mixed precision
@pytest.mark.parametrize("scheme", [1, 2])
def test_mixed_precision_matches_fp64_oracle(scheme):
    """FP32 correction cycles inside FP64 defect correction reach the same
    FP64 fixed point: relative L2 difference to the FP64 oracle <= 1e-9."""
    N = 128
    po, pg = both(scheme, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, radius_cells=N / 8, seed=3)
    st = api.Stepper(N, N, pg, tol=1e-10, precision=L.MPFC_MIXED, max_cycles=60)
    phi_g, prev_g, psi_g, infos = api.run(st, dev(phi0), 5)
    phi_o, prev_o, psi_o, res = O.run(po, phi0, 5, tol=1e-12, max_cycles=300)
    assert all(i.status == 0 and i.outer_iters > 0 for i in infos)
    assert all(i.residual <= 1e-10 for i in infos)
    assert rel_l2(host(phi_g), phi_o) <= 1e-9
    for i, r in zip(infos, res):
        assert abs(i.energy_mod - r.energies[2]) <= 1e-9 * abs(r.energies[2])


@pytest.mark.parametrize("inner,nxt,nuc", [(3, 1, 0), (2, 4, 0), (3, 2, 1)])
def test_mixed_precision_later_outer_cycle_count(inner, nxt, nuc):
    """inner_cycles FP32 cycles in a step's first outer iteration and
    inner_cycles_next in each later one (nuc: smoothing passes of those
    cycles below the finest level, 0 = nu1, nu2): same FP64 fixed point
    (oracle, 1e-9), and the reported FP32 cycle count is inner + (outer - 1)
    nxt."""
    N = 128
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, radius_cells=N / 8, seed=3)
    st = api.Stepper(N, N, pg, tol=1e-10, precision=L.MPFC_MIXED, max_cycles=60,
                     inner_cycles=inner, inner_cycles_next=nxt, inner_nu_coarse=nuc)
    phi_g, _, _, infos = api.run(st, dev(phi0), 5)
    st.close()
    phi_o, _, _, _ = O.run(po, phi0, 5, tol=1e-12, max_cycles=300)
    for i in infos:
        assert i.status == 0 and i.residual <= 1e-10 and i.outer_iters >= 1
        assert i.n_cycles == inner + (i.outer_iters - 1) * nxt
    assert rel_l2(host(phi_g), phi_o) <= 1e-9


def test_inner_nu_coarse_ignored_without_tiled_levels():
    """A 32 x 32 grid has no tiled level (the persistent kernel takes the
    finest level too), so the FP32 cycles keep nu1, nu2 there: the steps equal
    those without the option bit for bit."""
    _, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.noise(32, 32, mean=0.07, amp=0.05, seed=23)
    out = []
    for nuc in (0, 1):
        st = api.Stepper(32, 32, pg, tol=1e-10, precision=L.MPFC_MIXED, energy=0,
                         inner_nu_coarse=nuc)
        phi, _, _, infos = api.run(st, dev(phi0), 3)
        st.close()
        out.append((host(phi), [i.n_cycles for i in infos]))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_mixed_precision_full_size_1024():
    """One mixed-precision step of the 1024^2 workload against the oracle."""
    N = 1024
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, seed=2)
    st = api.Stepper(N, N, pg, tol=1e-10, precision=L.MPFC_MIXED)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=100)
    assert info.status == 0 and info.residual <= 1e-10
    assert rel_l2(host(phi_g), r.phi) <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_2048(precision):
    """One step of the 2048^2 workload (scheme 2, h = pi/4, dt = 0.05,
    crystallites seed 3) in FP64 and in mixed precision (four FP32 V-cycles per
    FP64 outer iteration, the benchmark's setting), against the oracle's step
    solved to 1e-12 (eight cycles, a few seconds on the host)."""
    N = 2048
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = I.crystallites(N, N, math.pi / 4, seed=3)
    kw = dict(precision=L.MPFC_MIXED, inner_cycles=4) if precision else {}
    st = api.Stepper(N, N, pg, tol=1e-10, energy=0, **kw)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    phi_g, info = st.step(dev(phi0), dev(phi0), psi)
    r = O.step(po, phi0, phi0, np.zeros_like(phi0), tol=1e-12, max_cycles=100, energy=False)
    assert r.cycles > 0 and info.status == 0 and info.residual <= 1e-10
    assert rel_l2(host(phi_g), r.phi) <= (1e-9 if precision else 1e-10)
    assert rel_l2(host(psi), r.psi) <= 1e-6
    st.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_one_cycle_iterate_matches_oracle(precision):
    """After exactly one V-cycle (FP64) the fused kernels' iterate equals the
    oracle's one-cycle iterate element by element (same components, same
    red-black order); the mixed path is checked after one outer iteration
    against the oracle's converged answer direction (residual must drop)."""
    N = 256
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phik = I.crystallites(N, N, math.pi / 4, radius_cells=24, seed=5)
    prev = phik.copy()
    st = api.Stepper(N, N, pg, tol=1e-30, max_cycles=1, precision=precision, energy=0)
    psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
    mu = torch.empty_like(psi)
    ka = torch.empty_like(psi)
    phi_g, info = st.step(dev(phik), dev(prev), psi, mu=mu, kappa=ka, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED
    if precision == 0:
        S = O.source(po, phik, prev, np.zeros_like(phik))
        u0 = O.complete_guess(po, 2 * phik - prev, S, phik)
        u, hist, _ = O.fas_solve(po, u0, S, phik=phik, tol=1e-30, max_cycles=1)
        for a, b in zip((host(phi_g), host(mu), host(ka)), u):
            assert relmax(a, b) <= 1e-12
    else:
        assert info.history[1] < 0.1 * info.history[0]


@pytest.mark.parametrize("precision,energy", [(0, 1), (0, 0), (1, 1), (1, 0)])
def test_mu_kappa_outputs_match_oracle(precision, energy):
    """The optional mu and kappa outputs, written by the step's wrap-up from the
    copy of the iterate that holds the result (with mixed precision either of
    the two), equal the oracle's converged mu and kappa over three steps: the
    first with a cold -1 norm solve, the later ones warm-started."""
    N = 128
    po, pg = both(2, h=math.pi / 4, dt=0.05)
    phi = I.crystallites(N, N, math.pi / 4, radius_cells=N / 8, seed=4)
    prev, psi = phi.copy(), np.zeros_like(phi)
    st = api.Stepper(N, N, pg, tol=1e-10, precision=precision, energy=energy, max_cycles=60)
    phi_d, prev_d, psi_d = dev(phi), dev(prev), dev(psi)
    mu = torch.empty_like(psi_d)
    ka = torch.empty_like(psi_d)
    outer = set()
    for _ in range(3):
        mu.fill_(float("nan"))
        ka.fill_(float("nan"))
        nxt, info = st.step(phi_d, prev_d, psi_d, mu=mu, kappa=ka)
        r = O.step(po, phi, prev, psi, guess=1, tol=1e-12, max_cycles=300, energy=False)
        assert info.status == 0 and r.cycles >= 0
        assert rel_l2(host(mu), r.mu) <= 1e-8
        assert rel_l2(host(ka), r.kappa) <= 1e-8
        outer.add(info.outer_iters)
        prev, phi, psi = phi, r.phi, r.psi
        prev_d, phi_d = phi_d, nxt
    if precision == 1:
        assert max(outer) >= 1


def test_mu_kappa_outputs_must_not_alias():
    _, pg = both(2, h=math.pi / 4, dt=0.05)
    phi0 = dev(I.noise(32, 32, mean=0.1, amp=0.1, seed=82))
    st = api.Stepper(32, 32, pg, energy=0)
    psi = torch.zeros_like(phi0)
    out = torch.empty_like(phi0)
    for mu, ka in ((psi, None), (None, phi0), (out, None), (out2 := torch.empty_like(phi0), out2)):
        with pytest.raises(L.MpfcError):
            st.step(phi0, phi0, psi, phi_np1=out, mu=mu, kappa=ka)


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_tile_shape_invariance(shape, monkeypatch):
    """Every tile shape gives the same iterate after a fixed number of
    V-cycles: red-black updates within a colour are independent and each
    cell's arithmetic does not depend on the tiling.  Agreement is bitwise
    except where the compiler contracts a multiply-add differently in one
    template instantiation (rounding level)."""
    N = 256
    _, pg = both(2, h=math.pi / 4, dt=0.05)
    phik = I.crystallites(N, N, math.pi / 4, radius_cells=24, seed=9)

    def run(env_shape):
        if env_shape is None:
            monkeypatch.delenv("MPFC_TILE_SHAPE", raising=False)
        else:
            monkeypatch.setenv("MPFC_TILE_SHAPE", str(env_shape))
        st = api.Stepper(N, N, pg, tol=1e-30, max_cycles=3, energy=0)
        psi = torch.zeros(N, N, dtype=torch.float64, device=DEV)
        phi, info = st.step(dev(phik), dev(phik), psi, allow_fail=True)
        assert info.n_cycles == 3
        return host(phi)

    ref = run(None)
    got = run(shape)
    diff = float(np.max(np.abs(ref - got)))
    print(f"shape {shape}: max |diff| = {diff:.3e}", flush=True)
    assert diff <= 1e-13 * float(np.max(np.abs(ref))), diff


@pytest.mark.parametrize("m,n", [(128, 128), (64, 128)])
@pytest.mark.parametrize("shape", list(range(7)))
@pytest.mark.parametrize("scheme", [1, 2])
def test_every_tile_shape_one_cycle_matches_oracle(scheme, shape, m, n, monkeypatch):
    """Each tile shape, forced on every level, gives the oracle's one-cycle
    iterate element by element (coarse down launches complete the right-hand
    side from u as loaded; regression test for a missing barrier that let a
    pass overwrite u before every wave had read it, seen only for tiles whose
    workgroups own an uneven number of blocks per wave)."""
    po, pg = both(scheme, h=0.5, dt=0.1)
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=13)
    monkeypatch.setenv("MPFC_TILE_SHAPE", str(shape))
    st = api.Stepper(m, n, pg, tol=1e-30, max_cycles=1, energy=0)
    psi = torch.zeros(n, m, dtype=torch.float64, device=DEV)
    phi, info = st.step(dev(phik), dev(phik), psi, allow_fail=True)
    assert info.n_cycles == 1
    pk = phik if scheme == 2 else None
    S = O.source(po, phik, phik, np.zeros_like(phik))
    u0 = O.complete_guess(po, phik.copy(), S, pk)
    u, _, _ = O.fas_solve(po, u0, S, phik=pk, tol=1e-30, max_cycles=1)
    assert relmax(host(phi), u[0]) <= 1e-12
