"""The learned initial guess on the GPU (BF16 matrix-core kernels) against the
FP64 CPU reference network (oracle/cnn.py), and inside the time step.

Bars: BF16 operands carry 8 significant bits, so forward outputs and
gradients agree with the FP64 reference to about 1e-2 relative (the tests use
3e-2 for outputs and 5e-2 per gradient array); Adam runs in FP32 and matches
the reference update of the same gradient to 1e-5.  Inside the step the
solution does not depend on the guess (Sec. 3, unique solvability), so a step
from the learned guess must agree with one from extrapolation to the solver
tolerance, and a network that cannot beat extrapolation must fall back to it
exactly.
"""
import math

import numpy as np
import pytest

from oracle import cnn as N
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def samples(m, n, count, seed, dt=0.05):
    """(phi^{n-1}, phi^n, psi^n, phi^{n+1})."""
    out = []
    for k in range(count):
        a = I.noise(m, n, mean=0.1, amp=0.1, seed=seed + 4 * k)
        b = a + I.noise(m, n, mean=0.0, amp=0.01, seed=seed + 4 * k + 1)
        p = (b - a) / dt + I.noise(m, n, mean=0.0, amp=0.05, seed=seed + 4 * k + 3)
        c = 2 * b - a + I.noise(m, n, mean=0.0, amp=0.002, seed=seed + 4 * k + 2)
        out.append((a, b, p, c))
    return out


def cols(S, *idx):
    return [[dev(s[i]) for s in S] for i in idx]


def make_blob(seed=3):
    """Hidden and output weights all random, small random biases."""
    blob = N.init_blob(seed, zero_last=False)
    rng = np.random.default_rng(seed + 100)
    off = N.HEADER
    for name, shape in N.layout():
        cnt = int(np.prod(shape))
        if name.startswith("b"):
            blob[off:off + cnt] = rng.uniform(-0.1, 0.1, cnt)
        off += cnt
    blob[5] = 0.5  # out_scale
    return blob


M, NN, B = 32, 64, 2


def test_predict_matches_oracle():
    blob = make_blob()
    S = samples(M, NN, B, 10)
    tr = api.CnnTrainer(M, NN, B, blob)
    got = tr.predict(*cols(S, 0, 1, 2))
    tr.close()
    for k, (a, b, p, _) in enumerate(S):
        ref = N.guess(blob, a, b, p)
        g = host(got[k])
        # the learned correction (the part the network adds to extrapolation)
        assert rel(g - (2 * b - a), ref - (2 * b - a)) <= 3e-2, k
        assert abs(np.mean(g) - np.mean(2 * b - a)) < 1e-14


def test_gradients_match_oracle():
    blob = make_blob(4)
    S = samples(M, NN, B, 20)
    tr = api.CnnTrainer(M, NN, B, blob)
    loss, g = tr.step(*cols(S, 0, 1, 2, 3), update=False, grad=True)
    tr.close()
    lref, gref = N.loss_and_grad(blob, S)
    assert abs(loss - lref) <= 3e-2 * lref
    off = 0
    for name, shape in N.layout():
        cnt = int(np.prod(shape))
        assert rel(g[off:off + cnt], gref[off:off + cnt]) <= 5e-2, name
        off += cnt


def test_adam_matches_oracle_on_gpu_gradients():
    blob = make_blob(5)
    S = samples(M, NN, B, 30)
    lr = 3e-3
    tr = api.CnnTrainer(M, NN, B, blob, lr=lr)
    args = cols(S, 0, 1, 2, 3)
    theta = blob[N.HEADER:].astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in (1, 2):
        _, g = tr.step(*args, update=True, grad=True)
        theta, m, v = N.adam(theta, g.astype(np.float64), m, v, t, lr)
        got = tr.blob()[N.HEADER:].astype(np.float64)
        assert np.max(np.abs(got - theta)) <= 1e-5 * max(1.0, np.max(np.abs(theta)))
    tr.close()


def test_training_reduces_loss():
    blob = N.init_blob(6)
    S = samples(M, NN, B, 40)
    tr = api.CnnTrainer(M, NN, B, blob, lr=3e-3)
    args = cols(S, 0, 1, 2, 3)
    first = tr.step(*args)
    for _ in range(60):
        last = tr.step(*args)
    tr.close()
    assert last < 0.5 * first


def crystal_run(stepper, steps, seed=5, N_=64):
    phi0 = I.crystallites(N_, N_, math.pi / 4, count=2, radius_cells=8, seed=seed)
    return api.run(stepper, dev(phi0), steps)


PARAMS = dict(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=2)


def test_fallback_is_exact():
    """A network whose output is zero reproduces extrapolation and counts
    every step as a fallback; a NaN network too; the states are bitwise those
    of the extrapolated guess."""
    p = api.Params(**PARAMS)
    ref = api.Stepper(64, 64, p, energy=0, guess=L.MPFC_GUESS_EXTRAP)
    phi_r, _, _, inf_r = crystal_run(ref, 4)
    for kind in ("zero", "nan"):
        blob = N.init_blob(7, zero_last=True)
        if kind == "nan":
            blob[N.HEADER + 700] = np.nan
        st = api.Stepper(64, 64, p, energy=0, guess=L.MPFC_GUESS_CNN)
        st.load_cnn(blob)
        phi, _, _, inf = crystal_run(st, 4)
        used, fb = st.cnn_counts()
        assert (used, fb) == (0, 4), kind
        assert np.array_equal(host(phi), host(phi_r)), kind
        assert [i.n_cycles for i in inf] == [i.n_cycles for i in inf_r]


def test_learned_guess_requires_a_network():
    st = api.Stepper(64, 64, api.Params(**PARAMS), energy=0, guess=L.MPFC_GUESS_CNN)
    x = dev(np.full((64, 64), 0.1))
    with pytest.raises(L.MpfcError):
        st.step(x, x, torch.zeros_like(x), torch.empty_like(x))
    with pytest.raises(L.MpfcError):
        st.load_cnn(np.zeros(10, dtype=np.float32))
    with pytest.raises(L.MpfcError):  # trained for another time step
        st.load_cnn(N.init_blob(1, dt=0.1))


def test_trained_network_gain():
    """The committed network (trained on solver runs from seeds 100+) on a
    held-out start (seed 5), 256^2, 40 steps: it cuts the initial residual of
    the step by more than 10x against extrapolation, never needs more
    V-cycles in total, and the states agree to the solver tolerance."""
    from paper_1208_2643_amd import guess_net
    blob = guess_net.load()
    p = api.Params(**PARAMS)
    phi0 = I.crystallites(256, 256, math.pi / 4, seed=5)
    out = {}
    for guess in (L.MPFC_GUESS_EXTRAP, L.MPFC_GUESS_CNN):
        st = api.Stepper(256, 256, p, energy=0, guess=guess)
        if guess == L.MPFC_GUESS_CNN:
            st.load_cnn(blob)
        phi, _, _, infos = api.run(st, dev(phi0), 40)
        counts = st.cnn_counts() if guess == L.MPFC_GUESS_CNN else None
        out[guess] = (host(phi), infos, counts)
    (pe, ie, _), (pc, ic, (used, fb)) = out[L.MPFC_GUESS_EXTRAP], out[L.MPFC_GUESS_CNN]
    r_e = np.median([i.history[0] for i in ie[2:]])
    r_c = np.median([i.history[0] for i in ic[2:]])
    assert r_c < 0.1 * r_e, (r_c, r_e)
    assert sum(i.n_cycles for i in ic) <= sum(i.n_cycles for i in ie)
    assert used >= 35 and used + fb == 40
    assert rel(pc, pe) < 1e-9


@pytest.mark.parametrize("m,n", [(16, 16), (32, 32), (16, 32)])
def test_learned_guess_on_untiled_grids(m, n):
    """Grids of at most 32 x 32 cells have no tiled level; the learned
    candidate still has its own copy of the finest level.  The steps agree
    with the extrapolated steps to the solver tolerance (the solution does not
    depend on the guess) and each starts from the learned or the extrapolated
    guess."""
    from paper_1208_2643_amd import guess_net
    p = api.Params(**PARAMS)
    phi0 = I.noise(m, n, mean=0.07, amp=0.05, seed=11)
    out = {}
    for guess in (L.MPFC_GUESS_EXTRAP, L.MPFC_GUESS_CNN):
        st = api.Stepper(m, n, p, energy=0, guess=guess, tol=1e-11)
        if guess == L.MPFC_GUESS_CNN:
            st.load_cnn(guess_net.load())
        phi, _, _, infos = api.run(st, dev(phi0), 4)
        assert all(i.status == 0 for i in infos)
        out[guess] = host(phi)
        if guess == L.MPFC_GUESS_CNN:
            used, fb = st.cnn_counts()
            assert used + fb == 4
    assert rel(out[L.MPFC_GUESS_CNN], out[L.MPFC_GUESS_EXTRAP]) < 1e-10


def test_learned_guess_with_mixed_precision():
    """The learned guess starting mixed-precision steps (FP32 correction
    cycles inside FP64 defect correction): the network's candidate is used,
    every step reaches the FP64 tolerance, and the states agree with FP64
    steps from the extrapolated guess to the mixed-precision bar (1e-9)."""
    from paper_1208_2643_amd import guess_net
    p = api.Params(**PARAMS)
    phi0 = I.crystallites(256, 256, math.pi / 4, seed=5)
    st = api.Stepper(256, 256, p, energy=0, guess=L.MPFC_GUESS_CNN, precision=L.MPFC_MIXED)
    st.load_cnn(guess_net.load())
    pm, _, _, im = api.run(st, dev(phi0), 12)
    used, fb = st.cnn_counts()
    st.close()
    st = api.Stepper(256, 256, p, energy=0, guess=L.MPFC_GUESS_EXTRAP)
    pe, _, _, ie = api.run(st, dev(phi0), 12)
    st.close()
    assert all(i.status == 0 and i.residual <= 1e-10 and i.outer_iters > 0 for i in im)
    assert used >= 10 and used + fb == 12
    assert rel(host(pm), host(pe)) < 1e-9


@pytest.mark.parametrize("precision", [L.MPFC_FP64, L.MPFC_MIXED])
def test_learned_guess_graph_replay_equals_direct_launches(precision):
    """The learned-guess set-up (the network, both candidates, their residuals
    and the choice) replays a captured graph whose kernels read the caller's
    arrays from the step's device table; with launch timing on, the same
    kernels are launched one by one.  Six steps of each, with the program's
    own eager work between them and the arrays rotating, give the same states
    (each context tunes its own tile shapes, which may regroup the norm's
    partial sums, hence a bar rather than bitwise equality) and the same
    choice of candidate in every step."""
    from paper_1208_2643_amd import guess_net
    p = api.Params(**PARAMS)
    phi0 = I.crystallites(128, 128, math.pi / 4, radius_cells=16, seed=5)

    def touch(phi, nxt, psi, info):
        assert info.status == 0
        float((nxt - phi).abs().sum())   # eager torch kernels, then a sync

    runs = []
    for direct in (False, True):
        st = api.Stepper(128, 128, p, energy=0, guess=L.MPFC_GUESS_CNN, precision=precision)
        st.load_cnn(guess_net.load())
        if direct:
            st.profile(True)
        phi, _, psi, infos = api.run(st, dev(phi0), 6, record=touch)
        runs.append((host(phi), host(psi), [i.history[0] for i in infos], st.cnn_counts()))
        st.close()
    (pa, sa, ha, ca), (pb, sb, hb, cb) = runs
    assert np.max(np.abs(pa - pb)) <= 1e-12
    assert np.max(np.abs(sa - sb)) <= 1e-10
    assert np.allclose(ha, hb, rtol=1e-9, atol=0)   # residual of the kept guess
    assert ca == cb and ca[0] >= 4
