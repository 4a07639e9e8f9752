"""The persistent coarse kernel's threshold (mpfc_opts.coarse_threshold):
with 256 the 32 x 32 level runs as fused tile launches instead of inside the
persistent kernel; the cycle is the same, so the one-cycle iterate equals the
oracle's element by element and steps equal the default threshold's."""
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


@pytest.mark.parametrize("scheme,m,n,thr", [(2, 64, 64, 256), (1, 128, 64, 256), (2, 64, 32, 512),
                                            (2, 32, 32, 256)])
def test_one_cycle_iterate_matches_oracle(scheme, m, n, thr):
    d = dict(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=scheme)
    po, pg = O.Params(**d), api.Params(**d)
    phik = I.noise(m, n, mean=0.1, amp=0.1, seed=41)
    prev = I.noise(m, n, mean=0.1, amp=0.1, seed=42)
    st = api.Stepper(m, n, pg, tol=1e-30, max_cycles=1, energy=0, coarse_threshold=thr)
    psi = torch.zeros(n, m, dtype=torch.float64, device=DEV)
    mu, ka = torch.empty_like(psi), torch.empty_like(psi)
    phi_g, info = st.step(dev(phik), dev(prev), psi, mu=mu, kappa=ka, allow_fail=True)
    assert info.status == L.MPFC_ENOTCONVERGED
    S = O.source(po, phik, prev, np.zeros_like(phik))
    u0 = O.complete_guess(po, 2 * phik - prev, S, phik)
    u, _, _ = O.fas_solve(po, u0, S, phik=phik, tol=1e-30, max_cycles=1)
    for a, b in zip((host(phi_g), host(mu), host(ka)), u):
        assert relmax(a, b) <= 1e-12
    st.close()


@pytest.mark.parametrize("precision", [L.MPFC_FP64, L.MPFC_MIXED])
def test_steps_equal_default_threshold(precision):
    N = 128
    p = api.Params(0.025, 0.9, 1.0, math.pi / 4, 0.05, 2)
    phi0 = I.crystallites(N, N, math.pi / 4, radius_cells=N / 8, seed=3)
    out = []
    for thr in (0, 256):
        st = api.Stepper(N, N, p, tol=1e-10, precision=precision, coarse_threshold=thr)
        phi, _, psi, infos = api.run(st, dev(phi0), 5)
        st.close()
        out.append((host(phi), [i.n_cycles for i in infos], infos[-1].energy_mod))
    assert out[0][1] == out[1][1]
    assert rel_l2(out[1][0], out[0][0]) <= 1e-12
    assert abs(out[1][2] - out[0][2]) <= 1e-12 * abs(out[0][2])
