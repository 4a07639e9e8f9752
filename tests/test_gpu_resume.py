"""Checkpoint and resume: a run interrupted after k steps, its state
(phi^k, phi^{k-1}, psi^k) written to a file, the solver context destroyed,
and the run continued from the file in a new context, equals the
uninterrupted run.  For the second-order scheme psi^k carries the run's
history (eq. discrete_2_b), so resuming from (phi^k, phi^{k-1}) alone would
not; the test checks that too."""
import math

import numpy as np
import pytest

from paper_1208_2643_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1208_2643_amd import api  # noqa: E402
from paper_1208_2643_amd import _lib as L  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def steps(st, phi, prev, psi, k):
    nxt = torch.empty_like(phi)
    infos = []
    for _ in range(k):
        _, info = st.step(phi, prev, psi, nxt)
        infos.append(info)
        prev, phi, nxt = phi, nxt, prev
    return phi, prev, psi, infos


@pytest.mark.parametrize("scheme,precision", [(2, L.MPFC_FP64), (1, L.MPFC_FP64),
                                              (2, L.MPFC_MIXED)])
def test_resume_equals_uninterrupted_run(scheme, precision, tmp_path):
    N, k1, k2 = 128, 6, 6
    p = api.Params(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=scheme)
    phi0 = torch.from_numpy(I.crystallites(N, N, p.h, radius_cells=12, seed=21)).to(DEV)
    kw = dict(tol=1e-11, precision=precision)
    st = api.Stepper(N, N, p, **kw)
    phi, prev, psi, ref_infos = steps(st, phi0.clone(), phi0.clone(), torch.zeros_like(phi0),
                                      k1 + k2)
    ref = phi.cpu().numpy()
    st.close()

    st = api.Stepper(N, N, p, **kw)
    phi, prev, psi, infos = steps(st, phi0.clone(), phi0.clone(), torch.zeros_like(phi0), k1)
    f = tmp_path / "state.npz"
    api.save_state(f, phi, prev, psi, k1, p)
    st.close()
    del phi, prev, psi

    phi, prev, psi, step, p2 = api.load_state(f)
    assert step == k1 and p2 == p
    st = api.Stepper(N, N, p2, **kw)
    phi, prev, psi, infos2 = steps(st, phi, prev, psi, k2)
    assert rel(phi.cpu().numpy(), ref) <= 1e-11
    # energies after resuming (the Poisson solve of the -1 norm starts cold in
    # the new context) equal the uninterrupted run's to its tolerance
    a, b = infos2[-1], ref_infos[-1]
    assert a.energy_status == 0
    for key in ("energy_F", "energy_pseudo", "energy_mod", "mass"):
        x, y = getattr(a, key), getattr(b, key)
        assert abs(x - y) <= 1e-9 * abs(y), key
    st.close()

    if scheme == 2:
        # psi is part of the state: restarting with psi = 0 changes the run
        phi, prev, _, _, _ = api.load_state(f)
        st = api.Stepper(N, N, p, **kw)
        phi, _, _, _ = steps(st, phi, prev, torch.zeros_like(phi), k2)
        assert rel(phi.cpu().numpy(), ref) > 1e-8
        st.close()
