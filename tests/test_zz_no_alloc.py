"""mpfc_op_smooth_noalloc (static device scratch, no allocation during the
call) against mpfc_op_smooth (scratch from hipMalloc), through the C ABI:
the same kernels run on the same inputs, so the results agree bit for bit.
Two calls in a row, the second on a smaller grid (the static array keeps the
first call's contents), and a grid beyond the array's size is refused."""
import ctypes
import math

import numpy as np
import pytest

from paper_1208_2643_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1208_2643_amd import _lib as L  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def smooth(fn, p, m, n, fields, sweeps, seed):
    """Copies of (phi, mu, kappa) smoothed in place by `fn`; returns them on the host."""
    phik, u, f = fields
    uu = [x.clone() for x in u]
    s = torch.cuda.current_stream()
    rc = fn(ctypes.byref(p), L.MPFC_NEWTON, m, n, ptr(phik), ptr(uu[0]), ptr(uu[1]), ptr(uu[2]),
            ptr(f[0]), ptr(f[1]), ptr(f[2]), sweeps, ctypes.c_void_p(s.cuda_stream))
    assert rc == 0, (rc, L.load().mpfc_last_error())
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in uu]


def fields(m, n, seed):
    phik = dev(I.noise(m, n, mean=0.1, amp=0.05, seed=seed))
    u = [dev(I.noise(m, n, mean=mean, amp=0.05, seed=seed + k + 1))
         for k, mean in enumerate((0.1, 0.0, 0.0))]
    f = [dev(I.noise(m, n, mean=0.0, amp=0.1, seed=seed + k + 4)) for k in range(3)]
    return phik, u, f


def test_noalloc_smooth_equals_allocating_smooth_twice():
    lib = L.load()
    p = L.mpfc_params(0.025, 0.9, 1.0, math.pi / 4, 0.05, 2, 0)
    # first a larger grid with an odd number of passes (the result is copied
    # back from the scratch), then a smaller one, not a power of two in x
    for (m, n, sweeps, seed) in ((256, 256, 3, 100), (96, 64, 2, 200)):
        fl = fields(m, n, seed)
        ref = smooth(lib.mpfc_op_smooth, p, m, n, fl, sweeps, seed)
        got = smooth(lib.mpfc_op_smooth_noalloc, p, m, n, fl, sweeps, seed)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (m, n)
        # the sweeps changed the fields
        assert not np.array_equal(got[0], fl[1][0].cpu().numpy())


def test_noalloc_smooth_refuses_grids_beyond_its_scratch():
    lib = L.load()
    p = L.mpfc_params(0.025, 0.9, 1.0, math.pi / 4, 0.05, 2, 0)
    x = torch.zeros(1024, 1024, dtype=torch.float64, device=DEV)
    q = ptr(x)
    rc = lib.mpfc_op_smooth_noalloc(ctypes.byref(p), L.MPFC_NEWTON, 1024, 1024, q, q, q, q, q, q,
                                    q, 1, None)
    assert rc == L.MPFC_EINVAL
    assert b"512 x 512" in lib.mpfc_last_error()
