"""CPU oracle for the MPFC convex-splitting time step (FP64).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously-correct CPU
implementation of what the GPU library computes.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product package never does, and the two share no code.

The arithmetic lives in ``mpfc_oracle.c`` (built with ``-ffp-contract=off``);
this module only marshals numpy arrays into it.  ``brute`` holds an
independent brute-force formulation used to pin the FAS solver on tiny grids.

Arrays are float64, C-contiguous, shape (n, m): row j holds cells (i=0..m-1, j)
so that x (index i) is fastest, matching the storage order of the paper's
cell-centred grid functions in the library.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


class _Model(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("h", ctypes.c_double), ("s", ctypes.c_double),
                ("M", ctypes.c_double), ("beta", ctypes.c_double), ("eps", ctypes.c_double)]


@dataclass
class Params:
    """Model and discretisation parameters (Sec. 3; App. B).  bc = (x, y)
    boundary conditions of the two axes: 0 periodic, 1 homogeneous Neumann
    (App. A)."""
    eps: float
    beta: float
    M: float
    h: float
    dt: float
    scheme: int
    bc: tuple = (0, 0)
    omega: float = 1.0  # relaxation factor of the smoother's cell update (1: App. B)

    @property
    def alpha(self) -> float:
        return 1.0 - self.eps

    def _c(self) -> _Model:
        return _Model(self.scheme, self.h, self.dt, self.M, self.beta, self.eps)


def load():
    """Load (building if needed) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    srcs = [os.path.join(_HERE, f) for f in ("mpfc_oracle.c", "mpfc3d_oracle.c")]
    if not os.path.exists(_LIBPATH) or any(os.path.getmtime(_LIBPATH) < os.path.getmtime(f)
                                           for f in srcs):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    i, d, v = ctypes.c_int, ctypes.c_double, None
    P = ctypes.POINTER(_Model)
    sigs = {
        "orc_laplacian": (v, [i, i, d, _dp, _dp]),
        "orc_coefficients": (v, [P, _dp, _dp]),
        "orc_source": (v, [P, i, i, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_operator": (v, [i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_residual": (v, [i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                             _dp]),
        "orc_norm3": (d, [i, i, d, _dp, _dp, _dp]),
        "orc_smooth_color": (v, [i, i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_smooth": (v, [i, i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_smooth_lex": (v, [i, i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_restrict": (v, [i, i, _dp, _dp]),
        "orc_prolong_add": (v, [i, i, _dp, _dp]),
        "orc_dense_newton": (i, [i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, i, _dp]),
        "orc_fas_solve": (i, [i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                              i, i, i, i, d, i, _dp, _dp]),
        "orc_complete_guess": (v, [i, i, i, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_psi_update": (v, [i, ctypes.c_size_t, d, _dp, _dp, _dp, _dp]),
        "orc_energy_F": (d, [i, i, d, d, _dp]),
        "orc_grad_sq": (d, [i, i, _dp]),
        "orc_poisson_cg": (i, [i, i, d, _dp, _dp, d, i]),
        "orc_norm_m1_sq": (d, [i, i, d, _dp]),
        "orc_energies": (v, [i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_step": (i, [P, i, i, i, _dp, _dp, _dp, i, i, i, i, i, d, i,
                         _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_set_bc": (v, [i, i]),
        # three dimensions (mpfc3d_oracle.c)
        "o3_laplacian": (v, [i, i, i, d, _dp, _dp]),
        "o3_source": (v, [i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp]),
        "o3_operator": (v, [i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "o3_residual": (v, [i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                            _dp]),
        "o3_norm3": (d, [i, i, i, d, _dp, _dp, _dp]),
        "o3_smooth": (v, [i, i, i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "o3_restrict": (v, [i, i, i, _dp, _dp]),
        "o3_prolong_add": (v, [i, i, i, _dp, _dp]),
        "o3_dense_newton": (i, [i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, i]),
        "o3_fas_solve": (i, [i, i, i, i, i, d, d, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, i, i, i,
                             i, d, i, _dp]),
        "o3_complete_guess": (v, [i, i, i, i, d, d, _dp, _dp, _dp, _dp, _dp, _dp]),
        "o3_grad_sq": (d, [i, i, i, d, _dp]),
        "o3_energy_F": (d, [i, i, i, d, d, _dp]),
        "o3_poisson_cg": (i, [i, i, i, d, _dp, _dp, d, i]),
        "o3_energies": (v, [i, i, i, d, d, d, _dp, _dp, _dp, _dp]),
        "o3_step": (i, [i, i, i, i, i, d, d, d, d, d, _dp, _dp, _dp, i, i, i, i, i, d, i,
                        _dp, _dp, _dp, _dp, _dp, _dp]),
        "orc_version": (i, []),
        "orc_num_threads": (i, []),
        "orc_set_threads": (None, [i]),
        "orc_set_omega": (None, [d]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def num_threads() -> int:
    return load().orc_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (timing only)."""
    load().orc_set_threads(int(n))


def _lib_bc(bc, omega=1.0):
    """The library with boundary conditions bc = (x, y) and the smoother's
    relaxation factor selected."""
    lib = load()
    lib.orc_set_bc(int(bc[0]), int(bc[1]))
    lib.orc_set_omega(float(omega))
    return lib


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _shape(a):
    n, m = a.shape
    return m, n


def _pin(p, pin, phihat=None, need_hat=False):
    """Pinning weight (and phi_hat) as arrays, checked (Sec. 4.6: scheme 2)."""
    if pin is None:
        return None, None
    if p.scheme != 2:
        raise ValueError("pinning is defined for the second-order scheme (Sec. 4.6)")
    w = _arr(pin)
    if need_hat and phihat is None:
        raise ValueError("pinning needs phi_hat")
    return w, (_arr(phihat) if phihat is not None else None)


# ---------------------------------------------------------------- operators
def coefficients(p: Params):
    """(c, d): c = sM/(beta+1/s), d = 1/(beta+1/s) (scheme 1) or with 2/s (scheme 2)."""
    c, d = ctypes.c_double(), ctypes.c_double()
    load().orc_coefficients(ctypes.byref(p._c()), ctypes.byref(c), ctypes.byref(d))
    return c.value, d.value


def laplacian(f, h, bc=(0, 0)):
    f = _arr(f)
    out = np.empty_like(f)
    m, n = _shape(f)
    _lib_bc(bc).orc_laplacian(m, n, h, _p(f), _p(out))
    return out


def source(p: Params, phik, phikm1=None, psik=None, pin=None, phihat=None):
    phik = _arr(phik)
    phikm1 = _arr(phikm1) if phikm1 is not None else phik
    psik = _arr(psik) if psik is not None else None
    w, ph = _pin(p, pin, phihat, need_hat=True)
    m, n = _shape(phik)
    S = [np.empty_like(phik) for _ in range(3)]
    _lib_bc(p.bc, p.omega).orc_source(ctypes.byref(p._c()), m, n, _p(phik), _p(phikm1), _p(psik),
                      *[_p(x) for x in S], _p(w), _p(ph))
    return S


def operator(p: Params, u, phik=None, h=None, pin=None):
    """N(u) on the grid of u (spacing h, default p.h)."""
    phi, mu, ka = (_arr(x) for x in u)
    m, n = _shape(phi)
    c, _ = coefficients(p)
    pk = _arr(phik) if (p.scheme == 2 and phik is not None) else None
    out = [np.empty_like(phi) for _ in range(3)]
    w, _ = _pin(p, pin)
    _lib_bc(p.bc, p.omega).orc_operator(p.scheme, m, n, p.h if h is None else h, c, p.alpha, _p(pk),
                        _p(phi), _p(mu), _p(ka), *[_p(x) for x in out], _p(w))
    return out


def residual(p: Params, u, f, phik=None, h=None, pin=None):
    phi, mu, ka = (_arr(x) for x in u)
    f1, f2, f3 = (_arr(x) for x in f)
    m, n = _shape(phi)
    c, _ = coefficients(p)
    pk = _arr(phik) if (p.scheme == 2 and phik is not None) else None
    out = [np.empty_like(phi) for _ in range(3)]
    w, _ = _pin(p, pin)
    _lib_bc(p.bc, p.omega).orc_residual(p.scheme, m, n, p.h if h is None else h, c, p.alpha, _p(pk),
                        _p(phi), _p(mu), _p(ka), _p(f1), _p(f2), _p(f3), *[_p(x) for x in out],
                        _p(w))
    return out


def norm3(r, h):
    r1, r2, r3 = (_arr(x) for x in r)
    m, n = _shape(r1)
    return load().orc_norm3(m, n, h, _p(r1), _p(r2), _p(r3))


def smooth(p: Params, u, f, phik=None, sweeps=1, newton=True, h=None, order="rb", pin=None):
    """Nonlinear Gauss-Seidel passes; returns the updated copy of u."""
    phi, mu, ka = (_arr(x).copy() for x in u)
    f1, f2, f3 = (_arr(x) for x in f)
    m, n = _shape(phi)
    c, _ = coefficients(p)
    pk = _arr(phik) if (p.scheme == 2 and phik is not None) else None
    lib = _lib_bc(p.bc, p.omega)
    fn = lib.orc_smooth if order == "rb" else lib.orc_smooth_lex
    w, _ = _pin(p, pin)
    fn(p.scheme, int(newton), sweeps, m, n, p.h if h is None else h, c, p.alpha, _p(pk),
       _p(phi), _p(mu), _p(ka), _p(f1), _p(f2), _p(f3), _p(w))
    return [phi, mu, ka]


def smooth_color(p: Params, u, f, color, phik=None, newton=True, h=None, pin=None):
    phi, mu, ka = (_arr(x).copy() for x in u)
    f1, f2, f3 = (_arr(x) for x in f)
    m, n = _shape(phi)
    c, _ = coefficients(p)
    pk = _arr(phik) if (p.scheme == 2 and phik is not None) else None
    _lib_bc(p.bc, p.omega).orc_smooth_color(p.scheme, int(newton), color, m, n, p.h if h is None else h, c,
                            p.alpha, _p(pk), _p(phi), _p(mu), _p(ka), _p(f1), _p(f2), _p(f3),
                            _p(_pin(p, pin)[0]))
    return [phi, mu, ka]


def restrict(fine):
    fine = _arr(fine)
    m, n = _shape(fine)
    out = np.empty((n // 2, m // 2))
    load().orc_restrict(m, n, _p(fine), _p(out))
    return out


def prolong_add(coarse, fine, bc=(0, 0)):
    """Return fine + bilinear interpolation of coarse."""
    coarse = _arr(coarse)
    fine = _arr(fine).copy()
    m, n = _shape(fine)
    _lib_bc(bc).orc_prolong_add(m, n, _p(coarse), _p(fine))
    return fine


def dense_newton(p: Params, u, f, phik=None, h=None, maxit=50, pin=None):
    phi, mu, ka = (_arr(x).copy() for x in u)
    f1, f2, f3 = (_arr(x) for x in f)
    m, n = _shape(phi)
    c, _ = coefficients(p)
    pk = _arr(phik) if (p.scheme == 2 and phik is not None) else None
    it = _lib_bc(p.bc, p.omega).orc_dense_newton(p.scheme, m, n, p.h if h is None else h, c, p.alpha, _p(pk),
                                 _p(phi), _p(mu), _p(ka), _p(f1), _p(f2), _p(f3), maxit,
                                 _p(_pin(p, pin)[0]))
    return [phi, mu, ka], it


def fas_solve(p: Params, u0, S, phik=None, nu1=2, nu2=2, coarsest=2, tol=1e-10,
              max_cycles=100, newton=True, pin=None, coarse_sweeps=0):
    """FAS V-cycles from the guess u0; returns (u, history, cycles).
    coarse_sweeps = K > 0 relaxes the coarsest grid by K red-black sweeps
    instead of solving it by dense Newton."""
    phi, mu, ka = (_arr(x).copy() for x in u0)
    S1, S2, S3 = (_arr(x) for x in S)
    m, n = _shape(phi)
    c, _ = coefficients(p)
    pk = _arr(phik) if p.scheme == 2 else None
    hist = np.zeros(max_cycles + 1)
    cyc = _lib_bc(p.bc, p.omega).orc_fas_solve(p.scheme, int(newton), m, n, p.h, c, p.alpha, _p(pk), _p(phi),
                               _p(mu), _p(ka), _p(S1), _p(S2), _p(S3), nu1, nu2, coarsest,
                               coarse_sweeps, tol, max_cycles, _p(hist), _p(_pin(p, pin)[0]))
    ncyc = cyc if cyc >= 0 else -cyc - 1
    return [phi, mu, ka], hist[: ncyc + 1], cyc


def complete_guess(p: Params, phi, S, phik=None, pin=None):
    phi = _arr(phi)
    m, n = _shape(phi)
    mu, ka = np.empty_like(phi), np.empty_like(phi)
    pk = _arr(phik) if p.scheme == 2 else None
    _lib_bc(p.bc, p.omega).orc_complete_guess(p.scheme, m, n, p.h, p.alpha, _p(pk), _p(phi), _p(mu), _p(ka),
                              _p(_arr(S[1])), _p(_arr(S[2])), _p(_pin(p, pin)[0]))
    return [phi.copy(), mu, ka]


def psi_update(p: Params, phinew, phik, psik):
    phinew, phik = _arr(phinew), _arr(phik)
    psik = _arr(psik) if psik is not None else None
    out = np.empty_like(phinew)
    _lib_bc(p.bc, p.omega).orc_psi_update(p.scheme, phinew.size, p.dt, _p(phinew), _p(phik), _p(psik), _p(out))
    return out


def energy_F(p: Params, phi):
    phi = _arr(phi)
    m, n = _shape(phi)
    return _lib_bc(p.bc, p.omega).orc_energy_F(m, n, p.h, p.eps, _p(phi))


def grad_sq(f, bc=(0, 0)):
    f = _arr(f)
    m, n = _shape(f)
    return _lib_bc(bc).orc_grad_sq(m, n, _p(f))


def poisson(b, h, rtol=1e-14, maxit=100000, bc=(0, 0)):
    b = _arr(b)
    m, n = _shape(b)
    w = np.empty_like(b)
    it = _lib_bc(bc).orc_poisson_cg(m, n, h, _p(b), _p(w), rtol, maxit)
    return w, it


def norm_m1_sq(psi, h, bc=(0, 0)):
    psi = _arr(psi)
    m, n = _shape(psi)
    return _lib_bc(bc).orc_norm_m1_sq(m, n, h, _p(psi))


def energies(p: Params, phinew, phik, psinew, pin=None, phihat=None):
    """(F, pseudo energy, modified energy, mass) after a step (with pinning,
    F includes h^2 sum W (phi - phi_hat)^2)."""
    phinew, phik, psinew = _arr(phinew), _arr(phik), _arr(psinew)
    m, n = _shape(phinew)
    out = np.zeros(4)
    w, ph = _pin(p, pin, phihat, need_hat=True)
    _lib_bc(p.bc, p.omega).orc_energies(m, n, p.h, p.eps, p.M, _p(phinew), _p(phik), _p(psinew), _p(out),
                               _p(w), _p(ph))
    return out


@dataclass
class StepResult:
    phi: np.ndarray
    mu: np.ndarray
    kappa: np.ndarray
    psi: np.ndarray
    history: np.ndarray
    cycles: int            # negative if the tolerance was not reached
    energies: np.ndarray   # F, pseudo energy, modified energy, mass


def step(p: Params, phik, phikm1=None, psik=None, guess=0, nu1=2, nu2=2, coarsest=2,
         tol=1e-10, max_cycles=100, newton=True, energy=True, pin=None,
         phihat=None, coarse_sweeps=0) -> StepResult:
    """One time step of the chosen scheme from (phi^k, phi^{k-1}, psi^k);
    pin / phihat: pinning weight W and prescribed configuration (Sec. 4.6)."""
    phik = _arr(phik)
    phikm1 = _arr(phikm1) if phikm1 is not None else phik
    psik = _arr(psik) if psik is not None else np.zeros_like(phik)
    m, n = _shape(phik)
    outs = [np.empty_like(phik) for _ in range(4)]
    hist = np.zeros(max_cycles + 1)
    en = np.zeros(4)
    cyc = _lib_bc(p.bc, p.omega).orc_step(ctypes.byref(p._c()), int(newton), m, n, _p(phik), _p(phikm1),
                          _p(psik), guess, nu1, nu2, coarsest, coarse_sweeps, tol, max_cycles,
                          *[_p(x) for x in outs], _p(hist), _p(en) if energy else None,
                          *[_p(x) for x in _pin(p, pin, phihat, need_hat=True)])
    ncyc = cyc if cyc >= 0 else -cyc - 1
    return StepResult(outs[0], outs[1], outs[2], outs[3], hist[: ncyc + 1], cyc, en)


def run(p: Params, phi0, steps, **kw):
    """Run `steps` time steps from phi^0 with psi^0 = 0, phi^{-1} = phi^0
    (Sec. 3.1, 3.2 initial conditions).  Returns (phi, phi_prev, psi, results)."""
    phi = _arr(phi0).copy()
    prev = phi.copy()
    psi = np.zeros_like(phi)
    results = []
    for _ in range(steps):
        r = step(p, phi, prev, psi, **kw)
        results.append(r)
        prev, phi, psi = phi, r.phi, r.psi
    return phi, prev, psi, results


# ---------------------------------------------------------------------------
# Three dimensions (mpfc3d_oracle.c): periodic m x n x l grids, arrays of shape
# (l, n, m) with x fastest.  Same parameters (bc must be periodic).

def _shape3(a):
    l, n, m = a.shape
    return m, n, l


def laplacian3(f, h):
    f = _arr(f)
    out = np.empty_like(f)
    load().o3_laplacian(*_shape3(f), h, _p(f), _p(out))
    return out


def source3(p: Params, phik, phikm1=None, psik=None):
    phik = _arr(phik)
    phikm1 = _arr(phikm1) if phikm1 is not None else phik
    psik = _arr(psik) if psik is not None else None
    _, d = coefficients(p)
    S = [np.empty_like(phik) for _ in range(3)]
    load().o3_source(p.scheme, *_shape3(phik), p.h, d, p.alpha, _p(phik), _p(phikm1), _p(psik),
                     *[_p(x) for x in S])
    return S


def operator3(p: Params, u, phik=None, h=None):
    phi, mu, ka = (_arr(x) for x in u)
    c, _ = coefficients(p)
    pk = _arr(phik) if p.scheme == 2 else None
    N = [np.empty_like(phi) for _ in range(3)]
    load().o3_operator(p.scheme, *_shape3(phi), p.h if h is None else h, c, p.alpha, _p(pk),
                       _p(phi), _p(mu), _p(ka), *[_p(x) for x in N])
    return N


def complete_guess3(p: Params, phi, S, phik=None):
    phi = _arr(phi)
    mu, ka = np.empty_like(phi), np.empty_like(phi)
    pk = _arr(phik) if p.scheme == 2 else None
    load().o3_complete_guess(p.scheme, *_shape3(phi), p.h, p.alpha, _p(pk), _p(phi), _p(mu),
                             _p(ka), _p(_arr(S[1])), _p(_arr(S[2])))
    return [phi.copy(), mu, ka]


def smooth3(p: Params, u, f, phik=None, sweeps=1, newton=True):
    phi, mu, ka = (_arr(x).copy() for x in u)
    c, _ = coefficients(p)
    pk = _arr(phik) if p.scheme == 2 else None
    load().o3_smooth(p.scheme, int(newton), sweeps, *_shape3(phi), p.h, c, p.alpha, _p(pk),
                     _p(phi), _p(mu), _p(ka), *[_p(_arr(x)) for x in f])
    return [phi, mu, ka]


def fas_solve3(p: Params, u0, S, phik=None, nu1=2, nu2=2, coarsest=2, tol=1e-10,
               max_cycles=100, newton=True, coarse_sweeps=0):
    phi, mu, ka = (_arr(x).copy() for x in u0)
    S1, S2, S3 = (_arr(x) for x in S)
    c, _ = coefficients(p)
    pk = _arr(phik) if p.scheme == 2 else None
    hist = np.zeros(max_cycles + 1)
    cyc = load().o3_fas_solve(p.scheme, int(newton), *_shape3(phi), p.h, c, p.alpha, _p(pk),
                              _p(phi), _p(mu), _p(ka), _p(S1), _p(S2), _p(S3), nu1, nu2,
                              coarsest, coarse_sweeps, tol, max_cycles, _p(hist))
    ncyc = cyc if cyc >= 0 else -cyc - 1
    return [phi, mu, ka], hist[: ncyc + 1], cyc


def energies3(p: Params, phinew, phik, psinew):
    phinew, phik, psinew = _arr(phinew), _arr(phik), _arr(psinew)
    out = np.zeros(4)
    load().o3_energies(*_shape3(phinew), p.h, p.eps, p.M, _p(phinew), _p(phik), _p(psinew),
                       _p(out))
    return out


def grad_sq3(f, h):
    f = _arr(f)
    return load().o3_grad_sq(*_shape3(f), h, _p(f))


def step3(p: Params, phik, phikm1=None, psik=None, guess=0, nu1=2, nu2=2, coarsest=2,
          coarse_sweeps=0, tol=1e-10, max_cycles=100, newton=True, energy=True) -> StepResult:
    """One time step in three dimensions (periodic)."""
    assert tuple(p.bc) == (0, 0), "the three-dimensional oracle is periodic"
    phik = _arr(phik)
    phikm1 = _arr(phikm1) if phikm1 is not None else phik
    psik = _arr(psik) if psik is not None else np.zeros_like(phik)
    outs = [np.empty_like(phik) for _ in range(4)]
    hist = np.zeros(max_cycles + 1)
    en = np.zeros(4)
    cyc = load().o3_step(p.scheme, int(newton), *_shape3(phik), p.h, p.dt, p.M, p.beta, p.eps,
                         _p(phik), _p(phikm1), _p(psik), guess, nu1, nu2, coarsest,
                         coarse_sweeps, tol, max_cycles, *[_p(x) for x in outs], _p(hist),
                         _p(en) if energy else None)
    ncyc = cyc if cyc >= 0 else -cyc - 1
    return StepResult(outs[0], outs[1], outs[2], outs[3], hist[: ncyc + 1], cyc, en)


def run3(p: Params, phi0, steps, **kw):
    phi = _arr(phi0).copy()
    prev = phi.copy()
    psi = np.zeros_like(phi)
    results = []
    for _ in range(steps):
        r = step3(p, phi, prev, psi, **kw)
        results.append(r)
        prev, phi, psi = phi, r.phi, r.psi
    return phi, prev, psi, results

