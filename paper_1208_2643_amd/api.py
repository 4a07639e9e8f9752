"""Python front end of libmpfc: PyTorch supplies device memory and the stream.

``Stepper`` wraps one solver context (one grid size and parameter set) and
advances the state (phi^k, phi^{k-1}, psi^k) of either convex-splitting scheme
by one implicit step per call; all arithmetic runs in the library's HIP
kernels.  There is no CPU fallback: without a GPU or without the built
library these calls raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


@dataclass
class Params:
    """Model/discretisation parameters (Sec. 2-3): alpha = 1 - eps.  bc:
    boundary conditions, MPFC_BC_NEUMANN_X | MPFC_BC_NEUMANN_Y bits (App. A;
    0 = periodic in both directions)."""
    eps: float
    beta: float
    M: float
    h: float
    dt: float
    scheme: int
    bc: int = 0

    def c(self) -> L.mpfc_params:
        return L.mpfc_params(self.eps, self.beta, self.M, self.h, self.dt, self.scheme, self.bc)


@dataclass
class StepInfo:
    status: int
    n_cycles: int
    residual: float
    history: np.ndarray
    energy_F: float
    energy_pseudo: float
    energy_mod: float
    mass: float
    outer_iters: int
    energy_status: int = 0   # MPFC_ENOTCONVERGED if the -1 norm's Poisson solve did not converge


def make_opts(**kw) -> L.mpfc_opts:
    """Solver options (mpfc_opts, include/mpfc.h) from the library's defaults
    with the given fields replaced: nu1, nu2, max_cycles, tol, precision,
    guess, linearization, coarsest, energy, diverge, inner_cycles,
    coarse_sweeps, omega (smoother relaxation, 1 = App. B), coarse_threshold,
    inner_cycles_next (FP32 cycles of each outer iteration after the first;
    0 = inner_cycles), inner_nu_coarse (smoothing passes of those FP32
    cycles on the levels below the finest; 0 = nu1, nu2)."""
    o = L.default_opts()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Stepper:
    """One solver context for an n x m grid (tensors of shape (n, m), x fastest)."""

    def __init__(self, m: int, n: int, params: Params, stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpfc needs a HIP GPU; none is visible")
        self.lib = L.load()
        self.m, self.n = m, n
        self.params = params
        self.opts = make_opts(**opts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = ctypes.c_void_p()
        L.check(self.lib.mpfc_create(ctypes.byref(ctx), m, n, ctypes.byref(params.c()),
                                     ctypes.byref(self.opts), _stream(self.stream)))
        self.ctx = ctx
        self._hist = np.zeros(self.opts.max_cycles + 1)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mpfc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, phi_n, phi_nm1, psi, phi_np1=None, mu=None, kappa=None, allow_fail=False):
        """Advance one step.  psi is updated in place to psi^{k+1}; returns
        (phi_np1, StepInfo)."""
        if phi_np1 is None:
            phi_np1 = torch.empty_like(phi_n)
        info = L.mpfc_info()
        info.residual_history = self._hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rc = self.lib.mpfc_step(self.ctx, _ptr(phi_n), _ptr(phi_nm1), _ptr(psi), _ptr(phi_np1),
                                _ptr(mu), _ptr(kappa), ctypes.byref(info))
        allow = (L.MPFC_ENOTCONVERGED, L.MPFC_ENONFINITE, L.MPFC_EDIVERGED) if allow_fail else ()
        L.check(rc, allow)
        nh = (info.outer_iters if self.opts.precision == L.MPFC_MIXED else info.n_cycles) + 1
        si = StepInfo(rc, info.n_cycles, info.residual, self._hist[:nh].copy(),
                      info.energy_F, info.energy_pseudo, info.energy_mod, info.mass,
                      info.outer_iters, info.energy_status)
        return phi_np1, si

    def profile(self, on: bool = True):
        """Time the two finest-level launches of every V-cycle with HIP events."""
        L.check(self.lib.mpfc_prof_enable(self.ctx, 1 if on else 0))

    def profile_read(self, which: int, reset: bool = True):
        """(total ms, launches, finest cells) of the timed down (0) or up (1) launches."""
        ms, n, cells = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_longlong()
        L.check(self.lib.mpfc_prof_read(self.ctx, which, ctypes.byref(ms), ctypes.byref(n),
                                        ctypes.byref(cells), 1 if reset else 0))
        return ms.value, n.value, cells.value

    def load_cnn(self, blob):
        """Load a learned-guess network (float32 blob); used when guess=MPFC_GUESS_CNN."""
        b = np.ascontiguousarray(blob, dtype=np.float32)
        L.check(self.lib.mpfc_cnn_load(self.ctx, b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       b.size))

    def cnn_counts(self):
        """(steps started from the learned guess, fallbacks to extrapolation)."""
        u, f = ctypes.c_longlong(), ctypes.c_longlong()
        L.check(self.lib.mpfc_cnn_counts(self.ctx, ctypes.byref(u), ctypes.byref(f)))
        return u.value, f.value

    def set_pinning(self, weight=None, phihat=None):
        """Pinning term of Sec. 4.6 (scheme 2, FP64, Newton): weight W >= 0 and
        prescribed configuration phi_hat, (n, m) float64 device tensors copied
        by the call; weight None switches it off."""
        if weight is None:
            L.check(self.lib.mpfc_set_pinning(self.ctx, None, None))
            return
        for t in (weight, phihat):
            if t is None or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("weight and phihat must be contiguous float64 CUDA tensors")
            if tuple(t.shape) != (self.n, self.m):
                raise ValueError("weight and phihat must have the grid's shape (n, m)")
        L.check(self.lib.mpfc_set_pinning(self.ctx, _ptr(weight), _ptr(phihat)))

    def tile_shape(self, level: int = 0, which: int = 0):
        """(tx, ty, halo) of the tiled launch `which` (0 down, 1 up) on `level`."""
        tx, ty, h = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        L.check(self.lib.mpfc_tile_shape(self.ctx, level, which, ctypes.byref(tx), ctypes.byref(ty),
                                         ctypes.byref(h)))
        return tx.value, ty.value, h.value

    def energies(self, phi, phi_prev, psi):
        out = (ctypes.c_double * 4)()
        L.check(self.lib.mpfc_energies(self.ctx, _ptr(phi), _ptr(phi_prev), _ptr(psi), out))
        return np.array(out[:])


class Stepper3:
    """Solver context for a periodic m x n x l grid in three dimensions
    (tensors of shape (l, n, m), x fastest); same options and step
    semantics as Stepper."""

    def __init__(self, m: int, n: int, l: int, params: Params, stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpfc needs a HIP GPU; none is visible")
        self.lib = L.load()
        self.m, self.n, self.l = m, n, l
        self.params = params
        self.opts = make_opts(**opts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = ctypes.c_void_p()
        L.check(self.lib.mpfc3d_create(ctypes.byref(ctx), m, n, l, ctypes.byref(params.c()),
                                       ctypes.byref(self.opts), _stream(self.stream)))
        self.ctx = ctx
        self._hist = np.zeros(self.opts.max_cycles + 1)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mpfc3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, phi_n, phi_nm1, psi, phi_np1=None, mu=None, kappa=None, allow_fail=False):
        if phi_np1 is None:
            phi_np1 = torch.empty_like(phi_n)
        info = L.mpfc_info()
        info.residual_history = self._hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rc = self.lib.mpfc3d_step(self.ctx, _ptr(phi_n), _ptr(phi_nm1), _ptr(psi), _ptr(phi_np1),
                                  _ptr(mu), _ptr(kappa), ctypes.byref(info))
        allow = (L.MPFC_ENOTCONVERGED, L.MPFC_ENONFINITE, L.MPFC_EDIVERGED) if allow_fail else ()
        L.check(rc, allow)
        si = StepInfo(rc, info.n_cycles, info.residual, self._hist[:info.n_cycles + 1].copy(),
                      info.energy_F, info.energy_pseudo, info.energy_mod, info.mass, 0,
                      info.energy_status)
        return phi_np1, si

    def profile(self, on: bool = True):
        """Time the finest level's red-black half-sweep launches with HIP events."""
        L.check(self.lib.mpfc3d_prof_enable(self.ctx, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        ms, n, cells = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_longlong()
        L.check(self.lib.mpfc3d_prof_read(self.ctx, ctypes.byref(ms), ctypes.byref(n),
                                          ctypes.byref(cells), 1 if reset else 0))
        return ms.value, n.value, cells.value


class Batch:
    """Many independent simulations advanced together (mpfc_batch_*).

    `sims` is a list of (m, n, Params) with one scheme; every option applies
    to all of them.  Fields are lists of (n, m) float64 GPU tensors, one per
    simulation."""

    def __init__(self, sims, stream=None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpfc needs a HIP GPU; none is visible")
        self.lib = L.load()
        self.sims = [(int(m), int(n), p) for m, n, p in sims]
        self.nsim = len(self.sims)
        self.opts = make_opts(**opts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        desc = (L.mpfc_sim_desc * self.nsim)()
        for k, (m, n, p) in enumerate(self.sims):
            desc[k].m, desc[k].n, desc[k].p = m, n, p.c()
        b = ctypes.c_void_p()
        L.check(self.lib.mpfc_batch_create(ctypes.byref(b), self.nsim, desc,
                                           ctypes.byref(self.opts), _stream(self.stream)))
        self.b = b
        self._hist = np.zeros((self.nsim, self.opts.max_cycles + 1))

    def close(self):
        if getattr(self, "b", None):
            self.lib.mpfc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _arr(self, ts, allow_none=False):
        if ts is None:
            if allow_none:
                return None
            raise ValueError("a list of tensors is required")
        if len(ts) != self.nsim:
            raise ValueError(f"expected {self.nsim} tensors, got {len(ts)}")
        a = (ctypes.c_void_p * self.nsim)()
        for k, t in enumerate(ts):
            m, n, _ = self.sims[k]
            if t is not None and tuple(t.shape) != (n, m):
                raise ValueError(f"simulation {k}: expected shape {(n, m)}, got {tuple(t.shape)}")
            a[k] = _ptr(t).value if t is not None else None
        return a

    def step(self, phi_n, phi_nm1, psi, phi_np1, allow_fail=False, history=True):
        """Advance every simulation one step (psi in place); returns a list of StepInfo."""
        infos = (L.mpfc_info * self.nsim)()
        if history:
            for k in range(self.nsim):
                infos[k].residual_history = self._hist[k].ctypes.data_as(
                    ctypes.POINTER(ctypes.c_double))
        rc = self.lib.mpfc_batch_step(self.b, self._arr(phi_n), self._arr(phi_nm1, True),
                                      self._arr(psi), self._arr(phi_np1), infos)
        allow = (L.MPFC_ENOTCONVERGED, L.MPFC_ENONFINITE, L.MPFC_EDIVERGED) if allow_fail else ()
        L.check(rc, allow)
        out = []
        for k in range(self.nsim):
            I = infos[k]
            hist = self._hist[k][: I.outer_iters + 1 if self.opts.precision == L.MPFC_MIXED
                                 else I.n_cycles + 1].copy() if history else np.zeros(0)
            out.append(StepInfo(I.status, I.n_cycles, I.residual, hist, 0.0, 0.0, 0.0, 0.0,
                                I.outer_iters))
        return out


def _ptrs(ts):
    a = (ctypes.c_void_p * len(ts))()
    for k, t in enumerate(ts):
        a[k] = _ptr(t).value
    return a


class CnnTrainer:
    """GPU trainer of the learned-guess network (mpfc_cnn_*): batches of
    `batch` samples (phi^{n-1}, phi^n, psi^n, phi^{n+1}) of an (n, m) grid."""

    def __init__(self, m: int, n: int, batch: int, blob, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpfc needs a HIP GPU; none is visible")
        self.lib = L.load()
        self.m, self.n, self.batch = m, n, batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        b = np.ascontiguousarray(blob, dtype=np.float32)
        hp = L.mpfc_cnn_hparams(lr, beta1, beta2, eps)
        t = ctypes.c_void_p()
        L.check(self.lib.mpfc_cnn_trainer_create(
            ctypes.byref(t), m, n, batch, b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), b.size,
            ctypes.byref(hp), _stream(self.stream)))
        self.t = t
        self.nparams = self.lib.mpfc_cnn_blob_size() - 8

    def close(self):
        if getattr(self, "t", None):
            self.lib.mpfc_cnn_trainer_destroy(self.t)
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, pm1, p0, psi, pp1, update=True, grad=False):
        """Loss before the step (and the gradient, float32, blob order)."""
        loss = ctypes.c_double()
        g = np.zeros(self.nparams, dtype=np.float32) if grad else None
        L.check(self.lib.mpfc_cnn_train_step(
            self.t, _ptrs(pm1), _ptrs(p0), _ptrs(psi), _ptrs(pp1), 1 if update else 0,
            ctypes.byref(loss),
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if grad else None))
        return (loss.value, g) if grad else loss.value

    def set_lr(self, lr: float):
        L.check(self.lib.mpfc_cnn_trainer_set_lr(self.t, lr))

    def predict(self, pm1, p0, psi):
        out = [torch.empty_like(t) for t in p0]
        L.check(self.lib.mpfc_cnn_predict(self.t, _ptrs(pm1), _ptrs(p0), _ptrs(psi), _ptrs(out)))
        return out

    def blob(self):
        b = np.zeros(self.nparams + 8, dtype=np.float32)
        L.check(self.lib.mpfc_cnn_trainer_blob(self.t, b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                               b.size))
        return b


def run_batch(batch: Batch, phi0s, steps: int):
    """Run `steps` steps of every simulation from phi^0 (psi^0 = 0, phi^{-1} = phi^0)."""
    phi = [t.clone() for t in phi0s]
    prev = [t.clone() for t in phi0s]
    psi = [torch.zeros_like(t) for t in phi0s]
    nxt = [torch.empty_like(t) for t in phi0s]
    infos = []
    for _ in range(steps):
        infos.append(batch.step(phi, prev, psi, nxt))
        prev, phi, nxt = phi, nxt, prev
    return phi, prev, psi, infos


def run(stepper: Stepper, phi0: torch.Tensor, steps: int, record=None):
    """Run `steps` steps from phi^0 with psi^0 = 0 and phi^{-1} = phi^0."""
    phi = phi0.clone()
    prev = phi0.clone()
    psi = torch.zeros_like(phi0)
    nxt = torch.empty_like(phi0)
    infos = []
    for _ in range(steps):
        _, info = stepper.step(phi, prev, psi, nxt)
        infos.append(info)
        if record is not None:
            record(phi, nxt, psi, info)
        prev, phi, nxt = phi, nxt, prev
    return phi, prev, psi, infos


# ---- checkpoint / resume ------------------------------------------------------
# The whole state of a run is (phi^k, phi^{k-1}, psi^k) and the step count: for
# the second-order scheme psi^k carries the run's history (eq. discrete_2_b),
# so it is saved with the two phi's.  A context holds nothing a resumed run
# needs (its Poisson warm start and cycle prediction only save work).
def save_state(path, phi, phi_prev, psi, step: int, params: Params) -> None:
    """Write a run's state to `path` (numpy .npz, FP64, no pickled objects)."""
    np.savez(path, phi=phi.detach().cpu().numpy(), phi_prev=phi_prev.detach().cpu().numpy(),
             psi=psi.detach().cpu().numpy(), step=np.int64(step),
             params=np.array([params.eps, params.beta, params.M, params.h, params.dt,
                              params.scheme, params.bc], dtype=np.float64))


def load_state(path, device="cuda:0"):
    """(phi, phi_prev, psi, step, params) from a file written by save_state."""
    with np.load(path, allow_pickle=False) as z:
        pr = z["params"]
        params = Params(float(pr[0]), float(pr[1]), float(pr[2]), float(pr[3]), float(pr[4]),
                        int(pr[5]), int(pr[6]))
        dev = torch.device(device)
        return (torch.from_numpy(z["phi"]).to(dev), torch.from_numpy(z["phi_prev"]).to(dev),
                torch.from_numpy(z["psi"]).to(dev), int(z["step"]), params)


# ---- operator-level wrappers (one V-cycle operation each) -------------------
def _at_spacing(p: Params, h):
    """The parameters with the grid spacing of the level the operator acts on."""
    return p if h is None else Params(p.eps, p.beta, p.M, h, p.dt, p.scheme, p.bc)


def op_smooth(p: Params, u, f, phik=None, sweeps=1, newton=True, h=None):
    lib = L.load()
    phi, mu, ka = u
    n, m = phi.shape
    L.check(lib.mpfc_op_smooth(ctypes.byref(_at_spacing(p, h).c()),
                               L.MPFC_NEWTON if newton else L.MPFC_PICARD, m, n, _ptr(phik),
                               _ptr(phi), _ptr(mu), _ptr(ka), _ptr(f[0]), _ptr(f[1]), _ptr(f[2]),
                               sweeps, _stream()))


def op_residual(p: Params, u, f, phik=None, h=None):
    lib = L.load()
    phi, mu, ka = u
    n, m = phi.shape
    r = [torch.empty_like(phi) for _ in range(3)]
    L.check(lib.mpfc_op_residual(ctypes.byref(_at_spacing(p, h).c()), m, n, _ptr(phik),
                                 _ptr(phi), _ptr(mu), _ptr(ka), _ptr(f[0]), _ptr(f[1]),
                                 _ptr(f[2]), _ptr(r[0]), _ptr(r[1]), _ptr(r[2]), _stream()))
    return r


def op_source(p: Params, phik, phikm1, psik):
    lib = L.load()
    n, m = phik.shape
    S = [torch.empty_like(phik) for _ in range(3)]
    L.check(lib.mpfc_op_source(ctypes.byref(p.c()), m, n, _ptr(phik), _ptr(phikm1), _ptr(psik),
                               _ptr(S[0]), _ptr(S[1]), _ptr(S[2]), _stream()))
    return S


def op_restrict(fine):
    lib = L.load()
    n, m = fine.shape
    out = torch.empty((n // 2, m // 2), dtype=fine.dtype, device=fine.device)
    L.check(lib.mpfc_op_restrict(m, n, _ptr(fine), _ptr(out), _stream()))
    return out
