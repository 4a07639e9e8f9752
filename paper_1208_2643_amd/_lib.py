"""ctypes binding of libmpfc.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/mpfc.h under the
same name.  Device arrays are passed as raw pointers (for example
``tensor.data_ptr()`` of a PyTorch CUDA/ROCm tensor); the stream is a
hipStream_t handle as an integer (``torch.cuda.current_stream().cuda_stream``).

The library must have been built (``python -m paper_1208_2643_amd.build`` or
``__graft_entry__.build()``); importing fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmpfc.so")

MPFC_OK = 0
MPFC_EINVAL = -1
MPFC_ENOTCONVERGED = -2
MPFC_ENONFINITE = -3
MPFC_EDIVERGED = -4
MPFC_ENOMEM = -5
MPFC_EHIP = -6

MPFC_FP64, MPFC_MIXED = 0, 1
MPFC_GUESS_PREV, MPFC_GUESS_EXTRAP, MPFC_GUESS_CNN = 0, 1, 2
MPFC_NEWTON, MPFC_PICARD = 0, 1


class mpfc_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("beta", ctypes.c_double), ("M", ctypes.c_double),
                ("h", ctypes.c_double), ("dt", ctypes.c_double), ("scheme", ctypes.c_int),
                ("bc", ctypes.c_int)]


class mpfc_opts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int), ("guess", ctypes.c_int),
                ("linearization", ctypes.c_int), ("coarsest", ctypes.c_int),
                ("energy", ctypes.c_int), ("diverge", ctypes.c_double),
                ("inner_cycles", ctypes.c_int), ("coarse_sweeps", ctypes.c_int),
                ("omega", ctypes.c_double), ("coarse_threshold", ctypes.c_int),
                ("inner_cycles_next", ctypes.c_int), ("inner_nu_coarse", ctypes.c_int)]


class mpfc_info(ctypes.Structure):
    _fields_ = [("energy_F", ctypes.c_double), ("energy_pseudo", ctypes.c_double),
                ("energy_mod", ctypes.c_double), ("mass", ctypes.c_double),
                ("residual", ctypes.c_double), ("n_cycles", ctypes.c_int),
                ("status", ctypes.c_int), ("outer_iters", ctypes.c_int), ("energy_status", ctypes.c_int),
                ("residual_history", ctypes.POINTER(ctypes.c_double))]


class mpfc_sim_desc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("p", mpfc_params)]


MPFC_BATCH_MAX = 4096
MPFC_BC_PERIODIC, MPFC_BC_NEUMANN_X, MPFC_BC_NEUMANN_Y = 0, 1, 2


class mpfc_cnn_hparams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class MpfcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpfc error {code}: {msg}")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

# name -> (restype, argtypes); every symbol declared in include/mpfc.h
SIGNATURES = {
    "mpfc_default_opts": (None, [ctypes.POINTER(mpfc_opts)]),
    "mpfc_validate": (_i, [_i, _i, ctypes.POINTER(mpfc_params), ctypes.POINTER(mpfc_opts)]),
    "mpfc_create": (_i, [ctypes.POINTER(_vp), _i, _i, ctypes.POINTER(mpfc_params),
                         ctypes.POINTER(mpfc_opts), _vp]),
    "mpfc_step": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(mpfc_info)]),
    "mpfc_energies": (_i, [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "mpfc_prof_enable": (_i, [_vp, _i]),
    "mpfc_prof_read": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong),
                            ctypes.POINTER(ctypes.c_longlong), _i]),
    "mpfc_destroy": (None, [_vp]),
    "mpfc_tile_shape": (_i, [_vp, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "mpfc_set_pinning": (_i, [_vp, _vp, _vp]),
    "mpfc_strerror": (ctypes.c_char_p, [_i]),
    "mpfc_last_error": (ctypes.c_char_p, []),
    "mpfc_version": (_i, []),
    "mpfc_op_smooth": (_i, [ctypes.POINTER(mpfc_params), _i, _i, _i, _vp, _vp, _vp, _vp, _vp,
                            _vp, _vp, _i, _vp]),
    "mpfc_op_smooth_noalloc": (_i, [ctypes.POINTER(mpfc_params), _i, _i, _i, _vp, _vp, _vp, _vp,
                                    _vp, _vp, _vp, _i, _vp]),
    "mpfc_op_residual": (_i, [ctypes.POINTER(mpfc_params), _i, _i, _vp, _vp, _vp, _vp, _vp, _vp,
                              _vp, _vp, _vp, _vp, _vp]),
    "mpfc_op_source": (_i, [ctypes.POINTER(mpfc_params), _i, _i, _vp, _vp, _vp, _vp, _vp, _vp,
                            _vp]),
    "mpfc_op_restrict": (_i, [_i, _i, _vp, _vp, _vp]),
    "mpfc_batch_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(mpfc_sim_desc),
                               ctypes.POINTER(mpfc_opts), _vp]),
    "mpfc_batch_step": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                             ctypes.POINTER(_vp), ctypes.POINTER(mpfc_info)]),
    "mpfc_batch_size": (_i, [_vp]),
    "mpfc_batch_destroy": (None, [_vp]),
    "mpfc_cnn_blob_size": (_i, []),
    "mpfc_cnn_load": (_i, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
    "mpfc_cnn_counts": (_i, [_vp, ctypes.POINTER(ctypes.c_longlong),
                             ctypes.POINTER(ctypes.c_longlong)]),
    "mpfc_cnn_trainer_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, ctypes.POINTER(ctypes.c_float),
                                     ctypes.c_size_t, ctypes.POINTER(mpfc_cnn_hparams), _vp]),
    "mpfc_cnn_train_step": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_vp), _i, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_float)]),
    "mpfc_cnn_predict": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                              ctypes.POINTER(_vp)]),
    "mpfc_cnn_trainer_blob": (_i, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
    "mpfc_cnn_trainer_destroy": (None, [_vp]),
    "mpfc_cnn_trainer_set_lr": (_i, [_vp, ctypes.c_float]),
    "mpfc3d_validate": (_i, [_i, _i, _i, ctypes.POINTER(mpfc_params), ctypes.POINTER(mpfc_opts)]),
    "mpfc3d_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, ctypes.POINTER(mpfc_params),
                           ctypes.POINTER(mpfc_opts), _vp]),
    "mpfc3d_step": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(mpfc_info)]),
    "mpfc3d_prof_enable": (_i, [_vp, _i]),
    "mpfc3d_prof_read": (_i, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong),
                              ctypes.POINTER(ctypes.c_longlong), _i]),
    "mpfc3d_destroy": (None, [_vp]),
}


def load():
    """Load libmpfc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is missing: build it with `python -m paper_1208_2643_amd.build`")
    lib = ctypes.CDLL(LIBPATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int, allow=()):
    if rc != MPFC_OK and rc not in allow:
        lib = load()
        raise MpfcError(rc, f"{lib.mpfc_strerror(rc).decode()}: {lib.mpfc_last_error().decode()}")
    return rc


def default_opts() -> mpfc_opts:
    o = mpfc_opts()
    load().mpfc_default_opts(ctypes.byref(o))
    return o
