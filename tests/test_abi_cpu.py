"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol declared in include/mpfc.h, and rejects invalid configurations
on the host before any HIP call."""
import ctypes
import math
import os
import re

import pytest

from paper_1208_2643_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mpfc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpfc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_symbols()
    assert "mpfc_step" in names and "mpfc_create" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"binding lacks {name}"


def test_version_and_strerror():
    lib = L.load()
    assert lib.mpfc_version() == 1
    for code in range(-6, 1):
        assert lib.mpfc_strerror(code)
    assert lib.mpfc_strerror(-99) == b"unknown error"


def good():
    p = L.mpfc_params(0.025, 0.9, 1.0, math.pi / 4, 0.05, 2)
    o = L.default_opts()
    return p, o


def test_defaults():
    o = L.default_opts()
    assert (o.inner_cycles, o.inner_cycles_next, o.inner_nu_coarse) == (3, 0, 0)
    assert (o.nu1, o.nu2, o.max_cycles, o.tol, o.coarsest, o.coarse_sweeps) == \
        (2, 2, 100, 1e-10, 2, 2)
    p, o = good()
    assert L.load().mpfc_validate(1024, 1024, ctypes.byref(p), ctypes.byref(o)) == 0


@pytest.mark.parametrize("field,value", [("dt", 0.0), ("dt", -1.0), ("h", 0.0), ("M", 0.0),
                                         ("beta", -0.1), ("scheme", 3), ("eps", 1.5),
                                         ("h", float("nan"))])
def test_invalid_params_rejected(field, value):
    p, o = good()
    setattr(p, field, value)
    assert L.load().mpfc_validate(64, 64, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("m,n", [(0, 64), (48, 66), (64, 102), (1, 1), (2, 128), (64, 256),
                                 (6, 8), (404, 404)])
def test_invalid_sizes_rejected(m, n):
    """Sides must be powers of two (aspect ratio at most 2) or multiples of 4
    whose coarsest level (coarsened while both sides stay even) has at most
    4096 cells (404 x 404 stops at 202 x 202)."""
    p, o = good()
    assert L.load().mpfc_validate(m, n, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("m,n", [(512, 400), (48, 64), (64, 100), (96, 96), (12, 4), (4000, 8)])
def test_general_sizes_accepted(m, n):
    p, o = good()
    assert L.load().mpfc_validate(m, n, ctypes.byref(p), ctypes.byref(o)) == 0


@pytest.mark.parametrize("field,value", [("precision", 1), ("guess", 2), ("nu1", 3), ("nu2", 3)])
def test_general_sizes_reject_unsupported_options(field, value):
    """Grids with a side that is not a power of two run the FP64 general-index
    kernels only: no mixed precision, no learned guess, halos up to nu = 2."""
    p, o = good()
    setattr(o, field, value)
    assert L.load().mpfc_validate(512, 400, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL
    assert L.load().mpfc_validate(512, 512, ctypes.byref(p), ctypes.byref(o)) == 0


@pytest.mark.parametrize("value", [0, 65])
def test_coarse_sweeps_range(value):
    p, o = good()
    o.coarse_sweeps = value
    assert L.load().mpfc_validate(512, 400, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("field,value", [("tol", 0.0), ("max_cycles", 0), ("nu1", -1),
                                         ("coarsest", 3), ("precision", 7), ("guess", 9),
                                         ("linearization", 5), ("diverge", 0.5),
                                         ("omega", 0.0), ("omega", 2.0), ("omega", float("nan")),
                                         ("inner_cycles", 0), ("inner_cycles", 17),
                                         ("inner_cycles_next", -1), ("inner_cycles_next", 17),
                                         ("inner_nu_coarse", -1), ("inner_nu_coarse", 3)])
def test_invalid_opts_rejected(field, value):
    p, o = good()
    setattr(o, field, value)
    assert L.load().mpfc_validate(64, 64, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


def test_create_rejects_before_any_hip_call():
    """mpfc_create validates on the host, so it fails cleanly without a GPU."""
    lib = L.load()
    p, o = good()
    p.dt = -1.0
    ctx = ctypes.c_void_p()
    assert lib.mpfc_create(ctypes.byref(ctx), 64, 64, ctypes.byref(p), ctypes.byref(o), None) \
        == L.MPFC_EINVAL
    assert ctx.value is None
    assert b"dt" in lib.mpfc_last_error()


def test_rectangular_and_small_grids_accepted():
    lib = L.load()
    p, o = good()
    for m, n in [(2, 2), (4, 8), (64, 128), (2048, 2048), (128, 64)]:
        assert lib.mpfc_validate(m, n, ctypes.byref(p), ctypes.byref(o)) == 0, (m, n)


def _descs(shapes, schemes=None):
    d = (L.mpfc_sim_desc * len(shapes))()
    for k, (m, n) in enumerate(shapes):
        d[k].m, d[k].n = m, n
        d[k].p = L.mpfc_params(0.025, 0.9, 1.0, math.pi / 4, 0.05,
                               schemes[k] if schemes else 2)
    return d


@pytest.mark.parametrize("shapes,schemes,nsim", [
    ([(64, 64), (128, 128)], [1, 2], 2),      # mixed schemes
    ([(64, 64), (32, 32)], None, 2),          # a grid of 1024 cells
    ([(64, 64), (48, 64)], None, 2),          # not a power of two
    ([(64, 64)], None, 0),                    # empty batch
    ([(64, 64)], None, L.MPFC_BATCH_MAX + 1),  # too many
])
def test_batch_create_rejects_before_any_hip_call(shapes, schemes, nsim):
    lib = L.load()
    o = L.default_opts()
    d = _descs(shapes, schemes)
    b = ctypes.c_void_p()
    assert lib.mpfc_batch_create(ctypes.byref(b), nsim, d, ctypes.byref(o), None) == L.MPFC_EINVAL
    assert not b.value
    assert lib.mpfc_last_error()


def test_batch_null_handles():
    lib = L.load()
    assert lib.mpfc_batch_size(None) == 0
    lib.mpfc_batch_destroy(None)
    assert lib.mpfc_batch_step(None, None, None, None, None, None) == L.MPFC_EINVAL


@pytest.mark.parametrize("bc", [-1, 4, 7])
def test_invalid_boundary_bits_rejected(bc):
    p, o = good()
    p.bc = bc
    assert L.load().mpfc_validate(64, 64, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("bc", [L.MPFC_BC_NEUMANN_X, L.MPFC_BC_NEUMANN_Y,
                                L.MPFC_BC_NEUMANN_X | L.MPFC_BC_NEUMANN_Y])
def test_neumann_boundaries_validate(bc):
    """Neumann and mixed boundary conditions (App. A) are accepted, except with
    the learned guess, whose convolutions are periodic."""
    p, o = good()
    p.bc = bc
    assert L.load().mpfc_validate(1024, 1024, ctypes.byref(p), ctypes.byref(o)) == 0
    o.guess = L.MPFC_GUESS_CNN
    assert L.load().mpfc_validate(1024, 1024, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("m,n,l", [(128, 128, 128), (2, 2, 2), (64, 32, 16), (8, 8, 64)])
def test_3d_sizes_accepted(m, n, l):
    p, o = good()
    assert L.load().mpfc3d_validate(m, n, l, ctypes.byref(p), ctypes.byref(o)) == 0


@pytest.mark.parametrize("m,n,l", [(96, 64, 64), (64, 64, 1), (0, 8, 8), (1024, 1024, 512)])
def test_3d_bad_sizes_rejected(m, n, l):
    p, o = good()
    assert L.load().mpfc3d_validate(m, n, l, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("kw", [dict(bc=1), dict(precision=1), dict(guess=2), dict(dt=-1.0),
                                dict(coarse_sweeps=0)])
def test_3d_unsupported_configurations_rejected(kw):
    """The three-dimensional step is periodic, FP64, without the learned guess;
    parameters and options are checked as for the two-dimensional step."""
    p, o = good()
    for k, v in kw.items():
        setattr(p if k in ("bc", "dt") else o, k, v)
    assert L.load().mpfc3d_validate(16, 16, 16, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL
    ctx = ctypes.c_void_p()
    assert L.load().mpfc3d_create(ctypes.byref(ctx), 16, 16, 16, ctypes.byref(p), ctypes.byref(o),
                                  None) == L.MPFC_EINVAL
    assert ctx.value is None



def test_operator_entry_points_validate_params_on_the_host():
    """The operator-level calls form the scheme's coefficients from mpfc_params
    in the library and reject invalid parameters before any HIP call."""
    lib = L.load()
    p, _ = good()
    z = ctypes.c_void_p(0)
    for field, value in (("dt", -1.0), ("h", 0.0), ("scheme", 5), ("bc", 9)):
        q = L.mpfc_params(p.eps, p.beta, p.M, p.h, p.dt, p.scheme, p.bc)
        setattr(q, field, value)
        assert lib.mpfc_op_smooth(ctypes.byref(q), 0, 64, 64, z, z, z, z, z, z, z, 1, None) \
            == L.MPFC_EINVAL, field
        assert lib.mpfc_op_residual(ctypes.byref(q), 64, 64, z, z, z, z, z, z, z, z, z, z,
                                    None) == L.MPFC_EINVAL, field
        assert lib.mpfc_op_source(ctypes.byref(q), 64, 64, z, z, z, z, z, z, None) \
            == L.MPFC_EINVAL, field
    assert lib.mpfc_op_smooth(None, 0, 64, 64, z, z, z, z, z, z, z, 1, None) == L.MPFC_EINVAL
    # valid parameters, missing arrays: still rejected on the host
    assert lib.mpfc_op_smooth(ctypes.byref(p), 0, 64, 64, z, z, z, z, z, z, z, 1, None) \
        == L.MPFC_EINVAL
    assert lib.mpfc_op_smooth(ctypes.byref(p), 7, 64, 64, z, z, z, z, z, z, z, 1, None) \
        == L.MPFC_EINVAL


def test_relaxation_factor_default_and_range():
    """omega defaults to App. B's update (1); under-relaxation validates in 2-D,
    the 3-D step takes omega = 1 only."""
    p, o = good()
    assert o.omega == 1.0
    o.omega = 0.8
    assert L.load().mpfc_validate(64, 64, ctypes.byref(p), ctypes.byref(o)) == 0
    assert L.load().mpfc_validate(512, 400, ctypes.byref(p), ctypes.byref(o)) == 0
    assert L.load().mpfc3d_validate(64, 64, 64, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL


@pytest.mark.parametrize("thr,ok", [(0, True), (256, True), (512, True), (1024, True),
                                    (128, False), (300, False), (2048, False), (-256, False)])
def test_coarse_threshold_values(thr, ok):
    p, o = good()
    assert o.coarse_threshold == 0
    o.coarse_threshold = thr
    rc = L.load().mpfc_validate(256, 256, ctypes.byref(p), ctypes.byref(o))
    assert rc == (0 if ok else L.MPFC_EINVAL)


def test_coarse_threshold_only_for_power_of_two_2d_single_grids():
    lib = L.load()
    p, o = good()
    o.coarse_threshold = 256
    assert lib.mpfc_validate(512, 400, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL
    assert lib.mpfc3d_validate(64, 64, 64, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL
    d = (L.mpfc_sim_desc * 1)()
    d[0].m, d[0].n, d[0].p = 64, 64, p
    b = ctypes.c_void_p()
    assert lib.mpfc_batch_create(ctypes.byref(b), 1, d, ctypes.byref(o), None) == L.MPFC_EINVAL
    assert not b.value


def test_inner_nu_coarse_bounded_by_the_finest_passes():
    """The FP32 inner cycles may smooth less below the finest level, never
    more (the tiles' halo is sized for nu1, nu2)."""
    p, o = good()
    lib = L.load()
    o.inner_nu_coarse = 1
    assert lib.mpfc_validate(64, 64, ctypes.byref(p), ctypes.byref(o)) == 0
    o.nu2 = 0
    assert lib.mpfc_validate(64, 64, ctypes.byref(p), ctypes.byref(o)) == L.MPFC_EINVAL
