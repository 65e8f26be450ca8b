"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/lbm.h declares, and rejects bad parameters before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lbm_create", "lbm_step", "lbm_macroscopic", "lbm_adjoint_step", "lbm_diagnostics",
              "lbm_init_equilibrium", "lbm_destroy", "lbm_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1202_6351_amd import _lib
    lib = _lib.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES), "binding and header disagree"


def _params(**kw):
    from paper_1202_6351_amd import Params
    base = dict(nx=100, ny=37, tau=0.8, storage="fp32")
    base.update(kw)
    return Params(**base)


def test_layout_pitch_and_bytes():
    from paper_1202_6351_amd import lattice_layout
    for storage, sz in (("fp64", 8), ("fp32", 4), ("fp16", 2), ("bf16", 2)):
        pitch, nbytes = lattice_layout(_params(storage=storage))
        assert pitch == 128 and nbytes == 9 * 37 * 128 * sz


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=0.4), "omega_nu"),
    (dict(omega3=2.0), "omega3"),
    (dict(nx=1), "grid"),
    (dict(bc=("periodic", "wall", "periodic", "periodic")), "periodic on one side"),
    (dict(wall_u=(0.0, 0.0, 0.1, 0.0)), "periodic side"),
    (dict(rho0=0.0), "rho0"),
    (dict(storage="fp32", rounding="stochastic"), "stochastic rounding needs"),
    (dict(fx=float("inf")), "body force"),
    (dict(nx=65536, ny=16384, storage="fp32"), "exceeds 4 GiB"),  # plane of exactly 2^32 bytes
])
def test_invalid_parameters_rejected(kw, msg):
    from paper_1202_6351_amd import _lib, lattice_layout
    with pytest.raises(_lib.LbmError) as ei:
        lattice_layout(_params(**kw))
    assert ei.value.status == _lib.LBM_EINVAL and msg in str(ei.value)


def test_create_rejects_null_and_misaligned_buffers():
    from paper_1202_6351_amd import _lib
    lib = _lib.lib()
    cp = _params().c()
    ctx = ctypes.c_void_p()
    st = lib.lbm_create(ctypes.byref(cp), None, None, None, None, ctypes.byref(ctx))
    assert st == _lib.LBM_EINVAL and not ctx.value
    assert b"lattice buffers" in lib.lbm_last_error(None)
    st = lib.lbm_create(ctypes.byref(cp), ctypes.c_void_p(0x1000 + 8), ctypes.c_void_p(0x20000),
                        None, None, ctypes.byref(ctx))
    assert st == _lib.LBM_EINVAL and b"aligned" in lib.lbm_last_error(None)


def test_largest_plane_accepted():
    """A plane one row below the 4 GiB limit of the 32-bit plane offsets."""
    from paper_1202_6351_amd import lattice_layout
    pitch, nbytes = lattice_layout(_params(nx=65536, ny=16383, storage="fp32"))
    assert pitch == 65536 and nbytes == 9 * 16383 * 65536 * 4



def test_explicit_buffer_steps_refuse_stochastic_rounding():
    """lbm_step_between and lbm_step_sequence take no step index, so they
    could not draw fresh stochastic-rounding bits per step: with that
    rounding they return LBM_EUNSUPPORTED before any device work (the
    buffers below are never touched)."""
    from paper_1202_6351_amd import _lib
    lib = _lib.lib()
    for storage in ("fp16", "bf16"):
        cp = _params(storage=storage, rounding="stochastic").c()
        ctx = ctypes.c_void_p()
        a, b, c = (ctypes.c_void_p(0x100000 * k) for k in (1, 2, 3))
        assert lib.lbm_create(ctypes.byref(cp), a, b, None, None, ctypes.byref(ctx)) == _lib.LBM_OK
        try:
            assert lib.lbm_step_between(ctx, a, c) == _lib.LBM_EUNSUPPORTED
            assert b"stochastic" in lib.lbm_last_error(ctx)
            arr = (ctypes.c_void_p * 2)(b.value, c.value)
            assert lib.lbm_step_sequence(ctx, a, arr, 2) == _lib.LBM_EUNSUPPORTED
        finally:
            lib.lbm_destroy(ctx)
