"""Host-side checks of libism.so that need no GPU: it loads, it exports every entry point
include/ism.h declares, the ctypes structs match the C layout, and invalid configurations
are rejected with the documented status codes before any device call."""
import ctypes
import os
import re

import pytest

from paper_1309_7128_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ism.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(ism_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.exported_names())


def test_struct_layout():
    # C layout: 6 int32, 2 double, 2 int32, 2 double, 5 int32 (+4 padding), 1 double,
    # 2 int32, 2 double, 1 int32 (+4 padding)
    assert ctypes.sizeof(L.IsmConfig) == 128
    assert L.IsmConfig.stall_drop.offset == 88 and L.IsmConfig.coarse_stencil.offset == 96
    assert L.IsmConfig.lx.offset == 24 and L.IsmConfig.rtol.offset == 48
    assert L.IsmConfig.cycling.offset == 100 and L.IsmConfig.fine_tol.offset == 112
    assert L.IsmConfig.coarse_gs.offset == 120
    # 4 int32, 2 int64, 3 double, 3 int32 (+4 padding)
    assert ctypes.sizeof(L.IsmStats) == 72 and L.IsmStats.coarse_iters.offset == 56
    assert L.IsmStats.coarse_syncs.offset == 64


def test_config_defaults():
    lib = L.load()
    cfg = L.IsmConfig()
    assert lib.ism_config_init(ctypes.byref(cfg), 256, 128, 2) == 0
    assert (cfg.nx, cfg.ny, cfg.batch, cfg.coarsen, cfg.nu) == (256, 128, 2, 16, 4)
    assert cfg.lx == 1.0 and cfg.ly == 0.5 and cfg.rtol == 1e-10 and cfg.fused == 1
    assert cfg.cycling == L.ISM_CYCLE_REPEAT and cfg.coarse_tol == 1e-5 and cfg.fine_tol == 1e-6
    assert cfg.coarse_gs == L.ISM_COARSE_GS_BLOCK
    assert lib.ism_config_init(None, 1, 1, 1) == L.ISM_ERR_INVALID


def _create(**kw):
    lib = L.load()
    cfg = L.IsmConfig()
    lib.ism_config_init(ctypes.byref(cfg), kw.pop("nx", 64), kw.pop("ny", 64), kw.pop("batch", 1))
    for k, v in kw.items():
        setattr(cfg, k, v)
    h = ctypes.c_void_p()
    code = lib.ism_create(ctypes.byref(cfg), None, ctypes.byref(h))
    return code, h, lib


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), L.ISM_ERR_INVALID),
    (dict(batch=0), L.ISM_ERR_INVALID),
    (dict(bc_x=7), L.ISM_ERR_INVALID),
    (dict(bc_y=5), L.ISM_ERR_INVALID),
    (dict(bc_x=-1), L.ISM_ERR_INVALID),
    (dict(precision=3), L.ISM_ERR_INVALID),
    (dict(nu=0), L.ISM_ERR_INVALID),
    (dict(rtol=0.0), L.ISM_ERR_INVALID),
    (dict(inner_rtol=1.5), L.ISM_ERR_INVALID),
    (dict(max_cycles=0), L.ISM_ERR_INVALID),
    (dict(lx=-1.0), L.ISM_ERR_INVALID),
    (dict(coarsen=12), L.ISM_ERR_UNSUPPORTED),
    # a grid that coarsen does not divide (padded) takes the ISM stencil, nx % 4 == 0, ny even
    (dict(nx=72, coarse_stencil=1), L.ISM_ERR_UNSUPPORTED),
    (dict(nx=72, coarse_stencil=2), L.ISM_ERR_UNSUPPORTED),
    (dict(nx=70, lx=70 / 64), L.ISM_ERR_UNSUPPORTED),
    (dict(ny=63, ly=63 / 64), L.ISM_ERR_UNSUPPORTED),
    (dict(ly=2.0), L.ISM_ERR_UNSUPPORTED),                    # non-square cells
    (dict(nu=5, fused=1), L.ISM_ERR_UNSUPPORTED),              # FP64 fused kernel: nu <= 4
    (dict(nu=6, fused=1, precision=1), L.ISM_ERR_UNSUPPORTED), # FP32 fused kernel: nu <= 5
    (dict(fused=4), L.ISM_ERR_INVALID),
    (dict(fused=-1), L.ISM_ERR_INVALID),
    (dict(stall_window=0), L.ISM_ERR_INVALID),
    (dict(stall_drop=1.0), L.ISM_ERR_INVALID),
    (dict(coarse_stencil=3), L.ISM_ERR_INVALID),
    (dict(coarse_stencil=2, precision=1), L.ISM_ERR_UNSUPPORTED),  # ACM is FP64 only
    (dict(cycling=2), L.ISM_ERR_INVALID),
    (dict(coarse_gs=2), L.ISM_ERR_INVALID),
    (dict(cycling=1, coarse_gs=-1), L.ISM_ERR_INVALID),
    (dict(cycling=1, coarse_tol=0.0), L.ISM_ERR_INVALID),
    (dict(cycling=1, fine_tol=-1.0), L.ISM_ERR_INVALID),
    (dict(cycling=1, coarse_stencil=2), L.ISM_ERR_UNSUPPORTED), # and needs a 9-point stencil
])
def test_invalid_configs_rejected_before_device(kw, code):
    got, h, lib = _create(**kw)
    assert got == code
    assert h.value is None
    assert lib.ism_last_error(None)  # a message is kept


def test_null_arguments():
    lib = L.load()
    h = ctypes.c_void_p()
    assert lib.ism_create(None, None, ctypes.byref(h)) == L.ISM_ERR_INVALID
    assert lib.ism_solve(None, None, None, None) == L.ISM_ERR_INVALID
    assert lib.ism_destroy(None) == L.ISM_OK
    assert lib.ism_status_string(L.ISM_NOT_CONVERGED) == b"not converged"


def test_static_solve_rejects_grids_beyond_its_scratch():
    # checked before any device call: 8192^2 mixed needs about 800 MB of workspace, more than
    # the static array; the ACM scheme is not available without a handle
    lib = L.load()
    cfg = L.IsmConfig()
    assert lib.ism_config_init(ctypes.byref(cfg), 8192, 8192, 1) == 0
    cfg.precision = L.ISM_PREC_MIXED
    st = L.IsmStats()
    rc = lib.ism_solve_static(ctypes.byref(cfg), 1, 1, ctypes.byref(st), None)
    assert rc == L.ISM_ERR_UNSUPPORTED
    assert b"static scratch" in lib.ism_last_error(None)
    assert lib.ism_config_init(ctypes.byref(cfg), 256, 256, 1) == 0
    cfg.coarse_stencil = L.ISM_COARSE_ACM
    assert lib.ism_solve_static(ctypes.byref(cfg), 1, 1, ctypes.byref(st), None) == L.ISM_ERR_UNSUPPORTED
    cfg.coarse_stencil = L.ISM_COARSE_ISM
    cfg.nx = 100  # not a multiple of the tile
    assert lib.ism_solve_static(ctypes.byref(cfg), 1, 1, ctypes.byref(st), None) == L.ISM_ERR_UNSUPPORTED
