"""The allocation-free solve (ism_solve_static) against ism_solve on a handle, through the C
ABI: the same kernels, tables and check schedule, so x and the iteration counts agree bit for
bit.  Two calls in a row on the one static scratch array, the second on a smaller grid, then
the first again (the array keeps the previous call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import ism_oracle as O
from paper_1309_7128_amd import _lib as L
from tests.gpu_util import announce, dev, host, solver

pytestmark = pytest.mark.gpu

_PREC = {"fp64": L.ISM_PREC_FP64, "mixed": L.ISM_PREC_MIXED}
_BC = {"neumann": L.ISM_BC_NEUMANN, "periodic": L.ISM_BC_PERIODIC,
       "dirichlet": L.ISM_BC_DIRICHLET, "neumann-dirichlet": L.ISM_BC_NEUMANN_DIRICHLET}


def _static_solve(b, nx, ny, batch, coarsen, prec, bc_x, bc_y, nu, rtol):
    lib = L.load()
    cfg = L.IsmConfig()
    assert lib.ism_config_init(ctypes.byref(cfg), nx, ny, batch) == 0
    cfg.coarsen, cfg.precision, cfg.nu, cfg.rtol = coarsen, _PREC[prec], nu, rtol
    cfg.bc_x, cfg.bc_y = _BC[bc_x], _BC[bc_y]
    x = torch.zeros_like(b)
    st = L.IsmStats()
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.ism_solve_static(ctypes.byref(cfg), ctypes.c_void_p(b.data_ptr()),
                              ctypes.c_void_p(x.data_ptr()), ctypes.byref(st),
                              ctypes.c_void_p(stream))
    assert rc == 0, lib.ism_last_error(None)
    return x, st.as_dict()


CASES = [
    # nx, ny, batch, n, precision, bc_x, bc_y, nu: the second is smaller than the first
    (768, 512, 2, 16, "mixed", "neumann", "neumann", 5),
    (256, 128, 1, 8, "fp64", "periodic", "neumann-dirichlet", 4),
    (768, 512, 2, 16, "mixed", "neumann", "neumann", 5),
]


def test_static_solve_matches_handle_solve():
    rng = np.random.default_rng(700)
    for nx, ny, batch, n, prec, bx, by, nu in CASES:
        announce("static_solve", nx, ny, batch, n, prec, bx, by, nu)
        b = dev(rng.standard_normal((batch, ny, nx)))
        x1, st1 = _static_solve(b, nx, ny, batch, n, prec, bx, by, nu, 1e-10)
        s = solver(nx=nx, ny=ny, batch=batch, coarsen=n, precision=prec, bc_x=bx, bc_y=by,
                   nu=nu, rtol=1e-10)
        x2, st2 = s.solve(b)
        assert st1["status"] == 0 and st2["status"] == 0
        for key in ("cycles", "outer_iters", "sweeps", "launches", "rel_res_l2", "rel_res_max"):
            assert st1[key] == st2[key], (key, st1[key], st2[key])
        xa, xb = host(x1), host(x2).reshape(batch, ny, nx)
        np.testing.assert_array_equal(xa, xb)
        bh = host(b)
        bcx = {"neumann": O.NEUMANN, "periodic": O.PERIODIC}[bx]
        bcy = {"neumann": O.NEUMANN, "neumann-dirichlet": O.NEUMANN_DIRICHLET}[by]
        for k in range(batch):
            assert O.relative_residual(bh[k], xa[k], 1.0 / nx, bcx, bcy) <= 1e-10
