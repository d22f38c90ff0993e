"""Python binding of the ISM solver: torch tensors in, the C ABI of libism.so underneath.

PyTorch supplies device memory and the HIP stream; every operation of the solver runs in the
library's HIP kernels.  Tensors must live on the GPU, be contiguous and have the dtype and
shape the C ABI documents; anything else raises.  There is no CPU path.
"""
from __future__ import annotations

import ctypes
import warnings

import torch

from . import _lib as L

_BC = {"neumann": L.ISM_BC_NEUMANN, "periodic": L.ISM_BC_PERIODIC,
       "dirichlet": L.ISM_BC_DIRICHLET, "neumann-dirichlet": L.ISM_BC_NEUMANN_DIRICHLET,
       "dirichlet-neumann": L.ISM_BC_DIRICHLET_NEUMANN}
_PREC = {"fp64": L.ISM_PREC_FP64, "mixed": L.ISM_PREC_MIXED}


class IsmError(RuntimeError):
    """A negative status from the library."""

    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class IsmNotConverged(RuntimeWarning):
    """The solve stopped at a cycle or outer-step cap before meeting rtol."""


def _check(code, handle=None, lib=None):
    if code < 0:
        lib = lib or L.load()
        txt = lib.ism_last_error(handle)
        raise IsmError(code, (txt or b"").decode() or lib.ism_status_string(code).decode())
    return code


class Solver:
    """One handle of the ISM pressure solver for a fixed grid (C ABI: ism_create).

    The solve is A x = b~ with A the cell-centred 5-point Laplacian of an nx x ny grid of
    square cells (size lx / nx), for `batch` independent grids.  bc_x / bc_y: "neumann",
    "periodic", "dirichlet" (zero pressure on both faces), "neumann-dirichlet" or
    "dirichlet-neumann" (low face first).  Without a Dirichlet face b~ = b - mean(b) and x
    is the zero-mean solution; with one, b~ = b."""

    def __init__(self, nx, ny, batch=1, bc_x="neumann", bc_y="neumann", coarsen=16, lx=1.0,
                 ly=None, precision="fp64", nu=4, rtol=1e-10, inner_rtol=1e-3,
                 max_cycles=100000, max_outer=50, check_every=0, fused=True, device=None,
                 raise_not_converged=False, stall_window=None, stall_drop=None,
                 coarse_stencil="ism", cycling="repeat", coarse_tol=None, fine_tol=None,
                 coarse_gs="block"):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the ISM solver runs on a GPU; torch.cuda is not available")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        cfg = L.IsmConfig()
        self._lib.ism_config_init(ctypes.byref(cfg), nx, ny, batch)
        cfg.bc_x, cfg.bc_y = _BC[bc_x], _BC[bc_y]
        cfg.coarsen = coarsen
        cfg.lx = lx
        cfg.ly = lx * ny / nx if ly is None else ly
        cfg.precision = _PREC[precision]
        cfg.nu = nu
        cfg.rtol = rtol
        cfg.inner_rtol = inner_rtol
        cfg.max_cycles = max_cycles
        cfg.max_outer = max_outer
        cfg.check_every = check_every
        # fused: True (the kernel chosen by grid size), False (one kernel per step), or
        # "walk" / "tile" to force one of the two fused kernels
        fused_modes = {True: L.ISM_FUSED_AUTO, False: L.ISM_FUSED_OFF, "auto": L.ISM_FUSED_AUTO,
                       "walk": L.ISM_FUSED_WALK, "tile": L.ISM_FUSED_TILE}
        if fused not in fused_modes:
            raise ValueError("fused must be True, False, 'auto', 'walk' or 'tile'")
        cfg.fused = fused_modes[fused]
        if stall_window is not None:
            cfg.stall_window = stall_window
        if stall_drop is not None:
            cfg.stall_drop = stall_drop
        cfg.coarse_stencil = {"ism": L.ISM_COARSE_ISM, "gmg5": L.ISM_COARSE_GMG5,
                              "acm": L.ISM_COARSE_ACM}[coarse_stencil]
        # "oneshot": the paper's accommodative cycling once per solve (block or multicolour GS
        # on the coarse grid to coarse_tol, then fine sweeps to fine_tol; both absolute
        # max-norms)
        cfg.cycling = {"repeat": L.ISM_CYCLE_REPEAT, "oneshot": L.ISM_CYCLE_ONESHOT}[cycling]
        if coarse_tol is not None:
            cfg.coarse_tol = coarse_tol
        if fine_tol is not None:
            cfg.fine_tol = fine_tol
        # the coarse iteration of one-shot cycling and coarse_gs(): "block" or "multicolour"
        cfg.coarse_gs = {"block": L.ISM_COARSE_GS_BLOCK,
                         "multicolour": L.ISM_COARSE_GS_MULTICOLOUR}[coarse_gs]
        self.cfg = cfg
        self.nx, self.ny, self.batch = nx, ny, batch
        self.bc_x, self.bc_y = bc_x, bc_y
        self.n = coarsen
        self.h = cfg.lx / nx
        self.raise_not_converged = raise_not_converged
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        _check(self._lib.ism_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(handle)), None, self._lib)
        self._h = handle

    # ---------------------------------------------------------------- helpers
    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("solver is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.ism_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def u_shape(self):
        nxu = self.nx if self.bc_x == "periodic" else self.nx + 1
        return (self.batch, self.ny, nxu)

    @property
    def v_shape(self):
        return (self.batch, self.ny + 1, self.nx)

    @property
    def cell_shape(self):
        return (self.batch, self.ny, self.nx)

    @property
    def coarse_shape(self):
        return (self.batch, -(-self.ny // self.n), -(-self.nx // self.n))

    def _arg(self, t, shape, dtype=torch.float64, name="array"):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape) and not (shape[0] == 1 and tuple(t.shape) == tuple(shape[1:])):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return ctypes.c_void_p(t.data_ptr())

    def _new(self, shape, dtype=torch.float64):
        return torch.empty(shape, dtype=dtype, device=self.device)

    @staticmethod
    def _dtype_code(t):
        if t.dtype == torch.float64:
            return L.ISM_F64
        if t.dtype == torch.float32:
            return L.ISM_F32
        raise ValueError("fine arrays must be float32 or float64")

    # ---------------------------------------------------------------- solves
    def solve(self, b, x=None, adjoint=False):
        """Solve A x = b~ (b - mean(b) without a Dirichlet face); x (optional) is the warm
        start and is overwritten.

        Returns (x, stats dict)."""
        if x is None:
            x = torch.zeros(self.cell_shape, dtype=torch.float64, device=self.device)
        pb = self._arg(b, self.cell_shape, name="b")
        px = self._arg(x, self.cell_shape, name="x")
        st = L.IsmStats()
        fn = self._lib.ism_solve_adjoint if adjoint else self._lib.ism_solve
        code = _check(fn(self.handle, pb, px, ctypes.byref(st)), self.handle, self._lib)
        if code == L.ISM_NOT_CONVERGED:
            msg = f"ISM solve stopped at {st.cycles} cycles, rel. residual {st.rel_res_l2:.3e}"
            if self.raise_not_converged:
                raise IsmError(code, msg)
            warnings.warn(msg, IsmNotConverged, stacklevel=2)
        return x, st.as_dict()

    def solve_adjoint(self, g, lam=None):
        return self.solve(g, lam, adjoint=True)

    # ---------------------------------------------------------------- MAC operators
    def div(self, u, v, out=None):
        out = self._new(self.cell_shape) if out is None else out
        _check(self._lib.ism_div(self.handle, self._arg(u, self.u_shape, name="u"),
                                 self._arg(v, self.v_shape, name="v"),
                                 self._arg(out, self.cell_shape, name="out")), self.handle)
        return out

    def grad(self, p):
        gu, gv = self._new(self.u_shape), self._new(self.v_shape)
        _check(self._lib.ism_grad(self.handle, self._arg(p, self.cell_shape, name="p"),
                                  self._arg(gu, self.u_shape), self._arg(gv, self.v_shape)),
               self.handle)
        return gu, gv

    def div_adjoint(self, lam):
        gu, gv = self._new(self.u_shape), self._new(self.v_shape)
        _check(self._lib.ism_div_adjoint(self.handle, self._arg(lam, self.cell_shape, name="lam"),
                                         self._arg(gu, self.u_shape), self._arg(gv, self.v_shape)),
               self.handle)
        return gu, gv

    def grad_adjoint(self, gu, gv):
        p = self._new(self.cell_shape)
        _check(self._lib.ism_grad_adjoint(self.handle, self._arg(gu, self.u_shape, name="gu"),
                                          self._arg(gv, self.v_shape, name="gv"),
                                          self._arg(p, self.cell_shape)), self.handle)
        return p

    # ---------------------------------------------------------------- time step
    def predict(self, u, v, p, dt, eta, walls=None):
        """Explicit predictor of Goda's scheme (Eq. 3): returns new (us, vs); walls =
        (v west, v east, u south, u north) tangential wall velocities."""
        us, vs = self._new(self.u_shape), self._new(self.v_shape)
        wl = None if walls is None else (ctypes.c_double * 4)(*[float(a) for a in walls])
        _check(self._lib.ism_predict(self.handle, self._arg(u, self.u_shape, name="u"),
                                     self._arg(v, self.v_shape, name="v"),
                                     self._arg(p, self.cell_shape, name="p"), float(dt), float(eta),
                                     None if wl is None else ctypes.cast(wl, ctypes.c_void_p),
                                     self._arg(us, self.u_shape), self._arg(vs, self.v_shape)),
               self.handle)
        return us, vs

    def correct(self, x, u, v, p):
        """u -= G x, v -= G x, p += x, in place."""
        _check(self._lib.ism_correct(self.handle, self._arg(x, self.cell_shape, name="x"),
                                     self._arg(u, self.u_shape, name="u"),
                                     self._arg(v, self.v_shape, name="v"),
                                     self._arg(p, self.cell_shape, name="p")), self.handle)
        return u, v, p

    def step(self, u, v, p, dt, eta, walls=None, x=None):
        """One projection time step (Sec. 2.2): predictor, pressure-change solve, correction.
        x (optional) warm-starts the pressure change.  Returns (u, v, p, x, stats)."""
        us, vs = self.predict(u, v, p, dt, eta, walls)
        b = self.div(us, vs)
        x, st = self.solve(b, x)
        p = p.clone()
        self.correct(x, us, vs, p)
        return us, vs, p, x, st

    # ---------------------------------------------------------------- stages
    def smooth(self, rhs, e, nsweeps=1):
        """nsweeps red-black sweeps on A' e = rhs, in place on e (float32 or float64)."""
        dt = self._dtype_code(e)
        _check(self._lib.ism_smooth(self.handle, dt, self._arg(rhs, self.cell_shape, e.dtype, "rhs"),
                                    self._arg(e, self.cell_shape, e.dtype, "e"), nsweeps), self.handle)
        return e

    def restrict(self, rhs, e, want_sumsq=False):
        dt = self._dtype_code(e)
        rc = self._new(self.coarse_shape)
        sq = self._new((self.batch,)) if want_sumsq else None
        _check(self._lib.ism_restrict(self.handle, dt, self._arg(rhs, self.cell_shape, e.dtype, "rhs"),
                                      self._arg(e, self.cell_shape, e.dtype, "e"),
                                      self._arg(rc, self.coarse_shape),
                                      None if sq is None else ctypes.c_void_p(sq.data_ptr())),
               self.handle)
        return (rc, sq) if want_sumsq else rc

    def prolong(self, E, e):
        dt = self._dtype_code(e)
        _check(self._lib.ism_prolong(self.handle, dt, self._arg(E, self.coarse_shape, name="E"),
                                     self._arg(e, self.cell_shape, e.dtype, "e")), self.handle)
        return e

    def coarse_solve(self, rc):
        E = self._new(self.coarse_shape)
        _check(self._lib.ism_coarse_solve(self.handle, self._arg(rc, self.coarse_shape, name="rc"),
                                          self._arg(E, self.coarse_shape)), self.handle)
        return E

    def cycle(self, rhs, e, rc, zero_e=False, want_sumsq=False):
        """One two-level cycle on A' e = rhs; e and rc are updated in place."""
        dt = self._dtype_code(e)
        sq = self._new((self.batch,)) if want_sumsq else None
        _check(self._lib.ism_cycle(self.handle, dt, self._arg(rhs, self.cell_shape, e.dtype, "rhs"),
                                   self._arg(e, self.cell_shape, e.dtype, "e"),
                                   self._arg(rc, self.coarse_shape, name="rc"), int(bool(zero_e)),
                                   None if sq is None else ctypes.c_void_p(sq.data_ptr())),
               self.handle)
        return (e, rc, sq) if want_sumsq else (e, rc)

    def coarse_gs(self, rc, tol, max_iter=100000):
        """Block or multicolour Gauss-Seidel (the handle's coarse_gs) on the coarse systems
        A_c E = rc to max |rc - A_c E| < tol.  Returns (E, iterations, converged)."""
        E = self._new(self.coarse_shape)
        it = ctypes.c_int32()
        code = _check(self._lib.ism_coarse_gs(self.handle, self._arg(rc, self.coarse_shape, name="rc"),
                                              self._arg(E, self.coarse_shape), float(tol),
                                              int(max_iter), ctypes.byref(it)), self.handle)
        return E, it.value, code == L.ISM_OK

    def coarse_stencil(self):
        ncy, ncx = self.coarse_shape[1:]
        coef = self._new((ncy, ncx, 3, 3))
        _check(self._lib.ism_coarse_stencil(self.handle, ctypes.c_void_p(coef.data_ptr())), self.handle)
        return coef

    def outer_residual(self, b, x):
        r = self._new(self.cell_shape)
        _check(self._lib.ism_outer_residual(self.handle, self._arg(b, self.cell_shape, name="b"),
                                            self._arg(x, self.cell_shape, name="x"),
                                            self._arg(r, self.cell_shape)), self.handle)
        return r

    def profile(self, enable=True, every=1):
        """Start (reset) or stop per-kernel-class event timing inside the library; every = n
        times every n-th launch of each class."""
        _check(self._lib.ism_profile(self.handle, int(every) if enable else 0), self.handle)

    def profile_read(self):
        """{class: (total_ms, launches)} since the last profile(True)."""
        out = {}
        for name, kind in L.KERNEL_CLASSES.items():
            ms, n = ctypes.c_double(), ctypes.c_int64()
            _check(self._lib.ism_profile_read(self.handle, kind, ctypes.byref(ms), ctypes.byref(n)),
                   self.handle)
            out[name] = (ms.value, n.value)
        return out

    def workspace_bytes(self):
        n = ctypes.c_size_t()
        _check(self._lib.ism_workspace_bytes(self.handle, ctypes.byref(n)), self.handle)
        return n.value
