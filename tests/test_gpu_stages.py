"""Step-by-step parity of the HIP kernels with the CPU oracle, through the C ABI.

Sizes span several workgroup tiles with ragged tails (the smoother tile is 64 x 32 cells, the
fused cycle tile 64 x 64, the restriction strip 64 x n).  Where the kernels evaluate the same
expression as the oracle in the same order (sweeps, prolongation, the MAC operators) the
comparison is bitwise; sums over tiles and the coarse transforms are compared with
tolerances derived from FP64 rounding.
"""
import numpy as np
import pytest
import torch

from oracle import ism_oracle as O
from tests.gpu_util import announce, dev, host, solver

pytestmark = pytest.mark.gpu
N, P, D = O.NEUMANN, O.PERIODIC, O.DIRICHLET
ND, DN = O.NEUMANN_DIRICHLET, O.DIRICHLET_NEUMANN
_CODE = {N: "N", P: "P", D: "D", ND: "ND", DN: "DN"}

# (nx, ny, n, bc_x, bc_y)
CASES = [
    (96, 80, 16, N, N),
    (128, 64, 8, P, N),
    (256, 192, 32, N, N),
    (64, 48, 4, P, N),
    (160, 96, 32, P, N),
    # large enough for the fused kernel's interior fast path (tiles whose halo touches no
    # wall and interpolates unclamped)
    (320, 256, 32, N, N),
    (320, 192, 16, P, N),
    (384, 320, 8, N, N),
    # zero-pressure (Dirichlet) walls: on every face, on one face of an axis, mixed
    (96, 80, 16, D, D),
    (128, 64, 8, P, ND),
    (64, 48, 4, DN, N),
    (320, 256, 32, DN, D),
    (384, 320, 8, ND, DN),
]
DTYPES = [(torch.float64, np.float64), (torch.float32, np.float32)]


def _ids(c):
    return f"{c[0]}x{c[1]}_n{c[2]}_{_CODE[c[3]]}-{_CODE[c[4]]}"


def _mk(case, batch=1, **kw):
    nx, ny, n, bx, by = case
    return solver(nx=nx, ny=ny, batch=batch, coarsen=n, bc_x=bx, bc_y=by, **kw)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_smooth_bitwise(case, tdt, ndt):
    announce("smooth", case, ndt.__name__)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(100)
    rhs = rng.standard_normal((ny, nx)).astype(ndt)
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    s = _mk(case)
    e = dev(e0, tdt)
    s.smooth(dev(rhs, tdt), e, nsweeps=3)
    ref = O.red_black_gs(e0, rhs, bx, by, sweeps=3)
    np.testing.assert_array_equal(host(e)[0] if host(e).ndim == 3 else host(e), ref)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_restrict(case, tdt, ndt):
    announce("restrict", case, ndt.__name__)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(101)
    rhs = rng.standard_normal((2, ny, nx)).astype(ndt)
    e = rng.standard_normal((2, ny, nx)).astype(ndt)
    s = _mk(case, batch=2)
    rc, sq = s.restrict(dev(rhs, tdt), dev(e, tdt), want_sumsq=True)
    rc, sq = host(rc), host(sq)
    for b in range(2):
        res = (rhs[b] - O.laplacian(e[b], bx, by)).astype(np.float64)
        ref = O.restrict_sum(res, n)
        scale = np.abs(res).max() * n * n
        np.testing.assert_allclose(rc[b], ref, rtol=0, atol=4e-16 * scale)
        np.testing.assert_allclose(sq[b], np.sum(res * res), rtol=1e-13)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_prolong_bitwise(case, tdt, ndt):
    announce("prolong", case, ndt.__name__)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(102)
    E = rng.standard_normal((ny // n, nx // n))
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    s = _mk(case)
    e = dev(e0, tdt)
    s.prolong(dev(E), e)
    ref = e0 + O.prolong_bilinear(E, n, bx, by, ndt)
    np.testing.assert_array_equal(host(e).reshape(ny, nx), ref)


@pytest.mark.parametrize("case", CASES + [(64, 64, 16, N, N), (64, 32, 16, P, N)], ids=_ids)
def test_coarse_stencil_matches_face_sums(case):
    announce("stencil", case)
    nx, ny, n, bx, by = case
    s = _mk(case)
    got = host(s.coarse_stencil())
    ref = O.coarse_stencil_ism(nx // n, ny // n, n, bx, by)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_coarse_solve(case):
    announce("coarse_solve", case)
    nx, ny, n, bx, by = case
    ncx, ncy = nx // n, ny // n
    rng = np.random.default_rng(103)
    Rc = rng.standard_normal((3, ncy, ncx))
    s = _mk(case, batch=3)
    E = host(s.coarse_solve(dev(Rc)))
    Ac = O.coarse_matrix(O.coarse_stencil_ism(ncx, ncy, n, bx, by), bx, by)
    cs = O.CoarseSolver(Ac)
    for b in range(3):
        ref = cs.solve(Rc[b])
        np.testing.assert_allclose(E[b], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        if cs.singular:
            assert abs(E[b].mean()) < 1e-13 * np.abs(ref).max()
        proj = Rc[b] - Rc[b].mean() if cs.singular else Rc[b]
        r = Ac @ E[b].ravel() - proj.ravel()
        assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(Rc[b])


@pytest.mark.parametrize("case", [(1280, 1088, 16, N, D), (2560, 1600, 32, P, N),
                                  (2304, 2112, 16, N, D), (4352, 1024, 32, P, DN)], ids=_ids)
def test_coarse_solve_mfma_path(case):
    """Coarse grids beyond 32 cells per axis (80 x 68, 80 x 50, 144 x 132, 136 x 32) take the
    four MFMA products instead of the one-workgroup solve; the same parity bar."""
    announce("coarse_solve_mfma", case)
    nx, ny, n, bx, by = case
    ncx, ncy = nx // n, ny // n
    rng = np.random.default_rng(113)
    Rc = rng.standard_normal((2, ncy, ncx))
    s = _mk(case, batch=2)
    E = host(s.coarse_solve(dev(Rc)))
    Ac = O.coarse_matrix(O.coarse_stencil_ism(ncx, ncy, n, bx, by), bx, by)
    cs = O.CoarseSolver(Ac)
    for b in range(2):
        ref = cs.solve(Rc[b])
        np.testing.assert_allclose(E[b], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("nu", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("fused", ["walk", "tile", False], ids=["walk", "tile", "unfused"])
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_cycle_sweeps_bitwise(case, nu, fused, tdt, ndt):
    """With a zero coarse right-hand side the correction is exactly zero, so a cycle is nu
    sweeps followed by the residual restriction: e must match the oracle bit for bit.  The
    fused FP64 kernel stops at nu = 4 (register budget): beyond it the call is refused."""
    announce("cycle_zero_coarse", case, nu, fused, ndt.__name__)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(104 + nu)
    rhs = rng.standard_normal((ny, nx)).astype(ndt)
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    s = _mk(case, nu=nu, fused=fused, precision="mixed" if nu > 4 else "fp64")
    if fused and ndt == np.float64 and nu > 4:
        from paper_1309_7128_amd.solver import IsmError

        rc = torch.zeros(s.coarse_shape, dtype=torch.float64, device="cuda")
        with pytest.raises(IsmError):
            s.cycle(dev(rhs, tdt), dev(e0, tdt), rc)
        return
    e = dev(e0, tdt)
    rc = torch.zeros(s.coarse_shape, dtype=torch.float64, device="cuda")
    s.cycle(dev(rhs, tdt), e, rc)
    ref = O.red_black_gs(e0, rhs, bx, by, sweeps=nu)
    np.testing.assert_array_equal(host(e).reshape(ny, nx), ref)
    res = (rhs - O.laplacian(ref, bx, by)).astype(np.float64)
    np.testing.assert_allclose(host(rc)[0], O.restrict_sum(res, n), rtol=0,
                               atol=4e-16 * np.abs(res).max() * n * n)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("fused", ["walk", "tile", False], ids=["walk", "tile", "unfused"])
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
@pytest.mark.parametrize("zero_e", [False, True], ids=["e", "zero_e"])
def test_cycle_matches_oracle(case, fused, tdt, ndt, zero_e):
    announce("cycle", case, fused, ndt.__name__, zero_e)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(110)
    rhs = rng.standard_normal((ny, nx)).astype(ndt)
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    rc0 = rng.standard_normal((ny // n, nx // n))
    s = _mk(case, nu=2, fused=fused)
    e = dev(e0, tdt)
    rc = dev(rc0[None])
    s.cycle(dev(rhs, tdt), e, rc, zero_e=zero_e)
    cs = O.CoarseSolver(O.coarse_matrix(O.coarse_stencil_ism(nx // n, ny // n, n, bx, by), bx, by))
    E = cs.solve(rc0)
    base = np.zeros_like(e0) if zero_e else e0
    ref = base + O.prolong_bilinear(E, n, bx, by, ndt)
    ref = O.red_black_gs(ref, rhs, bx, by, sweeps=2)
    got = host(e).reshape(ny, nx)
    # the only difference is the rounding of the coarse solve (<= 1e-12 relative), carried
    # through two sweeps; in FP32 it shows at most as an ulp of the result
    tol = (1e-11 if ndt == np.float64 else 4e-7) * np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=tol)
    res = (rhs - O.laplacian(got.astype(ndt), bx, by)).astype(np.float64)
    np.testing.assert_allclose(host(rc)[0], O.restrict_sum(res, n), rtol=0,
                               atol=4e-16 * np.abs(res).max() * n * n)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_fused_and_unfused_cycles_agree_bitwise(case):
    announce("fused_vs_unfused", case)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(111)
    rhs = dev(rng.standard_normal((ny, nx)), torch.float32)
    e0 = rng.standard_normal((ny, nx))
    rc0 = rng.standard_normal((1, ny // n, nx // n))
    outs = []
    for fused in ("walk", "tile", False):  # the two fused kernels and the unfused steps
        s = _mk(case, nu=3, fused=fused)
        e = dev(e0, torch.float32)
        rc = dev(rc0)
        for _ in range(3):
            s.cycle(rhs, e, rc)
        outs.append((host(e), host(rc)))
    for k in (1, 2):
        np.testing.assert_array_equal(outs[0][0], outs[k][0])
        np.testing.assert_allclose(outs[0][1], outs[k][1], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_outer_residual(case):
    announce("outer_residual", case)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(112)
    b = rng.standard_normal((2, ny, nx)) + 3.0
    x = rng.standard_normal((2, ny, nx))
    s = _mk(case, batch=2)
    r = host(s.outer_residual(dev(b), dev(x)))
    h = s.h
    for k in range(2):
        bt = b[k] - b[k].mean() if O.singular(bx, by) else b[k]
        ref = h * h * bt - O.laplacian(x[k], bx, by)
        np.testing.assert_allclose(r[k], ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_reduction_over_more_than_4096_chunks():
    """Grid means and norms are reduced in two stages: chunks of 4096 coarse-tile partials,
    then one workgroup per grid over the chunk results.  16400^2 cells at 4h make 4100^2
    tiles, 4105 chunks, and the second stage has to take all of them.  With b constant and
    x = 0 the outer residual h^2 (b - mean b) - A' x is zero up to the rounding of the mean;
    a chunk left out of the mean would leave h^2 times about 2e-3 in every cell."""
    n = 16400
    announce("reduction_4105_chunks", n)
    s = solver(nx=n, ny=n, coarsen=4)
    b = torch.ones((n, n), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    r = s.outer_residual(b, x)
    torch.cuda.synchronize()
    worst = float(r.abs().max())
    del r, b, x, s
    assert worst <= 4 * np.finfo(np.float64).eps * (1.0 / n) ** 2, worst


@pytest.mark.parametrize("bx,by", [(N, N), (P, N), (D, D), (ND, DN), (P, ND)])
def test_mac_operators_bitwise(bx, by):
    announce("mac", bx, by)
    nx, ny = 96, 80
    s = solver(nx=nx, ny=ny, batch=2, coarsen=16, bc_x=bx, bc_y=by, lx=1.5)
    h = s.h
    rng = np.random.default_rng(113)
    ush = (2,) + s.u_shape[1:]
    u, v = rng.standard_normal(ush), rng.standard_normal(s.v_shape)
    p = rng.standard_normal((2, ny, nx))
    b = host(s.div(dev(u), dev(v)))
    gu, gv = (host(t) for t in s.grad(dev(p)))
    du, dv = (host(t) for t in s.div_adjoint(dev(p)))
    gp = host(s.grad_adjoint(dev(u), dev(v)))
    for k in range(2):
        np.testing.assert_array_equal(b[k], O.div(u[k], v[k], h, bx))
        rgu, rgv = O.grad(p[k], h, bx, by)
        np.testing.assert_array_equal(gu[k], rgu)
        np.testing.assert_array_equal(gv[k], rgv)
        rdu, rdv = O.div_adjoint(p[k], h, bx)
        np.testing.assert_array_equal(du[k], rdu)
        np.testing.assert_array_equal(dv[k], rdv)
        np.testing.assert_allclose(gp[k], O.grad_adjoint(u[k], v[k], h, bx, by), rtol=0,
                                   atol=1e-15 * np.abs(gp[k]).max())


@pytest.mark.parametrize("case", CASES[:3] + [(128, 64, 8, P, ND), (96, 80, 16, D, D)], ids=_ids)
def test_gmg5_stencil_and_coarse_solve(case):
    announce("gmg5_stencil", case)
    nx, ny, n, bx, by = case
    s = _mk(case, batch=2, coarse_stencil="gmg5")
    got = host(s.coarse_stencil())
    ref = O.coarse_stencil_gmg5(nx // n, ny // n, n, bx, by)
    np.testing.assert_array_equal(got, ref)
    Rc = np.random.default_rng(120).standard_normal((2, ny // n, nx // n))
    E = host(s.coarse_solve(dev(Rc)))
    cs = O.CoarseSolver(O.coarse_matrix(ref, bx, by))
    for b in range(2):
        r = cs.solve(Rc[b])
        np.testing.assert_allclose(E[b], r, rtol=0, atol=1e-12 * np.abs(r).max())
