"""Grids that the tile size n does not divide (the padded domain: Sec. 3.3, Eq. 5, where the
rectangle sizes differ next to the padding, and Sec. 4.1).  The last tile of an axis is short
and its centre is its middle; every stage is compared with the oracle's padded forms through
the C ABI, bitwise where the kernels evaluate the oracle's expression in its order
(prolongation, sweeps), with FP64 rounding tolerances for sums and the coarse solve.

Without a Dirichlet face the coarse system is singular with the constants as null vectors on
both sides; the library's spectral solve returns the solution whose prolongation has zero mean
(the oracle's bordered solve the zero-mean E), so coarse solutions are compared up to a
constant, on right-hand sides that sum to zero.
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

# (nx, ny, n, bc_x, bc_y): nx a multiple of 4, ny even, n dividing neither or one axis
CASES = [
    (100, 70, 16, D, ND),
    (44, 36, 8, P, N),
    (72, 52, 32, DN, P),
    (40, 30, 16, P, D),
    (20, 12, 16, N, D),     # one short tile along y
    (96, 70, 16, N, N),     # x full, y padded
    (100, 64, 16, P, N),    # x padded, y full
    (64, 50, 4, N, DN),     # n = 4: only y can be padded
    # large enough for the fused kernel's plain walks away from the short tiles
    (1000, 500, 32, P, N),
    (340, 270, 16, N, N),
    (332, 262, 8, P, P),
    (424, 390, 32, DN, D),
]
DTYPES = [(torch.float64, np.float64), (torch.float32, np.float32)]


def _ids(c):
    return f"{c[0]}x{c[1]}_n{c[2]}_{_CODE[c[3]]}-{_CODE[c[4]]}"


def _mk(case, batch=1, **kw):
    nx, ny, n, bx, by = case
    return solver(nx=nx, ny=ny, batch=batch, coarsen=n, bc_x=bx, bc_y=by, lx=float(nx), **kw)


def _nc(case):
    nx, ny, n = case[:3]
    return -(-nx // n), -(-ny // n)


def _coarse_solver(case):
    nx, ny, n, bx, by = case
    ncx, ncy = _nc(case)
    C = O.coarse_stencil_ism(ncx, ncy, n, bx, by, fine_shape=(ny, nx))
    return O.CoarseSolver(O.coarse_matrix(C, bx, by))


def _to_library_gauge(E, case):
    """The oracle's zero-mean coarse solution shifted by the constant that gives its
    prolongation zero mean (singular systems only)."""
    nx, ny, n, bx, by = case
    if not O.singular(bx, by):
        return E
    return E - O.prolong_bilinear(E, n, bx, by, fine_shape=(ny, nx)).mean()


def test_cases_are_padded():
    for nx, ny, n, _, _ in CASES:
        assert nx % n or ny % n
        assert nx % 4 == 0 and ny % 2 == 0


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_prolong_bitwise(case, tdt, ndt):
    announce("padded_prolong", case, ndt.__name__)
    nx, ny, n, bx, by = case
    ncx, ncy = _nc(case)
    rng = np.random.default_rng(402)
    E = rng.standard_normal((ncy, ncx))
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    s = _mk(case)
    assert s.coarse_shape == (1, ncy, ncx)
    e = dev(e0, tdt)
    s.prolong(dev(E), e)
    ref = e0 + O.prolong_bilinear(E, n, bx, by, ndt, fine_shape=(ny, nx))
    np.testing.assert_array_equal(host(e).reshape(ny, nx), ref)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_restrict(case, tdt, ndt):
    announce("padded_restrict", case, ndt.__name__)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(401)
    rhs = rng.standard_normal((2, ny, nx)).astype(ndt)
    e = rng.standard_normal((2, ny, nx)).astype(ndt)
    s = _mk(case, batch=2)
    rc, sq = s.restrict(dev(rhs, tdt), dev(e, tdt), want_sumsq=True)
    rc, sq = host(rc), host(sq)
    for b in range(2):
        res = (rhs[b] - O.laplacian(e[b], bx, by)).astype(np.float64)
        ref = O.restrict_sum(res, n)
        assert ref.shape == _nc(case)[::-1]
        np.testing.assert_allclose(rc[b], ref, rtol=0, atol=4e-16 * np.abs(res).max() * n * n)
        np.testing.assert_allclose(sq[b], np.sum(res * res), rtol=1e-13)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_coarse_stencil_matches_face_sums(case):
    announce("padded_stencil", case)
    nx, ny, n, bx, by = case
    ncx, ncy = _nc(case)
    got = host(_mk(case).coarse_stencil())
    ref = O.coarse_stencil_ism(ncx, ncy, n, bx, by, fine_shape=(ny, nx))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("case", CASES + [(1000, 2000, 16, P, N), (1000, 2000, 32, P, N)],
                         ids=_ids)
def test_coarse_solve(case):
    """The host-built pencil tables solve the Galerkin system: against the oracle's LU up to
    a constant (singular systems), and P E with zero mean."""
    announce("padded_coarse_solve", case)
    nx, ny, n, bx, by = case
    ncx, ncy = _nc(case)
    rng = np.random.default_rng(403)
    Rc = rng.standard_normal((3, ncy, ncx))
    cs = _coarse_solver(case)
    if cs.singular:
        Rc -= Rc.mean(axis=(1, 2), keepdims=True)
    s = _mk(case, batch=3)
    E = host(s.coarse_solve(dev(Rc)))
    for b in range(3):
        ref = _to_library_gauge(cs.solve(Rc[b]), case)
        scale = np.abs(ref).max()
        np.testing.assert_allclose(E[b], ref, rtol=0, atol=1e-11 * scale)
        r = cs.Ac @ E[b].ravel() - Rc[b].ravel()
        assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(Rc[b])
        if cs.singular:
            pe = O.prolong_bilinear(E[b], n, bx, by, fine_shape=(ny, nx))
            # zero up to the rounding of the transforms (the constant mode's coefficient is
            # set to zero exactly)
            assert abs(pe.mean()) < 2e-12 * scale


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("nu", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("fused", ["walk", "tile", False], ids=["walk", "tile", "unfused"])
@pytest.mark.parametrize("tdt,ndt", DTYPES, ids=["f64", "f32"])
def test_cycle_sweeps_bitwise(case, nu, fused, tdt, ndt):
    """A zero coarse right-hand side gives an exactly zero correction: the cycle is nu
    sweeps and the restriction of the residual, e bitwise equal to the oracle's."""
    if fused and ndt == np.float64 and nu > 4:
        pytest.skip("the fused FP64 kernel takes nu <= 4 (refusal tested with full tiles)")
    announce("padded_cycle_zero_coarse", case, nu, fused, ndt.__name__)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(404 + nu)
    rhs = rng.standard_normal((ny, nx)).astype(ndt)
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    s = _mk(case, nu=nu, fused=fused, precision="mixed" if nu > 4 else "fp64")
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
    announce("padded_cycle", case, fused, ndt.__name__, zero_e)
    nx, ny, n, bx, by = case
    ncx, ncy = _nc(case)
    rng = np.random.default_rng(410)
    rhs = rng.standard_normal((ny, nx)).astype(ndt)
    e0 = rng.standard_normal((ny, nx)).astype(ndt)
    rc0 = rng.standard_normal((ncy, ncx))
    cs = _coarse_solver(case)
    if cs.singular:
        rc0 -= rc0.mean()
    s = _mk(case, nu=2, fused=fused)
    e = dev(e0, tdt)
    rc = dev(rc0[None])
    s.cycle(dev(rhs, tdt), e, rc, zero_e=zero_e)
    E = _to_library_gauge(cs.solve(rc0), case)
    base = np.zeros_like(e0) if zero_e else e0
    ref = base + O.prolong_bilinear(E, n, bx, by, ndt, fine_shape=(ny, nx))
    ref = O.red_black_gs(ref, rhs, bx, by, sweeps=2)
    got = host(e).reshape(ny, nx)
    tol = (1e-10 if ndt == np.float64 else 4e-7) * np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=0, atol=tol)
    res = (rhs - O.laplacian(got.astype(ndt), bx, by)).astype(np.float64)
    np.testing.assert_allclose(host(rc)[0], O.restrict_sum(res, n), rtol=0,
                               atol=4e-16 * np.abs(res).max() * n * n)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("tdt", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_fused_and_unfused_cycles_agree(case, tdt):
    """The first cycle (same coarse right-hand side) bitwise; later cycles start from
    restrictions summed in different orders, so in FP64 they agree to rounding (in FP32 the
    difference stays below the fine type's resolution here)."""
    announce("padded_fused_vs_unfused", case, tdt)
    nx, ny, n, bx, by = case
    ncx, ncy = _nc(case)
    rng = np.random.default_rng(411)
    rhs = dev(rng.standard_normal((ny, nx)), tdt)
    e0 = rng.standard_normal((ny, nx))
    rc0 = rng.standard_normal((1, ncy, ncx))
    first, outs = [], []
    for fused in ("walk", "tile", False):  # the two fused kernels and the unfused steps
        s = _mk(case, nu=3, fused=fused)
        e = dev(e0, tdt)
        rc = dev(rc0)
        for k in range(3):
            s.cycle(rhs, e, rc)
            if k == 0:
                first.append(host(e))
        outs.append((host(e), host(rc)))
    for k in (1, 2):
        np.testing.assert_array_equal(first[0], first[k])
        if tdt == torch.float32:
            np.testing.assert_array_equal(outs[0][0], outs[k][0])
            np.testing.assert_allclose(outs[0][1], outs[k][1], rtol=1e-12, atol=1e-14)
        else:
            np.testing.assert_allclose(outs[0][0], outs[k][0], rtol=0,
                                       atol=1e-11 * np.abs(outs[k][0]).max())
            np.testing.assert_allclose(outs[0][1], outs[k][1], rtol=0,
                                       atol=1e-10 * np.abs(outs[k][1]).max())


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_outer_residual(case):
    announce("padded_outer_residual", case)
    nx, ny, n, bx, by = case
    rng = np.random.default_rng(412)
    b = rng.standard_normal((2, ny, nx)) + 3.0
    x = rng.standard_normal((2, ny, nx))
    s = _mk(case, batch=2)
    r = host(s.outer_residual(dev(b), dev(x)))
    for k in range(2):
        bt = b[k] - b[k].mean() if O.singular(bx, by) else b[k]
        ref = s.h * s.h * bt - O.laplacian(x[k], bx, by)
        np.testing.assert_allclose(r[k], ref, rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("case", [(200, 150, 16, P, N), (340, 270, 16, N, N), (100, 70, 16, D, ND),
                                  (424, 390, 32, DN, D)], ids=_ids)
@pytest.mark.parametrize("fused", [True, False], ids=["fused", "unfused"])
def test_fp64_solve_matches_oracle_iteration(case, fused):
    """The FP64 ISM iteration on a padded grid: the oracle's cycle count, its solution."""
    announce("padded_fp64_solve", case, fused)
    nx, ny, n, bx, by = case
    b = np.random.default_rng(420).standard_normal((ny, nx))
    s = _mk(case, precision="fp64", rtol=1e-10, check_every=1, fused=fused, nu=2)
    x, st = s.solve(dev(b))
    x = host(x).reshape(ny, nx)
    assert st["status"] == 0
    assert O.relative_residual(b, x, s.h, bx, by) <= 1e-10
    xo, info = O.ism_solve(b, s.h, n, bx, by, nu=2, rtol=1e-10)
    assert abs(st["cycles"] - info["cycles"]) <= 1
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-8 * np.abs(xo).max())
    xs = O.exact_solve(b, s.h, bx, by)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_paper_grid_1000x2000(n, prec):
    """The paper's 1000 x 2000 grid (periodic in x, walls in y; Sec. 4.1), which neither 16 nor
    32 divides in x (and 32 not in y): the solve reaches the exact discrete solution."""
    announce("paper_grid", n, prec)
    nx, ny = 1000, 2000
    rng = np.random.default_rng(430 + n)
    b = rng.standard_normal((ny, nx))
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=P, bc_y=N, precision=prec, rtol=1e-10,
               lx=float(nx), nu=5 if prec == "mixed" else 4)
    x, st = s.solve(dev(b))
    print(st, flush=True)
    x = host(x).reshape(ny, nx)
    assert st["status"] == 0
    assert O.relative_residual(b, x, s.h, P, N) <= 1e-10
    xs = O.exact_solve(b, s.h, P, N, refine=1)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-6
    assert abs(x.mean()) < 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("case", [(44, 36, 8, P, N), (40, 30, 16, P, D), (20, 12, 16, N, D)], ids=_ids)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_small_padded_solves_against_dense(case, prec):
    announce("padded_dense", case, prec)
    nx, ny, n, bx, by = case
    b = np.random.default_rng(440).standard_normal((ny, nx))
    s = _mk(case, precision=prec, rtol=1e-10, nu=2)
    x, st = s.solve(dev(b))
    assert st["status"] == 0
    xd = O.dense_solve(b, s.h, bx, by)
    np.testing.assert_allclose(host(x).reshape(ny, nx), xd, rtol=0, atol=1e-7 * np.abs(xd).max())
