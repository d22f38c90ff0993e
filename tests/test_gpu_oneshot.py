"""The paper's own solver configuration on the GPU (Sec. 4, Sec. 4.3.1): block-iterative
Gauss-Seidel on the coarse grid to an absolute tolerance, and one-shot accommodative cycling
with its iteration and synchronization counts, against the oracle.

The coarse 9-point coefficients are sums of dyadic fractions and hence exact on both sides,
and both sides update the cells in the same order with the same arithmetic, so block GS
iterates agree bit for bit when the right-hand side reaches both unchanged (a Dirichlet
face).  Without one, each side removes the mean of R itself (different summation orders),
so the iterates agree to rounding and the counts to within one.
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

# (nx, ny, n, bc_x, bc_y): coarse grids of one partial tile, several tiles with ragged
# edges, periodic seams between tiles (a short periodic axis is split in two)
GS_CASES = [
    (192, 160, 16, D, D),        # 12 x 10 coarse: one partial tile
    (512, 384, 16, D, ND),       # 32 x 24: four tiles, the last row of tiles partial
    (640, 320, 16, P, DN),       # 40 x 20: periodic seam between tiles
    (192, 128, 16, P, D),        # 12 x 8: the periodic axis split into two tiles of 6
    (512, 384, 16, N, N),
    (320, 256, 16, P, N),
]


def bgs_block(ncx, ncy, bx, by):
    """The library's block-GS tiling, as include/ism.h states it: (by, bx) tiles of 16 x 16
    coarse cells, except that a periodic axis of at most 16 cells is split into two tiles of
    ceil(nc / 2), so that no tile spans a whole periodic axis."""
    def one(nc, bc):
        return (nc + 1) // 2 if bc == P and nc <= 16 else 16
    return one(ncy, by), one(ncx, bx)


def _ids(c):
    return f"{c[0]}x{c[1]}_n{c[2]}_{_CODE[c[3]]}-{_CODE[c[4]]}"


def _readbacks(stop_it):
    """Read-backs of a device-checked loop that stops at iteration stop_it, as include/ism.h
    states the schedule: batches of 4, 8, 16, 32, then 64 iterations, one read-back each."""
    count, done, batch = 0, 0, 4
    while done <= stop_it:
        done += batch
        batch = min(2 * batch, 64)
        count += 1
    return count


@pytest.mark.parametrize("case", GS_CASES, ids=_ids)
def test_coarse_block_gs_matches_oracle(case):
    announce("coarse_bgs", case)
    nx, ny, n, bx, by = case
    ncx, ncy = nx // n, ny // n
    rng = np.random.default_rng(400)
    Rc = rng.standard_normal((ncy, ncx))
    tol = 2e-3 * np.abs(Rc).max()
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=bx, bc_y=by)
    E, it, conv = s.coarse_gs(dev(Rc[None]), tol, max_iter=5000)
    E = host(E).reshape(ncy, ncx)
    C = O.coarse_stencil_ism(ncx, ncy, n, bx, by)
    ref, it_ref = O.block_gauss_seidel(C, Rc, tol, bgs_block(ncx, ncy, bx, by), bx, by)
    assert conv
    if O.singular(bx, by):
        assert abs(it - it_ref) <= 1
        if it == it_ref:
            np.testing.assert_allclose(E, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    else:
        assert it == it_ref
        np.testing.assert_array_equal(E, ref)


# (nx, ny, n, bc_x, bc_y): multicolour GS on coarse grids of 4 colours, 6 and 9 (odd periodic
# axes), a coarse axis of one cell, and a grid of many workgroups per colour
MC_CASES = [
    (192, 160, 16, D, D),        # 12 x 10, 4 colours
    (208, 160, 16, P, D),        # 13 x 10: odd periodic x, 6 colours
    (208, 176, 16, P, P),        # 13 x 11: 9 colours, singular
    (512, 384, 16, D, ND),       # 32 x 24
    (640, 320, 16, P, DN),       # 40 x 20
    (16, 96, 16, P, D),          # 1 x 6: the single x cell takes colour 2
    (320, 256, 16, N, N),
]


@pytest.mark.parametrize("case", MC_CASES, ids=_ids)
def test_coarse_multicolour_gs_matches_oracle(case):
    """Multicolour GS (Sec. 3.1, Sec. 4.3): both sides update each colour's cells from the same
    values with the same arithmetic, so the iterates agree bit for bit with a Dirichlet face
    (and to rounding, counts within one, without: each side removes the mean of R itself)."""
    announce("coarse_mcgs", case)
    nx, ny, n, bx, by = case
    ncx, ncy = nx // n, ny // n
    rng = np.random.default_rng(403)
    Rc = rng.standard_normal((ncy, ncx))
    tol = 2e-3 * np.abs(Rc).max()
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=bx, bc_y=by, coarse_gs="multicolour")
    E, it, conv = s.coarse_gs(dev(Rc[None]), tol, max_iter=5000)
    E = host(E).reshape(ncy, ncx)
    C = O.coarse_stencil_ism(ncx, ncy, n, bx, by)
    ref, it_ref, _ = O.multicolour_gauss_seidel(C, Rc, tol, bx, by)
    assert conv
    if O.singular(bx, by):
        assert abs(it - it_ref) <= 1
        if it == it_ref:
            np.testing.assert_allclose(E, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    else:
        assert it == it_ref
        np.testing.assert_array_equal(E, ref)


def test_coarse_multicolour_gs_many_workgroups():
    """256 x 128 coarse cells (128 workgroups in the residual launch, 32 per colour), batch of
    two: 40 iterations (tolerance 0, so the cap stops them) bit for bit, per grid."""
    announce("coarse_mcgs_large")
    nx, ny, n = 4096, 2048, 16
    s = solver(nx=nx, ny=ny, batch=2, coarsen=n, bc_x=D, bc_y=N, coarse_gs="multicolour")
    Rc = np.random.default_rng(404).standard_normal((2, ny // n, nx // n))
    E, it, conv = s.coarse_gs(dev(Rc), 0.0, max_iter=40)
    assert it == 40 and not conv
    C = O.coarse_stencil_ism(nx // n, ny // n, n, D, N)
    for k in range(2):
        ref, _, _ = O.multicolour_gauss_seidel(C, Rc[k], 0.0, D, N, max_iter=40)
        np.testing.assert_array_equal(host(E)[k], ref)


def test_coarse_multicolour_gs_gmg5_stencil():
    announce("coarse_mcgs_gmg5")
    nx, ny, n = 512, 384, 16
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=D, bc_y=ND, coarse_stencil="gmg5",
               coarse_gs="multicolour")
    Rc = np.random.default_rng(405).standard_normal((1, ny // n, nx // n))
    tol = 1e-3 * np.abs(Rc).max()
    E, it, conv = s.coarse_gs(dev(Rc), tol, max_iter=5000)
    ref, it_ref, _ = O.multicolour_gauss_seidel(O.coarse_stencil_gmg5(nx // n, ny // n, n, D, ND),
                                                Rc[0], tol, D, ND)
    assert conv and it == it_ref
    np.testing.assert_array_equal(host(E)[0], ref)


def test_coarse_block_gs_gmg5_stencil():
    """Block GS on the 5-point coarse stencil of the GMG variant (Sec. 4.3.2), bitwise."""
    announce("coarse_bgs_gmg5")
    nx, ny, n = 512, 384, 16
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=D, bc_y=ND, coarse_stencil="gmg5")
    Rc = np.random.default_rng(402).standard_normal((1, ny // n, nx // n))
    tol = 1e-3 * np.abs(Rc).max()
    E, it, conv = s.coarse_gs(dev(Rc), tol, max_iter=5000)
    ref, it_ref = O.block_gauss_seidel(O.coarse_stencil_gmg5(nx // n, ny // n, n, D, ND), Rc[0],
                                       tol, 16, D, ND)
    assert conv and it == it_ref
    np.testing.assert_array_equal(host(E)[0], ref)


def test_oneshot_batch_meets_every_criterion():
    """Grids of a batch iterate together until every one meets each criterion, so each ends
    below the fine criterion and the counts are at least each grid's own."""
    announce("oneshot_batch")
    nx, ny, n = 128, 96, 16
    h = 1.0 / nx
    bs = np.stack([_mac_rhs(420 + k, nx, ny, h, D) * (1.0 + k) for k in range(2)])
    m = np.abs(bs).max()
    s = solver(nx=nx, ny=ny, batch=2, coarsen=n, bc_x=D, bc_y=D, cycling="oneshot",
               coarse_tol=1e-2 * m, fine_tol=1e-4 * m)
    x, st = s.solve(dev(bs))
    x = host(x)
    assert st["status"] == 0
    for k in range(2):
        assert np.abs(bs[k] - O.laplacian(x[k], D, D) / h**2).max() < 1e-4 * m
        _, info = O.ism_solve_oneshot(bs[k], h, n, D, D, tol_c=1e-2 * m, tol_f=1e-4 * m)
        assert st["coarse_iters"] >= info["coarse_iters"] and st["fine_iters"] >= info["fine_iters"]


def test_coarse_block_gs_iteration_cap():
    announce("coarse_bgs_cap")
    s = solver(nx=256, ny=256, coarsen=16, bc_x=D, bc_y=D)
    Rc = np.random.default_rng(401).standard_normal((1, 16, 16))
    E, it, conv = s.coarse_gs(dev(Rc), 1e-14, max_iter=7)
    assert it == 7 and not conv
    C = O.coarse_stencil_ism(16, 16, 16, D, D)
    ref, _ = O.block_gauss_seidel(C, Rc[0], 0.0, 16, D, D, max_iter=7)
    np.testing.assert_array_equal(host(E)[0], ref)


def _mac_rhs(seed, nx, ny, h, bx):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, (ny, nx) if bx == P else (ny, nx + 1))
    v = rng.uniform(-1, 1, (ny + 1, nx))
    return O.div(u, v, h, bx)


@pytest.mark.parametrize("bx,by,n", [(D, D, 8), (P, ND, 16), (N, N, 8), (DN, N, 16)])
def test_oneshot_solve_matches_oracle(bx, by, n):
    announce("oneshot", bx, by, n)
    nx, ny = 128, 96
    h = 1.0 / nx
    b = _mac_rhs(410, nx, ny, h, bx)
    tol_c, tol_f = 1e-4 * np.abs(b).max(), 1e-6 * np.abs(b).max()
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=bx, bc_y=by, cycling="oneshot", coarse_tol=tol_c,
               fine_tol=tol_f, lx=1.0)
    x, st = s.solve(dev(b))
    x = host(x).reshape(ny, nx)
    xo, info = O.ism_solve_oneshot(b, h, n, bx, by, tol_c=tol_c, tol_f=tol_f,
                                   block=bgs_block(nx // n, ny // n, bx, by))
    print(st, info, flush=True)
    assert st["status"] == 0 and st["cycles"] == 1
    exact = not O.singular(bx, by)
    assert abs(st["coarse_iters"] - info["coarse_iters"]) <= (0 if exact else 1)
    assert abs(st["fine_iters"] - info["fine_iters"]) <= (0 if exact else 1)
    assert st["sweeps"] == st["fine_iters"]
    bt = b - b.mean() if O.singular(bx, by) else b
    assert np.abs(bt - O.laplacian(x, bx, by) / h**2).max() < tol_f
    if exact and st["fine_iters"] == info["fine_iters"]:
        np.testing.assert_allclose(x, xo, rtol=0, atol=1e-9 * np.abs(xo).max())
    # one read-back per batch of coarse and of fine iterations, plus a fixed few
    assert st["host_syncs"] <= _readbacks(st["coarse_iters"]) + _readbacks(st["fine_iters"]) + 4


def test_oneshot_coarse_criterion_trades_fine_work():
    """The shape of the paper's tables (Sec. 4.3.1, Tables A.1-A.3) on one synthetic time
    step: warm-started from the previous step's solution, a tighter coarse criterion costs
    coarse iterations and leaves less fine work; NCC_t = I_c + 2 I_f."""
    announce("oneshot_tradeoff")
    nx = ny = 128
    h = 1.0 / nx
    b0 = _mac_rhs(411, nx, ny, h, N)
    b1 = b0 + 0.05 * _mac_rhs(412, nx, ny, h, N)  # the next step's right-hand side
    x0 = O.exact_solve(b0, h)
    db = np.abs(b1 - b0).max()
    out = []
    for tol_c in (3e-1, 1e-2, 1e-4):
        s = solver(nx=nx, ny=ny, coarsen=16, cycling="oneshot", coarse_tol=tol_c * db,
                   fine_tol=1e-4 * db)
        x, st = s.solve(dev(b1), dev(x0))
        assert st["status"] == 0
        out.append((st["coarse_iters"], st["fine_iters"]))
        print(tol_c, st["coarse_iters"], st["fine_iters"], "NCC_t", st["coarse_iters"] + 2 * st["fine_iters"],
              flush=True)
    assert out[0][0] < out[1][0] < out[2][0]
    assert out[2][1] < out[0][1]


@pytest.mark.parametrize("bx,by,n,prec", [(D, D, 8, "fp64"), (P, ND, 16, "mixed"),
                                          (N, N, 8, "fp64"), (DN, P, 16, "mixed")])
def test_oneshot_multicolour_matches_oracle(bx, by, n, prec):
    """One-shot cycling with multicolour GS on the coarse grid: the counts, the coarse
    synchronizations (one per colour, Sec. 4.3) and the result against the oracle."""
    announce("oneshot_mc", bx, by, n, prec)
    nx, ny = 144, 96
    h = 1.0 / nx
    b = _mac_rhs(414, nx, ny, h, bx)
    tol_c, tol_f = 1e-4 * np.abs(b).max(), 1e-3 * np.abs(b).max()
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=bx, bc_y=by, cycling="oneshot", coarse_tol=tol_c,
               fine_tol=tol_f, lx=1.0, precision=prec, coarse_gs="multicolour")
    x, st = s.solve(dev(b))
    x = host(x).reshape(ny, nx)
    xo, info = O.ism_solve_oneshot(b, h, n, bx, by, tol_c=tol_c, tol_f=tol_f,
                                   precision="fp32" if prec == "mixed" else "fp64",
                                   coarse_gs="multicolour")
    print(st, info, flush=True)
    assert st["status"] == 0
    exact = not O.singular(bx, by)
    assert abs(st["coarse_iters"] - info["coarse_iters"]) <= (0 if exact else 1)
    assert abs(st["fine_iters"] - info["fine_iters"]) <= (0 if exact else 1)
    colours = info["ncc_c"] // max(info["coarse_iters"], 1)
    assert st["coarse_syncs"] == colours * st["coarse_iters"]
    bt = b - b.mean() if O.singular(bx, by) else b
    assert np.abs(bt - O.laplacian(x, bx, by) / h**2).max() < (1.01 if prec == "mixed" else 1.0) * tol_f
    if exact and st["fine_iters"] == info["fine_iters"]:
        np.testing.assert_allclose(x, xo, rtol=0, atol=1e-9 * np.abs(xo).max())


@pytest.mark.parametrize("prec,gs", [("fp64", "block"), ("mixed", "multicolour")])
def test_oneshot_many_coarse_tiles_matches_oracle(prec, gs):
    """320 x 256 at 4h: 5120 coarse tiles, so each fused fine pass leaves more per-tile maxima
    than one reduction chunk (4096) and the criterion takes the two-stage reduction.  A
    Dirichlet face: both counts exactly the oracle's."""
    announce("oneshot_many_tiles", prec, gs)
    nx, ny, n = 320, 256, 4
    h = 1.0 / nx
    b = _mac_rhs(415, nx, ny, h, D)
    tol_c, tol_f = 1e-2 * np.abs(b).max(), 1e-3 * np.abs(b).max()
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=D, bc_y=ND, cycling="oneshot", coarse_tol=tol_c,
               fine_tol=tol_f, lx=1.0, precision=prec, coarse_gs=gs)
    x, st = s.solve(dev(b))
    xo, info = O.ism_solve_oneshot(b, h, n, D, ND, tol_c=tol_c, tol_f=tol_f,
                                   block=bgs_block(nx // n, ny // n, D, ND),
                                   precision="fp32" if prec == "mixed" else "fp64", coarse_gs=gs)
    print(st, info, flush=True)
    assert st["status"] == 0
    assert st["coarse_iters"] == info["coarse_iters"] and st["fine_iters"] == info["fine_iters"]
    assert st["coarse_syncs"] == info["ncc_c"]
    x = host(x).reshape(ny, nx)
    assert np.abs(b - O.laplacian(x, D, ND) / h**2).max() < (1.01 if prec == "mixed" else 1.0) * tol_f
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-9 * np.abs(xo).max())


def test_coarse_multicolour_gs_iteration_cap():
    announce("coarse_mcgs_cap")
    s = solver(nx=256, ny=256, coarsen=16, bc_x=D, bc_y=D, coarse_gs="multicolour")
    Rc = np.random.default_rng(406).standard_normal((1, 16, 16))
    E, it, conv = s.coarse_gs(dev(Rc), 1e-14, max_iter=7)
    assert it == 7 and not conv
    C = O.coarse_stencil_ism(16, 16, 16, D, D)
    ref, _, _ = O.multicolour_gauss_seidel(C, Rc[0], 0.0, D, D, max_iter=7)
    np.testing.assert_array_equal(host(E)[0], ref)


@pytest.mark.parametrize("bx,by,n", [(D, D, 8), (P, ND, 16), (N, N, 8), (DN, N, 16)])
def test_oneshot_fp32_matches_oracle(bx, by, n):
    """The paper's single-precision solver (Sec. 4.2): the fine stage in FP32 as a correction,
    against the oracle's FP32 form.  The FP32 sweeps and residual maxima are bitwise those of
    the oracle, so with a Dirichlet face both counts are exact."""
    announce("oneshot_fp32", bx, by, n)
    nx, ny = 128, 96
    h = 1.0 / nx
    b = _mac_rhs(413, nx, ny, h, bx)
    tol_c, tol_f = 1e-4 * np.abs(b).max(), 1e-5 * np.abs(b).max()
    s = solver(nx=nx, ny=ny, coarsen=n, bc_x=bx, bc_y=by, cycling="oneshot", coarse_tol=tol_c,
               fine_tol=tol_f, lx=1.0, precision="mixed")
    x, st = s.solve(dev(b))
    x = host(x).reshape(ny, nx)
    xo, info = O.ism_solve_oneshot(b, h, n, bx, by, tol_c=tol_c, tol_f=tol_f,
                                   block=bgs_block(nx // n, ny // n, bx, by), precision="fp32")
    print(st, info, flush=True)
    assert st["status"] == 0
    exact = not O.singular(bx, by)
    assert abs(st["coarse_iters"] - info["coarse_iters"]) <= (0 if exact else 1)
    assert abs(st["fine_iters"] - info["fine_iters"]) <= (0 if exact else 1)
    bt = b - b.mean() if O.singular(bx, by) else b
    assert np.abs(bt - O.laplacian(x, bx, by) / h**2).max() < 1.01 * tol_f
    if exact and st["fine_iters"] == info["fine_iters"]:
        np.testing.assert_allclose(x, xo, rtol=0, atol=1e-12 * np.abs(xo).max())
    assert st["host_syncs"] <= _readbacks(st["coarse_iters"]) + _readbacks(st["fine_iters"]) + 4


def test_oneshot_iteration_cap():
    """max_cycles caps each stage: the fine stage stops at the cap, unconverged."""
    announce("oneshot_cap")
    nx = ny = 128
    h = 1.0 / nx
    b = _mac_rhs(414, nx, ny, h, D)
    s = solver(nx=nx, ny=ny, coarsen=16, bc_x=D, bc_y=D, cycling="oneshot",
               coarse_tol=1e-3 * np.abs(b).max(), fine_tol=1e-12 * np.abs(b).max(), max_cycles=37)
    x, st = s.solve(dev(b))
    assert st["status"] == 1 and st["fine_iters"] == 37
    _, info = O.ism_solve_oneshot(b, h, 16, D, D, tol_c=1e-3 * np.abs(b).max(),
                                  tol_f=1e-12 * np.abs(b).max(), max_fine=37)
    assert info["fine_iters"] == 37 and st["coarse_iters"] == info["coarse_iters"]


def test_oneshot_rejects_unsupported():
    from paper_1309_7128_amd.solver import IsmError

    with pytest.raises(IsmError):
        solver(nx=64, ny=64, coarsen=16, cycling="oneshot", coarse_stencil="acm")
