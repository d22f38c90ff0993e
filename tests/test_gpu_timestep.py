"""The projection time step of Goda's scheme on the GPU (Sec. 2.2, Eq. 3-4): the explicit
predictor bit for bit against the oracle's, one whole step against the oracle's step, and a
shear-driven cavity time loop in the shape of the paper's Benchmark I (Sec. 4.3.1)."""
import numpy as np
import pytest
import torch

from oracle import ism_oracle as O
from tests.gpu_util import announce, dev, host, solver

pytestmark = pytest.mark.gpu
N, P = O.NEUMANN, O.PERIODIC


def _fields(seed, nx, ny, bx, batch=1):
    rng = np.random.default_rng(seed)
    nxu = nx if bx == P else nx + 1
    u = rng.uniform(-1, 1, (batch, ny, nxu))
    v = rng.uniform(-1, 1, (batch, ny + 1, nx))
    if bx != P:
        u[:, :, 0] = u[:, :, -1] = 0.0
    v[:, 0, :] = v[:, -1, :] = 0.0
    p = rng.standard_normal((batch, ny, nx))
    return u, v, p


@pytest.mark.parametrize("bx,walls", [(N, (0.0, 0.0, 0.0, 1.0)), (N, (-0.3, 0.2, 0.5, -0.1)),
                                      (P, (0.0, 0.0, 0.25, -0.75))])
def test_predictor_bitwise(bx, walls):
    announce("predictor", bx, walls)
    nx, ny = 96, 80
    u, v, p = _fields(500, nx, ny, bx, batch=2)
    s = solver(nx=nx, ny=ny, batch=2, coarsen=16, bc_x=bx, lx=1.5)
    dt, eta = 0.01, 0.07
    us, vs = s.predict(dev(u), dev(v), dev(p), dt, eta, walls)
    us, vs = host(us), host(vs)
    for k in range(2):
        ru, rv = O.predictor(u[k], v[k], p[k], s.h, dt, eta, bx, walls)
        np.testing.assert_array_equal(us[k], ru)
        np.testing.assert_array_equal(vs[k], rv)


@pytest.mark.parametrize("bx", [N, P])
def test_projection_step_matches_oracle(bx):
    announce("projection_step", bx)
    nx, ny = 128, 96
    u, v, p = _fields(501, nx, ny, bx)
    walls = (0.0, 0.0, 0.0, 1.0)
    s = solver(nx=nx, ny=ny, coarsen=16, bc_x=bx, precision="fp64", rtol=1e-12, lx=1.0)
    dt, eta = 2e-3, 0.05
    un, vn, pn, x, st = s.step(dev(u), dev(v), dev(p), dt, eta, walls)
    ru, rv, rp = O.projection_step(u[0], v[0], p[0], s.h, dt, eta, bx, walls)
    un, vn, pn = host(un).reshape(ru.shape), host(vn).reshape(rv.shape), host(pn).reshape(rp.shape)
    # both sides solve A x = D v* (the library to a relative residual of 1e-12, the oracle
    # exactly); the error in x is bounded by cond(A) ~ (nx / pi)^2 times the residual
    scale = max(np.abs(ru).max(), np.abs(rv).max())
    np.testing.assert_allclose(un, ru, rtol=0, atol=1e-8 * scale)
    np.testing.assert_allclose(vn, rv, rtol=0, atol=1e-8 * scale)
    # the pressure change x = p_new - p is defined up to a constant in the singular case;
    # ||x - x*||_2 <= cond(A) ||b - A x|| / ||b|| ||x*||_2, with cond(A) = lambda_max /
    # lambda_min over the nonzero eigenvalues of this grid's Laplacian and the library's
    # relative residual below 1e-12
    lam = (O.laplacian_eigenvalues(nx, bx)[None, :] + O.laplacian_eigenvalues(ny, N)[:, None]).ravel()
    lam = np.abs(lam[np.abs(lam) > 1e-12])
    kappa = lam.max() / lam.min()
    assert st["rel_res_l2"] <= 1e-12
    xl, xo = pn - p[0], rp - p[0]
    dx = (xl - xl.mean()) - (xo - xo.mean())
    assert np.linalg.norm(dx) <= kappa * 1e-12 * np.linalg.norm(xo - xo.mean())
    b0 = np.abs(O.div(u[0], v[0], s.h, bx)).max()
    assert np.abs(O.div(un, vn, s.h, bx)).max() < 1e-9 * b0


def test_shear_driven_cavity_loop():
    """Benchmark I's set-up in shape (Sec. 4.3.1, Fig. 3): unit cells, dt = 1, viscosity 0.1,
    wall speed 0.1 (read as every wall sliding counter-clockwise), on 256^2; 30 steps from
    rest.  Every step leaves a divergence-free field and the flow spins up counter-clockwise."""
    announce("cavity_loop")
    nx = ny = 256
    U = 0.1
    walls = (-U, U, U, -U)
    s = solver(nx=nx, ny=ny, coarsen=16, precision="mixed", rtol=1e-8, lx=float(nx), nu=5)
    u = torch.zeros(s.u_shape, dtype=torch.float64, device="cuda")
    v = torch.zeros(s.v_shape, dtype=torch.float64, device="cuda")
    p = torch.zeros(s.cell_shape, dtype=torch.float64, device="cuda")
    x = None
    cycles = []
    for t in range(30):
        u, v, p, x, st = s.step(u, v, p, 1.0, 0.1, walls, x)
        assert st["status"] == 0
        cycles.append(st["cycles"])
        d = host(s.div(u, v))
        assert np.abs(d).max() < 1e-6 * U, (t, np.abs(d).max())
    uh, vh = host(u)[0], host(v)[0]
    assert np.isfinite(uh).all() and np.isfinite(vh).all()
    # next to the south wall the fluid is dragged along +x, next to the north wall along -x
    assert uh[0, nx // 2] > 0.0 and uh[-1, nx // 2] < 0.0
    assert vh[ny // 2, -1] > 0.0 and vh[ny // 2, 0] < 0.0
    # (the first step's right-hand side vanishes: the four sliding walls' corner
    # divergences cancel, so that solve takes no cycle)
    print("cycles per step", cycles, flush=True)
    assert cycles[0] == 0 and max(cycles[1:]) > 0
