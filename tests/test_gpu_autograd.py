"""The differentiable projection u -> u - G A^+ (D u - mean) and its hand-written backward
(adjoint ISM solve + D^T), checked against central finite differences and against the
oracle's dense and spectral adjoints."""
import numpy as np
import pytest
import torch

from oracle import ism_oracle as O
from paper_1309_7128_amd import inputs
from tests.gpu_util import announce, dev, host, solver

pytestmark = pytest.mark.gpu
N, P, D = O.NEUMANN, O.PERIODIC, O.DIRICHLET
ND = O.NEUMANN_DIRICHLET


def _oracle_grad(w_u, w_v, h, exact, bx=N, by=N):
    """d/du sum(w . (u - G A^+ Pi D u)) = w - D^T A^+ Pi G^T w (A, A^+ symmetric; Pi is the
    mean removal when A is singular, else the identity)."""
    g = O.grad_adjoint(w_u, w_v, h, bx, by)
    lam = exact(g)
    du, dv = O.div_adjoint(lam, h, bx)
    return w_u - du, w_v - dv


def test_fd_and_dense_adjoint_64():
    announce("fd64")
    from paper_1309_7128_amd.autograd import project

    nx = ny = 64
    u0, v0 = inputs.uniform_faces(7, nx, ny)
    rng = np.random.default_rng(8)
    wu, wv = rng.standard_normal(u0.shape), rng.standard_normal(v0.shape)
    s = solver(nx=nx, ny=ny, coarsen=16, precision="fp64", rtol=1e-12)
    h = s.h
    u = dev(u0).requires_grad_(True)
    v = dev(v0).requires_grad_(True)
    un, vn, p = project(u, v, s)
    loss = (dev(wu) * un).sum() + (dev(wv) * vn).sum()
    loss.backward()
    gu, gv = host(u.grad), host(v.grad)
    # dense adjoint (oracle)
    ru, rv = _oracle_grad(wu, wv, h, lambda g: O.dense_solve(g, h))
    scale = np.sqrt(np.sum(ru**2) + np.sum(rv**2))
    err = np.sqrt(np.sum((gu - ru) ** 2) + np.sum((gv - rv) ** 2)) / scale
    assert err < 1e-6, err
    # 32 directional central differences of the loss computed by the GPU forward
    dirs = np.random.default_rng(9)
    eps = 1e-3

    def L(uu, vv):
        with torch.no_grad():
            a, c, _ = project(dev(uu), dev(vv), s)
            return float((dev(wu) * a).sum() + (dev(wv) * c).sum())

    for _ in range(32):
        du, dv = dirs.standard_normal(u0.shape), dirs.standard_normal(v0.shape)
        fd = (L(u0 + eps * du, v0 + eps * dv) - L(u0 - eps * du, v0 - eps * dv)) / (2 * eps)
        an = np.sum(gu * du) + np.sum(gv * dv)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.sqrt(np.sum(du**2) + np.sum(dv**2)) * scale), (fd, an)


def test_fd_and_dense_adjoint_dirichlet_64():
    """The same gradient checks with zero-pressure walls (periodic x, Neumann bottom,
    Dirichlet top): the wall faces of the top carry the gradient 2 p / h."""
    announce("fd64_dirichlet")
    from paper_1309_7128_amd.autograd import project

    nx = ny = 64
    s = solver(nx=nx, ny=ny, coarsen=16, precision="fp64", rtol=1e-12, bc_x=P, bc_y=ND)
    h = s.h
    rng = np.random.default_rng(10)
    u0, v0 = rng.uniform(-1, 1, s.u_shape[1:]), rng.uniform(-1, 1, s.v_shape[1:])
    wu, wv = rng.standard_normal(u0.shape), rng.standard_normal(v0.shape)
    u = dev(u0).requires_grad_(True)
    v = dev(v0).requires_grad_(True)
    un, vn, p = project(u, v, s)
    # exactly divergence-free: with a Dirichlet face there is no mean to leave behind
    bn = O.div(host(un).reshape(u0.shape), host(vn).reshape(v0.shape), h, P)
    assert np.abs(bn).max() <= 1e-9 * np.abs(O.div(u0, v0, h, P)).max()
    loss = (dev(wu) * un).sum() + (dev(wv) * vn).sum()
    loss.backward()
    gu, gv = host(u.grad), host(v.grad)
    ru, rv = _oracle_grad(wu, wv, h, lambda g: O.dense_solve(g, h, P, ND), P, ND)
    scale = np.sqrt(np.sum(ru**2) + np.sum(rv**2))
    err = np.sqrt(np.sum((gu - ru) ** 2) + np.sum((gv - rv) ** 2)) / scale
    assert err < 1e-6, err

    def L(uu, vv):
        with torch.no_grad():
            a, c, _ = project(dev(uu), dev(vv), s)
            return float((dev(wu) * a).sum() + (dev(wv) * c).sum())

    dirs = np.random.default_rng(11)
    for _ in range(8):
        du, dv = dirs.standard_normal(u0.shape), dirs.standard_normal(v0.shape)
        fd = (L(u0 + 1e-3 * du, v0 + 1e-3 * dv) - L(u0 - 1e-3 * du, v0 - 1e-3 * dv)) / 2e-3
        an = np.sum(gu * du) + np.sum(gv * dv)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.sqrt(np.sum(du**2) + np.sum(dv**2)) * scale), (fd, an)


def test_projection_is_divergence_free():
    announce("divfree")
    from paper_1309_7128_amd.autograd import project

    nx, ny = 128, 96
    u0, v0 = inputs.smooth64(21, nx, ny, ly=ny / nx)
    s = solver(nx=nx, ny=ny, coarsen=16, precision="mixed", rtol=1e-10)
    un, vn, p = project(dev(u0), dev(v0), s)
    b = O.div(u0, v0, s.h)
    bn = O.div(host(un).reshape(u0.shape), host(vn).reshape(v0.shape), s.h)
    # what remains is the mean of the divergence (the net boundary flux)
    assert np.abs(bn - b.mean()).max() <= 1e-9 * np.abs(b).max()


def test_batch8x1024_gradient_vs_spectral_adjoint():
    announce("batch8x1024_grad")
    from paper_1309_7128_amd.autograd import project

    w = inputs.WORKLOADS["batch8x1024_mixed"]
    s = solver(nx=w.nx, ny=w.ny, batch=w.batch, coarsen=w.coarsen, precision="mixed", rtol=w.rtol)
    uv = [inputs.workload_fields(w.name, k) for k in range(w.batch)]
    ww = [inputs.batch_weights(k, uv[0][0].shape, uv[0][1].shape) for k in range(w.batch)]
    u = dev(np.stack([a for a, _ in uv])).requires_grad_(True)
    v = dev(np.stack([c for _, c in uv])).requires_grad_(True)
    wu = dev(np.stack([a for a, _ in ww]))
    wv = dev(np.stack([c for _, c in ww]))
    un, vn, p = project(u, v, s)
    ((wu * un).sum() + (wv * vn).sum()).backward()
    gu, gv = host(u.grad), host(v.grad)
    for k in range(w.batch):
        ru, rv = _oracle_grad(ww[k][0], ww[k][1], w.h, lambda g: O.exact_solve(g, w.h, refine=1))
        scale = np.sqrt(np.sum(ru**2) + np.sum(rv**2))
        err = np.sqrt(np.sum((gu[k] - ru) ** 2) + np.sum((gv[k] - rv) ** 2)) / scale
        print(k, f"grad rel err {err:.3e}", flush=True)
        assert err < 1e-6
