"""Plain CPU oracle of the interpolated stencil multigrid (ISM) pressure solve.

TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the CPU-baseline
leg of the benchmark may import this module.  The HIP library and its Python binding never
call it and it calls nothing of theirs: the two share no code, tables or constants.

Paper: G. Tegze and G. I. Toth, "A GPU cluster optimized multigrid scheme for computing
unsteady incompressible fluid flow".  Every function names the passage it follows.  The
pins that tie each function to something other than itself live in
``tests/test_oracle_pins.py``; a function without such a pin says "parity unpinned".

Conventions
-----------
* Fine grid of nx x ny cells of size h; arrays have shape (ny, nx): row j, column i,
  0-based, i along x.  Batches are handled by the caller, one grid at a time.
* ``laplacian`` is A' = h^2 A, the 5-point cell-centred Laplacian in difference form,
  (A'p)_C = (p_W - p_C) + (p_E - p_C) + (p_S - p_C) + (p_N - p_C), summed in that order.
  A periodic axis wraps.  Each face of a non-periodic axis is a wall of one of the two
  kinds Sec. 4.1 names besides periodic: "symmetric" (read as a homogeneous Neumann wall:
  the neighbour behind it contributes no term) or Dirichlet (zero pressure on the wall,
  read as the mirror ghost p_ghost = -p_C, so its term is (-p_C) - p_C).
* The pressure equation of Eq. 4 is solved as A x = b~.  Without a Dirichlet face the
  constants span the null space: then b~ = b - mean(b) and the solution returned is the
  zero-mean one.  With a Dirichlet face A is nonsingular and b~ = b.
* Coarse grid: tiles of n x n fine cells (Sec. 4: one work-group per coarse cell), coarse
  cell (J, I) covers rows nJ..nJ+n-1 and columns nI..nI+n-1; its centre is the tile centre
  (Fig. 1).
* Float arithmetic follows the dtype of the arrays passed in: float64 arrays give FP64
  arithmetic, float32 arrays give FP32 arithmetic (used to emulate the FP32 inner solve).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg

NEUMANN = "neumann"
PERIODIC = "periodic"
DIRICHLET = "dirichlet"                  # both faces of the axis
NEUMANN_DIRICHLET = "neumann-dirichlet"  # low face (west / south) Neumann, high face Dirichlet
DIRICHLET_NEUMANN = "dirichlet-neumann"  # low face Dirichlet, high face Neumann

_FACES = {NEUMANN: ("N", "N"), DIRICHLET: ("D", "D"), NEUMANN_DIRICHLET: ("N", "D"),
          DIRICHLET_NEUMANN: ("D", "N"), PERIODIC: None}


def faces(bc):
    """(low face, high face) of an axis, each "N" (no-flux wall) or "D" (zero-pressure
    wall); None for a periodic axis."""
    return _FACES[bc]


def singular(bc_x, bc_y):
    """True when A has the constants in its null space: no face is a Dirichlet wall."""
    return all(f is None or "D" not in f for f in (faces(bc_x), faces(bc_y)))


# --------------------------------------------------------------------------------------
# Fine-grid operators (Sec. 2.3: staggered grid, five-point pressure Laplacian)
# --------------------------------------------------------------------------------------

def _neighbours(p, bc_x, bc_y):
    """Values of the W, E, S, N neighbour of every cell, whether that neighbour exists, and
    whether the face towards it is a Dirichlet wall.

    A missing neighbour (behind a wall) has value 0 and ``present`` False."""
    zero = np.zeros((), dtype=p.dtype)
    out = {}
    for axis, bc, (lo_key, hi_key) in ((1, bc_x, ("W", "E")), (0, bc_y, ("S", "N"))):
        f = faces(bc)
        if f is None:
            allp = np.ones(p.shape, dtype=bool)
            none = np.zeros(p.shape, dtype=bool)
            out[lo_key] = (np.roll(p, 1, axis=axis), allp, none)
            out[hi_key] = (np.roll(p, -1, axis=axis), allp, none)
            continue
        lo = np.full_like(p, zero)
        hi = np.full_like(p, zero)
        plo = np.zeros(p.shape, dtype=bool)
        phi = np.zeros(p.shape, dtype=bool)
        dlo = np.zeros(p.shape, dtype=bool)
        dhi = np.zeros(p.shape, dtype=bool)
        if axis == 1:
            lo[:, 1:], plo[:, 1:], dlo[:, 0] = p[:, :-1], True, f[0] == "D"
            hi[:, :-1], phi[:, :-1], dhi[:, -1] = p[:, 1:], True, f[1] == "D"
        else:
            lo[1:, :], plo[1:, :], dlo[0, :] = p[:-1, :], True, f[0] == "D"
            hi[:-1, :], phi[:-1, :], dhi[-1, :] = p[1:, :], True, f[1] == "D"
        out[lo_key] = (lo, plo, dlo)
        out[hi_key] = (hi, phi, dhi)
    return out


def laplacian(p, bc_x=NEUMANN, bc_y=NEUMANN):
    """A'p: the sum of (p_nb - p_C) over the four faces, added as (W + E) + (S + N).

    Sec. 2.3 (five-point Laplacian) and Sec. 3.3 (its finite-volume reading: a sum of face
    fluxes).  A Neumann wall face carries no flux; a Dirichlet wall face carries
    (-p_C) - p_C, its ghost being the mirror -p_C (Sec. 4.1 lists Dirichlet walls).  Pinned
    by the closed-form eigenpairs of the discrete Laplacian and by an independently
    assembled dense matrix."""
    nb = _neighbours(p, bc_x, bc_y)
    zero = np.zeros((), dtype=p.dtype)
    d = {k: np.where(pres, val - p, np.where(dw, (-p) - p, zero))
         for k, (val, pres, dw) in nb.items()}
    return (d["W"] + d["E"]) + (d["S"] + d["N"])


def neighbour_count(nx, ny, bc_x=NEUMANN, bc_y=NEUMANN):
    """m_C, the magnitude of A's diagonal: 4, less one for each Neumann wall face of the
    cell, plus one for each Dirichlet wall face (its ghost -p_C adds a second -p_C)."""
    m = np.full((ny, nx), 4, dtype=np.int64)
    for bc, lo, hi in ((bc_x, (slice(None), 0), (slice(None), -1)),
                       (bc_y, (0, slice(None)), (-1, slice(None)))):
        f = faces(bc)
        if f is None:
            continue
        m[lo] += 1 if f[0] == "D" else -1
        m[hi] += 1 if f[1] == "D" else -1
    return m


def red_black_gs(p, rhs, bc_x=NEUMANN, bc_y=NEUMANN, sweeps=1):
    """Red-black Gauss-Seidel sweeps on A'p = rhs (Sec. 3.1; used on the fine grid, Sec. 4).

    A sweep updates the red cells ((i + j) even) and then the black cells.  A cell is set
    so that its own equation holds: p_C = (sum of existing neighbour values - rhs_C) / m_C,
    with the neighbour values added as (W + E) + (S + N) (a neighbour behind a wall
    counting 0), m_C the diagonal of ``neighbour_count`` and the division taken as a
    product with 1/m_C rounded to the working precision.  No over-relaxation factor is
    given in the paper; this is plain Gauss-Seidel.  Pinned by a cell-by-cell sequential
    sweep in red-black order on tiny grids and by the fixed point being the exact
    solution."""
    p = np.array(p, copy=True)
    rhs = np.asarray(rhs, dtype=p.dtype)
    ny, nx = p.shape
    m = neighbour_count(nx, ny, bc_x, bc_y)
    inv_m = np.ones((), dtype=p.dtype) / m.astype(p.dtype)
    jj, ii = np.indices((ny, nx))
    red = (ii + jj) % 2 == 0
    for _ in range(sweeps):
        for colour in (red, ~red):
            nb = _neighbours(p, bc_x, bc_y)
            s = (nb["W"][0] + nb["E"][0]) + (nb["S"][0] + nb["N"][0])
            new = (s - rhs) * inv_m
            p = np.where(colour, new, p)
    return p


# --------------------------------------------------------------------------------------
# MAC divergence and gradient (Sec. 2.2 projection step, Sec. 2.3 staggered grid)
# --------------------------------------------------------------------------------------

def div(u, v, h, bc_x=NEUMANN):
    """D[u; v]: cell divergence of face velocities, ((u_e - u_w) + (v_n - v_s)) / h.

    u has shape (ny, nx+1) (or (ny, nx) when periodic in x), v has shape (ny+1, nx).
    Pinned by the discrete divergence theorem and by D G = A."""
    if bc_x == PERIODIC:
        du = np.roll(u, -1, axis=1) - u
    else:
        du = u[:, 1:] - u[:, :-1]
    dv = v[1:, :] - v[:-1, :]
    return (du + dv) / h


def grad(p, h, bc_x=NEUMANN, bc_y=NEUMANN):
    """G p on the faces: (p_C - p_{west or south neighbour}) / h.

    A Neumann wall face carries no pressure gradient; on a Dirichlet wall face the missing
    neighbour is the mirror ghost -p, so the face gets (p - (-p)) / h on the west or south
    wall and ((-p) - p) / h on the east or north wall.  This is what makes D G equal to
    the cell-centred Laplacian with the same walls.  Pinned by D G = A."""
    ny, nx = p.shape
    if bc_x == PERIODIC:
        gu = (p - np.roll(p, 1, axis=1)) / h
    else:
        fx = faces(bc_x)
        gu = np.zeros((ny, nx + 1), dtype=p.dtype)
        gu[:, 1:nx] = (p[:, 1:] - p[:, :-1]) / h
        if fx[0] == "D":
            gu[:, 0] = (p[:, 0] - (-p[:, 0])) / h
        if fx[1] == "D":
            gu[:, nx] = ((-p[:, -1]) - p[:, -1]) / h
    gv = np.zeros((ny + 1, nx), dtype=p.dtype)
    if bc_y == PERIODIC:
        raise NotImplementedError("v faces are stored with ny+1 rows; periodic y is not used")
    fy = faces(bc_y)
    gv[1:ny, :] = (p[1:, :] - p[:-1, :]) / h
    if fy[0] == "D":
        gv[0, :] = (p[0, :] - (-p[0, :])) / h
    if fy[1] == "D":
        gv[ny, :] = ((-p[-1, :]) - p[-1, :]) / h
    return gu, gv


def div_adjoint(lam, h, bc_x=NEUMANN):
    """D^T lam, the transpose of ``div``: for an x-face f, (lam_{f-1} - lam_f) / h with the
    term of a missing cell left out.  Pinned by the dot-product identity
    <D w, lam> = <w, D^T lam>."""
    ny, nx = lam.shape
    if bc_x == PERIODIC:
        gu = (np.roll(lam, 1, axis=1) - lam) / h
    else:
        gu = np.zeros((ny, nx + 1), dtype=lam.dtype)
        gu[:, 1:] += lam
        gu[:, :-1] -= lam
        gu /= h
    gv = np.zeros((ny + 1, nx), dtype=lam.dtype)
    gv[1:, :] += lam
    gv[:-1, :] -= lam
    gv /= h
    return gu, gv


def grad_adjoint(gu, gv, h, bc_x=NEUMANN, bc_y=NEUMANN):
    """G^T w, the transpose of ``grad`` (a Dirichlet wall face adds twice its value to the
    cell next to it, with the sign of its gradient).  Pinned by <G p, w> = <p, G^T w>."""
    ny = gv.shape[0] - 1
    nx = gv.shape[1]
    out = np.zeros((ny, nx), dtype=gv.dtype)
    if bc_x == PERIODIC:
        out += gu - np.roll(gu, -1, axis=1)
    else:
        fx = faces(bc_x)
        out[:, 1:] += gu[:, 1:nx]
        out[:, :-1] -= gu[:, 1:nx]
        if fx[0] == "D":
            out[:, 0] += 2.0 * gu[:, 0]
        if fx[1] == "D":
            out[:, -1] -= 2.0 * gu[:, nx]
    fy = faces(bc_y)
    out[1:, :] += gv[1:ny, :]
    out[:-1, :] -= gv[1:ny, :]
    if fy[0] == "D":
        out[0, :] += 2.0 * gv[0, :]
    if fy[1] == "D":
        out[-1, :] -= 2.0 * gv[ny, :]
    return out / h


def predictor(u, v, p, h, dt, eta, bc_x=NEUMANN, walls=(0.0, 0.0, 0.0, 0.0)):
    """The explicit predictor of Goda's scheme (Sec. 2.2, Eq. 3) on the staggered grid with
    second-order central differences (Sec. 2.3):

        v* = v + dt (-(v . grad) v + eta lap v) - G p,

    p carrying the time step (p = dt times the pressure, so that the projection's solution
    x of A x = D v* updates it as p + x and the velocity as v* - G x).  The signs of Eq. 1
    and Eq. 3 are garbled in the text; this is the standard form they stand for.

    Layout as ``div``: u (ny, nx+1) (or (ny, nx) periodic in x), v (ny+1, nx).  At an interior
    u face (west face of cell (i, j)):
      dudx = (u_E - u_W) / (2h), dudy = (u_N - u_S) / (2h), lap = (((u_E + u_W) + u_N) + u_S
      - 4 u) / h^2, vbar = ((v_SW + v_SE) + (v_NW + v_NE)) / 4 (the four v faces around it),
      u* = u + dt (eta lap - (u dudx + vbar dudy)) - (p_C - p_W) / h,
    and the v faces alike with x and y exchanged (ubar from the four u faces around it).
    Walls: the normal velocity on a wall face is kept; a tangential neighbour behind a wall
    is the ghost 2 U_w - (the face's own value), U_w the wall's tangential velocity
    (walls = (v on the west wall, v on the east wall, u on the south wall, u on the north
    wall)); a periodic x axis wraps.  Returns (u*, v*).  Pinned by exactness on linear
    fields, second-order consistency and by the projection step."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    ny, nx = p.shape
    per = bc_x == PERIODIC
    vw, ve, us, un = (float(a) for a in walls)
    us_, vs_ = u.copy(), v.copy()
    two_h, hh = 2.0 * h, h * h
    # ---- u faces
    irange = range(nx) if per else range(1, nx)
    for j in range(ny):
        for i in irange:
            c = u[j, i]
            ue = u[j, (i + 1) % nx] if per else u[j, i + 1]
            uw = u[j, (i - 1) % nx] if per else u[j, i - 1]
            un_ = u[j + 1, i] if j + 1 < ny else 2.0 * un - c
            us_v = u[j - 1, i] if j > 0 else 2.0 * us - c
            im = (i - 1) % nx
            vbar = ((v[j, im] + v[j, i % nx]) + (v[j + 1, im] + v[j + 1, i % nx])) / 4.0
            dudx = (ue - uw) / two_h
            dudy = (un_ - us_v) / two_h
            lap = ((((ue + uw) + un_) + us_v) - 4.0 * c) / hh
            gp = (p[j, i % nx] - p[j, im]) / h
            us_[j, i] = c + dt * (eta * lap - (c * dudx + vbar * dudy)) - gp
    # ---- v faces (the wall rows j = 0 and j = ny keep their normal velocity)
    for j in range(1, ny):
        for i in range(nx):
            c = v[j, i]
            vn = v[j + 1, i]
            vs = v[j - 1, i]
            if per:
                ve_, vw_ = v[j, (i + 1) % nx], v[j, (i - 1) % nx]
            else:
                ve_ = v[j, i + 1] if i + 1 < nx else 2.0 * ve - c
                vw_ = v[j, i - 1] if i > 0 else 2.0 * vw - c
            ip = (i + 1) % nx if per else i + 1
            ubar = ((u[j - 1, i] + u[j - 1, ip]) + (u[j, i] + u[j, ip])) / 4.0
            dvdx = (ve_ - vw_) / two_h
            dvdy = (vn - vs) / two_h
            lap = ((((ve_ + vw_) + vn) + vs) - 4.0 * c) / hh
            gp = (p[j, i] - p[j - 1, i]) / h
            vs_[j, i] = c + dt * (eta * lap - (ubar * dvdx + c * dvdy)) - gp
    return us_, vs_


def projection_step(u, v, p, h, dt, eta, bc_x=NEUMANN, walls=(0.0, 0.0, 0.0, 0.0)):
    """One time step of Goda's incremental projection scheme (Sec. 2.2): the predictor
    (Eq. 3), the pressure-change equation A x = D v* (Eq. 4, solved exactly here), then
    v^{t+1} = v* - G x and p^{t+1} = p + x.  Returns (u, v, p)."""
    us, vs = predictor(u, v, p, h, dt, eta, bc_x, walls)
    b = div(us, vs, h, bc_x)
    x = exact_solve(b, h, bc_x, NEUMANN)
    gu, gv = grad(x, h, bc_x, NEUMANN)
    return us - gu, vs - gv, p + x


# --------------------------------------------------------------------------------------
# Grid transfer (Sec. 3.3, Eq. 5)
# --------------------------------------------------------------------------------------

def tile_layout(nf, n):
    """The coarse cells along one axis of nf fine cells (Sec. 3.3, Sec. 4.1): tiles of n
    cells from cell 0 on, the last one short when n does not divide nf (the padded domain:
    that coarse cell covers only the cells that exist).  Returns (nc, sizes, starts,
    centres); a coarse centre is the middle of its tile, in fine coordinates where fine cell
    i spans [i, i + 1]."""
    nc = -(-nf // n)
    sizes = np.full(nc, n, dtype=np.int64)
    sizes[-1] = nf - (nc - 1) * n
    starts = np.arange(nc, dtype=np.int64) * n
    return nc, sizes, starts, starts + sizes / 2.0


def restrict_sum(r, n):
    """R r: the sum of the fine values over each coarse tile (n x n, shorter in the last
    row or column of tiles when n does not divide the grid), in FP64.

    Sec. 3.3: the coarse right-hand side is the sum of quantities already computed on the
    fine grid (the agglomeration of ACM).  Pinned by conservation (sum R r = sum r) and by
    brute force."""
    ny, nx = r.shape
    r = np.asarray(r, dtype=np.float64)
    if nx % n == 0 and ny % n == 0:
        return r.reshape(ny // n, n, nx // n, n).sum(axis=(1, 3))
    sx, sy = tile_layout(nx, n)[2], tile_layout(ny, n)[2]
    return np.add.reduceat(np.add.reduceat(r, sy, axis=0), sx, axis=1)


def _interp_axis(nf, n, bc):
    """For every fine index along one axis: lower and upper coarse centre, the weight of
    the upper one (Eq. 5 coordinates divided by the rectangle size) and the sign each
    centre value is taken with.

    The coarse centre I sits in the middle of its tile (n (I + 1/2) for a full tile); fine
    centre i sits at i + 1/2.  Between a wall and the first (last) coarse centre the
    rectangle reaches a ghost centre, the mirror image of that centre in the wall: an equal
    value behind a Neumann wall (the interpolant is held constant, zero normal slope) and the
    negated value behind a Dirichlet wall (the interpolant falls linearly to zero on the
    wall).  On a periodic axis the neighbour across the seam is the wrapped centre.  With a
    short last tile the rectangles next to it are shorter than n (Eq. 5: the rectangle size
    can differ because of padding), and t is the offset divided by the rectangle's size."""
    nc, _, _, c = tile_layout(nf, n)
    pos = np.arange(nf) + 0.5
    if nf % n == 0:  # uniform tiles: rectangles of n cells
        p = pos / n - 0.5
        lo = np.floor(p).astype(np.int64)
        t = p - lo
    else:
        lo = np.searchsorted(c, pos, side="right").astype(np.int64) - 1
        below = c[-1] - nf if bc == PERIODIC else -c[0]      # the centre before centre 0
        above = c[0] + nf if bc == PERIODIC else 2 * nf - c[-1]  # the centre after the last
        cl = np.where(lo < 0, below, c[np.clip(lo, 0, nc - 1)])
        ch = np.where(lo + 1 > nc - 1, above, c[np.clip(lo + 1, 0, nc - 1)])
        t = (pos - cl) / (ch - cl)
    hi = lo + 1
    s_lo = np.ones(nf)
    s_hi = np.ones(nf)
    if bc == PERIODIC:
        lo %= nc
        hi %= nc
    else:
        f = faces(bc)
        if f[0] == "D":
            s_lo[lo < 0] = -1.0
        if f[1] == "D":
            s_hi[hi > nc - 1] = -1.0
        lo = np.clip(lo, 0, nc - 1)
        hi = np.clip(hi, 0, nc - 1)
    return lo, hi, t, s_lo, s_hi


def prolong_bilinear(E, n, bc_x=NEUMANN, bc_y=NEUMANN, dtype=np.float64, fine_shape=None):
    """P E: bilinear interpolation of the coarse values to every fine cell centre.

    Eq. 5 with origin at the south-west centre Q11 of the surrounding rectangle, in
    coordinates scaled by the rectangle size: p = Q11 (1-x)(1-y) + Q21 x (1-y) + Q12 (1-x) y
    + Q22 x y, evaluated in nested form, first along x on the lower and upper coarse rows,
    then along y: p = (Q11 (1-x) + Q21 x)(1-y) + (Q12 (1-x) + Q22 x) y.  The same
    interpolation serves the coarse stencil and the prolongation (Sec. 3.3).

    dtype is the fine arithmetic.  The x step works on coarse rows (coarse-grid data, FP64)
    and is rounded to dtype; the y step, one per fine cell, is evaluated in dtype.  In FP64
    this is the plain FP64 evaluation.  fine_shape (ny, nx) gives a grid that n does not
    divide (short last tiles); by default the tiles are full.  Pinned by exactness on
    constants and bilinear fields, dyadic weights and the coarse-stencil identities (FP64),
    and by the FP32 result lying within its rounding bound of the FP64 one."""
    ncy, ncx = E.shape
    ny, nx = (ncy * n, ncx * n) if fine_shape is None else fine_shape
    ilo, ihi, tx, sxl, sxh = _interp_axis(nx, n, bc_x)
    jlo, jhi, ty, syl, syh = _interp_axis(ny, n, bc_y)
    E = np.asarray(E, dtype=np.float64)
    # along x, every coarse row (a ghost centre's value negated exactly by its sign)
    ex = (E[:, ilo] * sxl[None, :]) * (1 - tx)[None, :] + (E[:, ihi] * sxh[None, :]) * tx[None, :]
    ex = ex.astype(dtype)
    # along y in dtype (the weights are dyadic and the signs +-1, both exact in either type)
    wl, wh = (1 - ty).astype(dtype)[:, None], ty.astype(dtype)[:, None]
    sl, sh = syl.astype(dtype)[:, None], syh.astype(dtype)[:, None]
    return (ex[jlo, :] * sl) * wl + (ex[jhi, :] * sh) * wh


def inject_constant(E, n):
    """P0 E: piecewise-constant injection (ACM adds the coarse value to every fine cell of
    its block, Sec. 3.2)."""
    return np.kron(np.asarray(E, dtype=np.float64), np.ones((n, n)))


# --------------------------------------------------------------------------------------
# Coarse operators (Sec. 3.2 ACM agglomeration, Sec. 3.3 interpolated stencil)
# --------------------------------------------------------------------------------------

def _fold(C, ncx, ncy, bc_x, bc_y):
    """Move the coefficient of an off-grid (ghost) neighbour behind a wall onto the cell
    whose mirror image it is: added for a Neumann wall (equal ghost), subtracted for a
    Dirichlet wall (negated ghost)."""
    C = C.copy()
    fx, fy = faces(bc_x), faces(bc_y)
    if fx is not None:
        sw, se = (-1.0 if f == "D" else 1.0 for f in fx)
        C[:, 0, :, 1] += sw * C[:, 0, :, 0]
        C[:, 0, :, 0] = 0.0
        C[:, -1, :, 1] += se * C[:, -1, :, 2]
        C[:, -1, :, 2] = 0.0
    if fy is not None:
        ss, sn = (-1.0 if f == "D" else 1.0 for f in fy)
        C[0, :, 1, :] += ss * C[0, :, 0, :]
        C[0, :, 0, :] = 0.0
        C[-1, :, 1, :] += sn * C[-1, :, 2, :]
        C[-1, :, 2, :] = 0.0
    return C


def _open_faces(ncx, ncy, bc_x, bc_y):
    """Masks over the coarse cells: which of the E, W, N, S faces carry a flux (interior
    faces, periodic wraps and Dirichlet walls; a Neumann wall carries none)."""
    J, I = np.indices((ncy, ncx))
    fx, fy = faces(bc_x), faces(bc_y)
    per_x, per_y = fx is None, fy is None
    east = (I < ncx - 1) | per_x | (not per_x and fx[1] == "D")
    west = (I > 0) | per_x | (not per_x and fx[0] == "D")
    north = (J < ncy - 1) | per_y | (not per_y and fy[1] == "D")
    south = (J > 0) | per_y | (not per_y and fy[0] == "D")
    return east, west, north, south


def _centre(c, I, nf, bc):
    """Position of coarse centre I on an axis with centres c, for I in -1 .. nc: the ghost
    centres beyond the ends are the mirror images in the walls, or the wrapped centres on a
    periodic axis."""
    nc = len(c)
    if 0 <= I < nc:
        return c[I]
    if bc == PERIODIC:
        return c[-1] - nf if I < 0 else c[0] + nf
    return -c[0] if I < 0 else 2 * nf - c[-1]


def _coarse_stencil_ism_padded(nx, ny, n, bc_x, bc_y):
    """The Eq. 6/7 face sums of ``coarse_stencil_ism`` on a grid that n does not divide:
    the same sums, with each rectangle's own size (Eq. 5: the sizes differ next to a short
    last tile), written face by face and fine face by fine face."""
    ncx, sx, stx, cx = tile_layout(nx, n)
    ncy, sy, sty, cy = tile_layout(ny, n)
    C = np.zeros((ncy, ncx, 3, 3))
    east_open, west_open, north_open, south_open = _open_faces(ncx, ncy, bc_x, bc_y)

    def interp(c, k, nf, bc, I):
        """fine cell k of tile I along the other axis: lower centre offset (-1 or 0
        relative to I) and the weight of the upper centre"""
        pos = k + 0.5
        off = -1 if pos < c[I] else 0
        lo, hi = _centre(c, I + off, nf, bc), _centre(c, I + off + 1, nf, bc)
        return off, (pos - lo) / (hi - lo)

    for J in range(ncy):
        for I in range(ncx):
            # east (+1) and west (-1) faces: the fine rows of tile J
            for sign, is_open, d_lo in ((+1.0, east_open[J, I], 0), (-1.0, west_open[J, I], -1)):
                if not is_open:
                    continue
                dx = _centre(cx, I + d_lo + 1, nx, bc_x) - _centre(cx, I + d_lo, nx, bc_x)
                for k in range(sty[J], sty[J] + sy[J]):
                    off, y = interp(cy, k, ny, bc_y, J)
                    for dj, w in ((off, 1.0 - y), (off + 1, y)):
                        C[J, I, dj + 1, d_lo + 2] += sign * w / dx
                        C[J, I, dj + 1, d_lo + 1] -= sign * w / dx
            # north (+1) and south (-1) faces: the fine columns of tile I
            for sign, is_open, d_lo in ((+1.0, north_open[J, I], 0), (-1.0, south_open[J, I], -1)):
                if not is_open:
                    continue
                dy = _centre(cy, J + d_lo + 1, ny, bc_y) - _centre(cy, J + d_lo, ny, bc_y)
                for k in range(stx[I], stx[I] + sx[I]):
                    off, x = interp(cx, k, nx, bc_x, I)
                    for di, w in ((off, 1.0 - x), (off + 1, x)):
                        C[J, I, d_lo + 2, di + 1] += sign * w / dy
                        C[J, I, d_lo + 1, di + 1] -= sign * w / dy
    return _fold(C, ncx, ncy, bc_x, bc_y)


def coarse_stencil_ism(ncx, ncy, n, bc_x=NEUMANN, bc_y=NEUMANN, fine_shape=None):
    """The ISM coarse 9-point stencil, built by summing interpolated face fluxes.

    Sec. 3.3, Eq. 6 and Eq. 7.  For every coarse cell the equation is the sum, over the
    fine faces that lie on its four faces, of the outward pressure gradient of the
    bilinear interpolant of the coarse unknowns (interior fine fluxes cancel in the sum).
    On a face between centres I and I+1 in x, Eq. 6 gives for the fine row whose centre has
    scaled offset y from the lower centre Q11:
        dp/dx = ((Q21 - Q11)(1 - y) + (Q22 - Q12) y) / n      (in fine-cell units),
    and Eq. 7 the same with x and y exchanged.  A Neumann wall face carries no flux.  A
    Dirichlet wall face carries the Eq. 6 flux towards the negated ghost centre: the
    interpolant is linear through zero on the wall, so that flux equals the fine one,
    (-p) - p of the wall cell.

    Returns C with shape (ncy, ncx, 3, 3): C[J, I, dj+1, di+1] multiplies the unknown at
    (J+dj, I+di) (wrapped on a periodic axis).  fine_shape (ny, nx) gives a grid that n does
    not divide: its last tiles are short and so are the rectangles next to them.  Pinned by
    the brute-force product R A' P (with full and short tiles), the closed-form interior
    stencil 1/4 [[1,2,1],[2,-12,2],[1,2,1]] and the closed-form eigenvalues."""
    if fine_shape is not None and (fine_shape[0] != ncy * n or fine_shape[1] != ncx * n):
        ny, nx = fine_shape
        assert (ncy, ncx) == (tile_layout(ny, n)[0], tile_layout(nx, n)[0])
        return _coarse_stencil_ism_padded(nx, ny, n, bc_x, bc_y)
    C = np.zeros((ncy, ncx, 3, 3))
    J, I = np.indices((ncy, ncx))
    half = n // 2

    def add(mask, dj, di, val):
        # val is an array over (J, I) or a scalar; the stencil entry gets it where mask holds
        C[:, :, dj + 1, di + 1] += np.where(mask, val, 0.0)

    east_open, west_open, north_open, south_open = _open_faces(ncx, ncy, bc_x, bc_y)
    for k in range(n):
        # fine row nJ + k: lower interpolation centre J-1 (k < n/2) or J (k >= n/2)
        lo_off = -1 if k < half else 0
        y = (k + 0.5) / n - 0.5 - lo_off  # scaled offset from the lower centre
        w_lo, w_hi = (1.0 - y) / n, y / n
        for sign, mask, d_lo in ((+1.0, east_open, 0), (-1.0, west_open, -1)):
            # face between centres I + d_lo and I + d_lo + 1; outward sign +1 east, -1 west
            add(mask, lo_off, d_lo + 1, sign * w_lo)
            add(mask, lo_off, d_lo, -sign * w_lo)
            add(mask, lo_off + 1, d_lo + 1, sign * w_hi)
            add(mask, lo_off + 1, d_lo, -sign * w_hi)
        # fine column nI + k on the north and south faces (Eq. 7)
        x = y
        w_lo, w_hi = (1.0 - x) / n, x / n
        for sign, mask, d_lo in ((+1.0, north_open, 0), (-1.0, south_open, -1)):
            add(mask, d_lo + 1, lo_off, sign * w_lo)
            add(mask, d_lo, lo_off, -sign * w_lo)
            add(mask, d_lo + 1, lo_off + 1, sign * w_hi)
            add(mask, d_lo, lo_off + 1, -sign * w_hi)
    return _fold(C, ncx, ncy, bc_x, bc_y)


def coarse_stencil_acm(ncx, ncy, n, bc_x=NEUMANN, bc_y=NEUMANN):
    """ACM coarse stencil: the sum of the fine equations of a block with the pressure
    assumed constant over each coarse cell (Sec. 3.2; Sec. 3.3 contrasts it with ISM).

    Each of the n fine faces on a coarse face then carries E_nb - E_C, so the result is n
    times the 5-point stencil (Sec. 4: summing fine equations gives a 5-point stencil).
    Pinned by the brute-force product R A' P0."""
    C = np.zeros((ncy, ncx, 3, 3))
    east, west, north, south = _open_faces(ncx, ncy, bc_x, bc_y)
    opens = {(0, 1): east, (0, -1): west, (1, 0): north, (-1, 0): south}
    for (dj, di), mask in opens.items():
        for _ in range(n):  # one flux per fine face on the coarse face
            C[:, :, dj + 1, di + 1] += np.where(mask, 1.0, 0.0)
            C[:, :, 1, 1] -= np.where(mask, 1.0, 0.0)
    return _fold(C, ncx, ncy, bc_x, bc_y)


def coarse_stencil_gmg5(ncx, ncy, n, bc_x=NEUMANN, bc_y=NEUMANN):
    """Aggressive-coarsening GMG variant: the 5-point stencil rediscretized at spacing nh
    (Sec. 3.2 GMG; Sec. 4.3.2 compares ISM with this "five point coarse grid stencil").
    With the restriction summing h^2-scaled residuals (n^2 of them, so H^2 times the mean
    residual), the coarse equation in the same units has unit coefficients.  Pinned by the
    closed form K (x) I + I (x) K with each wall kind's end, its eigenpairs, and exactness
    H^2 lap p on quadratics."""
    return coarse_stencil_acm(ncx, ncy, 1, bc_x, bc_y)


def coarse_matrix(C, bc_x=NEUMANN, bc_y=NEUMANN):
    """Sparse matrix of a (ncy, ncx, 3, 3) stencil; unknown (J, I) has index J*ncx + I."""
    ncy, ncx = C.shape[:2]
    rows, cols, vals = [], [], []
    J, I = np.indices((ncy, ncx))
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            c = C[:, :, dj + 1, di + 1]
            jj = J + dj
            ii = I + di
            if bc_y == PERIODIC:
                jj %= ncy
            if bc_x == PERIODIC:
                ii %= ncx
            ok = (c != 0.0) & (jj >= 0) & (jj < ncy) & (ii >= 0) & (ii < ncx)
            rows.append((J * ncx + I)[ok])
            cols.append((jj * ncx + ii)[ok])
            vals.append(c[ok])
    N = ncx * ncy
    return scipy.sparse.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


class CoarseSolver:
    """Exact solve of A_c E = R_c (the limit of the paper's coarse iterations to a
    vanishing tolerance; a direct solve on the coarsest grid, Sec. 3.2).

    When the constants span the null space of A_c (no Dirichlet wall; detected from the
    row sums, or given), the system is bordered with the constraint sum(E) = 0, and the
    bordered solve returns the zero-mean E that satisfies A_c E = R_c - mean(R_c), the same
    projection as dropping the constant mode.  Otherwise A_c is nonsingular and is solved
    as it is.  Either system is factorized once by sparse LU (a library primitive).  The
    paper's host-side Gauss-Seidel to a tolerance is `gauss_seidel`."""

    def __init__(self, Ac, singular=None):
        N = Ac.shape[0]
        Ac = scipy.sparse.csr_matrix(Ac)
        if singular is None:
            singular = bool(np.allclose(np.asarray(Ac.sum(axis=1)).ravel(), 0.0, atol=1e-12))
        self.N = N
        self.Ac = Ac
        self.singular = singular
        if singular:
            ones = np.ones((N, 1))
            K = scipy.sparse.bmat([[Ac, ones], [ones.T, None]], format="csc")
        else:
            K = Ac.tocsc()
        self.lu = scipy.sparse.linalg.splu(K)

    def solve(self, Rc):
        shape = Rc.shape
        rhs = np.asarray(Rc, dtype=np.float64).ravel()
        if not self.singular:
            return self.lu.solve(rhs).reshape(shape)
        rhs = np.concatenate([rhs, [0.0]])
        return self.lu.solve(rhs)[: self.N].reshape(shape)

    def gauss_seidel(self, Rc, E0=None, tol_c=1e-6, max_iter=100000):
        """Lexicographic Gauss-Seidel on A_c E = R_c until the absolute maximum residual is
        below tol_c (Sec. 4: block-iterative GS on the host, which reduces to serial GS on
        one node; Sec. 4.3.1 accommodative criterion).  Returns (E, iterations).  An option of
        the oracle's ISM solve, not used by the library; pinned by Gauss-Seidel written row by
        row on the dense assembled matrix."""
        A = self.Ac
        b = np.asarray(Rc, dtype=np.float64).ravel()
        if self.singular:
            b = b - b.mean()
        E = np.zeros_like(b) if E0 is None else np.asarray(E0, dtype=np.float64).ravel().copy()
        L = scipy.sparse.tril(A, format="csr")
        U = A - L
        it = 0
        while np.max(np.abs(b - A @ E)) >= tol_c and it < max_iter:
            E = scipy.sparse.linalg.spsolve_triangular(L, b - U @ E, lower=True)
            it += 1
        return E.reshape(Rc.shape) - (E.mean() if self.singular else 0.0), it


def block_gauss_seidel(C, Rc, tol_c, block=16, bc_x=NEUMANN, bc_y=NEUMANN, E0=None,
                       max_iter=100000):
    """Block-iterative Gauss-Seidel on A_c E = R_c to an absolute tolerance (Sec. 4: the
    coarse grid is iterated by block GS, whose blocks run concurrently and which reduces to
    serial GS on a single block; Sec. 4.3.1: the coarse stage ends when the absolute maximum
    residual falls below its limit).

    The coarse grid is cut into tiles of block x block cells (or by x bx when block is a pair
    (by, bx)), aligned at cell 0 of each axis, that are updated concurrently.  Inside a tile
    the cells are visited in lexicographic order (I fastest), each set from its own equation
    with the tile's newest values; cells of other tiles keep their values from the previous
    iteration, so one iteration needs one synchronization.  On a periodic axis a neighbour is
    found by wrapping and belongs to whichever tile holds the wrapped cell.  A cell update is
    E_C = (R_C - sum over the 8 neighbours of c_nb E_nb) / c_C, the neighbours taken in the
    order (dj, di) = (-1,-1), (-1,0), (-1,1), (0,-1), (0,1), (1,-1), (1,0), (1,1) and the
    products summed left to right (C is the (ncy, ncx, 3, 3) stencil of ``coarse_stencil_*``;
    a periodic axis wraps).  Before each iteration the residual max|R_c - A_c E| is
    compared with tol_c.  Without a Dirichlet face R_c is first projected to zero mean, the
    compatibility condition of the singular system.  Returns (E, iterations).

    Pinned by a cell-by-cell loop in the same order (bitwise), by block = grid reducing to
    the lexicographic ``CoarseSolver.gauss_seidel`` and by convergence to the exact solve."""
    ncy, ncx = Rc.shape
    by, bx = (block, block) if np.isscalar(block) else (int(block[0]), int(block[1]))
    R = np.asarray(Rc, dtype=np.float64)
    if singular(bc_x, bc_y):
        R = R - R.mean()
    E = np.zeros((ncy, ncx)) if E0 is None else np.asarray(E0, dtype=np.float64).copy()
    per_x, per_y = faces(bc_x) is None, faces(bc_y) is None
    order = [(dj, di) for dj in (-1, 0, 1) for di in (-1, 0, 1) if (dj, di) != (0, 0)]
    J, I = np.indices((ncy, ncx))

    def neighbour(a, dj, di):
        """a at (J+dj, I+di) (0 off a walled grid, where the folded stencil has 0 too)."""
        jj, ii = J + dj, I + di
        if per_y:
            jj = jj % ncy
        if per_x:
            ii = ii % ncx
        ok = (jj >= 0) & (jj < ncy) & (ii >= 0) & (ii < ncx)
        return np.where(ok, a[np.clip(jj, 0, ncy - 1), np.clip(ii, 0, ncx - 1)], 0.0)

    def residual(E):
        acc = C[:, :, 1, 1] * E
        for dj, di in order:
            acc = acc + C[:, :, dj + 1, di + 1] * neighbour(E, dj, di)
        return R - acc

    # the visiting order inside a tile, and for each local position the cells it names
    # (one per tile) with their neighbours' flat indices and whether each lies in the tile
    flatE = np.arange(ncy * ncx).reshape(ncy, ncx)
    steps = []
    for lj in range(by):
        for li in range(bx):
            cj, ci = J[lj::by, li::bx].ravel(), I[lj::by, li::bx].ravel()
            if cj.size == 0:
                continue
            nbs = []
            for dj, di in order:
                jj, ii = cj + dj, ci + di
                if per_y:
                    jj = jj % ncy
                if per_x:
                    ii = ii % ncx
                ok = (jj >= 0) & (jj < ncy) & (ii >= 0) & (ii < ncx)
                jc, ic = np.clip(jj, 0, ncy - 1), np.clip(ii, 0, ncx - 1)
                same = ok & (jc // by == cj // by) & (ic // bx == ci // bx)
                nbs.append((flatE[jc, ic], ok, same, C[cj, ci, dj + 1, di + 1]))
            steps.append((flatE[cj, ci], nbs, C[cj, ci, 1, 1]))
    it = 0
    while np.max(np.abs(residual(E))) >= tol_c and it < max_iter:
        new, old = E.ravel().copy(), E.ravel()
        Rf = R.ravel()
        for cells, nbs, cc in steps:
            acc = np.zeros(cells.size)
            for idx, ok, same, c in nbs:
                acc = acc + c * np.where(same, new[idx], np.where(ok, old[idx], 0.0))
            new[cells] = (Rf[cells] - acc) / cc
        E = new.reshape(ncy, ncx)
        it += 1
    return E, it


def axis_colours(nc, bc):
    """Colour of each cell along one coarse axis for multicolour ordering of a 9-point
    stencil (Sec. 3.1: red-black ordering serves the 5-point stencil, multicolour ordering
    higher-order ones): cell i takes i mod 2, so that neighbours along the axis differ;
    on a periodic axis of odd length the last cell would share colour 0 with its wrapped
    neighbour 0, so it takes a third colour, 2.  Returns (colours, count)."""
    q = np.arange(nc) % 2
    if faces(bc) is None and nc % 2 == 1:
        q[-1] = 2
        return q, 3
    return q, 2


def multicolour_gauss_seidel(C, Rc, tol_c, bc_x=NEUMANN, bc_y=NEUMANN, E0=None,
                             max_iter=100000):
    """Multicolour Gauss-Seidel on A_c E = R_c to an absolute tolerance (Sec. 3.1:
    multicolour ordering makes GS concurrent for stencils wider than five points; Sec. 4:
    GS on the coarse grid; Sec. 4.3.1: the coarse stage ends when the absolute maximum
    residual falls below its limit).

    Cell (J, I) has colour qy(J) * Qx + qx(I), with (qx, Qx) and (qy, Qy) from
    ``axis_colours`` for each axis: 4 colours, 6 or 9 when a periodic axis has odd length.
    Two cells that the 9-point stencil couples differ along some axis by one cell, so they
    never share a colour.  One iteration visits the colours in increasing order and sets
    every cell of a colour from its own equation with the values current at that moment
    (the new ones of earlier colours, the previous iteration's of later ones); one
    synchronization per colour.  The cell update and the residual test before each
    iteration are those of ``block_gauss_seidel`` (the same neighbour order and sums), and
    R_c is projected to zero mean when the system is singular.  Returns (E, iterations,
    number of colours).

    Pinned by a cell-by-cell loop over the colours (bitwise), by lexicographic GS on the
    matrix permuted to colour order (forward substitution with a library routine), by the
    colouring never coupling two cells of one colour, and by convergence to the exact
    solve."""
    ncy, ncx = Rc.shape
    R = np.asarray(Rc, dtype=np.float64)
    if singular(bc_x, bc_y):
        R = R - R.mean()
    E = np.zeros((ncy, ncx)) if E0 is None else np.asarray(E0, dtype=np.float64).copy()
    qx, Qx = axis_colours(ncx, bc_x)
    qy, Qy = axis_colours(ncy, bc_y)
    colour = qy[:, None] * Qx + qx[None, :]
    per_x, per_y = faces(bc_x) is None, faces(bc_y) is None
    order = [(dj, di) for dj in (-1, 0, 1) for di in (-1, 0, 1) if (dj, di) != (0, 0)]
    J, I = np.indices((ncy, ncx))

    def neighbour(a, dj, di):
        """a at (J+dj, I+di) (0 off a walled grid, where the folded stencil has 0 too)."""
        jj, ii = J + dj, I + di
        if per_y:
            jj = jj % ncy
        if per_x:
            ii = ii % ncx
        ok = (jj >= 0) & (jj < ncy) & (ii >= 0) & (ii < ncx)
        return np.where(ok, a[np.clip(jj, 0, ncy - 1), np.clip(ii, 0, ncx - 1)], 0.0)

    def residual(E):
        acc = C[:, :, 1, 1] * E
        for dj, di in order:
            acc = acc + C[:, :, dj + 1, di + 1] * neighbour(E, dj, di)
        return R - acc

    it = 0
    while np.max(np.abs(residual(E))) >= tol_c and it < max_iter:
        for k in range(Qx * Qy):
            acc = np.zeros((ncy, ncx))
            for dj, di in order:
                acc = acc + C[:, :, dj + 1, di + 1] * neighbour(E, dj, di)
            E = np.where(colour == k, (R - acc) / C[:, :, 1, 1], E)
        it += 1
    return E, it, Qx * Qy


def ism_solve_oneshot(b, h, n, bc_x=NEUMANN, bc_y=NEUMANN, tol_c=1e-5, tol_f=1e-6, x0=None,
                      block=16, max_fine=1000000, precision="fp64", coarse_gs="block"):
    """The paper's simplest accommodative cycling, once per call (Sec. 4.3.1): restrict the
    fine residual, iterate on the coarse grid by block GS (or, with coarse_gs="multicolour",
    by multicolour GS, the ordering Sec. 3.1 names for wider stencils) until its absolute
    maximum residual is below tol_c, prolongate and add, then iterate red-black GS on the
    fine grid until the absolute maximum of the fine residual is below tol_f.

    Units: both criteria are absolute maxima in the units of the pressure equation A x = b~
    (the paper's grids have h = 1, where they coincide with its figures): tol_f bounds
    max|b~ - A x| and tol_c bounds the residual of R A P E = R (b~ - A x), i.e. of the
    h^2-scaled coarse system divided by h^2.  The fine criterion is checked before every
    sweep.

    precision="fp32" runs the fine stage in the paper's single precision (Sec. 4.2) as a
    correction: r = h^2 b~ - A'x in FP64, its tile sums the coarse right-hand side (the coarse
    stage stays FP64, as on the host in the paper's setting), then e = P E and the red-black
    sweeps on A'e = fp32(r) entirely in FP32, the criterion on the FP32 residual
    max|fp32(r) - A'e| compared in FP64, and finally x + e in FP64.

    Returns (x, info) with info = dict(coarse_iters, fine_iters, ncc_c, ncc_f): one
    synchronization per coarse block-GS iteration and two per red-black fine iteration
    (Sec. 4.3: each colour of an ordering costs one), NCC_c = I_c (multicolour: the number
    of colours times I_c) and NCC_f = 2 I_f."""
    b = np.asarray(b, dtype=np.float64)
    ny, nx = b.shape
    bp = h * h * _project(b, bc_x, bc_y)
    x = np.zeros_like(bp) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    ncx, ncy = _coarse_shape(nx, ny, n)
    C = coarse_stencil_ism(ncx, ncy, n, bc_x, bc_y, (ny, nx))
    r = bp - laplacian(x, bc_x, bc_y)
    if coarse_gs == "block":
        E, ic = block_gauss_seidel(C, restrict_sum(r, n), tol_c * h * h, block, bc_x, bc_y)
        colours = 1
    elif coarse_gs == "multicolour":
        E, ic, colours = multicolour_gauss_seidel(C, restrict_sum(r, n), tol_c * h * h,
                                                  bc_x, bc_y)
    else:
        raise ValueError("coarse_gs must be 'block' or 'multicolour'")
    fi = 0
    if precision == "fp64":
        x = x + prolong_bilinear(E, n, bc_x, bc_y, fine_shape=(ny, nx))
        while np.max(np.abs(bp - laplacian(x, bc_x, bc_y))) >= tol_f * h * h and fi < max_fine:
            x = red_black_gs(x, bp, bc_x, bc_y, sweeps=1)
            fi += 1
    elif precision == "fp32":
        r32 = r.astype(np.float32)
        e = prolong_bilinear(E, n, bc_x, bc_y, np.float32, fine_shape=(ny, nx))
        while (float(np.max(np.abs(r32 - laplacian(e, bc_x, bc_y)))) >= tol_f * h * h
               and fi < max_fine):
            e = red_black_gs(e, r32, bc_x, bc_y, sweeps=1)
            fi += 1
        x = x + e.astype(np.float64)
    else:
        raise ValueError("precision must be 'fp64' or 'fp32'")
    return _project(x, bc_x, bc_y), dict(coarse_iters=ic, fine_iters=fi, ncc_c=colours * ic,
                                         ncc_f=2 * fi)


# --------------------------------------------------------------------------------------
# The exact discrete solution x* (what every solver must converge to)
# --------------------------------------------------------------------------------------

# The real trigonometric basis that diagonalizes the three-point operator along a walled
# axis, by its (low, high) faces: the mirror ghost of each wall fixes the cell-centred
# modes cos or sin(theta (i + 1/2)) and the allowed angles theta.
_TRANSFORM = {("N", "N"): ("dct", 2), ("D", "D"): ("dst", 2), ("N", "D"): ("dct", 4),
              ("D", "N"): ("dst", 4)}


def laplacian_eigenvalues(nf, bc):
    """Eigenvalues -4 sin^2(theta_k / 2) of the 1D three-point operator with the given
    boundary condition, in the order of its basis: theta_k = pi k / nf (Neumann walls,
    DCT-II), pi (k + 1) / nf (Dirichlet walls, DST-II), pi (k + 1/2) / nf (one wall of each
    kind, DCT-IV / DST-IV) and 2 pi k / nf (periodic, FFT order)."""
    k = np.arange(nf)
    f = faces(bc)
    if f is None:
        theta = 2.0 * np.pi * k / nf
    elif f == ("N", "N"):
        theta = np.pi * k / nf
    elif f == ("D", "D"):
        theta = np.pi * (k + 1.0) / nf
    else:
        theta = np.pi * (k + 0.5) / nf
    return -4.0 * np.sin(theta / 2.0) ** 2


def _spectral_solve(f, bc_x, bc_y):
    """Solution of A'x = f by diagonalizing A' (the real transform of ``_TRANSFORM`` on
    walled axes, the FFT on periodic ones); the zero-mean one when A' is singular."""
    ny, nx = f.shape
    lam = laplacian_eigenvalues(ny, bc_y)[:, None] + laplacian_eigenvalues(nx, bc_x)[None, :]
    sing = singular(bc_x, bc_y)
    if sing:
        lam[0, 0] = 1.0
    axes = ((0, faces(bc_y)), (1, faces(bc_x)))
    fh = np.asarray(f, dtype=np.float64)
    for axis, fc in axes:
        if fc is not None:
            kind, typ = _TRANSFORM[fc]
            fh = getattr(scipy.fft, kind)(fh, type=typ, norm="ortho", axis=axis)
    for axis, fc in axes:
        if fc is None:
            fh = np.fft.fft(fh, axis=axis)
    fh = fh / lam
    if sing:
        fh[0, 0] = 0.0
    for axis, fc in axes:
        if fc is None:
            fh = np.fft.ifft(fh, axis=axis)
    fh = np.real(fh)
    for axis, fc in axes:
        if fc is not None:
            kind, typ = _TRANSFORM[fc]
            fh = getattr(scipy.fft, "i" + kind)(fh, type=typ, norm="ortho", axis=axis)
    return fh


def _project(b, bc_x, bc_y):
    """b~: b less its mean when A is singular (the compatibility condition), else b."""
    b = np.asarray(b, dtype=np.float64)
    return b - b.mean() if singular(bc_x, bc_y) else b


def exact_solve(b, h, bc_x=NEUMANN, bc_y=NEUMANN, refine=2):
    """x*: the solution of A x = b~ (zero-mean when A is singular), by spectral
    diagonalization followed by `refine` steps of FP64 iterative refinement with the
    difference-form residual.

    Pinned by dense direct solves on small grids and by its residual."""
    bp = h * h * _project(b, bc_x, bc_y)
    x = _spectral_solve(bp, bc_x, bc_y)
    for _ in range(refine):
        x = x + _spectral_solve(bp - laplacian(x, bc_x, bc_y), bc_x, bc_y)
    return _project(x, bc_x, bc_y)


def dense_laplacian(nx, ny, bc_x=NEUMANN, bc_y=NEUMANN):
    """The matrix of A' assembled cell by cell from the neighbour lists (tiny grids)."""
    N = nx * ny
    A = np.zeros((N, N))
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            for dj, di in ((0, -1), (0, 1), (-1, 0), (1, 0)):
                jj, ii = j + dj, i + di
                if bc_x == PERIODIC:
                    ii %= nx
                if bc_y == PERIODIC:
                    jj %= ny
                if 0 <= ii < nx and 0 <= jj < ny:
                    A[c, jj * nx + ii] += 1.0
                    A[c, c] -= 1.0
                else:  # behind a wall: the ghost is +p_C (Neumann) or -p_C (Dirichlet)
                    fc = faces(bc_x) if di else faces(bc_y)
                    if fc[0 if (di < 0 or dj < 0) else 1] == "D":
                        A[c, c] -= 2.0
    return A


def dense_solve(b, h, bc_x=NEUMANN, bc_y=NEUMANN):
    """x* on a tiny grid by a dense solve (of the system bordered with sum(x) = 0 when A is
    singular)."""
    ny, nx = b.shape
    A = dense_laplacian(nx, ny, bc_x, bc_y)
    N = nx * ny
    rhs = (h * h * _project(b, bc_x, bc_y)).ravel()
    if not singular(bc_x, bc_y):
        return np.linalg.solve(A, rhs).reshape(ny, nx)
    K = np.zeros((N + 1, N + 1))
    K[:N, :N] = A
    K[:N, N] = 1.0
    K[N, :N] = 1.0
    return np.linalg.solve(K, np.concatenate([rhs, [0.0]]))[:N].reshape(ny, nx)


def relative_residual(b, x, h, bc_x=NEUMANN, bc_y=NEUMANN):
    """||b~ - A x||_2 / ||b~||_2, residual in difference form (FP64)."""
    bp = h * h * _project(b, bc_x, bc_y)
    r = bp - laplacian(np.asarray(x, dtype=np.float64), bc_x, bc_y)
    return float(np.linalg.norm(r) / np.linalg.norm(bp))


# --------------------------------------------------------------------------------------
# The ISM two-level cycle (Sec. 3.3 stencil, Sec. 3.4 sparse V cycle, Sec. 4.3.1 cycling)
# --------------------------------------------------------------------------------------

def _coarse_shape(nx, ny, n, kind="ism"):
    """(ncx, ncy) of a fine grid; only the ISM scheme takes grids that n does not divide."""
    if kind != "ism" and (nx % n or ny % n):
        raise ValueError("the comparison schemes need grids that are multiples of n")
    return tile_layout(nx, n)[0], tile_layout(ny, n)[0]


def _stencil(kind, ncx, ncy, n, bc_x, bc_y, fine_shape=None):
    if kind == "ism":
        return coarse_stencil_ism(ncx, ncy, n, bc_x, bc_y, fine_shape)
    return {"acm": coarse_stencil_acm, "gmg5": coarse_stencil_gmg5}[kind](ncx, ncy, n, bc_x, bc_y)


def _prolong(kind, E, n, bc_x, bc_y, fine_shape=None):
    if kind == "acm":
        return inject_constant(E, n)
    return prolong_bilinear(E, n, bc_x, bc_y, fine_shape=fine_shape)


def ism_solve(b, h, n, bc_x=NEUMANN, bc_y=NEUMANN, nu=2, rtol=1e-10, x0=None,
              max_cycles=100000, stencil="ism", coarse_tol=None):
    """FP64 two-level ISM solve of A x = b - mean(b).

    Sec. 3.4 (Fig. 2b): the fine grid is coupled directly to the n x n coarse grid.  Each
    cycle: restrict the fine residual by tile sums, solve the coarse equations built with
    the interpolated stencil, prolongate bilinearly and add (Sec. 3.3), then `nu` red-black
    Gauss-Seidel sweeps on the fine grid (Sec. 4).  The order (coarse first, then fine
    smoothing) is the paper's accommodative cycling (Sec. 4.3.1); here the coarse problem
    is solved exactly (or, with coarse_tol, by Gauss-Seidel to that absolute tolerance) and
    the fine stage has a fixed number of sweeps, repeated until
    ||b~ - A x|| <= rtol ||b~||.  stencil="acm" or "gmg5" swaps the coarse operator (and,
    for ACM, the prolongation) for the comparison schemes.

    Returns (x, info) with x zero-mean (when A is singular) and
    info = dict(cycles, sweeps, history)."""
    b = np.asarray(b, dtype=np.float64)
    ny, nx = b.shape
    bp = h * h * _project(b, bc_x, bc_y)
    x = np.zeros_like(bp) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    ncx, ncy = _coarse_shape(nx, ny, n, stencil)
    cs = CoarseSolver(coarse_matrix(_stencil(stencil, ncx, ncy, n, bc_x, bc_y, (ny, nx)), bc_x, bc_y))
    bnorm = np.linalg.norm(bp)
    r = bp - laplacian(x, bc_x, bc_y)
    hist = [float(np.linalg.norm(r) / bnorm)]
    cycles = 0
    while hist[-1] > rtol and cycles < max_cycles:
        Rc = restrict_sum(r, n)
        if coarse_tol is None:
            E = cs.solve(Rc)
        else:
            E, _ = cs.gauss_seidel(Rc, tol_c=coarse_tol)
        x = x + _prolong(stencil, E, n, bc_x, bc_y, (ny, nx))
        x = red_black_gs(x, bp, bc_x, bc_y, sweeps=nu)
        r = bp - laplacian(x, bc_x, bc_y)
        cycles += 1
        hist.append(float(np.linalg.norm(r) / bnorm))
    return _project(x, bc_x, bc_y), dict(cycles=cycles, sweeps=cycles * nu, history=hist)


def ism_solve_mixed(b, h, n, bc_x=NEUMANN, bc_y=NEUMANN, nu=2, rtol=1e-10, x0=None,
                    inner_rtol=1e-3, stall_window=8, stall_drop=0.02, max_inner=100000,
                    max_outer=50):
    """ISM with FP32 fine arithmetic inside an FP64 defect-correction loop (emulated).

    Not in the paper (its solver is FP32 throughout, Sec. 4.2).  Outer step in FP64:
    r = b' - A'x; stop if ||r|| <= rtol ||b'||.  Inner solve of A'e = r from e = 0: the fine
    arrays e and r32 = fp32(r) and every fine operation are FP32: smoothing, the residual and
    the prolongation (its x step on the FP64 coarse rows rounded to FP32, its y step and the
    addition to e in FP32); restriction sums and the coarse solve are FP64.  The first
    restriction sums the FP64 r.  The
    inner loop stops when ||r32 - A'e|| <= max(inner_rtol ||r||, rtol ||b'|| / 2), or when
    the residual fell by less than stall_drop over the last stall_window cycles, or at
    max_inner.  Then x += e in FP64.  Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    ny, nx = b.shape
    bp = h * h * _project(b, bc_x, bc_y)
    x = np.zeros_like(bp) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    ncx, ncy = _coarse_shape(nx, ny, n)
    cs = CoarseSolver(coarse_matrix(coarse_stencil_ism(ncx, ncy, n, bc_x, bc_y, (ny, nx)), bc_x, bc_y))
    bnorm = np.linalg.norm(bp)
    outer_hist, cycles, outer = [], 0, 0
    while True:
        r = bp - laplacian(x, bc_x, bc_y)
        rnorm = np.linalg.norm(r)
        outer_hist.append(float(rnorm / bnorm))
        if rnorm <= rtol * bnorm or outer >= max_outer:
            break
        outer += 1
        target = max(inner_rtol * rnorm, 0.5 * rtol * bnorm)
        r32 = r.astype(np.float32)
        Rc = restrict_sum(r, n)
        e = np.zeros_like(r32)
        inner_hist = []
        for _ in range(max_inner):
            E = cs.solve(Rc)
            e = e + prolong_bilinear(E, n, bc_x, bc_y, np.float32, (ny, nx))
            e = red_black_gs(e, r32, bc_x, bc_y, sweeps=nu)
            res = r32 - laplacian(e, bc_x, bc_y)
            res64 = res.astype(np.float64)
            Rc = restrict_sum(res64, n)
            cycles += 1
            inner_hist.append(float(np.linalg.norm(res64)))
            if inner_hist[-1] <= target:
                break
            if (len(inner_hist) > stall_window
                    and inner_hist[-1] > (1.0 - stall_drop) * inner_hist[-1 - stall_window]):
                break
        x = x + e.astype(np.float64)
    return _project(x, bc_x, bc_y), dict(cycles=cycles, sweeps=cycles * nu, outer=outer,
                                         history=outer_hist)


# --------------------------------------------------------------------------------------
# ACM V(0,1) with a 2h hierarchy (Sec. 3.2, Sec. 4, Sec. 4.3.1)
# --------------------------------------------------------------------------------------

def acm_solve(b, h, n, bc_x=NEUMANN, bc_y=NEUMANN, rtol=1e-10, x0=None, max_cycles=100000):
    """Additive correction multigrid with 2x2 agglomeration down to spacing n h.

    Sec. 3.2: each coarse equation is the sum of the fine equations it covers, and the
    coarse result is added back piecewise constant.  Sec. 4: the smoother is red-black GS on
    every level.  Sec. 4.3.1 fixes the cycle shape: the descent only restricts, and on the
    way up every level gets a single sweep after its correction.  Summing the
    2x2 fine equations of a 5-point operator gives twice the 5-point operator, so level l
    (spacing 2^l h) carries 2^l A'.  The coarsest level is solved exactly (zero mean).
    Launch count per cycle as a GPU implementation would issue them: per non-coarsest level
    one residual+restriction, one correction and one fused sweep, plus the coarsest solve.
    Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    ny, nx = b.shape
    L = int(round(math.log2(n)))
    bp = h * h * _project(b, bc_x, bc_y)
    x = np.zeros_like(bp) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    _coarse_shape(nx, ny, n, "acm")
    cs = CoarseSolver(coarse_matrix(coarse_stencil_acm(nx // n, ny // n, n, bc_x, bc_y),
                                    bc_x, bc_y))

    def vcycle(level, e, r):
        scale = float(2 ** level)
        if level == L:
            return cs.solve(r)
        res = r - scale * laplacian(e, bc_x, bc_y)
        ec = vcycle(level + 1, np.zeros((e.shape[0] // 2, e.shape[1] // 2)), restrict_sum(res, 2))
        e = e + inject_constant(ec, 2)
        return red_black_gs(e, r / scale, bc_x, bc_y, sweeps=1)

    bnorm = np.linalg.norm(bp)
    hist = [float(np.linalg.norm(bp - laplacian(x, bc_x, bc_y)) / bnorm)]
    cycles = 0
    while hist[-1] > rtol and cycles < max_cycles:
        x = vcycle(0, x, bp)
        cycles += 1
        hist.append(float(np.linalg.norm(bp - laplacian(x, bc_x, bc_y)) / bnorm))
    launches = cycles * (3 * L + 1)
    return _project(x, bc_x, bc_y), dict(cycles=cycles, sweeps=cycles, launches=launches,
                                         history=hist, levels=L)


# --------------------------------------------------------------------------------------
# Dense analysis on tiny grids
# --------------------------------------------------------------------------------------

def _columns(fn, ncols, shape):
    cols = []
    for k in range(ncols):
        e = np.zeros(ncols)
        e[k] = 1.0
        cols.append(np.asarray(fn(e.reshape(shape)), dtype=np.float64).ravel())
    return np.array(cols).T


def transfer_matrices(nx, ny, n, bc_x=NEUMANN, bc_y=NEUMANN, kind="ism"):
    """Dense R (Nc x N), P (N x Nc) and A' (N x N) built by applying the oracle's own
    functions to unit vectors."""
    ncx, ncy = _coarse_shape(nx, ny, n, kind)
    R = _columns(lambda f: restrict_sum(f, n), nx * ny, (ny, nx))
    P = _columns(lambda E: _prolong(kind, E, n, bc_x, bc_y, (ny, nx)), ncx * ncy, (ncy, ncx))
    A = _columns(lambda f: laplacian(f, bc_x, bc_y), nx * ny, (ny, nx))
    return R, P, A


def two_grid_matrix(nx, ny, n, nu, bc_x=NEUMANN, bc_y=NEUMANN, kind="ism"):
    """Error propagation of one cycle, T = S^nu (I - P A_c^+ R A'), on the zero-mean
    subspace when A is singular (tiny grids).  S is the red-black sweep applied to errors (zero right-hand
    side)."""
    R, P, A = transfer_matrices(nx, ny, n, bc_x, bc_y, kind)
    ncx, ncy = _coarse_shape(nx, ny, n, kind)
    C = _stencil(kind, ncx, ncy, n, bc_x, bc_y, (ny, nx))
    Ac = coarse_matrix(C, bc_x, bc_y).toarray()
    N = nx * ny
    S = _columns(lambda f: red_black_gs(f, np.zeros_like(f), bc_x, bc_y, 1), N, (ny, nx))
    K = np.eye(N) - P @ np.linalg.pinv(Ac) @ R @ A
    T = np.linalg.matrix_power(S, nu) @ K
    if not singular(bc_x, bc_y):
        return T
    Pi = np.eye(N) - np.ones((N, N)) / N
    return Pi @ T @ Pi


# --------------------------------------------------------------------------------------
# Cost accounting (Sec. 4.3)
# --------------------------------------------------------------------------------------

def cost_metrics(ncc_f, ncc_c, n):
    """The paper's per-step cost figures from its synchronization counts (Sec. 4.3).

    A fine red-black GS iteration needs two synchronizations (one per colour) and costs one
    Laplacian per fine control volume; a coarse Gauss-Seidel iteration needs one
    synchronization and costs 1/n^2 Laplacians per fine control volume, since the coarse
    grid has n^2 times fewer cells.  Hence NCC_t = NCC_f + NCC_c and
    N_Lap = NCC_f / 2 + NCC_c / n^2.  Pinned by the counts printed in Tables A.1 and A.3."""
    return dict(ncc_t=ncc_f + ncc_c, n_lap=ncc_f / 2.0 + ncc_c / float(n * n))
