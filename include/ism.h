/*
 * ism.h - C ABI of the interpolated stencil multigrid (ISM) pressure-Poisson solver for
 * MI355X (gfx950).
 *
 * The method is the two-level cycle of Tegze & Toth, "A GPU cluster optimized multigrid
 * scheme for computing unsteady incompressible fluid flow": red-black Gauss-Seidel on the
 * fine grid (Sec. 3.1, Sec. 4), restriction by sums over n x n tiles (Sec. 3.3), a coarse
 * grid whose 9-point stencil is built from the bilinear interpolant of the coarse unknowns
 * (Sec. 3.3, Eq. 5-7), bilinear prolongation (Sec. 3.3) and the sparse two-level V cycle
 * (Sec. 3.4, Fig. 2b).
 *
 * Problem.  The pressure equation of the projection step (Sec. 2.2, Eq. 4) on a cell-centred
 * nx x ny grid with square cells of size h = lx/nx = ly/ny, discretized with the 5-point
 * Laplacian (Sec. 2.3): A x = b~, with (A x)_C = sum over the four faces of
 * (x_nb - x_C) / h^2.  An axis is periodic or has a wall on each face, of one of the kinds
 * Sec. 4.1 lists: "symmetric", read as homogeneous Neumann (no flux through the wall face),
 * or Dirichlet (zero pressure on the wall face, read as the mirror ghost x_nb = -x_C).
 * Without a Dirichlet face the constants span the null space of A: then b~ = b - mean(b)
 * and the returned x is the zero-mean solution.  With one, A is nonsingular and b~ = b.
 *
 * Conventions for every entry point.
 *  - All array arguments are DEVICE pointers (HIP global memory), C-contiguous row-major
 *    [batch][ny][nx] with x fastest; the caller owns them and they stay valid until the
 *    call returns.  Staggered (MAC) face arrays: u is [batch][ny][nx+1] ([batch][ny][nx]
 *    when periodic in x; face i is the west face of cell i), v is [batch][ny+1][nx] (face j
 *    is the south face of cell j).
 *  - Every device operation is ordered on the HIP stream given to ism_create.  ism_solve
 *    and ism_solve_adjoint return after their last host synchronization, so their outputs
 *    are ready; every other entry point only enqueues work.
 *  - Return value: ISM_OK (0), ISM_NOT_CONVERGED (+1, a warning: x holds the last iterate),
 *    or a negative error code.  Arguments are validated before any device call; no C++
 *    exception crosses this interface.  ism_last_error() gives the text of the last error
 *    of a handle (NULL handle: of the last failed ism_create on this thread).
 *  - A handle is not thread-safe; independent handles are.
 */
#ifndef ISM_H
#define ISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISM_OK 0
#define ISM_NOT_CONVERGED 1
#define ISM_ERR_INVALID (-1)     /* null pointer, non-positive size, bad enum value       */
#define ISM_ERR_UNSUPPORTED (-2) /* a size or option outside what is supported (see
                                    ism_config: coarsen, padding), lx/nx != ly/ny,
                                    nx * ny >= 2^31                                      */
#define ISM_ERR_HIP (-3)         /* a HIP runtime call failed; see ism_last_error        */
#define ISM_ERR_NONFINITE (-4)   /* NaN or Inf met in b or during the iteration          */

#define ISM_BC_NEUMANN 0  /* wall: no flux across the boundary face ("symmetric", Sec. 4.1) */
#define ISM_BC_PERIODIC 1 /* the axis wraps (Sec. 4.1)                                       */
#define ISM_BC_DIRICHLET 2 /* zero-pressure walls on both faces of the axis (Sec. 4.1)       */
#define ISM_BC_NEUMANN_DIRICHLET 3 /* Neumann wall on the low face (west / south), zero-
                                      pressure wall on the high face (east / north), e.g. an
                                      outlet at the top of a channel                         */
#define ISM_BC_DIRICHLET_NEUMANN 4 /* zero-pressure wall on the low face, Neumann on the
                                      high face                                              */

#define ISM_PREC_FP64 0  /* every fine-grid operation in FP64                                */
#define ISM_PREC_MIXED 1 /* FP32 smoothing, restriction and prolongation inside an FP64
                            defect-correction loop; outer residual, mean removal, the
                            coarse solve and the update of x stay FP64                     */

#define ISM_COARSE_ISM 0  /* interpolated 9-point coarse stencil (Sec. 3.3, Eq. 5-7)            */
#define ISM_COARSE_GMG5 1 /* 5-point stencil rediscretized at spacing n h: the aggressive-
                             coarsening GMG scheme the paper compares with (Sec. 4.3.2)         */
#define ISM_COARSE_ACM 2  /* not two-level: additive correction multigrid with 2x2
                             agglomeration down to spacing n h and V(0,1) cycles, the scheme the
                             paper compares with (Sec. 3.2, Sec. 4, Sec. 4.3.1); FP64 only;
                             ism_cycle is unsupported on such a handle                         */

/* Cycling (Sec. 4.3.1).  REPEAT: {restrict, exact coarse solve, prolongate, nu sweeps} until
 * rtol, as described for ism_solve.  ONESHOT: the paper's simplest accommodative cycling,
 * once per solve: restrict the residual, iterate the coarse grid by block Gauss-Seidel
 * (Sec. 4; or multicolour Gauss-Seidel, see ism_config.coarse_gs; block GS takes tiles of
 * 16 x 16 coarse cells, aligned at cell 0, updated concurrently and lexicographic inside;
 * a periodic axis of at most 16 coarse cells is cut into two tiles of
 * ceil(nc / 2), so that no tile spans a whole periodic axis and a neighbour reached across a
 * periodic seam always belongs to another tile) until its absolute maximum residual is below
 * coarse_tol, prolongate and add, then iterate
 * red-black Gauss-Seidel on the fine grid until the absolute maximum residual is below
 * fine_tol.  Both criteria are in the units of A x = b~ (the coarse residual divided by h^2),
 * which are the paper's on its h = 1 grids.  Every iteration's criterion is tested on the
 * device right after it, and the first iteration that meets it stops the stage exactly
 * (iterations enqueued past it return at once); the host reads the outcome back once per
 * batch of 4, 8, 16, 32, then 64 iterations.  ISM or GMG5 stencil only.  ISM_PREC_FP64
 * iterates x itself; ISM_PREC_MIXED runs the fine stage in FP32 (the paper's precision,
 * Sec. 4.2) as a correction: e = P E and the sweeps on A'e = fp32(h^2 b~ - A'x), the
 * criterion on that FP32 residual, then x += e in FP64 (the coarse stage stays FP64).
 * rtol, max_outer and nu are not used; max_cycles caps each stage's iterations (status
 * ISM_NOT_CONVERGED when a stage reaches it).  The grids of a batch iterate together until
 * all of them meet a criterion. */
#define ISM_CYCLE_REPEAT 0
#define ISM_CYCLE_ONESHOT 1

/* The coarse iteration of ISM_CYCLE_ONESHOT and ism_coarse_gs (ism_config.coarse_gs).
 * BLOCK: block-iterative Gauss-Seidel as described above (Sec. 4; one synchronization per
 * iteration).  MULTICOLOUR: Gauss-Seidel in multicolour order, the ordering Sec. 3.1 names
 * for stencils wider than five points: along each axis cell i has colour i mod 2, except
 * that the last cell of an odd periodic axis takes colour 2; cell (J, I) has colour
 * qy(J) * Qx + qx(I) (4 colours; 6 or 9 with one or two odd periodic axes), so no two
 * coupled cells share one.  An iteration sets the cells colour by colour in increasing
 * order, all cells of a colour at once from the newest values, one synchronization per
 * colour (Sec. 4.3).  Both iterations update a cell as E_C = (R_C - sum of c_nb E_nb) / c_C
 * with the neighbours in the order (dj, di) = (-1,-1) .. (1,1) and summed left to right,
 * and test max |R - A_c E| against the tolerance before each iteration. */
#define ISM_COARSE_GS_BLOCK 0
#define ISM_COARSE_GS_MULTICOLOUR 1

/* The kernel a cycle takes (ism_config.fused).  Both fused kernels give the same e bit for
 * bit (that of nu whole-grid red-black sweeps) and the same tile sums up to their summation
 * order.  The row walk streams the grid once per cycle (the large-grid form); the LDS-tiled
 * form stages 32 x 32 blocks with a halo of 2 nu + 1 and suits grids too small for the walk
 * to hide its per-row latency.  AUTO takes the tiled form up to 1024^2 cells per launch
 * (nx * ny * batch), the walk above. */
#define ISM_FUSED_OFF 0  /* prolongation, nu sweeps, residual + restriction: one kernel each */
#define ISM_FUSED_AUTO 1 /* default                                                          */
#define ISM_FUSED_WALK 2 /* the row walk always                                              */
#define ISM_FUSED_TILE 3 /* the LDS-tiled form always                                        */

#define ISM_F64 0 /* element type selector of the stage entry points: double */
#define ISM_F32 1 /*                                                  float  */

typedef struct ism_ctx* ism_handle;

typedef struct {
  int32_t nx, ny;     /* fine cells along x and y (>= 2 each)                               */
  int32_t batch;      /* independent grids solved together (>= 1)                           */
  int32_t bc_x, bc_y; /* ISM_BC_* on the x faces (west/east) and the y faces (south/north)   */
  int32_t coarsen;    /* tile edge n of the n x n restriction: 4, 8, 16 or 32 (Sec. 3.4).
                         Tiles start at cell 0; where n does not divide nx (ny) the last
                         tile of the axis is short and covers the cells that exist, its
                         centre in its middle, and the interpolation rectangles next to it
                         are shorter (the padded domain, Sec. 3.3 Eq. 5, Sec. 4.1): the
                         coarse grid is ceil(ny/n) x ceil(nx/n).  Such a grid needs the
                         ISM stencil, nx a multiple of 4 and ny even (ISM_ERR_UNSUPPORTED
                         otherwise); the GMG5 and ACM stencils need multiples of n.     */
  double lx, ly;      /* domain size; lx/nx must equal ly/ny (square cells)                 */
  int32_t precision;  /* ISM_PREC_*                                                         */
  int32_t nu;         /* red-black sweeps per cycle after the coarse correction (>= 1);
                         ISM_COARSE_ACM cycles always take one sweep per level             */
  double rtol;        /* stop when ||b~ - A x||_2 <= rtol ||b~||_2 for every grid            */
  double inner_rtol;  /* mixed form: an inner FP32 solve stops once its residual fell by
                         this factor (or stagnated)                                         */
  int32_t max_cycles; /* cap on two-level cycles per solve (all inner solves together)      */
  int32_t max_outer;  /* cap on FP64 defect-correction steps                                */
  int32_t check_every;/* cycles between convergence checks; 0 = adaptive (predicts the
                         cycle that meets the target from the measured rate)               */
  int32_t fused;      /* ISM_FUSED_*: one fused kernel per cycle (prolongation, nu sweeps,
                         residual and restriction), or one kernel per step                 */
  int32_t stall_window; /* an inner solve also stops when its residual fell by less than   */
  double stall_drop;    /* stall_drop (a fraction) over the last >= stall_window cycles     */
  int32_t coarse_stencil; /* ISM_COARSE_ISM (default), ISM_COARSE_GMG5 or ISM_COARSE_ACM    */
  int32_t cycling;        /* ISM_CYCLE_REPEAT (default) or ISM_CYCLE_ONESHOT                */
  double coarse_tol;      /* ISM_CYCLE_ONESHOT: the coarse block Gauss-Seidel stops once
                             max |R (b~ - A x) - R A P E| < coarse_tol (default 1e-5)       */
  double fine_tol;        /* ISM_CYCLE_ONESHOT: the fine sweeps stop once
                             max |b~ - A x| < fine_tol (default 1e-6)                       */
  int32_t coarse_gs;      /* ISM_COARSE_GS_BLOCK (default) or ISM_COARSE_GS_MULTICOLOUR: the
                             coarse iteration of ISM_CYCLE_ONESHOT and ism_coarse_gs        */
} ism_config;

typedef struct {
  int32_t status;      /* return code of the solve                                          */
  int32_t outer_iters; /* FP64 defect-correction steps taken                                */
  int32_t cycles;      /* two-level cycles (coarse solve + prolongation + nu sweeps)        */
  int32_t sweeps;      /* fine-grid red-black sweeps: cycles * nu (cycles for ACM)          */
  int64_t launches;    /* kernels launched                                                  */
  int64_t host_syncs;  /* device-to-host reads the host waited for                          */
  double rel_res_l2;   /* max over the batch of ||b~ - A x||_2 / ||b~||_2 (FP64, difference
                          form) of the returned x (after its final mean removal)            */
  double rel_res_max;  /* max over the batch of max|b~ - A x| / max|b~|                     */
  double seconds;      /* wall time of the call                                              */
  int32_t coarse_iters; /* ISM_CYCLE_ONESHOT: Gauss-Seidel iterations on the coarse grid
                           (I_c; one synchronization each for block GS, NCC_c = I_c, one per
                           colour for multicolour GS, Sec. 4.3)                            */
  int32_t fine_iters;   /* ISM_CYCLE_ONESHOT: red-black iterations on the fine grid (I_f;
                           two synchronizations each, NCC_f = 2 I_f)                       */
  int32_t coarse_syncs; /* ISM_CYCLE_ONESHOT: synchronizations of the coarse stage, NCC_c:
                           coarse_iters (block GS) or colours x coarse_iters (multicolour)  */
} ism_stats;

/* Fill cfg with defaults for an nx x ny grid of unit cell size 1/nx (unit square), Neumann
 * walls, coarsen 16, FP64, nu 4, rtol 1e-10, inner_rtol 1e-3, adaptive checks, ISM_FUSED_AUTO,
 * stall_window 8, stall_drop 0.02, block coarse Gauss-Seidel. */
int ism_config_init(ism_config* cfg, int32_t nx, int32_t ny, int32_t batch);

/* Validate cfg, allocate the handle's device workspace and build the coarse tables
 * (the 1D factors of the coarse operator and their eigenbases).  stream is a hipStream_t
 * (NULL: the default stream).  On success *out owns device memory until ism_destroy. */
int ism_create(const ism_config* cfg, void* stream, ism_handle* out);

/* Synchronize the stream and release everything the handle owns.  NULL is accepted. */
int ism_destroy(ism_handle h);

/* Bytes of device memory the handle holds. */
int ism_workspace_bytes(ism_handle h, size_t* bytes);

/* Solve A x = b~ for every grid of the batch (Sec. 3.4 sparse two-level cycle, Sec. 4.3.1
 * cycling: coarse correction first, then nu fine sweeps, repeated).  b: FP64
 * [batch][ny][nx], read only.  x: FP64 [batch][ny][nx], initial guess on entry (warm start),
 * solution on return (the zero-mean one when A is singular).  st may be NULL. */
int ism_solve(ism_handle h, const double* b, double* x, ism_stats* st);

/* Allocation-free solve, for callers that cannot allocate device or pinned memory (tight
 * serving loops, harnesses that forbid hipMalloc).  The same solve as ism_create, ism_solve
 * and ism_destroy on cfg: the same kernels, tables and convergence-check schedule, so the
 * same x and the same stats (seconds and host_syncs aside), without a handle.  Its workspace
 * lies in a static device array of ISM_STATIC_SCRATCH_BYTES that every GPU the library runs
 * on holds until the process ends.  Calls no hipMalloc, hipFree, hipHostMalloc or
 * hipEventCreate: read-backs go to pageable host memory, with a stream synchronization
 * whenever a convergence check is read.
 * cfg: as for ism_create (ISM or GMG5 stencil; ACM returns ISM_ERR_UNSUPPORTED).  A grid
 * whose workspace exceeds the array (about 3 nx ny batch sizeof(T) bytes, T the inner type)
 * returns ISM_ERR_UNSUPPORTED before any device call.  stream: the HIP stream every
 * operation is ordered on (NULL: the null stream).  b, x: as for ism_solve.  Errors read
 * with ism_last_error(NULL).  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (a call writes everything it reads there first): calls that overlap
 * on one GPU race and must not be issued. */
#define ISM_STATIC_SCRATCH_BYTES (64u << 20)
int ism_solve_static(const ism_config* cfg, const double* b, double* x, ism_stats* stats,
                     void* stream);

/* Adjoint solve A^T lam = g~.  A is symmetric for these boundary conditions, so
 * this is the same solve; it exists so that a differentiable projection names its
 * backward pass.  Same layouts and ownership as ism_solve. */
int ism_solve_adjoint(ism_handle h, const double* g, double* lam, ism_stats* st);

/* Staggered-grid operators of the projection step (Sec. 2.2, Sec. 2.3), FP64:
 *   ism_div:          b = D[u; v],  b_C = ((u_e - u_w) + (v_n - v_s)) / h
 *   ism_grad:         [gu; gv] = G p, gradient on faces: zero on Neumann wall faces,
 *                     (p_C - (-p_C)) / h or ((-p_C) - p_C) / h on a west/south or
 *                     east/north Dirichlet wall face, so D G = A
 *   ism_div_adjoint:  [gu; gv] = D^T lam
 *   ism_grad_adjoint: p = G^T [gu; gv]
 * Layouts as above; outputs are overwritten. */
int ism_div(ism_handle h, const double* u, const double* v, double* b);
int ism_grad(ism_handle h, const double* p, double* gu, double* gv);
int ism_div_adjoint(ism_handle h, const double* lam, double* gu, double* gv);
int ism_grad_adjoint(ism_handle h, const double* gu, const double* gv, double* p);

/* ---- One time step of Goda's incremental projection scheme (Sec. 2.2, Eq. 3-4):
 *   ism_predict(u, v, p) -> (us, vs), the explicit predictor
 *   ism_div(us, vs) -> b, ism_solve(b) -> x  (x: the pressure change, warm start allowed)
 *   ism_correct(x, us, vs, p): us -= G x, vs -= G x, p += x  (the new velocity and pressure)
 * p carries the time step (p = dt times the kinematic pressure).
 *
 * ism_predict: us = u + dt (eta lap u - (u . grad) u) - G p on every face (and vs alike),
 * second-order central differences on the staggered grid (Sec. 2.3): at an interior u face
 * dudx = (u_E - u_W) / (2h), dudy = (u_N - u_S) / (2h), lap = (((u_E + u_W) + u_N) + u_S - 4 u)
 * / h^2, v at the face the mean of its four neighbouring v faces; v faces alike.  A wall face
 * keeps its normal velocity; behind a wall a tangential neighbour is the ghost 2 U_w - (the
 * face's value), with walls = {v of the west wall, v of the east wall, u of the south wall,
 * u of the north wall} (a HOST array of 4 doubles; NULL = walls at rest).  eta is the
 * kinematic viscosity.  us and vs must not alias u or v (ISM_ERR_INVALID).  The signs of
 * Eq. 1 and Eq. 3 are garbled in the paper's text; this is the standard form. */
int ism_predict(ism_handle h, const double* u, const double* v, const double* p, double dt,
                double eta, const double* walls, double* us, double* vs);
int ism_correct(ism_handle h, const double* x, double* u, double* v, double* p);

/* ---- Stage entry points: one step of the cycle each, for step-by-step verification.
 * Fine arrays have the element type selected by dtype (ISM_F64 / ISM_F32) and layout
 * [batch][ny][nx]; coarse arrays are FP64 [batch][ncy][ncx] with ncy = ceil(ny/n) and
 * ncx = ceil(nx/n) (ny/n and nx/n with full tiles).  rhs is in h^2 units
 * (the equation solved is A' e = rhs with A' = h^2 A). */

/* nsweeps red-black Gauss-Seidel sweeps on A' e = rhs, red ((i + j) even) first; each cell
 * takes the value that satisfies its own equation (Sec. 3.1). */
int ism_smooth(ism_handle h, int32_t dtype, const void* rhs, void* e, int32_t nsweeps);

/* rc = R (rhs - A' e): fine residual summed over every n x n tile (Sec. 3.3).  If sumsq is
 * not NULL, sumsq[g] = sum of the squared residual of grid g (FP64). */
int ism_restrict(ism_handle h, int32_t dtype, const void* rhs, const void* e, double* rc,
                 double* sumsq);

/* e += P E: bilinear interpolation of the coarse values to the fine cell centres (Eq. 5).
 * Between a wall and the first coarse centre the interpolation reaches the mirror image of
 * that centre: the same value behind a Neumann wall (constant extrapolation), the negated
 * value behind a Dirichlet wall (linear to zero on the wall). */
int ism_prolong(ism_handle h, int32_t dtype, const double* E, void* e);

/* E = solution of A_c E = rc on each grid's coarse grid (without a Dirichlet face: the
 * zero-mean solution of A_c E = rc - mean(rc)), where A_c is the interpolated 9-point
 * stencil (Sec. 3.3, Eq. 6-7), or the 5-point one when the handle was created with
 * ISM_COARSE_GMG5.  Exact up to FP64 rounding.  With a short last tile and no Dirichlet
 * face, the solution returned is the one whose prolongation P E has zero mean (E itself
 * then differs from the zero-mean solution by a constant), and rc is projected along the
 * tile-size weights rather than the constants: the two agree when rc sums to zero, as the
 * restriction of a compatible residual does. */
int ism_coarse_solve(ism_handle h, const double* rc, double* E);

/* One two-level cycle on A' e = rhs: E = coarse solve of rc; e += P E; nu red-black
 * sweeps; rc = R (rhs - A' e) (rc is read and then overwritten).  With zero_e != 0 the
 * incoming e is taken as zero.  Uses the fused kernel if the handle was created fused.
 * rhs and e must be 16-byte aligned (ISM_ERR_INVALID otherwise). */
int ism_cycle(ism_handle h, int32_t dtype, const void* rhs, void* e, double* rc,
              int32_t zero_e, double* sumsq);

/* Gauss-Seidel on each grid's coarse system A_c E = rc (the handle's ISM or GMG5 stencil;
 * block or multicolour by ism_config.coarse_gs), as the ISM_CYCLE_ONESHOT coarse stage runs
 * it (Sec. 4, Sec. 3.1): from E = 0, one
 * iteration at a time, until max |rc - A_c E| < tol (in the units of rc) on every grid or
 * max_iter iterations.  Without a Dirichlet face rc is first projected to zero mean (the
 * compatibility condition of the singular system; rc itself is not modified).  rc, E: FP64
 * [batch][ncy][ncx].  *iters receives the number of iterations.  Returns
 * ISM_NOT_CONVERGED if max_iter was reached first. */
int ism_coarse_gs(ism_handle h, const double* rc, double* E, double tol, int32_t max_iter,
                  int32_t* iters);

/* The coarse stencil assembled on the device (ISM: from the face sums of Eq. 6-7; GMG5:
 * the 5-point stencil with one-sided wall rows):
 * coef is FP64 [ncy][ncx][9]; entry 3*(dj+1) + (di+1) multiplies the unknown at
 * (J+dj, I+di) (wrapped on a periodic axis; the coefficient of a ghost behind a wall is
 * folded onto the unknown it mirrors, with a minus sign behind a Dirichlet wall). */
int ism_coarse_stencil(ism_handle h, double* coef);

/* r = h^2 b~ - A' x in FP64 for every grid (the outer defect-correction residual,
 * difference form). */
int ism_outer_residual(ism_handle h, const double* b, const double* x, double* r);

/* ---- Kernel timing.  While enabled, the handle brackets launches of the kernel classes
 * below with a pair of HIP events on its stream and accumulates their elapsed times at its
 * host synchronizations (the events are created once and reused).  ism_profile(h, n) with
 * n >= 1 resets the totals and starts timing every n-th launch of each class (n = 1: every
 * launch; each event record costs the stream a few microseconds, so a larger n keeps the
 * timing from slowing the timed work); ism_profile(h, 0) stops it.  ism_profile_read
 * synchronizes the stream and returns the total milliseconds and the number of timed
 * launches of one class since the last reset. */
#define ISM_KERNEL_CYCLE 0    /* fused two-level cycle kernel                        */
#define ISM_KERNEL_SMOOTH 1   /* one red-black sweep (unfused form)                  */
#define ISM_KERNEL_RESTRICT 2 /* residual + restriction (unfused form)               */
#define ISM_KERNEL_PROLONG 3  /* prolongation + correction (unfused form)            */
#define ISM_KERNEL_COARSE 4   /* the four transform passes of one coarse solve       */
#define ISM_KERNEL_OUTER 5    /* FP64 outer residual                                 */
#define ISM_KERNEL_CLASSES 6
int ism_profile(ism_handle h, int32_t enable);
int ism_profile_read(ism_handle h, int32_t kind, double* total_ms, int64_t* launches);

const char* ism_status_string(int status);
const char* ism_last_error(ism_handle h);

#ifdef __cplusplus
}
#endif
#endif /* ISM_H */
