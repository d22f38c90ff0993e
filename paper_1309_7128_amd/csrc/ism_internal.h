// Internal interface between the host orchestration (ism_api.cpp) and the kernel launchers
// (ism_kernels.hip).  Not installed; the public interface is include/ism.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace ism {

// Geometry of one handle, passed to every kernel by value.
struct Geo {
  int nx, ny, batch;   // fine grid and number of independent grids
  int n, ncx, ncy;     // tile edge and coarse grid
  int per_x, per_y;    // 1 if the axis is periodic
  int dmask;           // Dirichlet wall faces: bit 0 west, 1 east, 2 south, 3 north (others
                       // of a non-periodic axis are Neumann walls)
  int log2n;           // log2 of the tile edge
  long long plane;     // nx * ny
  long long cplane;    // ncx * ncy
  // Interpolation tables (Eq. 5), nx entries for the columns then ny for the rows: .x the
  // weight of the upper coarse centre, .y the lower centre (as a double; -1 below the first
  // centre) of each fine index in the grid.  Device memory of the handle's workspace.
  const void* itab;
};

enum Reduce { SUM = 0, MAX = 1 };

// Per-tile partial results written by the residual kernels, [batch][ncy][ncx] each.
struct Partials {
  double* sumsq;  // sum of squared residuals of the tile (or nullptr)
  double* maxabs; // max |residual| of the tile (or nullptr)
  double* bsumsq; // sum of squared right-hand side (outer residual, first call only)
  double* bmaxabs;
};

// ---- launchers (ism_kernels.hip); every one enqueues on `s` and returns hipGetLastError()
// One red-black sweep; e_in and e_out must not alias (workgroups read halos of their
// neighbours' tiles).
// The right-hand side is multiplied by rscale as it is read (a power of two on the ACM
// levels, so the product is exact).
// With part_max, also max |rhs - A'e_in| per tile into part_max[grid][tile]
// (rbgs_tiles(g) tiles per grid).  With stop, a device flag: the launch does nothing when
// *stop != 0 (set by launch_max_stop).
template <typename T>
hipError_t launch_rbgs(const Geo& g, const T* rhs, const T* e_in, T* e_out, hipStream_t s,
                       T rscale = T(1), double* part_max = nullptr, const double* stop = nullptr);
int rbgs_tiles(const Geo& g);

// ACM (FP64): out = 2x2 sums of (r - scale A'e) on the level grid g (e may be null) with
// per-output sums of squares; ef (+)= piecewise-constant injection of the level above.
hipError_t launch_agglomerate(const Geo& g, const double* r, const double* e, double scale,
                              double* out, double* psq, hipStream_t s);
hipError_t launch_inject(const Geo& g, const double* ec, double* ef, int assign, hipStream_t s);

template <typename T>
hipError_t launch_restrict(const Geo& g, const T* rhs, const T* e, double* rc, double* part_sumsq,
                           hipStream_t s);

template <typename T>
hipError_t launch_prolong(const Geo& g, const double* E, T* e, int assign, hipStream_t s);

// One fused cycle: e = (zero_e ? 0 : e) + P E, nu red-black sweeps on A'e = rhs, then
// rc = R (rhs - A'e) and per-coarse-tile sums of squares (ism_cycle_f32.hip and
// ism_cycle_f64.hip).  e_in and e_out must not alias.  nu <= fused_max_nu<T>().  With
// maxmode (nu = 1 only), psq receives per-tile maxima of |rhs - A'e| instead.  With stop, a
// device flag: the launch does nothing when *stop != 0.
template <typename T>
hipError_t launch_cycle_fused(const Geo& g, const T* rhs, const T* e_in, T* e_out,
                              const double* E, double* rc, double* part_sumsq, int nu,
                              int zero_e, hipStream_t s, const double* stop = nullptr,
                              int maxmode = 0);
template <typename T>
int fused_max_nu();
template <>
hipError_t launch_cycle_fused<float>(const Geo&, const float*, const float*, float*,
                                     const double*, double*, double*, int, int, hipStream_t,
                                     const double*, int);
template <>
hipError_t launch_cycle_fused<double>(const Geo&, const double*, const double*, double*,
                                      const double*, double*, double*, int, int, hipStream_t,
                                      const double*, int);
template <>
int fused_max_nu<float>();
template <>
int fused_max_nu<double>();

// The fused cycle of launch_cycle_fused (same arguments and results, 1 <= nu <=
// fused_max_nu<T>()), tiled in LDS: for grids too small for the row walk to hide its latency.
// 32 x 32 cells per workgroup with a halo of 2 nu + 1.
constexpr int kTile = 32;
template <typename T>
hipError_t launch_cycle_tile(const Geo& g, const T* rhs, const T* e_in, T* e_out, const double* E,
                             double* rc, double* part_sumsq, int nu, int zero_e, hipStream_t s,
                             const double* stop = nullptr, int maxmode = 0);

// The exact coarse solve in one workgroup per grid, for coarse grids of at most 32 cells per
// axis (coarse_small_fits); the same tables and result as the four products of k_gemm.
int coarse_small_fits(const Geo& g);
hipError_t launch_coarse_small(const Geo& g, const double* R, const double* Fx, const double* Fy,
                               const double* Vx, const double* Vy, const double* invLam,
                               double* E, hipStream_t s);

template <typename T>
hipError_t launch_outer_residual(const Geo& g, const double* b, const double* x,
                                 const double* mean_b, double h2, T* rT, double* rc,
                                 Partials p, hipStream_t s);

hipError_t launch_tile_sum(const Geo& g, const double* x, double* part, hipStream_t s);

// out[g * out_stride + slot] = scale * (sum or max of count partials of grid g); scratch
// holds batch * ceil(count / 4096) doubles for the chunk results.
hipError_t launch_finalize(const double* part, int count, long long part_stride, int batch,
                           Reduce op, double scale, double* out, int out_stride, int slot,
                           double* scratch, hipStream_t s);

template <typename T>
hipError_t launch_add_to(const Geo& g, double* x, const T* e, hipStream_t s);

hipError_t launch_sub_scalar(const Geo& g, double* x, const double* vals, int val_stride,
                             int slot, hipStream_t s);

// C[b] = op(A[b]) op(B[b]) (then times S elementwise if S != nullptr), FP64, row-major.
hipError_t launch_gemm(int M, int N, int K, int transA, const double* A, long long sA, int lda,
                       int transB, const double* B, long long sB, int ldb, double* C,
                       long long sC, int ldc, const double* S, int batch, hipStream_t s);

hipError_t launch_coarse_assemble(const Geo& g, int gmg5, double* coef, hipStream_t s);

// Fills the interpolation tables g.itab points to (nx + ny entries of double2).
hipError_t launch_interp_tables(const Geo& g, double2* tab, hipStream_t s);

// The exact coarse solve's tables: per-axis eigenbases Vx (ncx x ncx), Vy (ncy x ncy) and
// invLam (ncy x ncx) for stencil kind 0 ISM, 1 GMG5, 2 ACM; the constant mode's entry is 0
// when singular.
hipError_t launch_coarse_tables(const Geo& g, int kind, int singular, double* Vx, double* Vy,
                                double* invLam, hipStream_t s);

// Tables of the exact coarse solve along one axis (row-major nc x nc): the eigenbasis V
// (column k the k-th mode), the forward table F (F = V for an orthonormal V, else the left
// vectors of the pencil, F^T = V^-1 M^-1) and the mode factors k, m with
// 1/lambda = 1/(k_x m_y + m_x k_y) (ism_coarse_tables.cpp).
struct AxisTable {
  std::vector<double> V, F, k, m;
};

// The tables of an axis of nf fine cells in tiles of n (nc = ceil(nf / n) coarse cells):
// closed forms when n divides nf, else the eigen-decomposition of the axis's pencil (K, M).
// False, with a message in err, if the decomposition fails.
bool coarse_axis_table(int nf, int n, int nc, bool per, bool dlo, bool dhi, AxisTable& t,
                       std::string& err);

// p[0 .. count) = v (a kernel, not a memset node).
hipError_t launch_fill(double* p, long long count, double v, hipStream_t s);

// One block-iterative Gauss-Seidel iteration on each grid's coarse system (coef: the
// [ncy][ncx][9] stencil, shared by the batch): Eout from Ein, part_max[grid][tile] = max
// |R - A_c Ein| over the tile.  Ein and Eout must not alias.  coarse_bgs_tiles(g) tiles per
// grid.
int coarse_bgs_tiles(const Geo& g);
hipError_t launch_coarse_bgs(const Geo& g, const double* coef, const double* R, const double* Ein,
                             double* Eout, double* part_max, hipStream_t s,
                             const double* stop = nullptr);

// One multicolour Gauss-Seidel iteration on each grid's coarse system: Eout from Ein (which
// must not alias), the colours in increasing order, one launch each; part_max[grid][tile] =
// max |R - A_c Ein| over coarse_mc_tiles(g) tiles of cells per grid.  coarse_mc_colours(g)
// colours: 4, or 6 / 9 with one / two odd periodic axes.  Returns the number of kernels
// enqueued; *err the first launch error (hipSuccess if none).
int coarse_mc_colours(const Geo& g);
int coarse_mc_tiles(const Geo& g);
int launch_coarse_mc(const Geo& g, const double* coef, const double* R, const double* Ein,
                     double* Eout, double* part_max, hipStream_t s, const double* stop,
                     hipError_t* err);

// m[k] = max of part[k part_stride .. + count) for every grid k (values as launch_finalize's
// MAX), then the device-side stop test of iteration iter: if *state is 0 and every m[k] is
// below tol (or any is not finite), *state becomes 1 (2) and *at iter.  One workgroup (after
// launch_finalize's first stage into scratch when count exceeds one chunk).  Returns the
// kernels enqueued; *err the first launch error.
int launch_max_stop(const double* part, int count, long long part_stride, int batch, double* m,
                    double tol, int iter, double* state, double* at, double* scratch,
                    hipStream_t s, hipError_t* err);

hipError_t launch_div(const Geo& g, const double* u, const double* v, double h, double* b,
                      hipStream_t s);
hipError_t launch_grad(const Geo& g, const double* p, double h, double* gu, double* gv,
                       hipStream_t s);
hipError_t launch_div_adjoint(const Geo& g, const double* lam, double h, double* gu,
                              double* gv, hipStream_t s);
hipError_t launch_grad_adjoint(const Geo& g, const double* gu, const double* gv, double h,
                               double* p, hipStream_t s);
// Explicit predictor (us, vs must not alias u, v) and the projection's correction.
hipError_t launch_predict(const Geo& g, const double* u, const double* v, const double* p,
                          double h, double dt, double eta, const double walls[4], double* us,
                          double* vs, hipStream_t s);
hipError_t launch_correct(const Geo& g, const double* x, double h, double* u, double* v, double* p,
                          hipStream_t s);

}  // namespace ism
