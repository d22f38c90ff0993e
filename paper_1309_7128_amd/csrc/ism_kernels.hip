// HIP kernels of the interpolated stencil multigrid (ISM) solver, written for gfx950
// (MI355X: wave64, 160 KB LDS per CU, HBM3E).
//
// Every fine-grid kernel streams a 5-point stencil and is bound by HBM bandwidth; none of
// them is a dense contraction and none uses MFMA.  The one exception is k_gemm, the batched
// FP64 products of the exact coarse solve (dense eigenbasis transforms of the coarse grid),
// which runs on the FP64 matrix cores.  Fine arrays are row-major
// [batch][ny][nx]; a wave covers 64 consecutive cells of a row so every global access is a
// full 256 B (FP32) or 512 B (FP64) row segment.
//
// The arithmetic conventions all kernels share are stated in ism_device.h; the fused cycle
// kernel lives in ism_cycle.h.

#include "ism_device.h"

namespace ism {
namespace {

// ----------------------------------------------------------------------------------------
// One red-black sweep (red on the tile plus one ring, black on the tile), LDS-staged.
// Tile 64 x 32 cells per workgroup; e is staged with a halo of 2, rhs with a halo of 1.
// With part_max, the workgroup also writes max |rhs - A'ein| over its tile (the residual of
// the incoming iterate, from the staged values) to part_max[tile].
// ----------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rbgs(Geo g, const T* __restrict__ rhs,
                                                 const T* __restrict__ ein,
                                                 T* __restrict__ eout, T rscale,
                                                 double* __restrict__ part_max,
                                                 const double* __restrict__ stop) {
  // a sweep enqueued past the iteration a device-side check stopped at does nothing
  if (stop && *stop != 0.0) return;
  constexpr int TX = 64, TY = 32;
  constexpr int LE = TX + 4, HE = TY + 4;
  constexpr int LR = TX + 2, HR = TY + 2;
  __shared__ T se[HE * LE];
  __shared__ T sr[HR * LR];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const long long off = (long long)blockIdx.z * g.plane;
  const T* rb = rhs + off;
  const T* eb = ein + off;
  T* ob = eout + off;

  for (int t = threadIdx.x; t < HE * LE; t += kBlock) {
    int ly = t / LE, lx = t - ly * LE;
    int i = x0 + lx - 2, j = y0 + ly - 2;
    T v = T(0);
    if (map_cell(g, i, j)) v = eb[(long long)j * g.nx + i];
    se[t] = v;
  }
  for (int t = threadIdx.x; t < HR * LR; t += kBlock) {
    int ly = t / LR, lx = t - ly * LR;
    int i = x0 + lx - 1, j = y0 + ly - 1;
    T v = T(0);
    if (map_cell(g, i, j)) v = rb[(long long)j * g.nx + i] * rscale;
    sr[t] = v;
  }
  __syncthreads();
  if (part_max) {
    __shared__ double smax[kBlock / kWave];
    double m = 0.0;
    for (int t = threadIdx.x; t < TY * TX; t += kBlock) {
      const int r = t / TX, c = t - r * TX;
      const int i = x0 + c, j = y0 + r;
      if (i >= g.nx || j >= g.ny) continue;
      const int idx = (r + 2) * LE + c + 2;
      const T res = sr[(r + 1) * LR + (c + 1)] -
                    lap5<T>(se[idx], se[idx - 1], se[idx + 1], se[idx - LE], se[idx + LE],
                            cell_faces(g, i, j));
      m = fmax(m, fabs(double(res)));
    }
    m = wave_max_group(m, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) smax[threadIdx.x / kWave] = m;
    __syncthreads();  // the residual reads of se end before the red cells are overwritten
    if (threadIdx.x == 0) {
      for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, smax[w]);
      part_max[(long long)blockIdx.z * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] =
          fmax(m, smax[0]);
    }
  }

  // red cells of rows/cols 1 .. TY+2 / TX+2 of the staged region
  constexpr int RW = (TX + 2) / 2;
  for (int t = threadIdx.x; t < (TY + 2) * RW; t += kBlock) {
    int r = t / RW, k = t - r * RW;
    int ly = r + 1;
    int j = y0 + ly - 2;
    int lx = 1 + ((j + 1) & 1) + 2 * k;  // (i + j) even, x0 even
    int i = x0 + lx - 2;
    if (!map_cell(g, i, j)) continue;
    int idx = ly * LE + lx;
    T s = (se[idx - 1] + se[idx + 1]) + (se[idx - LE] + se[idx + LE]);
    se[idx] = (s - sr[(ly - 1) * LR + (lx - 1)]) * inv_count<T>(g, i, j);
  }
  __syncthreads();
  constexpr int BW = TX / 2;
  for (int t = threadIdx.x; t < TY * BW; t += kBlock) {
    int r = t / BW, k = t - r * BW;
    int ly = r + 2;
    int j = y0 + r;
    int lx = 2 + ((j + 1) & 1) + 2 * k;  // (i + j) odd
    int i = x0 + lx - 2;
    if (i >= g.nx || j >= g.ny) continue;
    int idx = ly * LE + lx;
    T s = (se[idx - 1] + se[idx + 1]) + (se[idx - LE] + se[idx + LE]);
    se[idx] = (s - sr[(ly - 1) * LR + (lx - 1)]) * inv_count<T>(g, i, j);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TY * TX; t += kBlock) {
    int r = t / TX, c = t - r * TX;
    int i = x0 + c, j = y0 + r;
    if (i < g.nx && j < g.ny) ob[(long long)j * g.nx + i] = se[(r + 2) * LE + c + 2];
  }
}

// ----------------------------------------------------------------------------------------
// Residual + restriction: rc = R (rhs - A'e).  A workgroup covers 64 columns by one row of
// coarse tiles (n rows); lane = column, wave w takes rows w, w+4, ...  Tile sums are formed
// with xor shuffles inside groups of n lanes, then across the 4 waves through LDS.
// ----------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(Geo g, const T* __restrict__ rhs,
                                                     const T* __restrict__ e,
                                                     double* __restrict__ rc,
                                                     double* __restrict__ psq) {
  __shared__ double s1[4][16], s2[4][16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int x0 = blockIdx.x * kWave, J = blockIdx.y;
  const long long off = (long long)blockIdx.z * g.plane;
  const T* rb = rhs + off;
  const T* eb = e + off;
  const int i = x0 + lane;
  double acc = 0.0, acc2 = 0.0;
  if (i < g.nx) {
    const int iw = g.per_x ? imod(i - 1, g.nx) : i - 1;
    const int ie = g.per_x ? imod(i + 1, g.nx) : i + 1;
    for (int r = wave; r < g.n && J * g.n + r < g.ny; r += 4) {
      const int j = J * g.n + r;
      const int js = g.per_y ? imod(j - 1, g.ny) : j - 1;
      const int jn = g.per_y ? imod(j + 1, g.ny) : j + 1;
      const CellFaces f = cell_faces(g, i, j);
      const T* row = eb + (long long)j * g.nx;
      T c = row[i];
      T w = f.hw ? row[iw] : T(0);
      T ee = f.he ? row[ie] : T(0);
      T s = f.hs ? eb[(long long)js * g.nx + i] : T(0);
      T nn = f.hn ? eb[(long long)jn * g.nx + i] : T(0);
      T res = rb[(long long)j * g.nx + i] - lap5<T>(c, w, ee, s, nn, f);
      double d = double(res);
      acc += d;
      acc2 += d * d;
    }
  }
  acc = wave_sum_group(acc, g.n);
  acc2 = wave_sum_group(acc2, g.n);
  if ((lane & (g.n - 1)) == 0) {
    s1[wave][lane >> g.log2n] = acc;
    s2[wave][lane >> g.log2n] = acc2;
  }
  __syncthreads();
  const int tiles = kWave >> g.log2n;
  if ((int)threadIdx.x < tiles) {
    const int I = (x0 >> g.log2n) + threadIdx.x;
    if (I < g.ncx) {
      const long long o = (long long)blockIdx.z * g.cplane + (long long)J * g.ncx + I;
      const int t = threadIdx.x;
      rc[o] = ((s1[0][t] + s1[1][t]) + s1[2][t]) + s1[3][t];
      if (psq) psq[o] = ((s2[0][t] + s2[1][t]) + s2[2][t]) + s2[3][t];
    }
  }
}

// ----------------------------------------------------------------------------------------
// Prolongation + correction: e (+)= P E, one thread per fine cell.
// ----------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(Geo g, const double* __restrict__ E,
                                                    T* __restrict__ e, int assign) {
  const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
  const int j = blockIdx.y * 4 + threadIdx.x / kWave;
  if (i >= g.nx || j >= g.ny) return;
  const T p = prolong_at<T>(g, E + (long long)blockIdx.z * g.cplane, i, j);
  T* ec = e + (long long)blockIdx.z * g.plane + (long long)j * g.nx + i;
  *ec = assign ? p : T(*ec + p);
}

// ----------------------------------------------------------------------------------------
// Fused cycle for small grids, tiled in LDS.  A workgroup stages a kTile x kTile block of e
// (with the coarse correction of Eq. 5 added) and of rhs, with a halo of H = 2 nu + 1 cells,
// and runs the 2 nu half-steps of nu red-black sweeps on it in LDS: each half-step leaves one
// more ring of the halo stale, so the block and the ring around it are exact after the last.
// Then it forms the residual of the block, sums it over the n x n coarse tiles in a fixed
// tree order and writes the block.  Every cell is set by the expressions of k_rbgs, so the
// result is that of nu whole-grid sweeps bit for bit.  It serves grids whose row walk (the
// other fused kernel) has too few waves to hide its per-row latency: a block's staging, 2 nu
// barriers and its reduction take a few microseconds, against the walk's tens.
// ----------------------------------------------------------------------------------------
constexpr int kTileBlock = 1024;  // threads of a k_cycle_tile workgroup

template <typename T, int NU>
__global__ __launch_bounds__(kTileBlock) void k_cycle_tile(Geo g, const T* __restrict__ rhs,
                                                       const T* __restrict__ ein,
                                                       T* __restrict__ eout,
                                                       const double* __restrict__ E,
                                                       double* __restrict__ rc,
                                                       double* __restrict__ psq, int zero_e,
                                                       const double* __restrict__ stop,
                                                       int maxmode) {
  constexpr int H = 2 * NU + 1, W = kTile + 2 * H, WI = W - 2, HW = WI / 2;
  static_assert(W % 2 == 0, "even staged width");
  __shared__ T se[W * W], sr[W * W], si[W * W];  // e, rhs, 1 / diagonal (0 behind a wall)
  __shared__ double p1[kBlock], p2[kBlock];       // per-thread partial sums, squares / maxima
  if (stop && *stop != 0.0) return;  // enqueued past a device-side stop
  const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
  const long long off = (long long)blockIdx.z * g.plane;
  const double* Eb = E + (long long)blockIdx.z * g.cplane;
  // stage: e (+)= P E, rhs and the inverse diagonal; cells behind a wall hold 0 throughout.
  // A thread's NS cells are formed first and stored after, so that their global reads are
  // all in flight together rather than one cell's latency after another's.
  constexpr int NS = (W * W + kTileBlock - 1) / kTileBlock;
  T ev[NS], rv[NS], iv[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int t = threadIdx.x + q * kTileBlock;
    const int ly = t / W, lx = t - ly * W;
    int i = x0 + lx - H, j = y0 + ly - H;
    ev[q] = T(0);
    rv[q] = T(0);
    iv[q] = T(0);
    if (t < W * W && map_cell(g, i, j)) {
      const long long a = off + (long long)j * g.nx + i;
      rv[q] = rhs[a];
      const T p = prolong_at<T>(g, Eb, i, j);
      ev[q] = zero_e ? p : T(ein[a] + p);
      iv[q] = inv_count<T>(g, i, j);
    }
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int t = threadIdx.x + q * kTileBlock;
    if (t < W * W) {
      se[t] = ev[q];
      sr[t] = rv[q];
      si[t] = iv[q];
    }
  }
  __syncthreads();
  // half-step k (red first) on the cells of its colour with four staged neighbours; x0 and
  // y0 are even, so a cell's colour is the parity of its staged coordinates.  A cell reads
  // only cells of the other colour, so a thread forms all its NH cells before storing any.
  constexpr int NH = (WI * HW + kTileBlock - 1) / kTileBlock;
#pragma unroll 1
  for (int k = 0; k < 2 * NU; ++k) {
    T nv[NH];
    int ni[NH];
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      const int t = threadIdx.x + q * kTileBlock;
      const int ly = 1 + t / HW;
      const int lx = 1 + 2 * (t - (ly - 1) * HW) + ((k + ly + 1) & 1);
      ni[q] = ly * W + lx;
      if (t < WI * HW) {
        const int idx = ni[q];
        const T sum = (se[idx - 1] + se[idx + 1]) + (se[idx - W] + se[idx + W]);
        nv[q] = (sum - sr[idx]) * si[idx];
      }
    }
#pragma unroll
    for (int q = 0; q < NH; ++q)
      if (threadIdx.x + q * kTileBlock < WI * HW) se[ni[q]] = nv[q];
    __syncthreads();
  }
  // the block's residual and write-back: thread t < kBlock takes row t / 8 and four cells of
  // it, which lie in one coarse tile (n >= 4); the other threads only join the barriers
  const bool rt = threadIdx.x < kBlock;
  const int r = (threadIdx.x >> 3) & (kTile - 1), c0 = (threadIdx.x & 7) * 4;
  const int j = y0 + r;
  double acc = 0.0, acc2 = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = x0 + c0 + q;
    if (!rt || i >= g.nx || j >= g.ny) continue;
    const int idx = (H + r) * W + H + c0 + q;
    const double d = double(sr[idx] - lap5<T>(se[idx], se[idx - 1], se[idx + 1], se[idx - W],
                                              se[idx + W], cell_faces(g, i, j)));
    acc += d;
    acc2 = maxmode ? fmax(acc2, fabs(d)) : acc2 + d * d;
    eout[off + (long long)j * g.nx + i] = se[idx];
  }
  // per coarse tile: its n rows x n/4 threads reduce pairwise, in a fixed order
  const int n = g.n, per = (n * n) >> 2;
  const int tile = (r >> g.log2n) * (kTile >> g.log2n) + (c0 >> g.log2n);
  const int k = (r & (n - 1)) * (n >> 2) + ((c0 & (n - 1)) >> 2);
  if (rt) {
    p1[tile * per + k] = acc;
    p2[tile * per + k] = acc2;
  }
  __syncthreads();
  for (int st = per >> 1; st > 0; st >>= 1) {
    if (rt && k < st) {
      p1[tile * per + k] += p1[tile * per + k + st];
      p2[tile * per + k] = maxmode ? fmax(p2[tile * per + k], p2[tile * per + k + st])
                                   : p2[tile * per + k] + p2[tile * per + k + st];
    }
    __syncthreads();
  }
  if (rt && k == 0) {
    const int I = (x0 + c0) >> g.log2n, J = j >> g.log2n;
    if (I < g.ncx && J < g.ncy) {
      const long long o = (long long)blockIdx.z * g.cplane + (long long)J * g.ncx + I;
      rc[o] = p1[tile * per];
      if (psq) psq[o] = p2[tile * per];
    }
  }
}

// ----------------------------------------------------------------------------------------
// The exact coarse solve of a small coarse grid (at most kSmallCoarse cells per axis) in one
// workgroup per grid: E = V_y ((F_y^T R_c F_x) .* Lambda^-1) V_x^T as four products through
// LDS, each output entry one FP64 dot product in index order.  One launch instead of four.
// ----------------------------------------------------------------------------------------
constexpr int kSmallCoarse = 32;

__global__ __launch_bounds__(kSmallCoarse * kSmallCoarse) void k_coarse_small(
    int ncx, int ncy, long long cplane, const double* __restrict__ R, const double* __restrict__ Fx,
    const double* __restrict__ Fy, const double* __restrict__ Vx, const double* __restrict__ Vy,
    const double* __restrict__ invLam, double* __restrict__ E) {
  __shared__ double A[kSmallCoarse * kSmallCoarse], B[kSmallCoarse * kSmallCoarse];
  const double* Rb = R + (long long)blockIdx.x * cplane;
  double* Eb = E + (long long)blockIdx.x * cplane;
  const int N = ncx * ncy, step = blockDim.x;
  for (int t = threadIdx.x; t < N; t += step) A[t] = Rb[t];
  __syncthreads();
  for (int t = threadIdx.x; t < N; t += step) {  // T1 = R_c F_x
    const int J = t / ncx, k = t - J * ncx;
    double acc = 0.0;
    for (int I = 0; I < ncx; ++I) acc = fma(A[J * ncx + I], Fx[I * ncx + k], acc);
    B[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N; t += step) {  // T2 = (F_y^T T1) .* Lambda^-1
    const int l = t / ncx, k = t - l * ncx;
    double acc = 0.0;
    for (int J = 0; J < ncy; ++J) acc = fma(Fy[J * ncy + l], B[J * ncx + k], acc);
    A[t] = acc * invLam[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N; t += step) {  // T3 = V_y T2
    const int J = t / ncx, k = t - J * ncx;
    double acc = 0.0;
    for (int l = 0; l < ncy; ++l) acc = fma(Vy[J * ncy + l], A[l * ncx + k], acc);
    B[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N; t += step) {  // E = T3 V_x^T
    const int J = t / ncx, I = t - J * ncx;
    double acc = 0.0;
    for (int k = 0; k < ncx; ++k) acc = fma(B[J * ncx + k], Vx[I * ncx + k], acc);
    Eb[t] = acc;
  }
}

// ----------------------------------------------------------------------------------------
// Outer FP64 residual: r = h^2 (b - mean b) - A'x, written as T, with per-tile sums of r
// (the first coarse right-hand side), sum of r^2, max |r| and, on request, the same two for
// the right-hand side.  Same workgroup layout as k_restrict.
// ----------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_outer_residual(Geo g, const double* __restrict__ b,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ mean_b,
                                                           double h2, T* __restrict__ rT,
                                                           double* __restrict__ rc,
                                                           Partials pt) {
  __shared__ double sh[6][4][16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int x0 = blockIdx.x * kWave, J = blockIdx.y;
  const long long off = (long long)blockIdx.z * g.plane;
  const double* bb = b + off;
  const double* xb = x + off;
  const double mb = mean_b[blockIdx.z];
  const int i = x0 + lane;
  double acc = 0.0, acc2 = 0.0, amax = 0.0, bsq = 0.0, bmax = 0.0;
  if (i < g.nx) {
    const int iw = g.per_x ? imod(i - 1, g.nx) : i - 1;
    const int ie = g.per_x ? imod(i + 1, g.nx) : i + 1;
    for (int r = wave; r < g.n && J * g.n + r < g.ny; r += 4) {
      const int j = J * g.n + r;
      const int js = g.per_y ? imod(j - 1, g.ny) : j - 1;
      const int jn = g.per_y ? imod(j + 1, g.ny) : j + 1;
      const CellFaces f = cell_faces(g, i, j);
      const double* row = xb + (long long)j * g.nx;
      double c = row[i];
      double w = f.hw ? row[iw] : 0.0;
      double ee = f.he ? row[ie] : 0.0;
      double s = f.hs ? xb[(long long)js * g.nx + i] : 0.0;
      double nn = f.hn ? xb[(long long)jn * g.nx + i] : 0.0;
      double bp = h2 * (bb[(long long)j * g.nx + i] - mb);
      double res = bp - lap5<double>(c, w, ee, s, nn, f);
      if (rT) rT[off + (long long)j * g.nx + i] = T(res);
      acc += res;
      acc2 += res * res;
      amax = fmax(amax, fabs(res));
      bsq += bp * bp;
      bmax = fmax(bmax, fabs(bp));
    }
  }
  acc = wave_sum_group(acc, g.n);
  acc2 = wave_sum_group(acc2, g.n);
  amax = wave_max_group(amax, g.n);
  bsq = wave_sum_group(bsq, g.n);
  bmax = wave_max_group(bmax, g.n);
  if ((lane & (g.n - 1)) == 0) {
    const int t = lane >> g.log2n;
    sh[0][wave][t] = acc;
    sh[1][wave][t] = acc2;
    sh[2][wave][t] = amax;
    sh[3][wave][t] = bsq;
    sh[4][wave][t] = bmax;
  }
  __syncthreads();
  const int tiles = kWave >> g.log2n;
  if ((int)threadIdx.x < tiles) {
    const int I = (x0 >> g.log2n) + threadIdx.x;
    if (I < g.ncx) {
      const long long o = (long long)blockIdx.z * g.cplane + (long long)J * g.ncx + I;
      const int t = threadIdx.x;
      if (rc) rc[o] = ((sh[0][0][t] + sh[0][1][t]) + sh[0][2][t]) + sh[0][3][t];
      if (pt.sumsq) pt.sumsq[o] = ((sh[1][0][t] + sh[1][1][t]) + sh[1][2][t]) + sh[1][3][t];
      if (pt.maxabs) pt.maxabs[o] = fmax(fmax(sh[2][0][t], sh[2][1][t]), fmax(sh[2][2][t], sh[2][3][t]));
      if (pt.bsumsq) pt.bsumsq[o] = ((sh[3][0][t] + sh[3][1][t]) + sh[3][2][t]) + sh[3][3][t];
      if (pt.bmaxabs) pt.bmaxabs[o] = fmax(fmax(sh[4][0][t], sh[4][1][t]), fmax(sh[4][2][t], sh[4][3][t]));
    }
  }
}

// Per-tile sums of a FP64 field (for means).
__global__ __launch_bounds__(kBlock) void k_tile_sum(Geo g, const double* __restrict__ x,
                                                     double* __restrict__ part) {
  __shared__ double s1[4][16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int x0 = blockIdx.x * kWave, J = blockIdx.y;
  const double* xb = x + (long long)blockIdx.z * g.plane;
  const int i = x0 + lane;
  double acc = 0.0;
  if (i < g.nx)
    for (int r = wave; r < g.n && J * g.n + r < g.ny; r += 4) acc += xb[(long long)(J * g.n + r) * g.nx + i];
  acc = wave_sum_group(acc, g.n);
  if ((lane & (g.n - 1)) == 0) s1[wave][lane >> g.log2n] = acc;
  __syncthreads();
  const int tiles = kWave >> g.log2n;
  if ((int)threadIdx.x < tiles) {
    const int I = (x0 >> g.log2n) + threadIdx.x;
    const int t = threadIdx.x;
    if (I < g.ncx)
      part[(long long)blockIdx.z * g.cplane + (long long)J * g.ncx + I] =
          ((s1[0][t] + s1[1][t]) + s1[2][t]) + s1[3][t];
  }
}

// Second reduction stage: the partials of each grid are reduced in chunks of kChunk by
// gridDim.x workgroups, in a fixed order (reproducible); a further pass (same kernel, one
// workgroup per grid, over all the chunk results however many there are) reduces them when
// there is more than one chunk.
constexpr int kChunk = 4096;

// One thread's share of a strided reduction: a = op(a, p[i]) for i = first, first + kBlock,
// ... below end, in that order.  The loads of kChunk / kBlock consecutive terms are all issued
// before the first of them is combined, so the thread waits on memory once per group instead
// of once per term; the result is the same as term by term.
__device__ __forceinline__ double strided_reduce(const double* __restrict__ p, int first, int end,
                                                 bool is_max) {
  constexpr int K = kChunk / kBlock;
  double a = 0.0;
  for (int base = first; base < end; base += K * kBlock) {
    double v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int i = base + j * kBlock;
      v[j] = i < end ? p[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (base + j * kBlock < end) a = is_max ? fmax(a, v[j]) : a + v[j];
    }
  }
  return a;
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ part, int count,
                                                     long long stride, int op, double scale,
                                                     double* __restrict__ out, int out_stride,
                                                     int slot) {
  __shared__ double sh[kBlock];
  const double* p = part + (long long)blockIdx.y * stride;
  // one workgroup per grid (a single stage, or the pass over the chunk results) takes every
  // term, however many chunks the first stage made
  const int lo = blockIdx.x * kChunk, hi = gridDim.x == 1 ? count : min(count, lo + kChunk);
  sh[threadIdx.x] = strided_reduce(p, lo + int(threadIdx.x), hi, op == MAX);
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double o = sh[threadIdx.x + w];
      sh[threadIdx.x] = op == MAX ? fmax(sh[threadIdx.x], o) : sh[threadIdx.x] + o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (gridDim.x == 1) out[(long long)blockIdx.y * out_stride + slot] = sh[0] * scale;
    else out[(long long)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_to(long long total, double* __restrict__ x,
                                                   const T* __restrict__ e) {
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock)
    x[k] += double(e[k]);
}

__global__ __launch_bounds__(kBlock) void k_sub_scalar(long long plane, int batch,
                                                       double* __restrict__ x,
                                                       const double* __restrict__ vals,
                                                       int val_stride, int slot) {
  const long long total = plane * batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock)
    x[k] -= vals[(k / plane) * val_stride + slot];
}

// ----------------------------------------------------------------------------------------
// Small batched FP64 GEMM for the separable coarse solve: C = op(A) op(B) [.* S].
// A 16 x 16 output tile per workgroup (a 256 x 256 product spreads over 256 workgroups, one
// per CU).  The whole K panel of A and B (up to 256 deep per pass) is loaded in one batch so
// that all loads are in flight together, the next panel's while the current one is being
// multiplied; the 4 waves each accumulate a quarter of K on
// the matrix cores (V_MFMA_F64_16X16X4F64: a 16 x 4 by 4 x 16 product per instruction) and
// the quarters are added in wave order through LDS.
// ----------------------------------------------------------------------------------------
constexpr int kGemmTile = 16, kGemmK = 256;

template <int TA, int TB>
__global__ __launch_bounds__(kBlock) void k_gemm(int M, int N, int K, const double* __restrict__ A,
                                                 long long sA, int lda,
                                                 const double* __restrict__ B, long long sB,
                                                 int ldb, double* __restrict__ C, long long sC,
                                                 int ldc, const double* __restrict__ S) {
  __shared__ double As[kGemmK][kGemmTile + 1];  // [k][m]
  __shared__ double Bs[kGemmK][kGemmTile + 1];  // [k][n]
  __shared__ double red[4][kGemmTile][kGemmTile + 1];
  A += (long long)blockIdx.z * sA;
  B += (long long)blockIdx.z * sB;
  C += (long long)blockIdx.z * sC;
  const int m0 = blockIdx.y * kGemmTile, n0 = blockIdx.x * kGemmTile;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  // MFMA operands: lane l holds A[row l % 16][k l / 16] and B[k l / 16][col l % 16] of a
  // 4-deep step; the 16 x 16 result lies in lane l's four values r as row l / 16 + 4 r,
  // column l % 16
  const int li = lane & 15, lk = lane >> 4;
  typedef double Vec4d __attribute__((ext_vector_type(4)));
  Vec4d acc = {0.0, 0.0, 0.0, 0.0};
  constexpr int PER = kGemmTile * kGemmK / kBlock;  // panel elements per thread and operand
  // every load of both panels is issued before any is stored, so that one memory latency
  // covers the whole panel; loads are coalesced along the contiguous index of the matrix
  double ra[PER], rb[PER];
  auto load_panel = [&](int k0) {
    const int kc = min(kGemmK, K - k0);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * kBlock;
      {
        const int m = TA ? (t & (kGemmTile - 1)) : (t / kGemmK);
        const int k = TA ? (t / kGemmTile) : (t & (kGemmK - 1));
        const int gm = m0 + m, gk = k0 + k;
        ra[i] = (gm < M && k < kc) ? (TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk])
                                   : 0.0;
      }
      {
        const int nn = TB ? (t / kGemmK) : (t & (kGemmTile - 1));
        const int k = TB ? (t & (kGemmK - 1)) : (t / kGemmTile);
        const int gk = k0 + k, gn = n0 + nn;
        rb[i] = (k < kc && gn < N) ? (TB ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn])
                                   : 0.0;
      }
    }
  };
  load_panel(0);
  for (int k0 = 0; k0 < K; k0 += kGemmK) {
    const int kc = min(kGemmK, K - k0);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * kBlock;
      As[TA ? (t / kGemmTile) : (t & (kGemmK - 1))][TA ? (t & (kGemmTile - 1)) : (t / kGemmK)] = ra[i];
      Bs[TB ? (t & (kGemmK - 1)) : (t / kGemmTile)][TB ? (t / kGemmK) : (t & (kGemmTile - 1))] = rb[i];
    }
    __syncthreads();
    // the next panel's loads are in flight while this one runs on the matrix cores
    if (k0 + kGemmK < K) load_panel(k0 + kGemmK);
    // this wave's quarter of the panel, in steps of 4 (rows past kc hold zeros)
    const int q = (kc + 15) / 16 * 4;
    const int ka = wave * q;
    for (int kk = ka; kk < ka + q; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[kk + lk][li], Bs[kk + lk][li], acc, 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave][lk + 4 * r][li] = acc[r];
  __syncthreads();
  const int m = threadIdx.x / kGemmTile, nn = threadIdx.x & (kGemmTile - 1);
  const int gm = m0 + m, gn = n0 + nn;
  if (gm < M && gn < N) {
    double v = ((red[0][m][nn] + red[1][m][nn]) + red[2][m][nn]) + red[3][m][nn];
    if (S) v *= S[(long long)gm * N + gn];
    C[(long long)gm * ldc + gn] = v;
  }
}

// ----------------------------------------------------------------------------------------
// Coarse 9-point stencil from the face sums of Eq. 6 (x faces) and Eq. 7 (y faces): for
// each fine face on a coarse face, the outward derivative of the bilinear interpolant of
// the coarse unknowns.  A Neumann wall carries no flux; a Dirichlet wall carries the flux
// towards the negated ghost centre.  An off-grid (ghost) neighbour is folded onto the cell
// it mirrors, added (Neumann) or subtracted (Dirichlet).  One thread per coarse cell.
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_coarse_assemble(Geo g, int gmg5,
                                                            double* __restrict__ coef) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= g.ncx * g.ncy) return;
  const int J = cell / g.ncx, I = cell - J * g.ncx;
  double c[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) c[a][b] = 0.0;
  const int n = g.n;
  const bool openE = g.per_x || I < g.ncx - 1 || (g.dmask & kDirE);
  const bool openW = g.per_x || I > 0 || (g.dmask & kDirW);
  const bool openN = g.per_y || J < g.ncy - 1 || (g.dmask & kDirN);
  const bool openS = g.per_y || J > 0 || (g.dmask & kDirS);
  if (gmg5) {  // unit 5-point stencil at the coarse spacing
    if (openE) c[1][2] += 1.0, c[1][1] -= 1.0;
    if (openW) c[1][0] += 1.0, c[1][1] -= 1.0;
    if (openN) c[2][1] += 1.0, c[1][1] -= 1.0;
    if (openS) c[0][1] += 1.0, c[1][1] -= 1.0;
  }
  // Eq. 6 / Eq. 7 face sums, fine row by fine row (x faces) and fine column by fine column
  // (y faces): the fine centre k of the tile lies between coarse centres lo and lo + 1
  // (relative offset off = -1 or 0) with weight t of the upper one (interp_axis: the
  // rectangle's own size next to a short last tile), and the derivative across a face
  // divides by the distance of the two centres it separates (n with full tiles; a ghost
  // centre is the mirror image in the wall or the wrapped centre).
  const int x0 = I * n, y0 = J * n;
  const int kx = gmg5 ? 0 : min(n, g.nx - x0), ky = gmg5 ? 0 : min(n, g.ny - y0);
  const double dxE = 0.5 * double(centre2(I + 1, g.nx, n, g.ncx, g.per_x) - centre2(I, g.nx, n, g.ncx, g.per_x));
  const double dxW = 0.5 * double(centre2(I, g.nx, n, g.ncx, g.per_x) - centre2(I - 1, g.nx, n, g.ncx, g.per_x));
  const double dyN = 0.5 * double(centre2(J + 1, g.ny, n, g.ncy, g.per_y) - centre2(J, g.ny, n, g.ncy, g.per_y));
  const double dyS = 0.5 * double(centre2(J, g.ny, n, g.ncy, g.per_y) - centre2(J - 1, g.ny, n, g.ncy, g.per_y));
  for (int k = 0; k < max(kx, ky); ++k) {
    int lo;
    double t;
    if (k < ky) {  // x faces (Eq. 6): fine row y0 + k, columns I + d and I + d + 1
      interp_axis(y0 + k, g.ny, n, g.log2n, g.ncy, g.per_y, lo, t);
      const int off = lo - J;
      if (openE) {  // outward +x, columns 0 -> +1
        const double wl = (1.0 - t) / dxE, wh = t / dxE;
        c[off + 1][2] += wl;
        c[off + 1][1] -= wl;
        c[off + 2][2] += wh;
        c[off + 2][1] -= wh;
      }
      if (openW) {  // outward -x, columns -1 -> 0
        const double wl = (1.0 - t) / dxW, wh = t / dxW;
        c[off + 1][1] -= wl;
        c[off + 1][0] += wl;
        c[off + 2][1] -= wh;
        c[off + 2][0] += wh;
      }
    }
    if (k < kx) {  // y faces (Eq. 7): fine column x0 + k
      interp_axis(x0 + k, g.nx, n, g.log2n, g.ncx, g.per_x, lo, t);
      const int off = lo - I;
      if (openN) {
        const double wl = (1.0 - t) / dyN, wh = t / dyN;
        c[2][off + 1] += wl;
        c[1][off + 1] -= wl;
        c[2][off + 2] += wh;
        c[1][off + 2] -= wh;
      }
      if (openS) {
        const double wl = (1.0 - t) / dyS, wh = t / dyS;
        c[1][off + 1] -= wl;
        c[0][off + 1] += wl;
        c[1][off + 2] -= wh;
        c[0][off + 2] += wh;
      }
    }
  }
  if (!g.per_x) {
    const double sw = (g.dmask & kDirW) ? -1.0 : 1.0, se = (g.dmask & kDirE) ? -1.0 : 1.0;
    if (I == 0)
      for (int a = 0; a < 3; ++a) {
        c[a][1] += sw * c[a][0];
        c[a][0] = 0.0;
      }
    if (I == g.ncx - 1)
      for (int a = 0; a < 3; ++a) {
        c[a][1] += se * c[a][2];
        c[a][2] = 0.0;
      }
  }
  if (!g.per_y) {
    const double ss = (g.dmask & kDirS) ? -1.0 : 1.0, sn = (g.dmask & kDirN) ? -1.0 : 1.0;
    if (J == 0)
      for (int b = 0; b < 3; ++b) {
        c[1][b] += ss * c[0][b];
        c[0][b] = 0.0;
      }
    if (J == g.ncy - 1)
      for (int b = 0; b < 3; ++b) {
        c[1][b] += sn * c[2][b];
        c[2][b] = 0.0;
      }
  }
  double* o = coef + (long long)cell * 9;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) o[3 * a + b] = c[a][b];
}

// ----------------------------------------------------------------------------------------
// One block-iterative Gauss-Seidel iteration on the coarse system A_c E = R (Sec. 4: the
// coarse grid is iterated by block GS, one synchronization per iteration).  A workgroup
// owns a tile of tx x ty coarse cells (at most kCB x kCB, aligned at cell 0): the tile and
// a ring of neighbours are staged in LDS with the values of the previous iteration, then
// the tile's cells are updated in lexicographic order (I fastest) in place, so a cell sees
// the new values of its tile's predecessors and the old values of everything else.  The
// host picks tiles narrower than every periodic axis (bgs_tile), so a neighbour reached
// across a periodic seam always belongs to another tile and is read from the ring.
// Lexicographic order is run as hyperplanes li + 2 lj = s, s = 0 .. (tx - 1) + 2 (ty - 1):
// the 9-point neighbours that precede a cell lie on earlier hyperplanes and those that
// follow on later ones, so each hyperplane is one parallel step.  Update:
// E_C = (R_C - sum of c_nb E_nb) / c_C, neighbours in the
// order (dj, di) = (-1,-1) .. (1,1) without the centre, summed left to right.  Before the
// update each cell forms the residual of the incoming iterate, R_C - (c_C E_C + sum ...),
// and the workgroup writes the maximum of its magnitude to part_max[tile].
// ----------------------------------------------------------------------------------------
constexpr int kCB = 16;

__global__ __launch_bounds__(kBlock) void k_coarse_bgs(Geo g, const double* __restrict__ coef,
                                                       const double* __restrict__ R,
                                                       const double* __restrict__ Ein,
                                                       double* __restrict__ Eout,
                                                       double* __restrict__ part_max, int tx,
                                                       int ty, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;  // enqueued past a device-side stop
  constexpr int LW = kCB + 2;
  __shared__ double sE[LW * LW];
  __shared__ double smax[kBlock / kWave];
  const int li = threadIdx.x % kCB, lj = threadIdx.x / kCB;
  const int I0 = blockIdx.x * tx, J0 = blockIdx.y * ty;
  const long long cb = (long long)blockIdx.z * g.cplane;
  const int I = I0 + li, J = J0 + lj;
  const bool active = li < tx && lj < ty && I < g.ncx && J < g.ncy;
  // stage the tile and its ring (ring positions are other tiles' cells, or 0 off the grid;
  // slots beyond a narrower tile's ring are staged too and never read)
  for (int t = threadIdx.x; t < LW * LW; t += kBlock) {
    const int rj = t / LW, ri = t - rj * LW;
    int jj = J0 + rj - 1, ii = I0 + ri - 1;
    bool ok = true;
    if (g.per_y) jj = imod(jj, g.ncy);
    else ok = ok && jj >= 0 && jj < g.ncy;
    if (g.per_x) ii = imod(ii, g.ncx);
    else ok = ok && ii >= 0 && ii < g.ncx;
    sE[t] = ok ? Ein[cb + (long long)jj * g.ncx + ii] : 0.0;
  }
  // the LDS slot of each neighbour
  int nb[9];
  double c[9];
  double r = 0.0;
  if (active) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      nb[k] = (lj + k / 3) * LW + li + k % 3;
      c[k] = coef[((long long)J * g.ncx + I) * 9 + k];
    }
    r = R[cb + (long long)J * g.ncx + I];
  }
  __syncthreads();
  double amax = 0.0;
  if (active) {
    double acc = c[4] * sE[nb[4]];
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (k != 4) acc = acc + c[k] * sE[nb[k]];
    amax = fabs(r - acc);
  }
  amax = wave_max_group(amax, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) smax[threadIdx.x / kWave] = amax;
  // hyperplane steps: each begins after the previous one's LDS writes (and, for s = 0, after
  // the residual reads of the incoming iterate)
  const int step = li + 2 * lj;
  for (int s = 0; s < tx + 2 * ty - 2; ++s) {
    __syncthreads();
    if (active && step == s) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (k != 4) acc = acc + c[k] * sE[nb[k]];
      sE[nb[4]] = (r - acc) / c[4];
    }
  }
  __syncthreads();
  if (active) Eout[cb + (long long)J * g.ncx + I] = sE[nb[4]];
  if (threadIdx.x == 0) {
    double m = smax[0];
    for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, smax[w]);
    part_max[(long long)blockIdx.z * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = m;
  }
}

// ----------------------------------------------------------------------------------------
// Multicolour Gauss-Seidel on the coarse system A_c E = R (Sec. 3.1: multicolour ordering
// iterates stencils wider than five points concurrently; Sec. 4.3: one synchronization per
// colour).  Along each axis cell i has colour i mod 2, except that the last cell of an odd
// periodic axis takes colour 2 (its wrapped neighbour is cell 0); cell (J, I) has colour
// qy(J) * Qx + qx(I).  Two cells the 9-point stencil couples never share a colour, so a
// colour's cells are updated concurrently, each reading only cells of other colours.  An
// iteration is one launch per colour, in increasing colour order: the first launch forms
// the residual of the incoming iterate at every cell (maxima per workgroup) and writes
// Eout, colour 0 updated and every other cell copied; the next launches update their
// colour in place in Eout.  Residual: R_C - (c_C E_C + sum of c_nb E_nb); update:
// E_C = (R_C - sum of c_nb E_nb) / c_C, both with the neighbours in the order
// (dj, di) = (-1,-1) .. (1,1) without the centre and summed left to right, as block GS.
// ----------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ int mc_axis_colours(int nc, bool per) {
  return per && (nc & 1) ? 3 : 2;
}
// cells of colour q along an axis of nc cells that has Q colours, and the m-th of them
__host__ __device__ __forceinline__ int mc_axis_count(int nc, int Q, int q) {
  return q == 2 ? 1 : (Q == 3 && q == 0 ? (nc - 1) / 2 : (nc - q + 1) / 2);
}
__device__ __forceinline__ int mc_axis_cell(int nc, int q, int m) { return q == 2 ? nc - 1 : q + 2 * m; }
__device__ __forceinline__ int mc_axis_colour(int i, int nc, int Q) {
  return (Q == 3 && i == nc - 1) ? 2 : (i & 1);
}

// The 8 neighbour values of cell (J, I) of plane Eb in stencil order (0 off a walled grid).
__device__ __forceinline__ void mc_neighbours(const Geo& g, const double* __restrict__ Eb, int J,
                                              int I, double v[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    int jj = J + k / 3 - 1, ii = I + k % 3 - 1;
    bool ok = true;
    if (g.per_y) jj = jj < 0 ? jj + g.ncy : (jj >= g.ncy ? jj - g.ncy : jj);
    else ok = jj >= 0 && jj < g.ncy;
    if (g.per_x) ii = ii < 0 ? ii + g.ncx : (ii >= g.ncx ? ii - g.ncx : ii);
    else ok = ok && ii >= 0 && ii < g.ncx;
    v[k] = ok ? Eb[(long long)jj * g.ncx + ii] : 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_coarse_mc_first(Geo g, const double* __restrict__ coef,
                                                            const double* __restrict__ R,
                                                            const double* __restrict__ Ein,
                                                            double* __restrict__ Eout,
                                                            double* __restrict__ part_max, int Qx,
                                                            int Qy, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;  // enqueued past a device-side stop
  __shared__ double smax[kBlock / kWave];
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  const long long cb = (long long)blockIdx.z * g.cplane;
  double amax = 0.0;
  if (cell < g.cplane) {
    const int J = cell / g.ncx, I = cell - J * g.ncx;
    const double* c = coef + (long long)cell * 9;
    double v[9];
    mc_neighbours(g, Ein + cb, J, I, v);
    const double r = R[cb + cell], e = Ein[cb + cell];
    double acc = c[4] * e, sum = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if (k == 4) continue;
      acc = acc + c[k] * v[k];
      sum = sum + c[k] * v[k];
    }
    amax = fabs(r - acc);
    const bool first = mc_axis_colour(J, g.ncy, Qy) == 0 && mc_axis_colour(I, g.ncx, Qx) == 0;
    Eout[cb + cell] = first ? (r - sum) / c[4] : e;
  }
  amax = wave_max_group(amax, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) smax[threadIdx.x / kWave] = amax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smax[0];
    for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, smax[w]);
    part_max[(long long)blockIdx.z * gridDim.x + blockIdx.x] = m;
  }
}

// Colour (qy, qx) of one iteration, in place: thread t updates the t-th cell of the colour
// (cx cells of it per row of the colour).
__global__ __launch_bounds__(kBlock) void k_coarse_mc_colour(Geo g, const double* __restrict__ coef,
                                                             const double* __restrict__ R,
                                                             double* __restrict__ E, int qy, int qx,
                                                             int cx, int count,
                                                             const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= count) return;
  const int my = t / cx, mx = t - my * cx;
  const int J = mc_axis_cell(g.ncy, qy, my), I = mc_axis_cell(g.ncx, qx, mx);
  const long long cb = (long long)blockIdx.z * g.cplane;
  const long long cell = (long long)J * g.ncx + I;
  const double* c = coef + cell * 9;
  double v[9];
  mc_neighbours(g, E + cb, J, I, v);
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    sum = sum + c[k] * v[k];
  }
  E[cb + cell] = (R[cb + cell] - sum) / c[4];
}

// ----------------------------------------------------------------------------------------
// Staggered-grid operators (FP64).  nxu = number of u faces per row.
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_div(Geo g, const double* __restrict__ u,
                                                const double* __restrict__ v, double h,
                                                double* __restrict__ b) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long total = g.plane * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / g.plane;
    const int rem = int(k - bi * g.plane);
    const int j = rem / g.nx, i = rem - j * g.nx;
    const double* ub = u + bi * (long long)g.ny * nxu + (long long)j * nxu;
    const double* vb = v + bi * (long long)(g.ny + 1) * g.nx;
    const int ie = g.per_x ? (i + 1 == g.nx ? 0 : i + 1) : i + 1;
    const double du = ub[ie] - ub[i];
    const double dv = vb[(long long)(j + 1) * g.nx + i] - vb[(long long)j * g.nx + i];
    b[k] = (du + dv) / h;
  }
}

// G p on u face f of row j (pr = that row of p): (p_C - p_W) / h; zero on a Neumann wall
// face; the mirror ghost -p behind a Dirichlet wall face.
__device__ __forceinline__ double grad_u_face(const Geo& g, const double* pr, int f, double h) {
  if (g.per_x) return (pr[f] - pr[f == 0 ? g.nx - 1 : f - 1]) / h;
  if (f == 0) return (g.dmask & kDirW) ? (pr[0] - (-pr[0])) / h : 0.0;
  if (f == g.nx) return (g.dmask & kDirE) ? ((-pr[g.nx - 1]) - pr[g.nx - 1]) / h : 0.0;
  return (pr[f] - pr[f - 1]) / h;
}

// G p on v face f of column i (pb = the grid's p).
__device__ __forceinline__ double grad_v_face(const Geo& g, const double* pb, int f, int i, double h) {
  if (f == 0) {
    const double q = pb[i];
    return (g.dmask & kDirS) ? (q - (-q)) / h : 0.0;
  }
  if (f == g.ny) {
    const double q = pb[(long long)(g.ny - 1) * g.nx + i];
    return (g.dmask & kDirN) ? ((-q) - q) / h : 0.0;
  }
  return (pb[(long long)f * g.nx + i] - pb[(long long)(f - 1) * g.nx + i]) / h;
}

__global__ __launch_bounds__(kBlock) void k_grad_u(Geo g, const double* __restrict__ p, double h,
                                                   double* __restrict__ gu) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long per = (long long)g.ny * nxu, total = per * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int j = rem / nxu, f = rem - j * nxu;
    gu[k] = grad_u_face(g, p + bi * g.plane + (long long)j * g.nx, f, h);
  }
}

__global__ __launch_bounds__(kBlock) void k_grad_v(Geo g, const double* __restrict__ p, double h,
                                                   double* __restrict__ gv) {
  const long long per = (long long)(g.ny + 1) * g.nx, total = per * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int f = rem / g.nx, i = rem - f * g.nx;
    gv[k] = grad_v_face(g, p + bi * g.plane, f, i, h);
  }
}

// ----------------------------------------------------------------------------------------
// Explicit predictor of Goda's scheme (Sec. 2.2, Eq. 3) with second-order central
// differences on the staggered grid (Sec. 2.3), FP64, one thread per face:
//   v* = v + dt (eta lap v - (v . grad) v) - G p,
// p carrying the time step.  Interior u face (west face of cell (i, j)):
//   dudx = (u_E - u_W) / (2h), dudy = (u_N - u_S) / (2h),
//   lap = (((u_E + u_W) + u_N) + u_S - 4 u) / h^2, vbar = ((v_SW + v_SE) + (v_NW + v_NE)) / 4,
//   u* = u + dt (eta lap - (u dudx + vbar dudy)) - (p_C - p_W) / h;
// v faces alike with x and y exchanged.  A wall face keeps its normal velocity; a tangential
// neighbour behind a wall is the ghost 2 U_w - (the face's own value); a periodic x axis
// wraps.  wall = tangential velocities (west wall v, east wall v, south wall u, north wall u).
// ----------------------------------------------------------------------------------------
struct Walls {
  double vw, ve, us, un;
};

__global__ __launch_bounds__(kBlock) void k_predict_u(Geo g, const double* __restrict__ u,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ p, double h,
                                                      double dt, double eta, Walls wl,
                                                      double* __restrict__ us) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long per = (long long)g.ny * nxu, total = per * g.batch;
  const double two_h = 2.0 * h, hh = h * h;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int j = rem / nxu, i = rem - j * nxu;
    const double* ub = u + bi * per;
    const double c = ub[(long long)j * nxu + i];
    if (!g.per_x && (i == 0 || i == g.nx)) {  // wall face: normal velocity kept
      us[k] = c;
      continue;
    }
    const double* vb = v + bi * (long long)(g.ny + 1) * g.nx;
    const double* pr = p + bi * g.plane + (long long)j * g.nx;
    const int ie = g.per_x ? (i + 1 == g.nx ? 0 : i + 1) : i + 1;
    const int im = g.per_x ? (i == 0 ? g.nx - 1 : i - 1) : i - 1;
    const double ue = ub[(long long)j * nxu + ie], uw = ub[(long long)j * nxu + im];
    const double un = j + 1 < g.ny ? ub[(long long)(j + 1) * nxu + i] : 2.0 * wl.un - c;
    const double usv = j > 0 ? ub[(long long)(j - 1) * nxu + i] : 2.0 * wl.us - c;
    const double vbar = ((vb[(long long)j * g.nx + im] + vb[(long long)j * g.nx + i]) +
                         (vb[(long long)(j + 1) * g.nx + im] + vb[(long long)(j + 1) * g.nx + i])) /
                        4.0;
    const double dudx = (ue - uw) / two_h, dudy = (un - usv) / two_h;
    const double lap = ((((ue + uw) + un) + usv) - 4.0 * c) / hh;
    const double gp = (pr[i] - pr[im]) / h;
    us[k] = c + dt * (eta * lap - (c * dudx + vbar * dudy)) - gp;
  }
}

__global__ __launch_bounds__(kBlock) void k_predict_v(Geo g, const double* __restrict__ u,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ p, double h,
                                                      double dt, double eta, Walls wl,
                                                      double* __restrict__ vs) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long per = (long long)(g.ny + 1) * g.nx, total = per * g.batch;
  const double two_h = 2.0 * h, hh = h * h;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int j = rem / g.nx, i = rem - j * g.nx;
    const double* vb = v + bi * per;
    const double c = vb[(long long)j * g.nx + i];
    if (j == 0 || j == g.ny) {  // wall face: normal velocity kept
      vs[k] = c;
      continue;
    }
    const double* ub = u + bi * (long long)g.ny * nxu;
    const double* pb = p + bi * g.plane;
    const double vn = vb[(long long)(j + 1) * g.nx + i], vsv = vb[(long long)(j - 1) * g.nx + i];
    double ve, vw;
    if (g.per_x) {
      ve = vb[(long long)j * g.nx + (i + 1 == g.nx ? 0 : i + 1)];
      vw = vb[(long long)j * g.nx + (i == 0 ? g.nx - 1 : i - 1)];
    } else {
      ve = i + 1 < g.nx ? vb[(long long)j * g.nx + i + 1] : 2.0 * wl.ve - c;
      vw = i > 0 ? vb[(long long)j * g.nx + i - 1] : 2.0 * wl.vw - c;
    }
    const int ip = g.per_x ? (i + 1 == g.nx ? 0 : i + 1) : i + 1;
    const double ubar = ((ub[(long long)(j - 1) * nxu + i] + ub[(long long)(j - 1) * nxu + ip]) +
                         (ub[(long long)j * nxu + i] + ub[(long long)j * nxu + ip])) /
                        4.0;
    const double dvdx = (ve - vw) / two_h, dvdy = (vn - vsv) / two_h;
    const double lap = ((((ve + vw) + vn) + vsv) - 4.0 * c) / hh;
    const double gp = (pb[(long long)j * g.nx + i] - pb[(long long)(j - 1) * g.nx + i]) / h;
    vs[k] = c + dt * (eta * lap - (ubar * dvdx + c * dvdy)) - gp;
  }
}

// Correction of the projection step: u -= G x, v -= G x (the handle's G), p += x.
__global__ __launch_bounds__(kBlock) void k_correct(Geo g, const double* __restrict__ x, double h,
                                                    double* __restrict__ u, double* __restrict__ v,
                                                    double* __restrict__ p) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long pu = (long long)g.ny * nxu, pv = (long long)(g.ny + 1) * g.nx;
  const long long tu = pu * g.batch, tv = pv * g.batch, tp = g.plane * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < tu + tv + tp;
       k += (long long)gridDim.x * kBlock) {
    if (k < tu) {
      const long long bi = k / pu;
      const int rem = int(k - bi * pu);
      const int j = rem / nxu, f = rem - j * nxu;
      u[k] = u[k] - grad_u_face(g, x + bi * g.plane + (long long)j * g.nx, f, h);
    } else if (k < tu + tv) {
      const long long q = k - tu, bi = q / pv;
      const int rem = int(q - bi * pv);
      const int f = rem / g.nx, i = rem - f * g.nx;
      v[q] = v[q] - grad_v_face(g, x + bi * g.plane, f, i, h);
    } else {
      const long long q = k - tu - tv;
      p[q] = p[q] + x[q];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_div_adjoint_u(Geo g, const double* __restrict__ lam,
                                                          double h, double* __restrict__ gu) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long per = (long long)g.ny * nxu, total = per * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int j = rem / nxu, f = rem - j * nxu;
    const double* lr = lam + bi * g.plane + (long long)j * g.nx;
    double a, c;
    if (g.per_x) {
      a = lr[f == 0 ? g.nx - 1 : f - 1];
      c = lr[f];
    } else {
      a = f >= 1 ? lr[f - 1] : 0.0;
      c = f <= g.nx - 1 ? lr[f] : 0.0;
    }
    gu[k] = (a - c) / h;
  }
}

__global__ __launch_bounds__(kBlock) void k_div_adjoint_v(Geo g, const double* __restrict__ lam,
                                                          double h, double* __restrict__ gv) {
  const long long per = (long long)(g.ny + 1) * g.nx, total = per * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int f = rem / g.nx, i = rem - f * g.nx;
    const double* lb = lam + bi * g.plane;
    const double a = f >= 1 ? lb[(long long)(f - 1) * g.nx + i] : 0.0;
    const double c = f <= g.ny - 1 ? lb[(long long)f * g.nx + i] : 0.0;
    gv[k] = (a - c) / h;
  }
}

__global__ __launch_bounds__(kBlock) void k_grad_adjoint(Geo g, const double* __restrict__ gu,
                                                         const double* __restrict__ gv, double h,
                                                         double* __restrict__ p) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long total = g.plane * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / g.plane;
    const int rem = int(k - bi * g.plane);
    const int j = rem / g.nx, i = rem - j * g.nx;
    const double* ur = gu + bi * (long long)g.ny * nxu + (long long)j * nxu;
    const double* vb = gv + bi * (long long)(g.ny + 1) * g.nx;
    double t = 0.0;
    if (g.per_x) {
      t = ur[i] - ur[i + 1 == g.nx ? 0 : i + 1];
    } else {
      if (i >= 1) t += ur[i];
      if (i <= g.nx - 2) t -= ur[i + 1];
      // a Dirichlet wall face's gradient is +-2 p / h of the cell next to it
      if (i == 0 && (g.dmask & kDirW)) t += 2.0 * ur[0];
      if (i == g.nx - 1 && (g.dmask & kDirE)) t -= 2.0 * ur[g.nx];
    }
    if (j >= 1) t += vb[(long long)j * g.nx + i];
    if (j <= g.ny - 2) t -= vb[(long long)(j + 1) * g.nx + i];
    if (j == 0 && (g.dmask & kDirS)) t += 2.0 * vb[i];
    if (j == g.ny - 1 && (g.dmask & kDirN)) t -= 2.0 * vb[(long long)g.ny * g.nx + i];
    p[k] = t / h;
  }
}

// ----------------------------------------------------------------------------------------
// Additive correction multigrid (the comparison scheme, Sec. 3.2 and Sec. 4), FP64.
// ----------------------------------------------------------------------------------------

// out = 2x2 sums of (r - scale * A'e) over the level grid g (e may be null: sums of r), and
// per output cell the sum of the squared residuals of its 4 cells.
__global__ __launch_bounds__(kBlock) void k_agglomerate(Geo g, const double* __restrict__ r,
                                                        const double* __restrict__ e, double scale,
                                                        double* __restrict__ out,
                                                        double* __restrict__ psq) {
  const int cx = g.nx / 2, cy = g.ny / 2;
  const long long cpl = (long long)cx * cy, total = cpl * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / cpl;
    const int rem = int(k - bi * cpl);
    const int J = rem / cx, I = rem - J * cx;
    const double* rb = r + bi * g.plane;
    const double* eb = e ? e + bi * g.plane : nullptr;
    double sum = 0.0, sq = 0.0;
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        const int i = 2 * I + di, j = 2 * J + dj;
        double res = rb[(long long)j * g.nx + i];
        if (eb) {
          const CellFaces fc = cell_faces(g, i, j);
          const double* row = eb + (long long)j * g.nx;
          const double c = row[i];
          const double w = fc.hw ? row[g.per_x ? imod(i - 1, g.nx) : i - 1] : 0.0;
          const double ee = fc.he ? row[g.per_x ? imod(i + 1, g.nx) : i + 1] : 0.0;
          const double sv = fc.hs ? eb[(long long)(g.per_y ? imod(j - 1, g.ny) : j - 1) * g.nx + i] : 0.0;
          const double nv = fc.hn ? eb[(long long)(g.per_y ? imod(j + 1, g.ny) : j + 1) * g.nx + i] : 0.0;
          res = res - scale * lap5<double>(c, w, ee, sv, nv, fc);
        }
        sum += res;
        sq += res * res;
      }
    out[k] = sum;
    if (psq) psq[k] = sq;
  }
}

// ef (+)= the value of the coarse cell that contains each fine cell (ACM's correction: the
// coarse result is added without interpolation, Sec. 3.2).  g is the fine level.
__global__ __launch_bounds__(kBlock) void k_inject(Geo g, const double* __restrict__ ec,
                                                   double* __restrict__ ef, int assign) {
  const int cx = g.nx / 2;
  const long long cpl = (long long)cx * (g.ny / 2), total = g.plane * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / g.plane;
    const int rem = int(k - bi * g.plane);
    const int j = rem / g.nx, i = rem - j * g.nx;
    const double v = ec[bi * cpl + (long long)(j >> 1) * cx + (i >> 1)];
    ef[k] = assign ? v : ef[k] + v;
  }
}

inline unsigned grid_stride_blocks(long long total) {
  long long b = (total + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return unsigned(b);
}

inline dim3 strip_grid(const Geo& g) {
  return dim3((g.nx + kWave - 1) / kWave, g.ncy, g.batch);
}

// ----------------------------------------------------------------------------------------
// Tables of the exact coarse solve.  Each axis has the 1D factors K = [1 -2 1] and
// M = [1 6 1] / 8 = I + K / 8 with the axis's end rule: circulant when periodic; at a
// Neumann end K = -1 and M = 7/8; at a Dirichlet end K = -3 and M = 5/8.  Column k of the
// axis table V (row-major nc x nc, V[I nc + k]) is an orthonormal eigenvector of both, with
// angle theta_k: lambda_K = -2 (1 - cos theta), lambda_M = (3 + cos theta) / 4.  The mirror
// ghost of each wall end fixes the modes: cos or sin(theta (I + 1/2)) for a Neumann or
// Dirichlet low end, with theta nc = pi k (two Neumann ends), pi (k + 1) (two Dirichlet
// ends) or pi (k + 1/2) (one of each); a periodic axis takes the constant, then cos and sin
// pairs of angle 2 pi m / nc, then (nc even) the alternating mode.  invLam[l ncx + k] is
// 1 / lambda of mode (k, l): ISM K_x M_y + M_x K_y, GMG5 K_x + K_y, ACM n (K_x + K_y); 0 for
// the constant mode of a singular system.
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_coarse_tables(Geo g, int kind, int singular,
                                                          double* __restrict__ Vx,
                                                          double* __restrict__ Vy,
                                                          double* __restrict__ invLam) {
  const long long nvx = (long long)g.ncx * g.ncx, nvy = (long long)g.ncy * g.ncy;
  const long long total = nvx + nvy + g.cplane;
  const bool xlo = g.dmask & kDirW, xhi = g.dmask & kDirE, ylo = g.dmask & kDirS,
             yhi = g.dmask & kDirN;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total;
       t += (long long)gridDim.x * kBlock) {
    if (t < nvx) {
      const int I = int(t / g.ncx), k = int(t - (long long)I * g.ncx);
      Vx[t] = axis_mode(g.ncx, g.per_x, xlo, xhi, k, I).value;
    } else if (t < nvx + nvy) {
      const long long u = t - nvx;
      const int I = int(u / g.ncy), k = int(u - (long long)I * g.ncy);
      Vy[u] = axis_mode(g.ncy, g.per_y, ylo, yhi, k, I).value;
    } else {
      const long long u = t - nvx - nvy;
      const int l = int(u / g.ncx), k = int(u - (long long)l * g.ncx);
      const double cx = cos(axis_mode(g.ncx, g.per_x, xlo, xhi, k, 0).theta);
      const double cy = cos(axis_mode(g.ncy, g.per_y, ylo, yhi, l, 0).theta);
      const double kx = -2.0 * (1.0 - cx), mx = (3.0 + cx) / 4.0;
      const double ky = -2.0 * (1.0 - cy), my = (3.0 + cy) / 4.0;
      const double lam = kind == 1 ? kx + ky : kind == 2 ? double(g.n) * (kx + ky) : kx * my + mx * ky;
      invLam[u] = (singular && l == 0 && k == 0) ? 0.0 : 1.0 / lam;
    }
  }
}

// The interpolation tables of Geo::itab: entry i < nx for column i, nx + j for row j.
__global__ __launch_bounds__(kBlock) void k_interp_tables(Geo g, double2* __restrict__ tab) {
  const int total = g.nx + g.ny;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < total; k += gridDim.x * kBlock) {
    int lo;
    double t;
    if (k < g.nx) interp_axis(k, g.nx, g.n, g.log2n, g.ncx, g.per_x, lo, t);
    else interp_axis(k - g.nx, g.ny, g.n, g.log2n, g.ncy, g.per_y, lo, t);
    tab[k] = make_double2(t, double(lo));
  }
}

// The per-grid maxima of an iteration's partials and its device-side convergence test in one
// workgroup: m[k] = max of part[k stride .. k stride + count) for every grid k (strided per
// thread, then a fixed tree, as k_finalize), then the first iteration at which every grid is
// below tol (or any value is not finite) sets state to 1 (2) and records the iteration; later
// iterations leave both alone.
__global__ __launch_bounds__(kBlock) void k_max_stop(const double* __restrict__ part, int count,
                                                     long long stride, int batch,
                                                     double* __restrict__ m, double tol, int iter,
                                                     double* __restrict__ state,
                                                     double* __restrict__ at) {
  __shared__ double sh[kBlock];
  bool all = true, bad = false;
  for (int k = 0; k < batch; ++k) {
    const double* p = part + (long long)k * stride;
    sh[threadIdx.x] = strided_reduce(p, int(threadIdx.x), count, true);
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
      __syncthreads();
    }
    const double v = sh[0];
    if (threadIdx.x == 0) m[k] = v;
    bad = bad || !isfinite(v);
    all = all && v < tol;
    __syncthreads();  // sh is reused by the next grid
  }
  if (threadIdx.x == 0 && *state == 0.0 && (bad || all)) {
    *state = bad ? 2.0 : 1.0;
    *at = double(iter);
  }
}

__global__ __launch_bounds__(kBlock) void k_fill(double* __restrict__ p, long long count,
                                                 double v) {
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < count;
       t += (long long)gridDim.x * kBlock)
    p[t] = v;
}

}  // namespace

// ---------------------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_rbgs(const Geo& g, const T* rhs, const T* ein, T* eout, hipStream_t s, T rscale,
                       double* part_max, const double* stop) {
  dim3 grid((g.nx + 63) / 64, (g.ny + 31) / 32, g.batch);
  hipLaunchKernelGGL(k_rbgs<T>, grid, dim3(kBlock), 0, s, g, rhs, ein, eout, rscale, part_max, stop);
  return hipGetLastError();
}

int rbgs_tiles(const Geo& g) { return ((g.nx + 63) / 64) * ((g.ny + 31) / 32); }

hipError_t launch_agglomerate(const Geo& g, const double* r, const double* e, double scale,
                              double* out, double* psq, hipStream_t s) {
  const long long total = (long long)(g.nx / 2) * (g.ny / 2) * g.batch;
  hipLaunchKernelGGL(k_agglomerate, dim3(grid_stride_blocks(total)), dim3(kBlock), 0, s, g, r, e,
                     scale, out, psq);
  return hipGetLastError();
}

hipError_t launch_inject(const Geo& g, const double* ec, double* ef, int assign, hipStream_t s) {
  const long long total = g.plane * g.batch;
  hipLaunchKernelGGL(k_inject, dim3(grid_stride_blocks(total)), dim3(kBlock), 0, s, g, ec, ef, assign);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const Geo& g, const T* rhs, const T* e, double* rc, double* psq,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_restrict<T>, strip_grid(g), dim3(kBlock), 0, s, g, rhs, e, rc, psq);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Geo& g, const double* E, T* e, int assign, hipStream_t s) {
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, g.batch);
  hipLaunchKernelGGL(k_prolong<T>, grid, dim3(kBlock), 0, s, g, E, e, assign);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_outer_residual(const Geo& g, const double* b, const double* x,
                                 const double* mean_b, double h2, T* rT, double* rc, Partials p,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_outer_residual<T>, strip_grid(g), dim3(kBlock), 0, s, g, b, x, mean_b, h2,
                     rT, rc, p);
  return hipGetLastError();
}

hipError_t launch_tile_sum(const Geo& g, const double* x, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_sum, strip_grid(g), dim3(kBlock), 0, s, g, x, part);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* part, int count, long long part_stride, int batch,
                           Reduce op, double scale, double* out, int out_stride, int slot,
                           double* scratch, hipStream_t s) {
  const int chunks = (count + kChunk - 1) / kChunk;
  if (chunks <= 1) {
    hipLaunchKernelGGL(k_finalize, dim3(1, batch), dim3(kBlock), 0, s, part, count, part_stride,
                       int(op), scale, out, out_stride, slot);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_finalize, dim3(chunks, batch), dim3(kBlock), 0, s, part, count, part_stride,
                     int(op), 1.0, scratch, 0, 0);
  hipLaunchKernelGGL(k_finalize, dim3(1, batch), dim3(kBlock), 0, s, scratch, chunks,
                     (long long)chunks, int(op), scale, out, out_stride, slot);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_add_to(const Geo& g, double* x, const T* e, hipStream_t s) {
  const long long total = g.plane * g.batch;
  hipLaunchKernelGGL(k_add_to<T>, dim3(grid_stride_blocks(total)), dim3(kBlock), 0, s, total, x, e);
  return hipGetLastError();
}

hipError_t launch_sub_scalar(const Geo& g, double* x, const double* vals, int val_stride, int slot,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_sub_scalar, dim3(grid_stride_blocks(g.plane * g.batch)), dim3(kBlock), 0, s,
                     g.plane, g.batch, x, vals, val_stride, slot);
  return hipGetLastError();
}

hipError_t launch_gemm(int M, int N, int K, int transA, const double* A, long long sA, int lda,
                       int transB, const double* B, long long sB, int ldb, double* C, long long sC,
                       int ldc, const double* S, int batch, hipStream_t s) {
  dim3 grid((N + kGemmTile - 1) / kGemmTile, (M + kGemmTile - 1) / kGemmTile, batch);
  dim3 block(kBlock);
  if (!transA && !transB)
    hipLaunchKernelGGL((k_gemm<0, 0>), grid, block, 0, s, M, N, K, A, sA, lda, B, sB, ldb, C, sC, ldc, S);
  else if (transA && !transB)
    hipLaunchKernelGGL((k_gemm<1, 0>), grid, block, 0, s, M, N, K, A, sA, lda, B, sB, ldb, C, sC, ldc, S);
  else if (!transA && transB)
    hipLaunchKernelGGL((k_gemm<0, 1>), grid, block, 0, s, M, N, K, A, sA, lda, B, sB, ldb, C, sC, ldc, S);
  else
    hipLaunchKernelGGL((k_gemm<1, 1>), grid, block, 0, s, M, N, K, A, sA, lda, B, sB, ldb, C, sC, ldc, S);
  return hipGetLastError();
}

hipError_t launch_coarse_assemble(const Geo& g, int gmg5, double* coef, hipStream_t s) {
  const int cells = g.ncx * g.ncy;
  hipLaunchKernelGGL(k_coarse_assemble, dim3((cells + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g,
                     gmg5, coef);
  return hipGetLastError();
}

hipError_t launch_coarse_tables(const Geo& g, int kind, int singular, double* Vx, double* Vy,
                                double* invLam, hipStream_t s) {
  const long long total = (long long)g.ncx * g.ncx + (long long)g.ncy * g.ncy + g.cplane;
  hipLaunchKernelGGL(k_coarse_tables, dim3(grid_stride_blocks(total)), dim3(kBlock), 0, s, g, kind,
                     singular, Vx, Vy, invLam);
  return hipGetLastError();
}

hipError_t launch_interp_tables(const Geo& g, double2* tab, hipStream_t s) {
  hipLaunchKernelGGL(k_interp_tables, dim3(grid_stride_blocks(g.nx + g.ny)), dim3(kBlock), 0, s, g,
                     tab);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long long count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_stride_blocks(count)), dim3(kBlock), 0, s, p, count, v);
  return hipGetLastError();
}

// Block-GS tile width on an axis of nc coarse cells: kCB, except that a periodic axis of at
// most kCB cells is split into two tiles, so that no tile spans a whole periodic axis.
int bgs_tile(int nc, bool periodic) { return periodic && nc <= kCB ? (nc + 1) / 2 : kCB; }

int coarse_bgs_tiles(const Geo& g) {
  const int tx = bgs_tile(g.ncx, g.per_x), ty = bgs_tile(g.ncy, g.per_y);
  return ((g.ncx + tx - 1) / tx) * ((g.ncy + ty - 1) / ty);
}

hipError_t launch_coarse_bgs(const Geo& g, const double* coef, const double* R, const double* Ein,
                             double* Eout, double* part_max, hipStream_t s, const double* stop) {
  const int tx = bgs_tile(g.ncx, g.per_x), ty = bgs_tile(g.ncy, g.per_y);
  dim3 grid((g.ncx + tx - 1) / tx, (g.ncy + ty - 1) / ty, g.batch);
  hipLaunchKernelGGL(k_coarse_bgs, grid, dim3(kBlock), 0, s, g, coef, R, Ein, Eout, part_max, tx,
                     ty, stop);
  return hipGetLastError();
}

int coarse_mc_colours(const Geo& g) {
  return mc_axis_colours(g.ncx, g.per_x) * mc_axis_colours(g.ncy, g.per_y);
}

int coarse_mc_tiles(const Geo& g) { return int((g.cplane + kBlock - 1) / kBlock); }

int launch_coarse_mc(const Geo& g, const double* coef, const double* R, const double* Ein,
                     double* Eout, double* part_max, hipStream_t s, const double* stop,
                     hipError_t* err) {
  const int Qx = mc_axis_colours(g.ncx, g.per_x), Qy = mc_axis_colours(g.ncy, g.per_y);
  hipLaunchKernelGGL(k_coarse_mc_first, dim3(coarse_mc_tiles(g), 1, g.batch), dim3(kBlock), 0, s,
                     g, coef, R, Ein, Eout, part_max, Qx, Qy, stop);
  int launched = 1;
  if ((*err = hipGetLastError()) != hipSuccess) return launched;
  for (int k = 1; k < Qx * Qy; ++k) {
    const int qy = k / Qx, qx = k - qy * Qx;
    const int cx = mc_axis_count(g.ncx, Qx, qx), count = cx * mc_axis_count(g.ncy, Qy, qy);
    if (count == 0) continue;  // a coarse axis of one cell has no cell of colour 0 or 1
    hipLaunchKernelGGL(k_coarse_mc_colour, dim3((count + kBlock - 1) / kBlock, 1, g.batch),
                       dim3(kBlock), 0, s, g, coef, R, Eout, qy, qx, cx, count, stop);
    ++launched;
    if ((*err = hipGetLastError()) != hipSuccess) return launched;
  }
  return launched;
}

template <typename T, int NU>
hipError_t cycle_tile_nu(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                         double* rc, double* psq, int nu, int zero_e, hipStream_t s,
                         const double* stop, int maxmode) {
  if constexpr (NU == 0) {
    return hipErrorInvalidValue;
  } else {
    if (nu != NU)
      return cycle_tile_nu<T, NU - 1>(g, rhs, ein, eout, E, rc, psq, nu, zero_e, s, stop, maxmode);
    dim3 grid((g.nx + kTile - 1) / kTile, (g.ny + kTile - 1) / kTile, g.batch);
    hipLaunchKernelGGL((k_cycle_tile<T, NU>), grid, dim3(kTileBlock), 0, s, g, rhs, ein, eout, E, rc, psq,
                       zero_e, stop, maxmode);
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_cycle_tile(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                             double* rc, double* psq, int nu, int zero_e, hipStream_t s,
                             const double* stop, int maxmode) {
  if (g.n < 4 || g.n > kTile) return hipErrorInvalidValue;
  return cycle_tile_nu<T, sizeof(T) == 4 ? 5 : 4>(g, rhs, ein, eout, E, rc, psq, nu, zero_e, s,
                                                   stop, maxmode);
}

int coarse_small_fits(const Geo& g) { return g.ncx <= kSmallCoarse && g.ncy <= kSmallCoarse; }

hipError_t launch_coarse_small(const Geo& g, const double* R, const double* Fx, const double* Fy,
                               const double* Vx, const double* Vy, const double* invLam,
                               double* E, hipStream_t s) {
  if (!coarse_small_fits(g)) return hipErrorInvalidValue;
  // one thread per coarse cell (at least kBlock): the four products' dot products then run
  // side by side rather than several after one another in each thread
  const int cells = int(g.cplane), threads = std::max(kBlock, (cells + kWave - 1) / kWave * kWave);
  hipLaunchKernelGGL(k_coarse_small, dim3(g.batch), dim3(threads), 0, s, g.ncx, g.ncy, g.cplane, R,
                     Fx, Fy, Vx, Vy, invLam, E);
  return hipGetLastError();
}

int launch_max_stop(const double* part, int count, long long part_stride, int batch, double* m,
                    double tol, int iter, double* state, double* at, double* scratch,
                    hipStream_t s, hipError_t* err) {
  const int chunks = (count + kChunk - 1) / kChunk;
  int launched = 0;
  if (chunks > 1) {  // first stage as launch_finalize's
    hipLaunchKernelGGL(k_finalize, dim3(chunks, batch), dim3(kBlock), 0, s, part, count,
                       part_stride, int(MAX), 1.0, scratch, 0, 0);
    ++launched;
    if ((*err = hipGetLastError()) != hipSuccess) return launched;
    part = scratch;
    count = chunks;
    part_stride = chunks;
  }
  hipLaunchKernelGGL(k_max_stop, dim3(1), dim3(kBlock), 0, s, part, count, part_stride, batch, m,
                     tol, iter, state, at);
  *err = hipGetLastError();
  return launched + 1;
}

hipError_t launch_div(const Geo& g, const double* u, const double* v, double h, double* b,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_div, dim3(grid_stride_blocks(g.plane * g.batch)), dim3(kBlock), 0, s, g, u,
                     v, h, b);
  return hipGetLastError();
}

hipError_t launch_grad(const Geo& g, const double* p, double h, double* gu, double* gv,
                       hipStream_t s) {
  const long long nu_ = (long long)g.ny * (g.per_x ? g.nx : g.nx + 1) * g.batch;
  const long long nv_ = (long long)(g.ny + 1) * g.nx * g.batch;
  hipLaunchKernelGGL(k_grad_u, dim3(grid_stride_blocks(nu_)), dim3(kBlock), 0, s, g, p, h, gu);
  hipLaunchKernelGGL(k_grad_v, dim3(grid_stride_blocks(nv_)), dim3(kBlock), 0, s, g, p, h, gv);
  return hipGetLastError();
}

hipError_t launch_predict(const Geo& g, const double* u, const double* v, const double* p,
                          double h, double dt, double eta, const double walls[4], double* us,
                          double* vs, hipStream_t s) {
  const Walls wl{walls[0], walls[1], walls[2], walls[3]};
  const long long nu_ = (long long)g.ny * (g.per_x ? g.nx : g.nx + 1) * g.batch;
  const long long nv_ = (long long)(g.ny + 1) * g.nx * g.batch;
  hipLaunchKernelGGL(k_predict_u, dim3(grid_stride_blocks(nu_)), dim3(kBlock), 0, s, g, u, v, p, h,
                     dt, eta, wl, us);
  hipLaunchKernelGGL(k_predict_v, dim3(grid_stride_blocks(nv_)), dim3(kBlock), 0, s, g, u, v, p, h,
                     dt, eta, wl, vs);
  return hipGetLastError();
}

hipError_t launch_correct(const Geo& g, const double* x, double h, double* u, double* v, double* p,
                          hipStream_t s) {
  const long long total = (long long)g.ny * (g.per_x ? g.nx : g.nx + 1) * g.batch +
                          (long long)(g.ny + 1) * g.nx * g.batch + g.plane * g.batch;
  hipLaunchKernelGGL(k_correct, dim3(grid_stride_blocks(total)), dim3(kBlock), 0, s, g, x, h, u, v, p);
  return hipGetLastError();
}

hipError_t launch_div_adjoint(const Geo& g, const double* lam, double h, double* gu, double* gv,
                              hipStream_t s) {
  const long long nu_ = (long long)g.ny * (g.per_x ? g.nx : g.nx + 1) * g.batch;
  const long long nv_ = (long long)(g.ny + 1) * g.nx * g.batch;
  hipLaunchKernelGGL(k_div_adjoint_u, dim3(grid_stride_blocks(nu_)), dim3(kBlock), 0, s, g, lam, h, gu);
  hipLaunchKernelGGL(k_div_adjoint_v, dim3(grid_stride_blocks(nv_)), dim3(kBlock), 0, s, g, lam, h, gv);
  return hipGetLastError();
}

hipError_t launch_grad_adjoint(const Geo& g, const double* gu, const double* gv, double h,
                               double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_adjoint, dim3(grid_stride_blocks(g.plane * g.batch)), dim3(kBlock), 0,
                     s, g, gu, gv, h, p);
  return hipGetLastError();
}

template hipError_t launch_cycle_tile<float>(const Geo&, const float*, const float*, float*,
                                             const double*, double*, double*, int, int,
                                             hipStream_t, const double*, int);
template hipError_t launch_cycle_tile<double>(const Geo&, const double*, const double*, double*,
                                              const double*, double*, double*, int, int,
                                              hipStream_t, const double*, int);
template hipError_t launch_rbgs<float>(const Geo&, const float*, const float*, float*, hipStream_t, float,
                                       double*, const double*);
template hipError_t launch_rbgs<double>(const Geo&, const double*, const double*, double*, hipStream_t,
                                        double, double*, const double*);
template hipError_t launch_restrict<float>(const Geo&, const float*, const float*, double*, double*, hipStream_t);
template hipError_t launch_restrict<double>(const Geo&, const double*, const double*, double*, double*, hipStream_t);
template hipError_t launch_prolong<float>(const Geo&, const double*, float*, int, hipStream_t);
template hipError_t launch_prolong<double>(const Geo&, const double*, double*, int, hipStream_t);
template hipError_t launch_outer_residual<float>(const Geo&, const double*, const double*,
                                                 const double*, double, float*, double*, Partials,
                                                 hipStream_t);
template hipError_t launch_outer_residual<double>(const Geo&, const double*, const double*,
                                                  const double*, double, double*, double*, Partials,
                                                  hipStream_t);
template hipError_t launch_add_to<float>(const Geo&, double*, const float*, hipStream_t);
template hipError_t launch_add_to<double>(const Geo&, double*, const double*, hipStream_t);

}  // namespace ism
