// HIP kernels of the interpolated stencil multigrid (ISM) solver, written for gfx950
// (MI355X: wave64, 160 KB LDS per CU, HBM3E).
//
// Every fine-grid kernel streams a 5-point stencil and is bound by HBM bandwidth; none of
// them is a dense contraction, so nothing here uses MFMA.  Fine arrays are row-major
// [batch][ny][nx]; a wave covers 64 consecutive cells of a row so every global access is a
// full 256 B (FP32) or 512 B (FP64) row segment.
//
// Arithmetic conventions (shared by every kernel so that a cell value never depends on the
// kernel that produced it):
//  * A'e (the 5-point Laplacian times h^2) in difference form,
//    ((e_W - e_C) + (e_E - e_C)) + (e_S - e_C)) + (e_N - e_C), a wall neighbour's term being
//    absent (Sec. 2.3 stencil, Sec. 4.1 walls).
//  * Red-black Gauss-Seidel (Sec. 3.1): red is (i + j) even; a cell is set to
//    (((e_W + e_E) + e_S) + e_N - rhs_C) * (1 / m_C), m_C its number of existing neighbours
//    and a missing neighbour contributing 0.
//  * Bilinear prolongation (Eq. 5) evaluated in FP64 and added to the fine value in FP64,
//    then rounded to the fine type.
// The library is compiled with -ffp-contract=off so these expressions round exactly as
// written; products that are meant to fuse (the coarse transforms) call fma explicitly.

#include <hip/hip_runtime.h>

#include "ism_internal.h"

namespace ism {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;

__device__ __forceinline__ int imod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int floordiv(int a, int n) {
  return a >= 0 ? a / n : -((-a + n - 1) / n);
}

// Map an unwrapped cell coordinate onto the grid: wraps periodic axes, rejects cells behind
// a wall.
__device__ __forceinline__ bool map_cell(const Geo& g, int& i, int& j) {
  if (g.per_x) {
    i = imod(i, g.nx);
  } else if (i < 0 || i >= g.nx) {
    return false;
  }
  if (g.per_y) {
    j = imod(j, g.ny);
  } else if (j < 0 || j >= g.ny) {
    return false;
  }
  return true;
}

template <typename T>
__device__ __forceinline__ T inv_count(const Geo& g, int i, int j) {
  int m = 4;
  if (!g.per_x) m -= (i == 0) + (i == g.nx - 1);
  if (!g.per_y) m -= (j == 0) + (j == g.ny - 1);
  constexpr T third = T(1) / T(3);
  return m == 4 ? T(0.25) : (m == 3 ? third : (m == 2 ? T(0.5) : T(1)));
}

// A'e at a cell from its four neighbours, difference form; absent terms skipped.
template <typename T>
__device__ __forceinline__ T lap5(T c, T w, T e, T s, T n, bool hw, bool he, bool hs, bool hn) {
  T dw = hw ? T(w - c) : T(0);
  T de = he ? T(e - c) : T(0);
  T ds = hs ? T(s - c) : T(0);
  T dn = hn ? T(n - c) : T(0);
  return ((dw + de) + ds) + dn;
}

__device__ __forceinline__ double wave_sum_group(double v, int group) {
  for (int off = 1; off < group; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max_group(double v, int group) {
  for (int off = 1; off < group; off <<= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Interpolation coordinate along one axis (Eq. 5): fine index -> lower coarse index
// (unwrapped, may be -1 or the last+1) and the offset t = (2k+1)/(2n) of the fine centre
// from the lower coarse centre, in units of the rectangle size n.
__device__ __forceinline__ void interp_coord(int gi, int n, int& lo, double& t) {
  int s = gi - (n >> 1);
  lo = floordiv(s, n);
  int k = s - lo * n;
  t = double(2 * k + 1) / double(2 * n);
}

// Eq. 5 evaluated in nested form: interpolate along x on the lower and the upper coarse row,
// then along y, p = (Q11 (1-X) + Q21 X) (1-Y) + (Q12 (1-X) + Q22 X) Y, rounded in this order.
__device__ __forceinline__ double lerp(double a, double b, double t) { return a * (1.0 - t) + b * t; }

__device__ __forceinline__ double bilinear(double q11, double q21, double q12, double q22,
                                           double X, double Y) {
  return lerp(lerp(q11, q21, X), lerp(q12, q22, X), Y);
}

// ----------------------------------------------------------------------------------------
// One red-black sweep (red on the tile plus one ring, black on the tile), LDS-staged.
// Tile 64 x 32 cells per workgroup; e is staged with a halo of 2, rhs with a halo of 1.
// ----------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rbgs(Geo g, const T* __restrict__ rhs,
                                                 const T* __restrict__ ein,
                                                 T* __restrict__ eout, T rscale) {
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
    T s = ((se[idx - 1] + se[idx + 1]) + se[idx - LE]) + se[idx + LE];
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
    T s = ((se[idx - 1] + se[idx + 1]) + se[idx - LE]) + se[idx + LE];
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
    const bool hw = g.per_x || i > 0, he = g.per_x || i < g.nx - 1;
    for (int r = wave; r < g.n; r += 4) {
      const int j = J * g.n + r;
      const int js = g.per_y ? imod(j - 1, g.ny) : j - 1;
      const int jn = g.per_y ? imod(j + 1, g.ny) : j + 1;
      const bool hs = g.per_y || j > 0, hn = g.per_y || j < g.ny - 1;
      const T* row = eb + (long long)j * g.nx;
      T c = row[i];
      T w = hw ? row[iw] : T(0);
      T ee = he ? row[ie] : T(0);
      T s = hs ? eb[(long long)js * g.nx + i] : T(0);
      T nn = hn ? eb[(long long)jn * g.nx + i] : T(0);
      T res = rb[(long long)j * g.nx + i] - lap5<T>(c, w, ee, s, nn, hw, he, hs, hn);
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
  const double* Eb = E + (long long)blockIdx.z * g.cplane;
  int ilo, jlo;
  double X, Y;
  interp_coord(i, g.n, ilo, X);
  interp_coord(j, g.n, jlo, Y);
  int ihi = ilo + 1, jhi = jlo + 1;
  if (g.per_x) {
    ilo = imod(ilo, g.ncx);
    ihi = imod(ihi, g.ncx);
  } else {
    ilo = max(ilo, 0);
    ihi = min(ihi, g.ncx - 1);
  }
  if (g.per_y) {
    jlo = imod(jlo, g.ncy);
    jhi = imod(jhi, g.ncy);
  } else {
    jlo = max(jlo, 0);
    jhi = min(jhi, g.ncy - 1);
  }
  const double p = bilinear(Eb[jlo * g.ncx + ilo], Eb[jlo * g.ncx + ihi], Eb[jhi * g.ncx + ilo],
                            Eb[jhi * g.ncx + ihi], X, Y);
  T* ec = e + (long long)blockIdx.z * g.plane + (long long)j * g.nx + i;
  *ec = assign ? T(p) : T(double(*ec) + p);
}

// ----------------------------------------------------------------------------------------
// Fused two-level cycle kernel (temporal blocking of the red-black sweeps).
//
// A workgroup owns a 64 x TSY tile of fine cells (TSY = 64 for FP32, 32 for FP64 so that
// three workgroups fit in a CU's LDS either way).  It stages e on the tile grown by H = 2 NU + 1
// rows and PADX columns (PADX >= H - 1 + VEC, a multiple of the 16-byte chunk of VEC cells),
// and rhs on the cells a half-step may update, in LDS, adding the bilinear coarse correction
// to every staged e.  Every global access is a 16-byte chunk and all of a lane's loads are in
// flight together.  The 2 NU red/black half-steps then each update their colour on every
// staged chunk that has all its neighbours staged; a lane keeps the same chunks throughout.
// Values computed outside the ring H - 1 - s at half-step s come from stale neighbours, but
// no later half-step inside its own ring reads them, so after the last half-step e is exact
// on the tile plus one ring.  A red/black half-step reads only the other colour, so a halo
// cell gets exactly the value its owner computes.  The kernel then forms the residual on the
// tile, writes the tile of e and the sums of the residual (and its square) over each n x n
// coarse tile it contains.  Per cycle it reads e and rhs once and writes e once.
// Workgroups are numbered so that the consecutive workgroups one XCD receives (the hardware
// deals them out round-robin over the 8 XCDs) take neighbouring tiles, whose halos then
// meet in that XCD's L2.
// ----------------------------------------------------------------------------------------
template <typename T>
struct Chunk;
template <>
struct Chunk<float> {
  using type = float4;
};
template <>
struct Chunk<double> {
  using type = double2;
};

template <typename V>
__device__ __forceinline__ V zero_chunk() {
  V v;
  for (int k = 0; k < int(sizeof(V) / sizeof(v.x)); ++k) (&v.x)[k] = 0;
  return v;
}

template <typename T, int NU, int LOG2N, int TSY>
struct CycleTile {
  using V = typename Chunk<T>::type;
  static constexpr int VEC = 16 / sizeof(T);  // cells per 16-byte chunk
  static constexpr int TSX = 64;
  static constexpr int N = 1 << LOG2N;
  static constexpr int H = 2 * NU + 1;
  static constexpr int PADX = ((H - 1 + VEC + VEC - 1) / VEC) * VEC;
  static constexpr int LEX = TSX + 2 * PADX, LEY = TSY + 2 * H;  // staged region
  static constexpr int HX = LEX / 2;                             // cells per half-row
  static constexpr int CX = LEX / VEC;                           // global chunks per staged row
  static constexpr int HC = HX / VEC;                            // LDS chunks per half-row
  static constexpr int NE = (LEY * CX + kBlock - 1) / kBlock;    // e chunks staged per lane
  static constexpr int NRC = ((LEY - 2) * CX + kBlock - 1) / kBlock;  // rhs chunks per lane
  static constexpr int NUC = ((LEY - 2) * HC + kBlock - 1) / kBlock;  // updated chunks per lane
  static constexpr int CEX = LEX / N + 3, CEY = LEY / N + 3;
  static constexpr int RPW = TSY / 4;                 // tile rows per wave (residual)
  static constexpr int NBW = RPW >= N ? RPW / N : 1;  // coarse bands per wave
  static constexpr int WPB = N > RPW ? N / RPW : 1;   // waves per coarse band
  static constexpr int TPX = TSX / N, TPY = TSY / N;  // coarse tiles per workgroup tile
  static_assert(TSY % 4 == 0 && N <= TSY, "a workgroup tile must hold whole coarse tiles");
  static_assert(HX % VEC == 0, "half-rows must hold whole chunks");

  // Staged rows are stored split by column parity: [even columns | odd columns], so that a
  // red or black half-step works on contiguous chunks of one colour.
  struct Shared {
    alignas(16) T se[LEY * LEX];        // e, rows 0 .. LEY-1
    alignas(16) T sr[(LEY - 2) * LEX];  // rhs, rows 1 .. LEY-2
    double sE[CEY * CEX];   // coarse values around the staged region
    alignas(16) double sEx[CEY * LEX];  // the same, interpolated along x at every staged column
    double rowY[LEY];       // y weight of every staged row, 1 minus it ...
    double rowY1[LEY];
    int rowJ[LEY];          // ... and the offset of its lower coarse row in sEx
    double red1[4][NBW][TPX];
    double red2[4][NBW][TPX];
  };

  static __device__ __forceinline__ int at(int ly, int lx) { return ly * LEX + (lx & 1) * HX + (lx >> 1); }

  // a natural-order chunk of VEC cells (columns lx0 .. lx0+VEC-1) into the split row
  static __device__ __forceinline__ void put(T* row, int lx0, const V& v) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) row[(k & 1) * HX + ((lx0 + k) >> 1)] = (&v.x)[k];
  }

  // 1 / (number of existing neighbours) of a staged cell, 0 for a cell behind a wall (which
  // then stays 0, as a missing neighbour contributes nothing)
  static __device__ __forceinline__ T inv_at(const Geo& g, int i, int j) {
    if (!map_cell(g, i, j)) return T(0);
    return inv_count<T>(g, i, j);
  }

  // INTERIOR: the staged region lies inside the grid, touches no wall and interpolates from
  // unclamped coarse values.

  // Issue every global load of a tile (e with its halo, rhs on the rows a half-step updates)
  // into registers.
  template <bool INTERIOR>
  static __device__ __forceinline__ void load(const Geo& g, const T* __restrict__ rb,
                                              const T* __restrict__ eb, int zero_e, int x0, int y0,
                                              V (&ev)[NE], V (&rv)[NRC], int tid) {
    const int xs = x0 - PADX, ys = y0 - H;
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      const int q = tid + m * kBlock;
      ev[m] = zero_chunk<V>();
      if (q < LEY * CX && !zero_e) {
        const int ly = q / CX, c = q - ly * CX;
        int i = xs + VEC * c, j = ys + ly;
        if (INTERIOR || map_cell(g, i, j)) ev[m] = *reinterpret_cast<const V*>(eb + j * g.nx + i);
      }
    }
#pragma unroll
    for (int m = 0; m < NRC; ++m) {
      const int q = tid + m * kBlock;
      rv[m] = zero_chunk<V>();
      if (q < (LEY - 2) * CX) {
        const int ly = 1 + q / CX, c = q - (ly - 1) * CX;
        int i = xs + VEC * c, j = ys + ly;
        if (INTERIOR || map_cell(g, i, j)) rv[m] = *reinterpret_cast<const V*>(rb + j * g.nx + i);
      }
    }
  }

  // Coarse tables of the tile, then e + P E and rhs from the registers into LDS.
  template <bool INTERIOR>
  static __device__ __forceinline__ void stage(Shared& sh, const Geo& g,
                                               const double* __restrict__ Eb, int x0, int y0,
                                               int cI0, int cJ0, const V (&ev)[NE],
                                               const V (&rv)[NRC], int tid) {
    const int xs = x0 - PADX, ys = y0 - H;
    // coarse values around the staged region, with the boundary rule applied at load time
    for (int t = tid; t < CEY * CEX; t += kBlock) {
      int cj = t / CEX, ci = t - cj * CEX;
      int I = cI0 + ci, J = cJ0 + cj;
      if (!INTERIOR) {
        I = g.per_x ? imod(I, g.ncx) : min(max(I, 0), g.ncx - 1);
        J = g.per_y ? imod(J, g.ncy) : min(max(J, 0), g.ncy - 1);
      }
      sh.sE[t] = Eb[J * g.ncx + I];
    }
    for (int t = tid; t < LEY; t += kBlock) {
      int jlo;
      double Y;
      interp_coord(ys + t, N, jlo, Y);
      sh.rowY[t] = Y;
      sh.rowY1[t] = 1.0 - Y;
      sh.rowJ[t] = (jlo - cJ0) * LEX;
    }
    __syncthreads();
    for (int t = tid; t < CEY * LEX; t += kBlock) {
      int cj = t / LEX, lx = t - cj * LEX;
      int ilo;
      double X;
      interp_coord(xs + lx, N, ilo, X);
      const double* q = sh.sE + cj * CEX + (ilo - cI0);
      sh.sEx[t] = lerp(q[0], q[1], X);
    }
    __syncthreads();

    // staged e = e + P E (cells behind a wall stay 0), staged rhs
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      const int q = tid + m * kBlock;
      if (q < LEY * CX) {
        const int ly = q / CX, c = q - ly * CX;
        int i = xs + VEC * c, j = ys + ly;
        V v = zero_chunk<V>();
        if (INTERIOR || map_cell(g, i, j)) {
          // the chunk's interpolated values on the bounding coarse rows, read as 16-byte
          // vectors (contiguous across the wave), then the y weights: same rounding as lerp
          const double2* plo = reinterpret_cast<const double2*>(sh.sEx + sh.rowJ[ly] + VEC * c);
          const double2* phi = reinterpret_cast<const double2*>(sh.sEx + sh.rowJ[ly] + LEX + VEC * c);
          const double Y = sh.rowY[ly], Y1 = sh.rowY1[ly];
#pragma unroll
          for (int k2 = 0; k2 < VEC / 2; ++k2) {
            const double2 a = plo[k2], b = phi[k2];
            (&v.x)[2 * k2] = T(double((&ev[m].x)[2 * k2]) + (a.x * Y1 + b.x * Y));
            (&v.x)[2 * k2 + 1] = T(double((&ev[m].x)[2 * k2 + 1]) + (a.y * Y1 + b.y * Y));
          }
        }
        put(sh.se + ly * LEX, VEC * c, v);
      }
    }
#pragma unroll
    for (int m = 0; m < NRC; ++m) {
      const int q = tid + m * kBlock;
      if (q < (LEY - 2) * CX) {
        const int r = q / CX, c = q - r * CX;
        put(sh.sr + r * LEX, VEC * c, rv[m]);
      }
    }
    __syncthreads();
  }

  // Red/black half-steps, residual, write-back of the tile and its coarse-tile sums.
  template <bool INTERIOR>
  static __device__ __forceinline__ void compute(Shared& sh, const Geo& g, T* __restrict__ ob,
                                                 double* __restrict__ rc, double* __restrict__ psq,
                                                 int x0, int y0, int bz, int tid) {
    const int xs = x0 - PADX, ys = y0 - H;

    // 2 NU red/black half-steps: in rows 1 .. LEY-2 every chunk of the half-row holding the
    // colour is updated.  Edge chunks read a neighbour from outside their row; the garbage
    // they make spreads one column per half-step and never reaches the valid ring.
#pragma unroll 1
    for (int s = 0; s < 2 * NU; ++s) {
      const int colour = s & 1;
#pragma unroll
      for (int m = 0; m < NUC; ++m) {
        const int q = tid + m * kBlock;
        if (q < (LEY - 2) * HC) {
          const int ly = 1 + q / HC, h = q - (ly - 1) * HC;
          const int par = (colour + ly + 1) & 1;  // column parity of this colour in row ly
          const int t0 = VEC * h;
          const int xrow = ly * LEX + par * HX;        // this colour's half-row
          const int orow = ly * LEX + (1 - par) * HX;  // the other colour's
          const V on = *reinterpret_cast<const V*>(sh.se + orow + t0);
          const T ox = sh.se[orow + (par ? t0 + VEC : t0 - 1)];
          const V up = *reinterpret_cast<const V*>(sh.se + xrow + LEX + t0);
          const V dn = *reinterpret_cast<const V*>(sh.se + xrow - LEX + t0);
          const V rr = *reinterpret_cast<const V*>(sh.sr + (ly - 1) * LEX + par * HX + t0);
          V out;
#pragma unroll
          for (int k = 0; k < VEC; ++k) {
            // even cells (par 0) have their west neighbour one slot left in the odd half,
            // odd cells (par 1) their east neighbour one slot right in the even half
            const T lo = k == 0 ? ox : (&on.x)[k - 1];
            const T hi = k == VEC - 1 ? ox : (&on.x)[k + 1];
            const T w = par ? (&on.x)[k] : lo;
            const T e = par ? hi : (&on.x)[k];
            T inv = T(0.25);
            if (!INTERIOR) inv = inv_at(g, xs + 2 * (t0 + k) + par, ys + ly);
            const T sum = ((w + e) + (&dn.x)[k]) + (&up.x)[k];
            (&out.x)[k] = (sum - (&rr.x)[k]) * inv;
          }
          *reinterpret_cast<V*>(sh.se + xrow + t0) = out;
        }
      }
      __syncthreads();
    }

    // residual on the tile, write-back, per-coarse-tile sums
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int gi = x0 + lane;
    const int lx = PADX + lane;
    const bool hw = INTERIOR || g.per_x || gi > 0, he = INTERIOR || g.per_x || gi < g.nx - 1;
    double acc[NBW], acc2[NBW];
#pragma unroll
    for (int q = 0; q < NBW; ++q) acc[q] = acc2[q] = 0.0;
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int r = RPW * wave + rr;
      const int gj = y0 + r;
      const int ly = r + H;
      if (INTERIOR || (gi < g.nx && gj < g.ny)) {
        const bool hs = INTERIOR || g.per_y || gj > 0, hn = INTERIOR || g.per_y || gj < g.ny - 1;
        const T c = sh.se[at(ly, lx)];
        const T res = sh.sr[at(ly - 1, lx)] -
                      lap5<T>(c, sh.se[at(ly, lx - 1)], sh.se[at(ly, lx + 1)], sh.se[at(ly - 1, lx)],
                              sh.se[at(ly + 1, lx)], hw, he, hs, hn);
        ob[gj * g.nx + gi] = c;
        const double d = double(res);
        const int q = RPW >= N ? (rr >> LOG2N) : 0;
        acc[q] += d;
        acc2[q] += d * d;
      }
    }
#pragma unroll
    for (int q = 0; q < NBW; ++q) {
      double a = wave_sum_group(acc[q], N);
      double b = wave_sum_group(acc2[q], N);
      if ((lane & (N - 1)) == 0) {
        sh.red1[wave][q][lane >> LOG2N] = a;
        sh.red2[wave][q][lane >> LOG2N] = b;
      }
    }
    __syncthreads();
    if ((int)tid < TPX * TPY) {
      const int band = tid / TPX, tc = tid - band * TPX;
      double a = 0.0, b = 0.0;
      if (WPB > 1) {  // a coarse band spans WPB waves: add them in wave order
        for (int w = band * WPB; w < band * WPB + WPB; ++w) {
          a += sh.red1[w][0][tc];
          b += sh.red2[w][0][tc];
        }
      } else {
        const int w = band / NBW, q = band - w * NBW;
        a = sh.red1[w][q][tc];
        b = sh.red2[w][q][tc];
      }
      const int I = (x0 >> LOG2N) + tc, J = (y0 >> LOG2N) + band;
      if (INTERIOR || (I < g.ncx && J < g.ncy)) {
        const long long o = (long long)bz * g.cplane + (long long)J * g.ncx + I;
        rc[o] = a;
        if (psq) psq[o] = b;
      }
    }
  }
};

// Origin of tile (bx, by) and the coarse index of its first staged interpolation cell.
template <typename CT>
struct TileInfo {
  int x0, y0, cI0, cJ0;
  __device__ __forceinline__ TileInfo(int bx, int by, int tsy) {
    x0 = bx * CT::TSX;
    y0 = by * tsy;
    cI0 = floordiv(x0 - CT::PADX - (CT::N >> 1), CT::N);
    cJ0 = floordiv(y0 - CT::H - (CT::N >> 1), CT::N);
  }
};

// Interior tiles (whose staged region lies inside the grid away from the walls and
// interpolates from unclamped coarse values) form the rectangle [bx0, bx0+nbx) x
// [by0, by0+nby) of tile indices.  This persistent kernel runs them: gridDim.x workgroups per
// grid each walk a sequence of tiles, loading the next tile's e and rhs into registers while
// they sweep the current one.  When possible the workgroups on one XCD (the hardware deals
// workgroups out round-robin over the 8 XCDs) walk one contiguous band of tiles, so that
// neighbouring tiles' halos meet in that XCD's L2.  Every workgroup leaves the loop after its
// last tile; there is no inter-workgroup wait.
template <typename T, int NU, int LOG2N, int TSY>
__global__ __launch_bounds__(kBlock) void k_cycle_interior(Geo g, const T* __restrict__ rhs,
                                                           const T* __restrict__ ein,
                                                           T* __restrict__ eout,
                                                           const double* __restrict__ E,
                                                           double* __restrict__ rc,
                                                           double* __restrict__ psq, int zero_e,
                                                           int bx0, int by0, int nbx, int nby) {
  using CT = CycleTile<T, NU, LOG2N, TSY>;
  using V = typename CT::V;
  __shared__ typename CT::Shared sh;
  const int nt = nbx * nby;
  const int G = gridDim.x, b = blockIdx.x;
  const bool banded = (nt & 7) == 0 && (G & 7) == 0;
  auto tile_at = [&](int it) {  // the it-th tile of this workgroup, nt when none is left
    if (banded) {
      const int local = (b >> 3) + it * (G >> 3);
      return local < (nt >> 3) ? (b & 7) * (nt >> 3) + local : nt;
    }
    const int t = b + it * G;
    return t < nt ? t : nt;
  };
  const long long off = (long long)blockIdx.z * g.plane;
  const T* rb = rhs + off;
  const T* eb = ein + off;
  T* ob = eout + off;
  const double* Eb = E + (long long)blockIdx.z * g.cplane;

  V ev[CT::NE], rv[CT::NRC];
  int t = tile_at(0);
  if (t < nt) {
    const int by = t / nbx;
    TileInfo<CT> ti(bx0 + t - by * nbx, by0 + by, TSY);
    CT::template load<true>(g, rb, eb, zero_e, ti.x0, ti.y0, ev, rv, threadIdx.x);
  }
  for (int it = 0; t < nt; ++it) {
    // with few sweeps (where three workgroups fit a CU's LDS) the lane index is re-read each
    // iteration, opaque to the compiler, so that the per-chunk index arithmetic is recomputed
    // per tile instead of being hoisted out of the tile loop into registers
    int tid = threadIdx.x;
    if (NU <= 2) asm volatile("" : "+v"(tid));
    const int by = t / nbx;
    const TileInfo<CT> ti(bx0 + t - by * nbx, by0 + by, TSY);
    const int tn = tile_at(it + 1);
    __syncthreads();  // the previous tile is done with LDS
    CT::template stage<true>(sh, g, Eb, ti.x0, ti.y0, ti.cI0, ti.cJ0, ev, rv, tid);
    if (tn < nt) {  // prefetch the next tile while this one is swept
      const int byn = tn / nbx;
      TileInfo<CT> tj(bx0 + tn - byn * nbx, by0 + byn, TSY);
      CT::template load<true>(g, rb, eb, zero_e, tj.x0, tj.y0, ev, rv, tid);
    }
    if (NU <= 2) asm volatile("" : "+v"(tid));
    CT::template compute<true>(sh, g, ob, rc, psq, ti.x0, ti.y0, blockIdx.z, tid);
    t = tn;
  }
}

// The tiles outside the interior rectangle (the frame next to the walls, or every tile of a
// small grid): one workgroup per tile, with the boundary rules applied cell by cell.
template <typename T, int NU, int LOG2N, int TSY>
__global__ __launch_bounds__(kBlock) void k_cycle_edge(Geo g, const T* __restrict__ rhs,
                                                       const T* __restrict__ ein,
                                                       T* __restrict__ eout,
                                                       const double* __restrict__ E,
                                                       double* __restrict__ rc,
                                                       double* __restrict__ psq, int zero_e,
                                                       int tiles_x, int tiles_y, int bx0, int by0,
                                                       int nbx, int nby) {
  using CT = CycleTile<T, NU, LOG2N, TSY>;
  using V = typename CT::V;
  __shared__ typename CT::Shared sh;
  // frame tile f: the rows below the rectangle, the rows above it, then the columns left and
  // right of it in the rectangle's rows
  int f = blockIdx.x, bx, by;
  const int below = by0 * tiles_x, above = (tiles_y - by0 - nby) * tiles_x;
  if (f < below) {
    by = f / tiles_x;
    bx = f - by * tiles_x;
  } else if ((f -= below) < above) {
    by = by0 + nby + f / tiles_x;
    bx = f % tiles_x;
  } else {
    f -= above;
    const int side = tiles_x - nbx;  // frame tiles per rectangle row
    by = by0 + f / side;
    const int k = f % side;
    bx = k < bx0 ? k : k + nbx;
  }
  const long long off = (long long)blockIdx.z * g.plane;
  const TileInfo<CT> ti(bx, by, TSY);
  V ev[CT::NE], rv[CT::NRC];
  CT::template load<false>(g, rhs + off, ein + off, zero_e, ti.x0, ti.y0, ev, rv, threadIdx.x);
  CT::template stage<false>(sh, g, E + (long long)blockIdx.z * g.cplane, ti.x0, ti.y0, ti.cI0,
                            ti.cJ0, ev, rv, threadIdx.x);
  CT::template compute<false>(sh, g, eout + off, rc, psq, ti.x0, ti.y0, blockIdx.z, threadIdx.x);
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
    const bool hw = g.per_x || i > 0, he = g.per_x || i < g.nx - 1;
    for (int r = wave; r < g.n; r += 4) {
      const int j = J * g.n + r;
      const int js = g.per_y ? imod(j - 1, g.ny) : j - 1;
      const int jn = g.per_y ? imod(j + 1, g.ny) : j + 1;
      const bool hs = g.per_y || j > 0, hn = g.per_y || j < g.ny - 1;
      const double* row = xb + (long long)j * g.nx;
      double c = row[i];
      double w = hw ? row[iw] : 0.0;
      double ee = he ? row[ie] : 0.0;
      double s = hs ? xb[(long long)js * g.nx + i] : 0.0;
      double nn = hn ? xb[(long long)jn * g.nx + i] : 0.0;
      double bp = h2 * (bb[(long long)j * g.nx + i] - mb);
      double res = bp - lap5<double>(c, w, ee, s, nn, hw, he, hs, hn);
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
    for (int r = wave; r < g.n; r += 4) acc += xb[(long long)(J * g.n + r) * g.nx + i];
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
// workgroup per grid) reduces the chunk results when there is more than one chunk.
constexpr int kChunk = 4096;

__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ part, int count,
                                                     long long stride, int op, double scale,
                                                     double* __restrict__ out, int out_stride,
                                                     int slot) {
  __shared__ double sh[kBlock];
  const double* p = part + (long long)blockIdx.y * stride;
  const int lo = blockIdx.x * kChunk, hi = min(count, lo + kChunk);
  double a = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kBlock) a = op == MAX ? fmax(a, p[i]) : a + p[i];
  sh[threadIdx.x] = a;
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
// that all loads are in flight together; the 4 waves then each accumulate a quarter of K
// (a lane owns a 2 x 2 block) and the quarters are added in wave order through LDS.
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
  const int tx = lane & 7, ty = lane >> 3;  // lane computes rows ty, ty+8 and cols tx, tx+8
  double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
  for (int k0 = 0; k0 < K; k0 += kGemmK) {
    const int kc = min(kGemmK, K - k0);
#pragma unroll 4
    for (int t = threadIdx.x; t < kGemmTile * kGemmK; t += kBlock) {
      {  // A panel, coalesced along the contiguous index of the stored matrix
        const int m = TA ? (t & (kGemmTile - 1)) : (t / kGemmK);
        const int k = TA ? (t / kGemmTile) : (t & (kGemmK - 1));
        const int gm = m0 + m, gk = k0 + k;
        double v = 0.0;
        if (gm < M && k < kc) v = TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
        As[k][m] = v;
      }
      {
        const int nn = TB ? (t / kGemmK) : (t & (kGemmTile - 1));
        const int k = TB ? (t & (kGemmK - 1)) : (t / kGemmTile);
        const int gk = k0 + k, gn = n0 + nn;
        double v = 0.0;
        if (k < kc && gn < N) v = TB ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn];
        Bs[k][nn] = v;
      }
    }
    __syncthreads();
    const int q = (kc + 3) / 4;  // this wave's quarter of the panel
    const int ka = wave * q, kb = min(kc, ka + q);
#pragma unroll 8
    for (int kk = ka; kk < kb; ++kk) {
      const double a0 = As[kk][ty], a1 = As[kk][ty + 8];
      const double b0 = Bs[kk][tx], b1 = Bs[kk][tx + 8];
      c00 = fma(a0, b0, c00);
      c01 = fma(a0, b1, c01);
      c10 = fma(a1, b0, c10);
      c11 = fma(a1, b1, c11);
    }
    __syncthreads();
  }
  red[wave][ty][tx] = c00;
  red[wave][ty][tx + 8] = c01;
  red[wave][ty + 8][tx] = c10;
  red[wave][ty + 8][tx + 8] = c11;
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
// the coarse unknowns; walls carry no flux and the clamped interpolation folds an
// off-grid neighbour onto the cell itself.  One thread per coarse cell.
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_coarse_assemble(Geo g, int gmg5,
                                                            double* __restrict__ coef) {
  const int cell = blockIdx.x * kBlock + threadIdx.x;
  if (cell >= g.ncx * g.ncy) return;
  const int J = cell / g.ncx, I = cell - J * g.ncx;
  double c[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) c[a][b] = 0.0;
  const int n = g.n, half = n / 2;
  const bool openE = g.per_x || I < g.ncx - 1, openW = g.per_x || I > 0;
  const bool openN = g.per_y || J < g.ncy - 1, openS = g.per_y || J > 0;
  if (gmg5) {  // unit 5-point stencil at the coarse spacing, no flux through a wall
    if (openE) c[1][2] += 1.0, c[1][1] -= 1.0;
    if (openW) c[1][0] += 1.0, c[1][1] -= 1.0;
    if (openN) c[2][1] += 1.0, c[1][1] -= 1.0;
    if (openS) c[0][1] += 1.0, c[1][1] -= 1.0;
  }
  for (int k = 0; k < (gmg5 ? 0 : n); ++k) {
    // along the face, the fine centre k of the coarse cell lies between coarse centres
    // lo and lo + 1 (relative offsets -1/0 or 0/+1) at scaled distance t from the lower one
    const int lo = k < half ? -1 : 0;
    const double t = double(2 * k + 1 + (k < half ? n : -n)) / double(2 * n);
    const double wl = (1.0 - t) / double(n), wh = t / double(n);
    // x faces (Eq. 6): derivative across the face between columns d and d+1 (relative)
    if (openE) {  // outward +x, columns 0 -> +1
      c[lo + 1][2] += wl;
      c[lo + 1][1] -= wl;
      c[lo + 2][2] += wh;
      c[lo + 2][1] -= wh;
    }
    if (openW) {  // outward -x, columns -1 -> 0
      c[lo + 1][1] -= wl;
      c[lo + 1][0] += wl;
      c[lo + 2][1] -= wh;
      c[lo + 2][0] += wh;
    }
    // y faces (Eq. 7)
    if (openN) {
      c[2][lo + 1] += wl;
      c[1][lo + 1] -= wl;
      c[2][lo + 2] += wh;
      c[1][lo + 2] -= wh;
    }
    if (openS) {
      c[1][lo + 1] -= wl;
      c[0][lo + 1] += wl;
      c[1][lo + 2] -= wh;
      c[0][lo + 2] += wh;
    }
  }
  if (!g.per_x) {
    if (I == 0)
      for (int a = 0; a < 3; ++a) {
        c[a][1] += c[a][0];
        c[a][0] = 0.0;
      }
    if (I == g.ncx - 1)
      for (int a = 0; a < 3; ++a) {
        c[a][1] += c[a][2];
        c[a][2] = 0.0;
      }
  }
  if (!g.per_y) {
    if (J == 0)
      for (int b = 0; b < 3; ++b) {
        c[1][b] += c[0][b];
        c[0][b] = 0.0;
      }
    if (J == g.ncy - 1)
      for (int b = 0; b < 3; ++b) {
        c[1][b] += c[2][b];
        c[2][b] = 0.0;
      }
  }
  double* o = coef + (long long)cell * 9;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) o[3 * a + b] = c[a][b];
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

__global__ __launch_bounds__(kBlock) void k_grad_u(Geo g, const double* __restrict__ p, double h,
                                                   double* __restrict__ gu) {
  const int nxu = g.per_x ? g.nx : g.nx + 1;
  const long long per = (long long)g.ny * nxu, total = per * g.batch;
  for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < total;
       k += (long long)gridDim.x * kBlock) {
    const long long bi = k / per;
    const int rem = int(k - bi * per);
    const int j = rem / nxu, f = rem - j * nxu;
    const double* pr = p + bi * g.plane + (long long)j * g.nx;
    double val;
    if (g.per_x) val = (pr[f] - pr[f == 0 ? g.nx - 1 : f - 1]) / h;
    else val = (f == 0 || f == g.nx) ? 0.0 : (pr[f] - pr[f - 1]) / h;
    gu[k] = val;
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
    const double* pb = p + bi * g.plane;
    gv[k] = (f == 0 || f == g.ny) ? 0.0
                                  : (pb[(long long)f * g.nx + i] - pb[(long long)(f - 1) * g.nx + i]) / h;
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
    }
    if (j >= 1) t += vb[(long long)j * g.nx + i];
    if (j <= g.ny - 2) t -= vb[(long long)(j + 1) * g.nx + i];
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
          const bool hw = g.per_x || i > 0, he = g.per_x || i < g.nx - 1;
          const bool hs = g.per_y || j > 0, hn = g.per_y || j < g.ny - 1;
          const double* row = eb + (long long)j * g.nx;
          const double c = row[i];
          const double w = hw ? row[g.per_x ? imod(i - 1, g.nx) : i - 1] : 0.0;
          const double ee = he ? row[g.per_x ? imod(i + 1, g.nx) : i + 1] : 0.0;
          const double sv = hs ? eb[(long long)(g.per_y ? imod(j - 1, g.ny) : j - 1) * g.nx + i] : 0.0;
          const double nv = hn ? eb[(long long)(g.per_y ? imod(j + 1, g.ny) : j + 1) * g.nx + i] : 0.0;
          res = res - scale * lap5<double>(c, w, ee, sv, nv, hw, he, hs, hn);
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

// Resident workgroups of a kernel on the whole device (compute units x workgroups per CU).
template <typename K>
int resident_workgroups(K kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess)
    return 0;
  return cus * (per_cu > 0 ? per_cu : 1);
}

// Host copy of the interior test of one tile axis: the staged span [o - pad, o + len + pad)
// lies in [1, n - 1) and its interpolation reads coarse cells [c0, c0 + ce) inside [0, nc).
inline bool axis_interior(int o, int len, int pad, int N, int ce, int n, int nc) {
  const int s = o - pad - N / 2;
  const int c0 = s >= 0 ? s / N : -((-s + N - 1) / N);
  return o - pad >= 1 && o + len + pad + 1 <= n && c0 >= 0 && c0 + ce <= nc;
}

template <typename T, int NU, int LOG2N>
hipError_t cycle_dispatch3(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                           double* rc, double* psq, int zero_e, hipStream_t s) {
  constexpr int TSY = sizeof(T) == 4 ? 64 : 32;
  using CT = CycleTile<T, NU, LOG2N, TSY>;
  const int tx = (g.nx + 63) / 64, ty = (g.ny + TSY - 1) / TSY;
  // the interior rectangle of tiles (the test is separable in x and y)
  int bx0 = tx, bx1 = tx, by0 = ty, by1 = ty;
  for (int b = 0; b < tx; ++b)
    if (axis_interior(b * CT::TSX, CT::TSX, CT::PADX, CT::N, CT::CEX, g.nx, g.ncx)) {
      bx0 = bx0 == tx ? b : bx0;
      bx1 = b + 1;
    }
  for (int b = 0; b < ty; ++b)
    if (axis_interior(b * TSY, TSY, CT::H, CT::N, CT::CEY, g.ny, g.ncy)) {
      by0 = by0 == ty ? b : by0;
      by1 = b + 1;
    }
  int nbx = bx1 - bx0, nby = by1 - by0;
  if (nbx <= 0 || nby <= 0) {
    bx0 = by0 = 0;
    nbx = nby = 0;
  }
  const int nt = nbx * nby;
  if (nt > 0) {
    auto kernel = k_cycle_interior<T, NU, LOG2N, TSY>;
    static int resident = 0;  // per kernel instantiation, computed on first use
    if (resident == 0) resident = resident_workgroups(kernel);
    int G = resident;
    if (G <= 0) return hipErrorInvalidValue;
    G = (G + g.batch - 1) / g.batch;  // workgroups per grid
    if (G >= 8) G &= ~7;
    // with few sweeps per cycle one tile per workgroup (more workgroups in flight) measured
    // faster than the persistent walk; with more sweeps the prefetch pays
    G = (NU <= 2 || G > nt) ? nt : G;
    hipLaunchKernelGGL(kernel, dim3(G, 1, g.batch), dim3(kBlock), 0, s, g, rhs, ein, eout, E, rc,
                       psq, zero_e, bx0, by0, nbx, nby);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  const int frame = tx * ty - nt;
  if (frame > 0)
    hipLaunchKernelGGL((k_cycle_edge<T, NU, LOG2N, TSY>), dim3(frame, 1, g.batch), dim3(kBlock), 0, s,
                       g, rhs, ein, eout, E, rc, psq, zero_e, tx, ty, bx0, by0, nbx, nby);
  return hipGetLastError();
}

template <typename T, int NU>
hipError_t cycle_dispatch2(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                           double* rc, double* psq, int zero_e, hipStream_t s) {
  switch (g.log2n) {
    case 2: return cycle_dispatch3<T, NU, 2>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    case 3: return cycle_dispatch3<T, NU, 3>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    case 4: return cycle_dispatch3<T, NU, 4>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    case 5: return cycle_dispatch3<T, NU, 5>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// ---------------------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_rbgs(const Geo& g, const T* rhs, const T* ein, T* eout, hipStream_t s, T rscale) {
  dim3 grid((g.nx + 63) / 64, (g.ny + 31) / 32, g.batch);
  hipLaunchKernelGGL(k_rbgs<T>, grid, dim3(kBlock), 0, s, g, rhs, ein, eout, rscale);
  return hipGetLastError();
}

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

int fused_max_nu() { return 4; }

template <typename T>
hipError_t launch_cycle_fused(const Geo& g, const T* rhs, const T* ein, T* eout,
                              const double* E, double* rc, double* psq, int nu, int zero_e,
                              hipStream_t s) {
  switch (nu) {
    case 1: return cycle_dispatch2<T, 1>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    case 2: return cycle_dispatch2<T, 2>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    case 3: return cycle_dispatch2<T, 3>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    case 4: return cycle_dispatch2<T, 4>(g, rhs, ein, eout, E, rc, psq, zero_e, s);
    default: return hipErrorInvalidValue;
  }
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

template hipError_t launch_rbgs<float>(const Geo&, const float*, const float*, float*, hipStream_t, float);
template hipError_t launch_rbgs<double>(const Geo&, const double*, const double*, double*, hipStream_t, double);
template hipError_t launch_restrict<float>(const Geo&, const float*, const float*, double*, double*, hipStream_t);
template hipError_t launch_restrict<double>(const Geo&, const double*, const double*, double*, double*, hipStream_t);
template hipError_t launch_prolong<float>(const Geo&, const double*, float*, int, hipStream_t);
template hipError_t launch_prolong<double>(const Geo&, const double*, double*, int, hipStream_t);
template hipError_t launch_cycle_fused<float>(const Geo&, const float*, const float*, float*,
                                              const double*, double*, double*, int, int, hipStream_t);
template hipError_t launch_cycle_fused<double>(const Geo&, const double*, const double*, double*,
                                               const double*, double*, double*, int, int, hipStream_t);
template hipError_t launch_outer_residual<float>(const Geo&, const double*, const double*,
                                                 const double*, double, float*, double*, Partials,
                                                 hipStream_t);
template hipError_t launch_outer_residual<double>(const Geo&, const double*, const double*,
                                                  const double*, double, double*, double*, Partials,
                                                  hipStream_t);
template hipError_t launch_add_to<float>(const Geo&, double*, const float*, hipStream_t);
template hipError_t launch_add_to<double>(const Geo&, double*, const double*, hipStream_t);

}  // namespace ism
