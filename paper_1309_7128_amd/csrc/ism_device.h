// Device-side helpers shared by the kernel sources of the ISM solver: geometry of the
// cell-centred grid, the boundary rules and the arithmetic conventions every kernel follows.
//
// Arithmetic conventions (shared by every kernel so that a cell value never depends on the
// kernel that produced it):
//  * A'e (the 5-point Laplacian times h^2) in difference form, added per axis,
//    ((e_W - e_C) + (e_E - e_C)) + ((e_S - e_C) + (e_N - e_C)) (Sec. 2.3 stencil): the
//    order is symmetric in each axis, so it does not depend on the direction rows or
//    columns are visited in.  Behind
//    a Neumann wall the term is absent; behind a Dirichlet wall the neighbour is the mirror
//    ghost -e_C and the term is (-e_C) - e_C (Sec. 4.1 lists both wall kinds).
//  * Red-black Gauss-Seidel (Sec. 3.1): red is (i + j) even; a cell is set to
//    (((e_W + e_E) + (e_S + e_N)) - rhs_C) * (1 / m_C), a missing neighbour contributing 0 and
//    m_C the diagonal: 4, less one per Neumann wall face, plus one per Dirichlet wall face.
//  * Bilinear interpolation (Eq. 5) reaches a ghost coarse centre behind a wall: the
//    mirror image of the first centre, with the same value (Neumann) or the negated value
//    (Dirichlet).
//  * Bilinear prolongation (Eq. 5) in nested form: the x step on the coarse rows in FP64,
//    rounded to the fine type T; the y step and the addition to the fine value in T.
// The library is compiled with -ffp-contract=off so these expressions round exactly as
// written; products that are meant to fuse (the coarse transforms) call fma explicitly.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "ism_internal.h"

namespace ism {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;

__host__ __device__ __forceinline__ int imod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__host__ __device__ __forceinline__ int floordiv(int a, int n) {
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

enum : int { kDirW = 1, kDirE = 2, kDirS = 4, kDirN = 8 };

// The wall faces of a cell: whether each neighbour exists (h*) and, where it does not,
// whether the face is a Dirichlet wall (d*).
struct CellFaces {
  bool hw, he, hs, hn, dw, de, ds, dn;
};

__device__ __forceinline__ CellFaces cell_faces(const Geo& g, int i, int j) {
  CellFaces f;
  f.hw = g.per_x || i > 0;
  f.he = g.per_x || i < g.nx - 1;
  f.hs = g.per_y || j > 0;
  f.hn = g.per_y || j < g.ny - 1;
  f.dw = !f.hw && (g.dmask & kDirW);
  f.de = !f.he && (g.dmask & kDirE);
  f.ds = !f.hs && (g.dmask & kDirS);
  f.dn = !f.hn && (g.dmask & kDirN);
  return f;
}

// 1 / m for a diagonal m in 1 .. 6, each constant rounded once to T.
template <typename T>
__device__ __forceinline__ T inv_diag(int m) {
  constexpr T third = T(1) / T(3), fifth = T(1) / T(5), sixth = T(1) / T(6);
  return m == 4 ? T(0.25)
                : (m == 3 ? third
                          : (m == 5 ? fifth : (m == 2 ? T(0.5) : (m == 6 ? sixth : T(1)))));
}

template <typename T>
__device__ __forceinline__ T inv_count(const Geo& g, int i, int j) {
  const CellFaces f = cell_faces(g, i, j);
  const int m = 4 - (!f.hw && !f.dw) - (!f.he && !f.de) - (!f.hs && !f.ds) - (!f.hn && !f.dn) +
                f.dw + f.de + f.ds + f.dn;
  return inv_diag<T>(m);
}

// One face term of A'e: the difference to an existing neighbour, (-c) - c across a
// Dirichlet wall, nothing across a Neumann wall.
template <typename T>
__device__ __forceinline__ T face_term(T c, T v, bool has, bool dir) {
  return has ? T(v - c) : (dir ? T(T(-c) - c) : T(0));
}

// A'e at a cell from its four neighbours, difference form.
template <typename T>
__device__ __forceinline__ T lap5(T c, T w, T e, T s, T n, bool hw, bool he, bool hs, bool hn,
                                  bool dw = false, bool de = false, bool ds = false,
                                  bool dn = false) {
  return (face_term(c, w, hw, dw) + face_term(c, e, he, de)) +
         (face_term(c, s, hs, ds) + face_term(c, n, hn, dn));
}

template <typename T>
__device__ __forceinline__ T lap5(T c, T w, T e, T s, T n, const CellFaces& f) {
  return lap5<T>(c, w, e, s, n, f.hw, f.he, f.hs, f.hn, f.dw, f.de, f.ds, f.dn);
}

// Coarse index I of a non-periodic axis clamped into 0 .. nc - 1, and the sign of the
// value there: -1 for the ghost behind a Dirichlet wall (lo_dir / hi_dir).
__device__ __forceinline__ double ghost_clamp(int& I, int nc, bool lo_dir, bool hi_dir) {
  if (I < 0) {
    I = 0;
    return lo_dir ? -1.0 : 1.0;
  }
  if (I > nc - 1) {
    I = nc - 1;
    return hi_dir ? -1.0 : 1.0;
  }
  return 1.0;
}

__device__ __forceinline__ double wave_sum_group(double v, int group) {
  for (int off = 1; off < group; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max_group(double v, int group) {
  for (int off = 1; off < group; off <<= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Coarse centres along one axis of nf fine cells split into tiles of n from cell 0 on, the
// last tile short (m = nf - (nc - 1) n cells) when n does not divide nf: the padded domain,
// whose last coarse cell covers the cells that exist (Sec. 3.3, Sec. 4.1).  Positions are in
// doubled fine coordinates (fine cell i spans [2i, 2i + 2], its centre is 2i + 1), so every
// centre is an integer: 2 I n + n for a full tile, 2 (nc - 1) n + m for the last.  The
// centres -1 and nc beyond the ends are the mirror images of the first and last centre in
// the walls, or on a periodic axis the wrapped centres.
__host__ __device__ __forceinline__ int centre2(int I, int nf, int n, int nc, bool periodic) {
  const int last = 2 * (nc - 1) * n + (nf - (nc - 1) * n);
  const int first = nc > 1 ? n : last;
  if (I < 0) return periodic ? last - 2 * nf : -first;
  if (I >= nc) return periodic ? first + 2 * nf : 4 * nf - last;
  return I < nc - 1 ? 2 * I * n + n : last;
}

// Interpolation coordinate along one axis (Eq. 5): for fine index i (any integer on a
// periodic axis, where it is first wrapped into the grid), the lower coarse centre lo
// (unwrapped: on a periodic axis lo + k nc for i + k nf; -1 or nc - 1 beyond a wall) and the
// offset t of the fine centre from it, divided by the size of its rectangle.  With full tiles
// the rectangle is n cells and t = (2k + 1) / (2n); next to a short tile it is shorter.
__host__ __device__ __forceinline__ void interp_axis(int i, int nf, int n, int log2n, int nc, bool periodic,
                                            int& lo, double& t) {
  int shift = 0;
  if (periodic) {
    const int k = floordiv(i, nf);
    i -= k * nf;
    shift = k * nc;
  }
  const int p2 = 2 * i + 1;
  if (p2 < centre2(0, nf, n, nc, periodic)) {
    lo = -1;
  } else if (p2 >= centre2(nc - 1, nf, n, nc, periodic)) {
    lo = nc - 1;
  } else {
    lo = (i - (n >> 1)) >> log2n;  // between two centres of full tiles
  }
  const int c0 = centre2(lo, nf, n, nc, periodic), c1 = centre2(lo + 1, nf, n, nc, periodic);
  // a full rectangle (2n in doubled units, a power of two): the quotient is the exact product
  // with 1/(2n); a shorter one needs the division
  t = c1 - c0 == 2 * n ? double(p2 - c0) * (0.5 / double(n)) : double(p2 - c0) / double(c1 - c0);
  lo += shift;
}

// Mode k of a full axis of nc coarse cells (the common eigenvectors of the 1D coarse factors
// [1 -2 1] and [1 6 1]/8 with the axis's end rules): its angle theta and its entry at cell I,
// orthonormal.  A periodic axis takes the constant, then cos and sin pairs, then the
// alternating mode; a wall axis the cosine (Neumann) or sine (Dirichlet) modes fixed by the
// mirror ghost of each end.
struct AxisMode {
  double theta, value;  // the mode's angle and its entry at cell I
};

__host__ __device__ inline AxisMode axis_mode(int nc, bool per, bool dlo, bool dhi, int k, int I) {
  const double pi = 3.14159265358979323846;
  AxisMode m;
  if (per) {
    if (k == 0) {
      m.theta = 0.0;
      m.value = std::sqrt(1.0 / nc);
    } else if (nc % 2 == 0 && k == nc - 1) {
      m.theta = pi;
      m.value = (I % 2 ? -1.0 : 1.0) / std::sqrt(double(nc));
    } else {
      const int q = (k + 1) / 2;
      m.theta = 2.0 * pi * q / nc;
      const double a = 2.0 * pi * q * I / nc;
      m.value = std::sqrt(2.0 / nc) * ((k & 1) ? std::cos(a) : std::sin(a));
    }
    return m;
  }
  double sc = std::sqrt(2.0 / nc), kk = k;
  if (!dlo && !dhi) {
    if (k == 0) sc = std::sqrt(1.0 / nc);
  } else if (dlo && dhi) {
    kk = k + 1;
    if (k == nc - 1) sc = std::sqrt(1.0 / nc);
  } else {
    kk = k + 0.5;
  }
  m.theta = pi * kk / nc;
  const double a = pi * kk * (I + 0.5) / nc;
  m.value = sc * (dlo ? std::sin(a) : std::cos(a));
  return m;
}

// Eq. 5 evaluated in nested form: interpolate along x on the lower and the upper coarse row,
// then along y, p = (Q11 (1-X) + Q21 X) (1-Y) + (Q12 (1-X) + Q22 X) Y, rounded in this order
// (one linear step of it here).
__device__ __forceinline__ double lerp(double a, double b, double t) { return a * (1.0 - t) + b * t; }

// (P E) at fine cell (i, j) of the grid (Eq. 5), from the grid's coarse values Eb: the x step
// on the two coarse rows in FP64, rounded to T, the y step in T.  A ghost centre behind a wall
// takes the mirrored value (negated behind a Dirichlet wall); the signs multiply exactly, so
// negating a corner value commutes with the rounding.
template <typename T>
__device__ __forceinline__ T prolong_at(const Geo& g, const double* __restrict__ Eb, int i, int j) {
  int ilo, jlo;
  double X, Y;
  interp_axis(i, g.nx, g.n, g.log2n, g.ncx, g.per_x, ilo, X);
  interp_axis(j, g.ny, g.n, g.log2n, g.ncy, g.per_y, jlo, Y);
  int ihi = ilo + 1, jhi = jlo + 1;
  double sil = 1.0, sih = 1.0, sjl = 1.0, sjh = 1.0;
  if (g.per_x) {
    ilo = imod(ilo, g.ncx);
    ihi = imod(ihi, g.ncx);
  } else {
    sil = ghost_clamp(ilo, g.ncx, g.dmask & kDirW, g.dmask & kDirE);
    sih = ghost_clamp(ihi, g.ncx, g.dmask & kDirW, g.dmask & kDirE);
  }
  if (g.per_y) {
    jlo = imod(jlo, g.ncy);
    jhi = imod(jhi, g.ncy);
  } else {
    sjl = ghost_clamp(jlo, g.ncy, g.dmask & kDirS, g.dmask & kDirN);
    sjh = ghost_clamp(jhi, g.ncy, g.dmask & kDirS, g.dmask & kDirN);
  }
  const T lo = T(lerp(sjl * sil * Eb[jlo * g.ncx + ilo], sjl * sih * Eb[jlo * g.ncx + ihi], X));
  const T hi = T(lerp(sjh * sil * Eb[jhi * g.ncx + ilo], sjh * sih * Eb[jhi * g.ncx + ihi], X));
  return lo * T(1.0 - Y) + hi * T(Y);
}

}  // namespace
}  // namespace ism
