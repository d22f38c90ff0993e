// Device-side helpers shared by the kernel sources of the ISM solver: geometry of the
// cell-centred grid, the boundary rules and the arithmetic conventions every kernel follows.
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
#pragma once

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

}  // namespace
}  // namespace ism
