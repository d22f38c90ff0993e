// Host construction of the exact coarse solve's tables for grids that the tile size does not
// divide (Sec. 3.3, Eq. 5: the interpolation rectangles next to the short last tile differ;
// Sec. 4.1: automated padding).
//
// The coarse operator R A' P stays separable, A_c = K_x (x) M_y + M_x (x) K_y, with per axis
// K = n R D P and M = R P / n (R the tile sums, D the fine three-point operator with the
// axis's end rule, P the 1D linear interpolation of Eq. 5; the factors n cancel in the
// products).  With full tiles K and M are the Toeplitz [1 -2 1] and [1 6 1]/8 with
// closed-form common eigenvectors (built on the device for such grids).  With a
// short last tile K stays symmetric but M does not, so each padded axis is diagonalized
// through the pencil K v = mu M v: C = M^-1 K has real eigenvalues mu and eigenvectors V.
// With left vectors U^T = V^-1 M^-1 (so that U^T M V = I and U^T K V = diag(mu)) the coarse
// solve is
//   E = V_y [ (U_y^T R_c U_x) ./ (mu_x + mu_y) ] V_x^T,
// the same four products as with full tiles, with forward tables F = U and mode factors
// (k, m) = (mu, 1).  A full axis keeps its closed form (F = V orthonormal, (k, m) the
// eigenvalues of K and M), and 1/lambda = 1/(k_x m_y + m_x k_y) covers every combination.
//
// The eigenvectors come from a real Schur form: Householder reduction to Hessenberg form,
// shifted QR sweeps with Givens rotations (Wilkinson shift, exceptional shifts on stalls) and
// deflation; the spectrum of these pencils is real, so the Schur form is triangular and the
// eigenvectors follow by back substitution.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "ism.h"
#include "ism_device.h"

namespace ism {

namespace {

using Mat = std::vector<double>;  // row-major n x n

// LU factorization with partial pivoting of the n x n matrix a (in place); false if singular.
bool lu_factor(int n, Mat& a, std::vector<int>& piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[size_t(i) * n + k]) > std::fabs(a[size_t(p) * n + k])) p = i;
    piv[k] = p;
    if (a[size_t(p) * n + k] == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[size_t(k) * n + j], a[size_t(p) * n + j]);
    for (int i = k + 1; i < n; ++i) {
      const double f = a[size_t(i) * n + k] / a[size_t(k) * n + k];
      a[size_t(i) * n + k] = f;
      for (int j = k + 1; j < n; ++j) a[size_t(i) * n + j] -= f * a[size_t(k) * n + j];
    }
  }
  return true;
}

// Solves A X = B for the factored A; B is n x m, row-major, overwritten by X.
void lu_solve(int n, const Mat& lu, const std::vector<int>& piv, Mat& b, int m) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k)
      for (int j = 0; j < m; ++j) std::swap(b[size_t(k) * m + j], b[size_t(piv[k]) * m + j]);
  for (int i = 1; i < n; ++i)
    for (int k = 0; k < i; ++k) {
      const double f = lu[size_t(i) * n + k];
      if (f != 0.0)
        for (int j = 0; j < m; ++j) b[size_t(i) * m + j] -= f * b[size_t(k) * m + j];
    }
  for (int i = n - 1; i >= 0; --i) {
    for (int k = i + 1; k < n; ++k) {
      const double f = lu[size_t(i) * n + k];
      if (f != 0.0)
        for (int j = 0; j < m; ++j) b[size_t(i) * m + j] -= f * b[size_t(k) * m + j];
    }
    const double d = lu[size_t(i) * n + i];
    for (int j = 0; j < m; ++j) b[size_t(i) * m + j] /= d;
  }
}

// Reduces a (n x n) to upper Hessenberg form H = Q^T a Q in place; q receives Q.
void hessenberg(int n, Mat& a, Mat& q) {
  q.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) q[size_t(i) * n + i] = 1.0;
  std::vector<double> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double norm = 0.0;
    for (int i = k + 1; i < n; ++i) norm += a[size_t(i) * n + k] * a[size_t(i) * n + k];
    norm = std::sqrt(norm);
    if (norm == 0.0) continue;
    const double x0 = a[size_t(k + 1) * n + k];
    const double alpha = x0 >= 0.0 ? -norm : norm;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = a[size_t(i) * n + k] - (i == k + 1 ? alpha : 0.0);
      vn += v[i] * v[i];
    }
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // a <- (I - 2 v v^T) a (rows k+1..), then a <- a (I - 2 v v^T), q <- q (I - 2 v v^T)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * a[size_t(i) * n + j];
      for (int i = k + 1; i < n; ++i) a[size_t(i) * n + j] -= 2.0 * v[i] * s;
    }
    for (int i = 0; i < n; ++i) {
      double s = 0.0, t = 0.0;
      for (int j = k + 1; j < n; ++j) {
        s += a[size_t(i) * n + j] * v[j];
        t += q[size_t(i) * n + j] * v[j];
      }
      for (int j = k + 1; j < n; ++j) {
        a[size_t(i) * n + j] -= 2.0 * s * v[j];
        q[size_t(i) * n + j] -= 2.0 * t * v[j];
      }
    }
  }
}

// Shifted QR sweeps on the Hessenberg h (n x n), accumulating the rotations into z, until h
// is upper triangular (a real spectrum).  False if the iteration does not converge or a 2 x 2
// block with complex eigenvalues remains.
bool schur_real(int n, Mat& h, Mat& z) {
  const double eps = 1e-15;
  int hi = n - 1, it = 0;
  auto H = [&](int i, int j) -> double& { return h[size_t(i) * n + j]; };
  while (hi > 0) {
    if (std::fabs(H(hi, hi - 1)) <= eps * (std::fabs(H(hi, hi)) + std::fabs(H(hi - 1, hi - 1)))) {
      H(hi, hi - 1) = 0.0;
      --hi;
      it = 0;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(H(lo, lo - 1)) > eps * (std::fabs(H(lo, lo)) + std::fabs(H(lo - 1, lo - 1))))
      --lo;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer its last entry
    const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    const double tr = a + d, det = a * d - b * c, disc = 0.25 * tr * tr - det;
    double mu;
    if (disc >= 0.0) {
      const double r = std::sqrt(disc), l1 = 0.5 * tr + r, l2 = 0.5 * tr - r;
      mu = std::fabs(l1 - d) < std::fabs(l2 - d) ? l1 : l2;
    } else {
      mu = 0.5 * tr;
    }
    if (it > 0 && it % 11 == 0) mu = d + std::fabs(H(hi, hi - 1));  // exceptional shift
    if (++it > 100 * n) return false;
    double x = H(lo, lo) - mu, y = H(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, y);
      const double cs = r == 0.0 ? 1.0 : x / r, sn = r == 0.0 ? 0.0 : y / r;
      for (int j = std::max(lo, k - 1); j < n; ++j) {  // rows k, k+1
        const double u = H(k, j), w = H(k + 1, j);
        H(k, j) = cs * u + sn * w;
        H(k + 1, j) = -sn * u + cs * w;
      }
      const int i1 = std::min(hi, k + 2);
      for (int i = 0; i <= i1; ++i) {  // columns k, k+1
        const double u = H(i, k), w = H(i, k + 1);
        H(i, k) = cs * u + sn * w;
        H(i, k + 1) = -sn * u + cs * w;
      }
      for (int i = 0; i < n; ++i) {
        const double u = z[size_t(i) * n + k], w = z[size_t(i) * n + k + 1];
        z[size_t(i) * n + k] = cs * u + sn * w;
        z[size_t(i) * n + k + 1] = -sn * u + cs * w;
      }
      if (k + 1 < hi) {
        x = H(k + 1, k);
        y = H(k + 2, k);
      }
    }
  }
  return true;
}

// Real eigenvalues mu and unit eigenvectors V (columns) of the n x n matrix c.
bool eig_real(int n, Mat c, std::vector<double>& mu, Mat& V) {
  Mat z;
  hessenberg(n, c, z);
  if (!schur_real(n, c, z)) return false;
  // eigenvectors of the triangular form by back substitution, then V = Z Y
  Mat y(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    y[size_t(j) * n + j] = 1.0;
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += c[size_t(i) * n + k] * y[size_t(k) * n + j];
      double den = c[size_t(i) * n + i] - c[size_t(j) * n + j];
      if (std::fabs(den) < 1e-300) den = 1e-300;
      y[size_t(i) * n + j] = -s / den;
    }
  }
  mu.resize(n);
  V.assign(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    mu[j] = c[size_t(j) * n + j];
    double norm = 0.0;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k <= j; ++k) s += z[size_t(i) * n + k] * y[size_t(k) * n + j];
      V[size_t(i) * n + j] = s;
      norm += s * s;
    }
    norm = std::sqrt(norm);
    for (int i = 0; i < n; ++i) V[size_t(i) * n + j] /= norm;
  }
  return true;
}

// Closed-form tables of a full axis: the orthonormal modes of axis_mode (F = V) and the
// eigenvalues of K = [1 -2 1] and M = [1 6 1]/8 on them.
void closed_axis(int nc, bool per, bool dlo, bool dhi, AxisTable& t) {
  t.V.assign(size_t(nc) * nc, 0.0);
  t.k.assign(nc, 0.0);
  t.m.assign(nc, 0.0);
  for (int k = 0; k < nc; ++k) {
    for (int I = 0; I < nc; ++I) t.V[size_t(I) * nc + k] = axis_mode(nc, per, dlo, dhi, k, I).value;
    const double c = std::cos(axis_mode(nc, per, dlo, dhi, k, 0).theta);
    t.k[k] = -2.0 * (1.0 - c);
    t.m[k] = (3.0 + c) / 4.0;
  }
  t.F = t.V;
}

// The 1D factors n R D P and R P / n (nc x nc) of an axis with nf fine cells in tiles of n.
void axis_pencil(int nf, int n, int nc, bool per, bool dlo, bool dhi, Mat& K, Mat& M) {
  int log2n = 0;
  while ((1 << log2n) < n) ++log2n;
  // P as (lower index, upper index, their weights) per fine cell, ghosts folded
  std::vector<int> lo(nf), hi(nf);
  std::vector<double> wl(nf), wh(nf);
  for (int i = 0; i < nf; ++i) {
    int l;
    double t;
    interp_axis(i, nf, n, log2n, nc, per, l, t);
    int h = l + 1;
    double sl = 1.0, sh = 1.0;
    if (per) {
      l = imod(l, nc);
      h = imod(h, nc);
    } else {
      if (l < 0) { l = 0; sl = dlo ? -1.0 : 1.0; }
      if (h > nc - 1) { h = nc - 1; sh = dhi ? -1.0 : 1.0; }
    }
    lo[i] = l;
    hi[i] = h;
    wl[i] = sl * (1.0 - t);
    wh[i] = sh * t;
  }
  K.assign(size_t(nc) * nc, 0.0);
  M.assign(size_t(nc) * nc, 0.0);
  std::vector<double> row(nc);
  for (int i = 0; i < nf; ++i) {
    const int I = i / n;  // the tile of fine cell i
    M[size_t(I) * nc + lo[i]] += wl[i];
    M[size_t(I) * nc + hi[i]] += wh[i];
    // (D P)[i] = sum over the two faces of cell i of (P[nb] - P[i]); a Dirichlet wall face
    // adds (-P[i]) - P[i], a Neumann wall face nothing
    std::fill(row.begin(), row.end(), 0.0);
    for (int side = -1; side <= 1; side += 2) {
      int j = i + side;
      if (per) {
        j = imod(j, nf);
      } else if (j < 0 || j >= nf) {
        if ((j < 0 && dlo) || (j >= nf && dhi)) {
          row[lo[i]] -= 2.0 * wl[i];
          row[hi[i]] -= 2.0 * wh[i];
        }
        continue;
      }
      row[lo[j]] += wl[j];
      row[hi[j]] += wh[j];
      row[lo[i]] -= wl[i];
      row[hi[i]] -= wh[i];
    }
    for (int J = 0; J < nc; ++J) K[size_t(I) * nc + J] += row[J];
  }
  // scaled to the closed forms' normalization, n K and M / n ([1 -2 1] and [1 6 1] / 8 with
  // full tiles), so that the two kinds of axis combine: K_x (x) M_y is unchanged
  for (size_t e = 0; e < K.size(); ++e) {
    K[e] *= double(n);
    M[e] /= double(n);
  }
}

// Pencil tables of a padded axis; false with a message if the eigen-decomposition fails.
bool pencil_axis(int nf, int n, int nc, bool per, bool dlo, bool dhi, AxisTable& t,
                 std::string& err) {
  Mat K, M;
  axis_pencil(nf, n, nc, per, dlo, dhi, K, M);
  Mat lu = M;
  std::vector<int> piv;
  if (!lu_factor(nc, lu, piv)) return err = "padded axis: the interpolation factor M is singular", false;
  Mat C = K;  // C = M^-1 K
  lu_solve(nc, lu, piv, C, nc);
  std::vector<double> mu;
  Mat V;
  if (!eig_real(nc, C, mu, V)) return err = "padded axis: eigen-decomposition did not converge", false;
  // modes in order of decreasing eigenvalue: the constant mode (mu = 0) of a Neumann or
  // periodic axis first, as with full tiles
  std::vector<int> ord(nc);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return mu[a] > mu[b]; });
  t.V.assign(size_t(nc) * nc, 0.0);
  t.k.assign(nc, 0.0);
  t.m.assign(nc, 1.0);
  for (int k = 0; k < nc; ++k) {
    t.k[k] = mu[ord[k]];
    for (int I = 0; I < nc; ++I) t.V[size_t(I) * nc + k] = V[size_t(I) * nc + ord[k]];
  }
  // the constant mode of a singular axis is exactly mu = 0
  if (!dlo && !dhi && std::fabs(t.k[0]) < 1e-12) t.k[0] = 0.0;
  // U^T = V^-1 M^-1, i.e. U = M^-T V^-T: solve M^T X = V^-T column by column, X = U
  Mat vlu = t.V;
  std::vector<int> vpiv;
  if (!lu_factor(nc, vlu, vpiv)) return err = "padded axis: singular eigenvector matrix", false;
  Mat vinv(size_t(nc) * nc, 0.0);
  for (int i = 0; i < nc; ++i) vinv[size_t(i) * nc + i] = 1.0;
  lu_solve(nc, vlu, vpiv, vinv, nc);  // V^-1
  Mat mt(size_t(nc) * nc);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) mt[size_t(i) * nc + j] = M[size_t(j) * nc + i];
  std::vector<int> mpiv;
  if (!lu_factor(nc, mt, mpiv)) return err = "padded axis: the interpolation factor M is singular", false;
  Mat rhs(size_t(nc) * nc);  // V^-T
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) rhs[size_t(i) * nc + j] = vinv[size_t(j) * nc + i];
  lu_solve(nc, mt, mpiv, rhs, nc);
  t.F = rhs;  // F[I][k] = U[I][k]
  return true;
}

}  // namespace

bool coarse_axis_table(int nf, int n, int nc, bool per, bool dlo, bool dhi, AxisTable& t,
                       std::string& err) {
  if (nf % n == 0) {
    closed_axis(nc, per, dlo, dhi, t);
    return true;
  }
  return pencil_axis(nf, n, nc, per, dlo, dhi, t, err);
}

}  // namespace ism
