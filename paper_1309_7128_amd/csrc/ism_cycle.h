// The fused two-level cycle kernel of the ISM solver (prolongation, red-black sweeps,
// residual and restriction in one pass over the grid), as templates; ism_cycle_f32.hip and
// ism_cycle_f64.hip instantiate them for the two fine-grid types.
#pragma once

#include <algorithm>
#include <cmath>

#include "ism_device.h"

namespace ism {
namespace {

// ----------------------------------------------------------------------------------------
// Fused two-level cycle kernel: row-pipelined temporal blocking in registers.
//
// One wave owns a strip of LW = 64 CPL columns (CPL consecutive cells per lane) and a run of
// L output rows, and walks along the strip one row at a time (up, or down for every other
// chunk) holding a ring of P rows of e and rhs in registers.  When row t enters it receives
// the bilinear coarse correction (Eq. 5).  Then half-step k = 1 .. 2 NU (odd k red, even k
// black) updates its colour on the row that entered k steps earlier: at that moment the row
// after it has just had half-step k - 1 and the row before it still waits for half-step
// k + 1, so every cell sees exactly the neighbours the k-th half-step of a whole-grid sweep
// would give it.  The row that entered 2 NU + 1 steps earlier is then final: its residual is formed,
// summed over the n x n coarse tiles, and the row is written out.  East and west neighbours
// across lanes come from DPP wavefront shifts, so the half-steps touch neither LDS nor
// memory.  The strip's PX >= 2 NU + 1 outer columns on each side and its first H rows absorb
// the stale values its edges inject (they spread one cell per half-step); the VW = LW - 2 PX
// valid columns start on a coarse tile boundary.  Per cycle e and rhs are read once (plus
// halos) and e is written once.
// ----------------------------------------------------------------------------------------
constexpr int stream_pad(int h, int n, int cpl, int lw) {
  int px = (h + cpl - 1) / cpl * cpl;
  while ((lw - 2 * px) % n != 0) px += cpl;
  return px;
}

template <typename T, int NU, int LOG2N>
struct Stream {
  static constexpr int CPL = 4;           // cells per lane
  static constexpr int LW = kWave * CPL;  // columns per strip
  static constexpr int N = 1 << LOG2N;
  static constexpr int H = 2 * NU + 1;    // reach of one cycle (2 NU half-steps + residual)
  static constexpr int PX = stream_pad(H, N, CPL, LW);
  static constexpr int VW = LW - 2 * PX;  // valid columns per strip
  // rows read ahead, through a per-wave LDS ring of DL slots (16-byte chunks per lane of e
  // and rhs in each); 4 in FP32 at n = 16, where a fifth slot would leave room for only two
  // workgroups per CU (the staged coarse block is larger there): 107 us against 119 us per
  // launch on the 4096 x 8192 jet
  static constexpr int C16 = CPL * int(sizeof(T)) / 16;
  static constexpr int DL = sizeof(T) == 4 ? (N == 16 ? 4 : 5) : 3;
  static constexpr int SLOT = 2 * C16 * kWave * 16;  // bytes per ring slot
  // register ring rows: 2 NU + 3 live, even (fixed row parity per slot)
  static constexpr int P = 2 * NU + 4;
  static constexpr int L = N >= 8 ? 128 : 64;  // output rows per unit (half that by a wall)
  // coarse rows and columns one walk interpolates from, at most (staged in LDS per wave):
  // with full tiles (L + 2 H) / N + 3 rows and LW / N + 3 columns; next to a short last tile
  // of a periodic axis the lower centres of a walk's first and last cells can each move out
  // by one
  static constexpr int NR = (L + 2 * H) / N + 5;
  static constexpr int NC = LW / N + 4;
  static_assert(N >= CPL && VW >= N && VW % N == 0 && PX % CPL == 0, "strip geometry");
  static_assert(P % 2 == 0 && P >= 2 * NU + 3, "ring length");
  // LDS of a workgroup of kBlock / kWave waves (coarse block, x-interpolated rows, read-ahead
  // ring) and the waves per SIMD the launch is compiled for: as many as the 160 KiB of LDS
  // per CU allow (one wave per SIMD per workgroup), at most three in FP32 and two in FP64,
  // the most the ring's registers leave room for
  static constexpr int LDS_BYTES =
      (kBlock / kWave) * (NR * NC * 8 + 2 * C16 * kWave * 16 + DL * SLOT);
  static constexpr int WAVES_LDS = (160 * 1024) / LDS_BYTES;
  static constexpr int WAVES_REG = sizeof(T) == 4 ? 3 : 2;
  static constexpr int WAVES = WAVES_LDS < 1 ? 1 : (WAVES_LDS < WAVES_REG ? WAVES_LDS : WAVES_REG);
};


template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
};
template <>
struct Vec16<double> {
  using type = double2;
};

template <typename T, int C>
__device__ __forceinline__ void load_cells(const T* __restrict__ p, T (&v)[C]) {
  using V = typename Vec16<T>::type;
  constexpr int K = 16 / sizeof(T);
#pragma unroll
  for (int q = 0; q < C / K; ++q) {
    const V x = reinterpret_cast<const V*>(p)[q];
#pragma unroll
    for (int k = 0; k < K; ++k) v[q * K + k] = (&x.x)[k];
  }
}

template <typename T, int C>
__device__ __forceinline__ void store_cells(T* __restrict__ p, const T (&v)[C]) {
  using V = typename Vec16<T>::type;
  constexpr int K = 16 / sizeof(T);
#pragma unroll
  for (int q = 0; q < C / K; ++q) {
    V x;
#pragma unroll
    for (int k = 0; k < K; ++k) (&x.x)[k] = v[q * K + k];
    reinterpret_cast<V*>(p)[q] = x;
  }
}

// A value known to be the same in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(b & 0xffffffffll)));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((long long)lo | ((long long)hi << 32));
}

// The value of lane l - 1 (wave_shr:1) or lane l + 1 (wave_shl:1); lanes without a source
// get 0.
constexpr int kDppFromLeft = 0x138, kDppFromRight = 0x130;

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, 0xf, 0xf, false));
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)lo | ((long long)hi << 32));
}

// LDS byte offset of a pointer into __shared__ memory.
typedef __attribute__((address_space(3))) char LdsChar;
typedef unsigned Vec4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned lds_offset(const void* p) {
  return (unsigned)(uintptr_t)(const LdsChar*)p;
}

// 16 bytes per lane from global memory into LDS: lane i's bytes at g land at LDS byte offset
// lds + 16 i (an LDS-DMA load, M0 holding the base; lds must be wave-uniform).  Issued as
// inline assembly so that the compiler, which otherwise waits for every such load in flight
// before any LDS read, leaves the waits to the caller.  The LDS it writes is touched only by
// these statements and lds_take (volatile, so kept in program order), and the global memory
// it reads is not written by the kernel, so no memory clobber is needed.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const void* g, unsigned lds) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(g), "s"(lds) : "m0");
}
#pragma clang diagnostic pop

// Wait until at most NV vector-memory operations are outstanding, then read K 16-byte chunks
// per lane from LDS at a, a + 1024, ... and wait for them.
template <int NV, int K>
__device__ __forceinline__ void lds_take(unsigned a, Vec4u (&v)[K]) {
  static_assert(K == 2 || K == 4, "two or four chunks");
  if constexpr (K == 2) {
    asm volatile(
        "s_waitcnt vmcnt(%3)\n\tds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:1024\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1])
        : "v"(a), "n"(NV));
  } else {
    asm volatile(
        "s_waitcnt vmcnt(%5)\n\tds_read_b128 %0, %4\n\tds_read_b128 %1, %4 offset:1024\n\t"
        "ds_read_b128 %2, %4 offset:2048\n\tds_read_b128 %3, %4 offset:3072\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])
        : "v"(a), "n"(NV));
  }
}

// The CPL cells of one array held in 16-byte chunks c0, c0 + 1, ...
template <typename T, int CPL, int K>
__device__ __forceinline__ void unpack_cells(const Vec4u (&v)[K], int c0, T (&out)[CPL]) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int p = 0; p < CPL; ++p) out[p] = __uint_as_float(v[c0 + p / 4][p % 4]);
  } else {
#pragma unroll
    for (int p = 0; p < CPL; ++p) {
      const Vec4u& c = v[c0 + p / 2];
      out[p] = __hiloint2double(int(c[2 * (p % 2) + 1]), int(c[2 * (p % 2)]));
    }
  }
}

// Kinds of walk.  PLAIN: every row and column the walk reads exists in the grid (possibly
// wrapped), so every cell has four neighbours and diagonal 4.  ROWS: the rows may reach
// past a wall in y (or off the grid); every column exists.  EDGE: the strip also reads
// columns behind a wall in x, handled lane by lane.  The *_TAB kinds are ROWS and EDGE on a
// grid that the tile size does not divide, which read the interpolation tables; keeping
// them apart keeps the walks that other grids run compact (their code shares the
// instruction cache with the plain walks).
enum WalkKind { kPlain = 0, kRows = 1, kEdge = 2, kRowsTab = 3, kEdgeTab = 4 };

// One wave's walk along its strip: output rows y0 .. y0 + min(L, ny - y0) - 1 of the strip
// whose first read column is xs, walking up (rows ys = y0 - H .. y0 + L + H - 1) or, with
// down, down (rows y0 + L + H .. ys: one extra row at the top so that every ring slot sees
// rows of the same parity either way).  A red-black sweep does not depend on the order its
// rows are visited in, so both walks give the same cells bit for bit; the coarse-tile sums
// add the rows in walk order.  Neighbouring chunks walk in opposite directions so that both
// reach the rows around their common boundary at about the same time, and the second read
// of those halo rows can hit in cache.
//
// A PLAIN walk keeps rhs / 4 in its ring instead of rhs (exact: a power of two) and sets a
// cell to fma(sum, 1/4, -rhs/4), which rounds (sum - rhs) / 4 once: bit for bit the value
// (sum - rhs) * (1/4) of the other walks, one operation instead of two.  Its residual
// fma(rhs/4, 4, -A'e) is likewise exactly rhs - A'e rounded once.  (Both hold while rhs / 4
// stays a normal number, i.e. |rhs| >= 2^-124 or rhs = 0.)
template <typename T, int NU, int LOG2N, int KIND>
__device__ __forceinline__ void cycle_walk(const Geo& g, const T* __restrict__ rb,
                                           const T* __restrict__ eb, T* __restrict__ ob,
                                           const double* __restrict__ Eb, double* __restrict__ rc,
                                           double* __restrict__ psq, double* __restrict__ sE,
                                           typename Vec16<T>::type* __restrict__ sX,
                                           Vec4u* __restrict__ sR, long long coff, int zero_e,
                                           int xs, int y0, int L, bool down,
                                           const double2* __restrict__ tabx,
                                           const double2* __restrict__ taby, int maxmode) {
  using S = Stream<T, NU, LOG2N>;
  using V16 = typename Vec16<T>::type;
  constexpr bool EDGE = KIND == kEdge || KIND == kEdgeTab, PLAIN = KIND == kPlain;
  constexpr bool TAB = KIND == kRowsTab || KIND == kEdgeTab;
  constexpr int CPL = S::CPL, N = S::N, H = S::H, PX = S::PX, VW = S::VW, P = S::P;
  constexpr int G = N / CPL;  // lanes per coarse tile
  const int lane = threadIdx.x & (kWave - 1);
  // Inverse diagonals, uniform over the walk.  The diagonal is 4, less one per Neumann wall
  // face, plus one per Dirichlet wall face (its ghost -e counts twice).  y part of the first
  // and last row (2 on a periodic axis), x part of the west and east wall cells; then
  // 1 / diagonal for the first, middle and last row of an interior cell (ic*) and of the
  // wall cells (iw*, ie*).
  const int mys = g.per_y ? 2 : ((g.dmask & kDirS) ? 3 : 1);
  const int myn = g.per_y ? 2 : ((g.dmask & kDirN) ? 3 : 1);
  const int mxw = (g.dmask & kDirW) ? 3 : 1, mxe = (g.dmask & kDirE) ? 3 : 1;
  const T icS = inv_diag<T>(2 + mys), icN = inv_diag<T>(2 + myn);
  const T iwS = inv_diag<T>(mxw + mys), iwM = inv_diag<T>(mxw + 2), iwN = inv_diag<T>(mxw + myn);
  const T ieS = inv_diag<T>(mxe + mys), ieM = inv_diag<T>(mxe + 2), ieN = inv_diag<T>(mxe + myn);
  const int ys = y0 - H;
  const int yend = y0 + min(L, g.ny - y0) + H;  // rows ys .. yend - 1 are output or halo
  const int nrows = yend - ys + (down ? 1 : 0);  // rows the walk reads
  const int dir = down ? -1 : 1;
  const int t0 = down ? yend : ys;  // first row read; row of step s: t0 + dir s

  // this lane's first column (unwrapped), the column it is read from, whether it exists
  const int cu = xs + CPL * lane;
  bool col_in = true;
  int cw = cu;
  if (g.per_x) {
    cw = imod(cu, g.nx);
  } else if (EDGE) {
    col_in = cu >= 0 && cu < g.nx;
    cw = col_in ? cu : 0;
  }
  const bool lane_out = lane >= PX / CPL && lane < (PX + VW) / CPL && cu < g.nx;
  // whether the lane's cells exist (unwrapped): the others add nothing to a coarse tile sum
  // (they matter where a short last tile shares its lane group with columns past the grid)
  const bool lane_sum = cu >= 0 && cu < g.nx;

  // The coarse values the walk interpolates from (Eq. 5, boundary rule applied), staged in
  // this wave's LDS block: rows crow(ys) .. crow(yend) + 1, columns from the lower
  // neighbour of the strip's first column on.  Only this wave reads them.
  // Fine row t's lower coarse row and y weight (Eq. 5).  Where every rectangle is full (n
  // rows: an axis that n divides, and every row a plain walk reads) a shift and a dyadic
  // weight, also for rows past a wall or a periodic seam.  On an axis with a short last tile
  // the walk reads the axis's table (entry .x the weight, .y the lower centre of the
  // wrapped or clamped row), the lower centre unwrapped again on a periodic axis.
  const bool tab_y = TAB && (g.ny & (N - 1)), tab_x = TAB && (g.nx & (N - 1));
  auto row_interp = [&](int t, int& lo, double& w) {
    if (!tab_y) {
      lo = (t - N / 2) >> LOG2N;
      w = double(2 * ((t - N / 2) & (N - 1)) + 1) * (1.0 / double(2 * N));
    } else {
      int shift = 0, tw;
      if (g.per_y) {
        const int k = floordiv(t, g.ny);
        tw = t - k * g.ny;
        shift = k * g.ncy;
      } else {
        tw = min(max(t, 0), g.ny - 1);
      }
      const double2 e = taby[tw];
      lo = int(e.y) + shift;
      w = e.x;
    }
  };
  auto crow = [&](int t) {
    int lo;
    double w;
    row_interp(t, lo, w);
    return lo;
  };
  const int J0 = crow(ys);
  // the lower centre of column xs, the strip's first
  int I0;
  if (!tab_x) {
    I0 = (xs - N / 2) >> LOG2N;
  } else {
    int shift = 0, cb;
    if (g.per_x) {
      const int k = floordiv(xs, g.nx);
      cb = xs - k * g.nx;
      shift = k * g.ncx;
    } else {
      cb = min(max(xs, 0), g.nx - 1);
    }
    I0 = int(tabx[cb].y) + shift;
  }
  {
    // (the bound on the staged rows holds by the geometry; the clamp keeps it in memory)
    const int nr = min(crow(yend) + 2 - J0, S::NR);
    for (int i = lane; i < nr * S::NC; i += kWave) {
      const int rr = i / S::NC, c = i - rr * S::NC;
      int J = J0 + rr, I = I0 + c;
      // a ghost centre behind a wall mirrors the first one, negated behind a Dirichlet wall
      double sg = 1.0;
      if (g.per_y) J = imod(J, g.ncy);
      else sg = ghost_clamp(J, g.ncy, g.dmask & kDirS, g.dmask & kDirN);
      if (g.per_x) I = imod(I, g.ncx);
      else sg *= ghost_clamp(I, g.ncx, g.dmask & kDirW, g.dmask & kDirE);
      sE[i] = sg * Eb[(long long)J * g.ncx + I];
    }
    // the block is written and read by this wave only: order its writes before the reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // The ring: e and rhs (PLAIN: rhs / 4) of the last P rows read, the row of step s in slot
  // s mod P,
  // and per slot the row's inverse diagonals (uniform): for cells with both x-neighbours,
  // and (EDGE) for the west and east wall cells; 0 for rows off the grid and rows not read
  // yet, which the half-steps then leave at 0.
  T e[P][CPL], r[P][CPL];
  T invs[P], iws[P], ies[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    invs[q] = iws[q] = ies[q] = T(0);
#pragma unroll
    for (int p = 0; p < CPL; ++p) e[q][p] = r[q][p] = T(0);
  }
  // Coarse rows J interpolated along x at the lane's cells (FP64, rounded to T), kept in LDS
  // buffer J & 1 (each lane reads back only what it wrote): [buffer][16-byte chunk][lane].
  constexpr int K16 = 16 / int(sizeof(T)), C16X = CPL / K16;
  // with full rectangles, the lane's first lower centre relative to the staged block
  const int crel = ((cu - N / 2) >> LOG2N) - I0;
  auto put_x = [&](int J) {
    V16* d = sX + (J & 1) * C16X * kWave + lane;
    if (!tab_x) {
      // full rectangles: for n >= 8 all of a lane's cells lie between the same two coarse
      // centres, for n = 4 its first and last two cells between consecutive pairs
      constexpr int NEC = N >= 8 ? 2 : 3;
      constexpr double inv2n = 1.0 / double(2 * N);
      const double* qq = sE + (J - J0) * S::NC + crel;
      int c0 = cu;
      asm volatile("" : "+v"(c0));  // recomputed here, not held in registers for the walk
      double v[NEC];
#pragma unroll
      for (int k = 0; k < NEC; ++k) v[k] = qq[k];
#pragma unroll
      for (int cq = 0; cq < C16X; ++cq) {
        V16 w;
#pragma unroll
        for (int k = 0; k < K16; ++k) {
          const int p = cq * K16 + k;
          const double X = double(2 * ((c0 + p - N / 2) & (N - 1)) + 1) * inv2n;
          const int m = N >= 8 ? 0 : (p >> 1);
          (&w.x)[k] = T(lerp(v[m], v[m + 1], X));
        }
        d[cq * kWave] = w;
      }
    } else {
      // the axis's table at the lane's columns (wrapped or clamped; a lane's CPL cells lie in
      // one period of a periodic axis, nx being a multiple of CPL), one cell at a time and
      // each value stored at once: the ring holds most registers, and this path must not
      // raise the kernel's register count
      const double* q = sE + (J - J0) * S::NC - I0;
      int c0 = cu;
      asm volatile("" : "+v"(c0));
      int cb = c0, shift = 0;
      if (g.per_x) {
        const int k = floordiv(c0, g.nx);
        cb = c0 - k * g.nx;
        shift = k * g.ncx;
      }
      T* dt = reinterpret_cast<T*>(d);
#pragma unroll 1
      for (int p = 0; p < CPL; ++p) {
        const double2 e = tabx[g.per_x ? cb + p : min(max(cb + p, 0), g.nx - 1)];
        const int lo = int(e.y) + shift;
        dt[(p / K16) * kWave * K16 + p % K16] = T(lerp(q[lo], q[lo + 1], e.x));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  int jc = crow(t0);
  put_x(jc);
  put_x(jc + 1);
  // the next row to read, wrapped or clamped into the grid
  int jn = g.per_y ? imod(t0, g.ny) : min(max(t0, 0), g.ny - 1);
  // Rows are read DL ahead by LDS-DMA into this wave's LDS ring (slot (step) mod DL:
  // the C16 chunks of e, then those of rhs) and enter the register ring when used.  Every row
  // issues the same 2 C16 loads (e is read even when it is ignored), and every output row
  // C16 stores, after the loads of the row DL steps ahead.  Vector memory operations
  // complete in issue order, so when row t enters, the operations issued after its loads
  // (the loads of the next DL - 1 rows, and the stores of the last DL - 1 iterations once
  // output has begun) may still be outstanding: waiting until no more than that many are
  // guarantees row t landed.  Fewer than counted (before output begins) would be unsafe, so
  // the count with stores applies only from the step whose DL - 1 predecessors all stored;
  // extra stores (the coarse-tile sums) only make a wait longer.
  constexpr int DL = S::DL, C16 = S::C16;
  constexpr int NWAIT = 2 * C16 * (DL - 1), NWAIT_OUT = 3 * C16 * (DL - 1);
  const int st_out = 2 * H + (down ? 1 : 0) + DL - 1;  // steps from which NWAIT_OUT holds
  const unsigned ring0 = lds_offset(sR);
  int qs = 0;  // LDS slot of the next row to enter
  auto fetch = [&](int t, int slot) {
    const long long a = (long long)jn * g.nx + cw;
    const unsigned base = ring0 + unsigned(slot) * S::SLOT;
#pragma unroll
    for (int c = 0; c < C16; ++c) {
      dma16(eb + a + c * (16 / int(sizeof(T))), base + c * 1024);
      dma16(rb + a + c * (16 / int(sizeof(T))), base + (C16 + c) * 1024);
    }
    if (g.per_y) jn = down ? (jn == 0 ? g.ny - 1 : jn - 1) : (jn + 1 == g.ny ? 0 : jn + 1);
    else jn = min(max(t + dir, 0), g.ny - 1);
  };
#pragma unroll
  for (int q = 0; q < DL; ++q) fetch(t0 + dir * q, q);
  double acc = 0.0, acc2 = 0.0;

  for (int sb = 0; sb < nrows; sb += P) {
#pragma unroll
    for (int ph = 0; ph < P; ++ph) {
      const int st = sb + ph;
      if (st < nrows) {
        const int t = t0 + dir * st;
        // t0 is odd (ys = y0 - H and yend = y0 + L + H, y0 and L even, H odd) and P even, so
        // the parity of t is fixed per slot
        const int tpar = (1 + ph) & 1;
        // EDGE: the lane's first column, opaque so that the per-cell wall arithmetic below is
        // redone each row rather than held in registers for the walk
        int cx = cu;
        if (EDGE) asm volatile("" : "+v"(cx));

        // row t enters: e = (zero_e ? 0 : e) + P E; cells behind a wall hold 0
        {
          // the row's lower coarse row and y weight (Eq. 5)
          int jrow;
          double Yd;
          row_interp(t, jrow, Yd);
          if (jrow != jc) {  // next pair of coarse rows
            jc = jrow;
            put_x(down ? jc : jc + 1);
          }
          T xlo[CPL], xhi[CPL];
          {
            const V16* a = sX + (jc & 1) * C16X * kWave + lane;
            const V16* b = sX + ((jc + 1) & 1) * C16X * kWave + lane;
#pragma unroll
            for (int q = 0; q < C16X; ++q) {
              const V16 u = a[q * kWave], w = b[q * kWave];
#pragma unroll
              for (int k = 0; k < K16; ++k) {
                xlo[q * K16 + k] = (&u.x)[k];
                xhi[q * K16 + k] = (&w.x)[k];
              }
            }
          }
          // the y step of Eq. 5 in T (weights from FP64, dyadic and exact unless the row lies
          // next to a short last tile, which only the table walks read; exact in T otherwise,
          // so 1 - Y is too)
          T Y, Y1;
          if constexpr (!TAB) {
            Y = T(Yd);
            Y1 = T(1) - Y;
          } else {
            Y = T(Yd);
            Y1 = T(1.0 - Yd);
          }
          {
            Vec4u v[2 * C16];
            const unsigned la = ring0 + unsigned(qs) * S::SLOT + 16u * unsigned(lane);
            if (st >= st_out) lds_take<NWAIT_OUT>(la, v);
            else lds_take<NWAIT>(la, v);
            T le[CPL];
            unpack_cells<T, CPL>(v, 0, le);
            unpack_cells<T, CPL>(v, C16, r[ph]);
#pragma unroll
            for (int p = 0; p < CPL; ++p) {
              const T e0 = zero_e ? T(0) : le[p];
              e[ph][p] = e0 + (xlo[p] * Y1 + xhi[p] * Y);
              if (PLAIN) r[ph][p] = r[ph][p] * T(0.25);
            }
          }
          const bool row_in = PLAIN || g.per_y || (t >= 0 && t < g.ny);
          if (!row_in) {
#pragma unroll
            for (int p = 0; p < CPL; ++p) e[ph][p] = r[ph][p] = T(0);
          }
          if (EDGE && !col_in) {
#pragma unroll
            for (int p = 0; p < CPL; ++p) e[ph][p] = r[ph][p] = T(0);
          }
          const bool first = !PLAIN && !g.per_y && t == 0, last = !PLAIN && !g.per_y && t == g.ny - 1;
          if (!PLAIN) invs[ph] = uniform(!row_in ? T(0) : (first ? icS : (last ? icN : T(0.25))));
          if (EDGE) {  // the wall cells of the row
            iws[ph] = uniform(!row_in ? T(0) : (first ? iwS : (last ? iwN : iwM)));
            ies[ph] = uniform(!row_in ? T(0) : (first ? ieS : (last ? ieN : ieM)));
          }
        }

        // half-step k (odd red, even black) on the row that entered k steps ago
#pragma unroll
        for (int k = 1; k <= 2 * NU; ++k) {
          const int sc = (ph - k + P) % P, sb = (ph - k - 1 + P) % P, sa = (ph - k + 1 + P) % P;
          const int colour = (k - 1) & 1;          // 0 red, 1 black
          const int p0 = (colour + tpar + k) & 1;  // the lane's cells p with (p + row) & 1 == colour
#pragma unroll
          for (int p = 0; p < CPL; ++p) {
            if ((p & 1) != p0) continue;
            const T w = p > 0 ? e[sc][p - 1] : lane_shift<kDppFromLeft>(e[sc][CPL - 1]);
            const T ea = p < CPL - 1 ? e[sc][p + 1] : lane_shift<kDppFromRight>(e[sc][0]);
            const T sum = (w + ea) + (e[sb][p] + e[sa][p]);
            if (PLAIN) {
              e[sc][p] = fma(sum, T(0.25), -r[sc][p]);
              continue;
            }
            T inv = invs[sc];
            if (EDGE) {
              // 1 / diagonal: the row's interior value, the row's wall-cell value at the wall
              // column, or 0 behind a wall (the cell then stays 0)
              const int i = cx + p;
              inv = i == 0 ? iws[sc] : inv;
              inv = i == g.nx - 1 ? ies[sc] : inv;
              inv = unsigned(i) < unsigned(g.nx) ? inv : T(0);
            }
            e[sc][p] = (sum - r[sc][p]) * inv;
          }
        }

        // row o, entered H steps ago, is final: residual, write-back, coarse-tile sums
        const int o = t - dir * H;
        if (st >= H && o >= y0 && o < yend - H) {
          const int so = (ph - H + P) % P, sb = (ph - H - 1 + P) % P, sa = (ph - H + 1 + P) % P;
          const bool hs = PLAIN || g.per_y || o > 0, hn = PLAIN || g.per_y || o < g.ny - 1;
          const bool ds = !hs && (g.dmask & kDirS), dn = !hn && (g.dmask & kDirN);
          // the rows in slots sb (entered one step before row o) and sa (one step after) are
          // its south and north neighbours walking up, north and south walking down
          const bool hb = down ? hn : hs, ha = down ? hs : hn, db = down ? dn : ds, da = down ? ds : dn;
          double d[CPL];
#pragma unroll
          for (int p = 0; p < CPL; ++p) {
            const T c = e[so][p];
            const T w = p > 0 ? e[so][p - 1] : lane_shift<kDppFromLeft>(e[so][CPL - 1]);
            const T ea = p < CPL - 1 ? e[so][p + 1] : lane_shift<kDppFromRight>(e[so][0]);
            if (PLAIN) {
              const T lap = ((w - c) + (ea - c)) + ((e[sb][p] - c) + (e[sa][p] - c));
              d[p] = double(fma(r[so][p], T(4), -lap));
            } else {
              const bool hw = !EDGE || cx + p > 0, he = !EDGE || cx + p < g.nx - 1;
              const bool dw = EDGE && cx + p == 0 && (g.dmask & kDirW);
              const bool de = EDGE && cx + p == g.nx - 1 && (g.dmask & kDirE);
              d[p] = double(r[so][p] - lap5<T>(c, w, ea, e[sb][p], e[sa][p], hw, he, hb, ha, dw,
                                               de, db, da));
            }
            acc += d[p];
          }
          if (psq) {  // only when a convergence check reads them: squared sums, or maxima of |d|
            // (the maxima only in the one-sweep kernel, the one-shot cycling's fine stage)
            if (NU == 1 && maxmode) {
#pragma unroll
              for (int p = 0; p < CPL; ++p) acc2 = fmax(acc2, fabs(d[p]));
            } else {
#pragma unroll
              for (int p = 0; p < CPL; ++p) acc2 += d[p] * d[p];
            }
          }
          if (lane_out) store_cells(ob + (long long)o * g.nx + cu, e[so]);
          // a tile's last row in walk order (walking up, the last row of the grid also ends a
          // short last tile, which only the table walks reach)
          if (((o - y0) & (N - 1)) == (down ? 0 : N - 1) || (TAB && !down && o == g.ny - 1)) {
            // with full tiles a lane group lies wholly inside or wholly outside the grid
            double a = !TAB || lane_sum ? acc : 0.0, q = !TAB || lane_sum ? acc2 : 0.0;
#pragma unroll
            for (int k = 1; k < G; k <<= 1) a += __shfl_down(a, k, kWave);
            if (psq) {
              if (NU == 1 && maxmode) {
#pragma unroll
                for (int k = 1; k < G; k <<= 1) q = fmax(q, __shfl_down(q, k, kWave));
              } else {
#pragma unroll
                for (int k = 1; k < G; k <<= 1) q += __shfl_down(q, k, kWave);
              }
            }
            if (lane_out && ((lane - PX / CPL) & (G - 1)) == 0) {
              const long long oc = coff + (long long)(o >> LOG2N) * g.ncx + (cu >> LOG2N);
              rc[oc] = a;
              if (psq) psq[oc] = q;
            }
            acc = acc2 = 0.0;
          }
        }

        // the row DL steps ahead into the LDS slot row t just left
        fetch(t + dir * DL, qs);
        qs = qs + 1 == DL ? 0 : qs + 1;
      }
    }
  }
  // the loads of rows past the end are still in flight into LDS: wait for them
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// One launch covers every strip.  Units (a strip and a chunk of rows) are numbered
// strip-fastest.  A strip's nb bands of n rows are split into C chunks of floor or ceil(nb / C)
// bands (chunk c starts at band c nb / C).  The first nblk_e workgroups take the strips that
// touch a wall (strip 0 and strips efirst + 1, efirst + 2, ...) in Ce chunks; the others take
// strips first, first + 1, ... in Ci chunks, dealt out so that each XCD (the hardware deals
// workgroups out round-robin over the 8 XCDs) runs one contiguous band of units.
template <typename T, int NU, int LOG2N>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Stream<T, NU, LOG2N>::WAVES)))
void k_cycle(Geo g, const T* __restrict__ rhs, const T* __restrict__ ein, T* __restrict__ eout,
             const double* __restrict__ E, double* __restrict__ rc, double* __restrict__ psq,
             int zero_e, int nb, int Ci, int nstrip, int first, int Ce, int nstrip_e, int efirst,
             int nblk_e, const double* __restrict__ stop, int maxmode) {
  // a launch enqueued past the iteration a device-side check stopped at does nothing
  if (stop && *stop != 0.0) return;
  using S = Stream<T, NU, LOG2N>;
  constexpr int WPB = kBlock / kWave;
  __shared__ double sE[WPB][S::NR * S::NC];
  __shared__ typename Vec16<T>::type sX[WPB][2 * S::C16 * kWave];
  __shared__ Vec4u sR[WPB][S::DL * S::SLOT / 16];
  static_assert(sizeof(sE) + sizeof(sX) + sizeof(sR) == S::LDS_BYTES, "LDS budget");
  const long long off = (long long)blockIdx.z * g.plane;
  const long long coff = (long long)blockIdx.z * g.cplane;
  const double2* tabx = reinterpret_cast<const double2*>(g.itab);
  const double2* taby = tabx + g.nx;
  // the wave index, made visibly wave-uniform so that everything derived from it (strip,
  // rows, the walk's row bookkeeping) lives in scalar registers and scalar branches
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
  const int b = blockIdx.x;
  if (b < nblk_e) {
    const int u = b * WPB + w;
    if (u >= nstrip_e * Ce) return;
    const int chunk = u / nstrip_e, sl = u - chunk * nstrip_e;
    const int strip = sl == 0 ? 0 : efirst + sl;
    const int b0 = chunk * nb / Ce, b1 = (chunk + 1) * nb / Ce;
    if ((g.nx | g.ny) & (S::N - 1))
      cycle_walk<T, NU, LOG2N, kEdgeTab>(g, rhs + off, ein + off, eout + off, E + coff, rc, psq,
                                         sE[w], sX[w], sR[w], coff, zero_e, strip * S::VW - S::PX,
                                         b0 * S::N, (b1 - b0) * S::N, chunk & 1, tabx, taby,
                                         maxmode);
    else
      cycle_walk<T, NU, LOG2N, kEdge>(g, rhs + off, ein + off, eout + off, E + coff, rc, psq,
                                      sE[w], sX[w], sR[w], coff, zero_e, strip * S::VW - S::PX,
                                      b0 * S::N, (b1 - b0) * S::N, chunk & 1, tabx, taby, maxmode);
    return;
  }
  int bi = b - nblk_e;
  const int nbi = gridDim.x - nblk_e;
  if ((nbi & 7) == 0) bi = (bi & 7) * (nbi >> 3) + (bi >> 3);
  const int u = bi * WPB + w;
  if (u >= nstrip * Ci) return;
  const int chunk = u / nstrip, sl = u - chunk * nstrip;
  const int b0 = chunk * nb / Ci, b1 = (chunk + 1) * nb / Ci;
  const int y0 = b0 * S::N, len = (b1 - b0) * S::N, xs = (first + sl) * S::VW - S::PX;
  const bool down = chunk & 1;  // odd chunks walk down
  // A chunk walks the plain way when every row and column it reads lies inside the grid (or
  // wraps) in full-size interpolation rectangles: below the centre of the last full tile
  // when n does not divide the axis, where the rectangles next to the short tile begin.
  const int ylo = y0 - S::H, yhi = y0 + len + S::H + (down ? 1 : 0);  // rows [ylo, yhi)
  const bool pad_y = g.ny & (S::N - 1), pad_x = g.nx & (S::N - 1);
  const int yfull = (g.ncy - 2) * S::N + S::N / 2, xfull = (g.ncx - 2) * S::N + S::N / 2;
  const bool rows_ok = pad_y ? (ylo >= 0 && yhi <= yfull) : (g.per_y || (ylo >= 0 && yhi <= g.ny));
  const bool cols_ok = !pad_x || (xs >= 0 && xs + S::LW <= xfull);
  if (rows_ok && cols_ok)
    cycle_walk<T, NU, LOG2N, kPlain>(g, rhs + off, ein + off, eout + off, E + coff, rc, psq,
                                     sE[w], sX[w], sR[w], coff, zero_e, xs, y0, len, down, tabx,
                                     taby, maxmode);
  else if (pad_x || pad_y)
    cycle_walk<T, NU, LOG2N, kRowsTab>(g, rhs + off, ein + off, eout + off, E + coff, rc, psq,
                                       sE[w], sX[w], sR[w], coff, zero_e, xs, y0, len, down, tabx,
                                       taby, maxmode);
  else
    cycle_walk<T, NU, LOG2N, kRows>(g, rhs + off, ein + off, eout + off, E + coff, rc, psq,
                                    sE[w], sX[w], sR[w], coff, zero_e, xs, y0, len, down, tabx,
                                    taby, maxmode);
}

template <typename T, int NU, int LOG2N>
hipError_t cycle_dispatch3(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                           double* rc, double* psq, int zero_e, hipStream_t s, const double* stop,
                           int maxmode) {
  using S = Stream<T, NU, LOG2N>;
  constexpr int WPB = kBlock / kWave;
  auto kernel = k_cycle<T, NU, LOG2N>;
  const int ns = (g.nx + S::VW - 1) / S::VW;
  // strips whose columns all exist: every strip of a periodic axis, else strips 1 .. kmax
  // with (k + 1) VW + PX <= nx; the others (strip 0 and those after kmax) touch a wall
  int first = 0, ni = ns, ne = 0, efirst = 0;
  if (!g.per_x) {
    const int kmax = g.nx >= S::PX ? (g.nx - S::PX) / S::VW - 1 : -1;
    first = 1;
    ni = kmax > 0 ? kmax : 0;
    efirst = ni;
    ne = ns - ni;
  }
  // Chunks of whole bands, all of one length where the band count allows it, between 32
  // rows (one band when bands are longer) and S::L rows; wall strips, whose rows cost more,
  // walk chunks half as long.  Among those lengths the launch takes the one whose number of
  // units (waves) is closest to kUnits, about 1.6 rounds of the chip's wave slots at three
  // waves per SIMD: enough waves that the hardware keeps every SIMD busy to the end, at the
  // price of more re-read halo rows.  Measured on 8192^2 (nu = 5, 32h): 2 bands per chunk
  // (4992 units) 194 us per launch, 4 bands (2496) 216 us, 1 band (9984) 204 us; chunk sets
  // mixing two lengths were slower than either (the longer chunks set the launch time).
  constexpr double kUnits = 4864.0;
  const int nb = (g.ny + S::N - 1) / S::N;  // bands of n rows, the last one short if n does not divide ny
  const int bmin = std::max(1, 32 / S::N), bmax = std::max(1, S::L / S::N);
  auto units = [&](int ci) { return double(ni * ci + ne * std::min(2 * ci, nb)) * g.batch; };
  int Ci = 0;
  double best = 0.0;
  for (int bands = bmin; bands <= bmax; ++bands) {
    if (nb % bands) continue;
    const double u = std::max(1.0, units(nb / bands));
    const double cost = std::fabs(std::log(u / kUnits));
    if (Ci == 0 || cost < best) {
      best = cost;
      Ci = nb / bands;
    }
  }
  if (Ci == 0) {  // no chunk length of whole bands divides the strip: floor or ceil lengths
    const int cmax = std::max(1, nb / bmin);
    const int per = std::max(1, (ni + 2 * ne) * g.batch);
    Ci = std::max((nb + bmax - 1) / bmax, std::min(cmax, int(kUnits / per)));
  }
  const int Ce = std::min(2 * Ci, nb);
  // wall blocks padded to a multiple of 8 so that the XCD of a block (its index mod 8) is
  // known to the band mapping of the others
  const int nblk_e = ne > 0 ? ((ne * Ce + WPB - 1) / WPB + 7) / 8 * 8 : 0;
  const int nblk_i = (ni * Ci + WPB - 1) / WPB;
  if (nblk_e + nblk_i == 0) return hipSuccess;
  hipLaunchKernelGGL(kernel, dim3(nblk_e + nblk_i, 1, g.batch), dim3(kBlock), 0, s, g, rhs, ein,
                     eout, E, rc, psq, zero_e, nb, Ci, ni, first, Ce, ne, efirst, nblk_e, stop,
                     maxmode);
  return hipGetLastError();
}

template <typename T, int NU>
hipError_t cycle_dispatch2(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                           double* rc, double* psq, int zero_e, hipStream_t s, const double* stop,
                           int maxmode) {
  switch (g.log2n) {
    case 2: return cycle_dispatch3<T, NU, 2>(g, rhs, ein, eout, E, rc, psq, zero_e, s, stop, maxmode);
    case 3: return cycle_dispatch3<T, NU, 3>(g, rhs, ein, eout, E, rc, psq, zero_e, s, stop, maxmode);
    case 4: return cycle_dispatch3<T, NU, 4>(g, rhs, ein, eout, E, rc, psq, zero_e, s, stop, maxmode);
    case 5: return cycle_dispatch3<T, NU, 5>(g, rhs, ein, eout, E, rc, psq, zero_e, s, stop, maxmode);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Every sweep count 1 .. MAXNU of the fused kernel for fine type T.
template <typename T, int MAXNU>
hipError_t launch_cycle_upto(const Geo& g, const T* rhs, const T* ein, T* eout, const double* E,
                             double* rc, double* psq, int nu, int zero_e, hipStream_t s,
                             const double* stop, int maxmode) {
  if constexpr (MAXNU == 0) {
    return hipErrorInvalidValue;
  } else {
    if (nu == MAXNU)
      return cycle_dispatch2<T, MAXNU>(g, rhs, ein, eout, E, rc, psq, zero_e, s, stop, maxmode);
    return launch_cycle_upto<T, MAXNU - 1>(g, rhs, ein, eout, E, rc, psq, nu, zero_e, s, stop,
                                           maxmode);
  }
}

}  // namespace ism
