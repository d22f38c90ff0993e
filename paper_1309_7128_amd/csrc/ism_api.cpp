// Host side of the ISM library: the C ABI of include/ism.h, argument validation, the
// device workspace, the coarse tables and the outer/inner iteration that strings the
// kernels together.  Every device operation is enqueued on the handle's stream; the host
// waits only for the few FP64 scalars that decide convergence.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ism.h"
#include "ism_internal.h"

using ism::Geo;
using ism::Partials;

namespace {

// Slots of the per-grid device scalars; the array is slot-major, [kSlots][batch].
// STOP and STOP_AT (entry 0 of each) hold the state of a device-checked loop: 0 running, 1
// converged, 2 a non-finite value met, and the iteration it stopped at.
enum Slot { MEAN_B = 0, RSQ, RMAX, BSQ, BMAX, ISQ, MEAN_X, CMAX, MEAN_R, STOP, STOP_AT, kSlots };

// Adaptive convergence checks in flight at once (pinned read-back slots) and the number of
// cycles the host enqueues past a check before it waits for that check's result.
constexpr int kChecks = 8, kLag = 2;

// Iterations a device-checked loop (the one-shot stages) enqueues between two read-backs: 4,
// doubling to 64, so that a loop of I iterations reads back about log2(I) + I / 64 times and
// enqueues at most 63 iterations past its stop, each of which exits at once.
constexpr int kBatchFirst = 4, kBatchMax = 64;

thread_local std::string g_create_error;

// An inner solve's residual target never goes below margin * rtol * ||b'||.  In FP64 the inner
// residual r - A'e is the outer residual up to rounding, so the margin is 1; the FP32 inner
// residual only estimates it, so the mixed form aims at half the tolerance.
constexpr double kInnerMarginFP64 = 1.0;
constexpr double kInnerMarginMixed = 0.5;

}  // namespace

struct ism_ctx {
  ism_config cfg{};
  hipStream_t stream = nullptr;
  Geo g{};
  double h = 0.0, h2 = 0.0;
  bool singular = true;  // no Dirichlet face: the constants span the null space of A
  size_t tsize = 8;  // bytes per element of the inner fine arrays
  // device memory (one allocation)
  char* block = nullptr;
  size_t bytes = 0;
  void* rT = nullptr;   // inner right-hand side, type T
  void* eA = nullptr;   // inner correction, ping
  void* eB = nullptr;   // inner correction, pong
  double *rc = nullptr, *E = nullptr, *t1 = nullptr, *t2 = nullptr;
  double *p_sq = nullptr, *p_max = nullptr, *p_bsq = nullptr, *p_bmax = nullptr, *p_sum = nullptr;
  double* scal = nullptr;  // [kSlots][batch]
  double* fin = nullptr;   // chunk results of the two-stage reductions
  double *Vx = nullptr, *Vy = nullptr, *invLam = nullptr;
  // forward tables of the coarse solve: Vx, Vy themselves with full tiles, the pencil's left
  // vectors when a tile size does not divide the axis (padded)
  double *Fx = nullptr, *Fy = nullptr;
  bool padded = false;
  double* coef = nullptr;  // coarse 9-point stencil [ncy][ncx][9] (block Gauss-Seidel)
  void* stage_tmp = nullptr;  // lazily allocated FP64-sized fine scratch for stage calls
  double* h_scal = nullptr;   // host mirror of scal, then kChecks slots of B check norms
  double* h_chk = nullptr;    // = h_scal + kSlots * batch
  // Pinned h_scal (a handle from ism_create): check norms go straight to h_chk behind an
  // event.  Otherwise (pageable host memory, no events) they are parked in d_chk on the
  // device and read back synchronously when the check is acted on.
  bool pinned = true;
  double* d_chk = nullptr;    // device check slots [kChecks][batch]
  double* d_hchk = nullptr;   // device address of the pinned h_chk (hipHostGetDevicePointer)
  std::vector<double> h_mem;  // pageable h_scal when not pinned
  std::vector<hipEvent_t> chk_ev;  // one per check slot (created on first use)
  // ACM hierarchy (coarse_stencil == ISM_COARSE_ACM): per level l = 1..L-1 the agglomerated
  // right-hand side and two correction buffers, plus level-0 squared-residual partials
  void* acm_mem = nullptr;
  std::vector<double*> acm_r, acm_ea, acm_eb;
  double* acm_psq = nullptr;
  std::string err;
  int64_t launches = 0, syncs = 0;
  // kernel timing (ism_profile): event pairs recorded around launches, resolved at syncs
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  bool prof = false;
  int prof_every = 1;                             // time every prof_every-th launch of a class
  int64_t prof_seen[ISM_KERNEL_CLASSES] = {};     // launches of each class since the reset
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<Pending> pending;
  double prof_ms[ISM_KERNEL_CLASSES] = {};
  int64_t prof_n[ISM_KERNEL_CLASSES] = {};
};

namespace {

int set_err(ism_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_err((ctx), ISM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH(ctx, expr)   \
  do {                      \
    (ctx)->launches++;      \
    HIPCHK(ctx, (expr));    \
  } while (0)

// ---- kernel timing
hipEvent_t prof_event(ism_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

hipEvent_t prof_start(ism_ctx* c, int kind) {
  if (!c->prof) return nullptr;
  if (c->prof_seen[kind]++ % c->prof_every != 0) return nullptr;  // not sampled
  hipEvent_t a = prof_event(c);
  if (a) (void)hipEventRecord(a, c->stream);
  return a;
}

void prof_stop(ism_ctx* c, int kind, hipEvent_t a) {
  if (!c->prof || !a) return;
  hipEvent_t b = prof_event(c);
  if (!b) return;
  (void)hipEventRecord(b, c->stream);
  c->pending.push_back({kind, a, b});
}

// Resolve the recorded pairs; only called after the stream has been synchronized.
void prof_collect(ism_ctx* c) {
  for (const auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_ms[p.kind] += ms;
      c->prof_n[p.kind]++;
    }
  }
  c->pending.clear();
  c->ev_used = 0;
}

bool is_pow2_coarsen(int n) { return n == 4 || n == 8 || n == 16 || n == 32; }

int validate(const ism_config* cfg, std::string& why) {
  if (!cfg) return why = "config is NULL", ISM_ERR_INVALID;
  if (cfg->nx <= 0 || cfg->ny <= 0 || cfg->batch <= 0)
    return why = "nx, ny and batch must be positive", ISM_ERR_INVALID;
  auto bc_ok = [](int bc) { return bc >= ISM_BC_NEUMANN && bc <= ISM_BC_DIRICHLET_NEUMANN; };
  if (!bc_ok(cfg->bc_x) || !bc_ok(cfg->bc_y))
    return why = "bc_x/bc_y must be one of the ISM_BC_* values", ISM_ERR_INVALID;
  if (cfg->precision != ISM_PREC_FP64 && cfg->precision != ISM_PREC_MIXED)
    return why = "precision must be ISM_PREC_FP64 or ISM_PREC_MIXED", ISM_ERR_INVALID;
  if (!(cfg->lx > 0.0) || !(cfg->ly > 0.0) || !std::isfinite(cfg->lx) || !std::isfinite(cfg->ly))
    return why = "lx and ly must be positive and finite", ISM_ERR_INVALID;
  if (cfg->nu < 1) return why = "nu must be >= 1", ISM_ERR_INVALID;
  if (!(cfg->rtol > 0.0)) return why = "rtol must be positive", ISM_ERR_INVALID;
  if (!(cfg->inner_rtol > 0.0) || !(cfg->inner_rtol < 1.0))
    return why = "inner_rtol must lie in (0, 1)", ISM_ERR_INVALID;
  if (cfg->max_cycles < 1 || cfg->max_outer < 1 || cfg->check_every < 0)
    return why = "max_cycles and max_outer must be >= 1, check_every >= 0", ISM_ERR_INVALID;
  if (cfg->fused < ISM_FUSED_OFF || cfg->fused > ISM_FUSED_TILE)
    return why = "fused must be one of the ISM_FUSED_* values", ISM_ERR_INVALID;
  if (cfg->coarse_stencil != ISM_COARSE_ISM && cfg->coarse_stencil != ISM_COARSE_GMG5 &&
      cfg->coarse_stencil != ISM_COARSE_ACM)
    return why = "coarse_stencil must be ISM_COARSE_ISM, ISM_COARSE_GMG5 or ISM_COARSE_ACM", ISM_ERR_INVALID;
  if (cfg->coarse_stencil == ISM_COARSE_ACM && cfg->precision != ISM_PREC_FP64)
    return why = "the ACM scheme runs in FP64 only", ISM_ERR_UNSUPPORTED;
  if (cfg->cycling != ISM_CYCLE_REPEAT && cfg->cycling != ISM_CYCLE_ONESHOT)
    return why = "cycling must be ISM_CYCLE_REPEAT or ISM_CYCLE_ONESHOT", ISM_ERR_INVALID;
  if (cfg->cycling == ISM_CYCLE_ONESHOT) {
    if (!(cfg->coarse_tol > 0.0) || !(cfg->fine_tol > 0.0) || !std::isfinite(cfg->coarse_tol) ||
        !std::isfinite(cfg->fine_tol))
      return why = "coarse_tol and fine_tol must be positive and finite", ISM_ERR_INVALID;
    if (cfg->coarse_stencil == ISM_COARSE_ACM)
      return why = "one-shot cycling takes the ISM or GMG5 stencil", ISM_ERR_UNSUPPORTED;
  }
  if (cfg->coarse_gs != ISM_COARSE_GS_BLOCK && cfg->coarse_gs != ISM_COARSE_GS_MULTICOLOUR)
    return why = "coarse_gs must be ISM_COARSE_GS_BLOCK or ISM_COARSE_GS_MULTICOLOUR", ISM_ERR_INVALID;
  if (cfg->stall_window < 1 || !(cfg->stall_drop >= 0.0) || !(cfg->stall_drop < 1.0))
    return why = "stall_window must be >= 1 and stall_drop in [0, 1)", ISM_ERR_INVALID;
  if (!is_pow2_coarsen(cfg->coarsen))
    return why = "coarsen must be 4, 8, 16 or 32", ISM_ERR_UNSUPPORTED;
  if (cfg->nx % cfg->coarsen || cfg->ny % cfg->coarsen) {
    // a short last tile (the padded domain of Sec. 4.1) is defined for the ISM stencil
    if (cfg->coarse_stencil != ISM_COARSE_ISM)
      return why = "nx or ny not a multiple of coarsen (padding) needs the ISM coarse stencil", ISM_ERR_UNSUPPORTED;
    if (cfg->nx % 4 || cfg->ny % 2)
      return why = "nx or ny not a multiple of coarsen (padding) needs nx a multiple of 4 and ny even", ISM_ERR_UNSUPPORTED;
  }
  if (cfg->nx < 2 || cfg->ny < 2) return why = "the grid needs at least 2 cells per axis", ISM_ERR_UNSUPPORTED;
  const double hx = cfg->lx / cfg->nx, hy = cfg->ly / cfg->ny;
  if (std::fabs(hx - hy) > 1e-12 * hx) return why = "cells must be square (lx/nx == ly/ny)", ISM_ERR_UNSUPPORTED;
  if (cfg->fused && cfg->coarse_stencil != ISM_COARSE_ACM) {
    const int maxnu = cfg->precision == ISM_PREC_FP64 ? ism::fused_max_nu<double>()
                                                        : ism::fused_max_nu<float>();
    if (cfg->nu > maxnu)
      return why = "the fused cycle kernel supports nu <= " + std::to_string(maxnu) +
                   " in this precision; use fused = 0", ISM_ERR_UNSUPPORTED;
  }
  if (double(cfg->nx) * cfg->ny >= 2147483648.0)
    return why = "one grid must have fewer than 2^31 cells", ISM_ERR_UNSUPPORTED;
  return ISM_OK;
}

template <typename T>
constexpr int dtype_of() {
  return sizeof(T) == 4 ? ISM_F32 : ISM_F64;
}

// ------------------------------------------------------------------ coarse solve (FP64)
// E = V_y ((F_y^T R_c F_x) .* Lambda^-1) V_x^T with the (0,0) entry of Lambda^-1 zero when
// A_c is singular.  With full tiles F = V (orthonormal): the zero-mean solution of
// K_x (x) M_y + M_x (x) K_y applied to E equal to R_c minus its mean.  With a short last
// tile F holds the left vectors of each padded axis's pencil; dropping the constant mode
// then gives the solution whose prolongation P E has zero mean, for R_c minus a multiple
// of the tile-size weights (equal to R_c when R_c sums to zero).
int coarse_solve(ism_ctx* c, const double* rc, double* E) {
  const Geo& g = c->g;
  const int nx = g.ncx, ny = g.ncy, B = g.batch;
  const long long cp = g.cplane;
  hipStream_t s = c->stream;
  if (ism::coarse_small_fits(g)) {
    LAUNCH(c, ism::launch_coarse_small(g, rc, c->Fx, c->Fy, c->Vx, c->Vy, c->invLam, E, s));
    return ISM_OK;
  }
  LAUNCH(c, ism::launch_gemm(ny, nx, nx, 0, rc, cp, nx, 0, c->Fx, 0, nx, c->t1, cp, nx, nullptr, B, s));
  LAUNCH(c, ism::launch_gemm(ny, nx, ny, 1, c->Fy, 0, ny, 0, c->t1, cp, nx, c->t2, cp, nx, c->invLam, B, s));
  LAUNCH(c, ism::launch_gemm(ny, nx, ny, 0, c->Vy, 0, ny, 0, c->t2, cp, nx, c->t1, cp, nx, nullptr, B, s));
  LAUNCH(c, ism::launch_gemm(ny, nx, nx, 0, c->t1, cp, nx, 1, c->Vx, 0, nx, E, cp, nx, nullptr, B, s));
  return ISM_OK;
}

// Which fused kernel a cycle takes (ISM_FUSED_AUTO): the LDS-tiled one up to kTileCells cells
// per launch, where the row walk has too few waves to hide its per-row latency, else the
// walk.  Measured on MI355X (whole solves per cycle, tiled against walked; FP64 nu = 4, FP32
// nu = 5): 256^2 at 16h 17 against 56 us (FP64), 20 against 46 (FP32); 1024^2 at 16h 56
// against 71 (FP64), 64 against 61 (FP32); 1280^2 at 16h 84 against 74 (FP64), 96 against
// 63 (FP32); 2048^2 171 against 78 (FP64).
constexpr double kTileCells = 1024.0 * 1024.0;

bool tile_cycle(const ism_ctx* c) {
  if (c->cfg.fused == ISM_FUSED_TILE) return true;
  if (c->cfg.fused == ISM_FUSED_WALK) return false;
  return double(c->g.plane) * c->g.batch <= kTileCells;
}

template <typename T>
hipError_t launch_fused(ism_ctx* c, const T* rhs, const T* ein, T* eout, const double* E,
                        double* rc, double* psq, int nu, int zero_e, const double* stop = nullptr,
                        int maxmode = 0) {
  if (tile_cycle(c))
    return ism::launch_cycle_tile<T>(c->g, rhs, ein, eout, E, rc, psq, nu, zero_e, c->stream, stop,
                                     maxmode);
  return ism::launch_cycle_fused<T>(c->g, rhs, ein, eout, E, rc, psq, nu, zero_e, c->stream, stop,
                                    maxmode);
}

int read_scalars(ism_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->h_scal, c->scal, sizeof(double) * kSlots * c->g.batch,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->syncs++;
  prof_collect(c);
  return ISM_OK;
}

int finalize(ism_ctx* c, const double* part, ism::Reduce op, double scale, int slot) {
  LAUNCH(c, ism::launch_finalize(part, int(c->g.cplane), c->g.cplane, c->g.batch, op, scale,
                                 c->scal + size_t(slot) * c->g.batch, 1, 0, c->fin, c->stream));
  return ISM_OK;
}

void* scratch_fine(ism_ctx* c) {
  if (!c->stage_tmp) {
    if (hipMalloc(&c->stage_tmp, size_t(c->g.plane) * c->g.batch * sizeof(double)) != hipSuccess)
      c->stage_tmp = nullptr;
  }
  return c->stage_tmp;
}

// One two-level cycle on A' e = rhs.  Reads e from *cur (ignored if zero_e), leaves the new
// correction in *cur (swapping with *spare), overwrites rc with R(rhs - A'e) and psq with the
// per-tile squared-residual sums.
template <typename T>
int run_cycle(ism_ctx* c, const T* rhs, T** cur, T** spare, double* rc, double* psq, int zero_e) {
  const Geo& g = c->g;
  hipStream_t s = c->stream;
  hipEvent_t ev = prof_start(c, ISM_KERNEL_COARSE);
  int rcode = coarse_solve(c, rc, c->E);
  if (rcode) return rcode;
  prof_stop(c, ISM_KERNEL_COARSE, ev);
  if (c->cfg.fused) {
    ev = prof_start(c, ISM_KERNEL_CYCLE);
    LAUNCH(c, launch_fused<T>(c, rhs, *cur, *spare, c->E, rc, psq, c->cfg.nu, zero_e));
    prof_stop(c, ISM_KERNEL_CYCLE, ev);
    std::swap(*cur, *spare);
    return ISM_OK;
  }
  ev = prof_start(c, ISM_KERNEL_PROLONG);
  LAUNCH(c, ism::launch_prolong<T>(g, c->E, *cur, zero_e, s));
  prof_stop(c, ISM_KERNEL_PROLONG, ev);
  for (int k = 0; k < c->cfg.nu; ++k) {
    ev = prof_start(c, ISM_KERNEL_SMOOTH);
    LAUNCH(c, ism::launch_rbgs<T>(g, rhs, *cur, *spare, s));
    prof_stop(c, ISM_KERNEL_SMOOTH, ev);
    std::swap(*cur, *spare);
  }
  ev = prof_start(c, ISM_KERNEL_RESTRICT);
  LAUNCH(c, ism::launch_restrict<T>(g, rhs, *cur, rc, psq, s));
  prof_stop(c, ISM_KERNEL_RESTRICT, ev);
  return ISM_OK;
}

// The most cycles between two convergence checks of a mixed inner solve, so that FP32
// stagnation is seen within about 1 ms of device work.  A deterministic function of the
// grid (a cycle is modelled as a 40 us launch floor plus 3.2 ps per cell, close to the
// fused kernel and coarse solve on MI355X), so that the cycles at which a solve checks and
// stops do not depend on host timing.
int mixed_check_cap(const Geo& g) {
  const double cells = double(g.plane) * g.batch;
  return std::max(4, int(1.0e-3 / (40e-6 + 3.2e-12 * cells)));
}

struct Check {
  int cycle;
  std::vector<double> res;
};

// Convergence bookkeeping of one inner solve: evaluates a check (the grid residual norms in
// the ISQ slot) and schedules the next one.
struct Monitor {
  ism_ctx* c;
  const std::vector<double>& target;
  bool mixed;
  std::vector<Check> hist;
  int next = 1;

  Monitor(ism_ctx* ctx, const std::vector<double>& tgt, bool is_mixed)
      : c(ctx), target(tgt), mixed(is_mixed) {}

  // After k cycles of this inner solve (the squared grid residual norms read back now):
  // < 0 error, 1 stop (target met, stagnation or cycle cap), 0 continue (next check
  // scheduled in `next`).
  int check(int k, int cycles) {
    int rcode = read_scalars(c);
    if (rcode) return rcode;
    return evaluate(k, cycles, c->h_scal + size_t(ISQ) * c->g.batch);
  }

  // The same decision from squared norms sq[batch] taken after cycle k.
  int evaluate(int k, int cycles, const double* sq) {
    const int B = c->g.batch;
    Check ck{k, std::vector<double>(B)};
    bool done = true, finite = true;
    for (int b = 0; b < B; ++b) {
      ck.res[b] = std::sqrt(sq[b]);
      finite = finite && std::isfinite(ck.res[b]);
      done = done && ck.res[b] <= target[b];
    }
    if (!finite) return set_err(c, ISM_ERR_NONFINITE, "non-finite residual in the inner iteration");
    hist.push_back(ck);
    if (done || cycles >= c->cfg.max_cycles) return 1;
    // stagnation: the newest check against the latest one at least stall_window cycles older
    const Check* old = nullptr;
    for (auto it = hist.rbegin(); it != hist.rend(); ++it)
      if (it->cycle <= k - c->cfg.stall_window) {
        old = &*it;
        break;
      }
    if (old) {
      bool stalled = true;
      for (int b = 0; b < B; ++b)
        if (ck.res[b] > target[b] && ck.res[b] < (1.0 - c->cfg.stall_drop) * old->res[b]) stalled = false;
      if (stalled) return 1;
    }
    int gap;
    if (c->cfg.check_every > 0) {
      gap = c->cfg.check_every;
    } else {
      // predict the cycle that meets every target from the rate since the previous check,
      // at most doubling the cycle count per check
      gap = 1;
      if (hist.size() >= 2) {
        const Check& p = hist[hist.size() - 2];
        double need = 1.0;
        for (int b = 0; b < B; ++b) {
          if (ck.res[b] <= target[b]) continue;
          const double rho = std::pow(ck.res[b] / p.res[b], 1.0 / double(k - p.cycle));
          if (!(rho < 1.0) || !(rho > 0.0)) continue;
          need = std::max(need, std::ceil(std::log(target[b] / ck.res[b]) / std::log(rho)));
        }
        gap = int(std::min(need, double(std::max(4, k))));
      }
      if (mixed) {  // keep stagnation visible: about 1 ms of device work between checks
        gap = std::min(gap, mixed_check_cap(c->g));
      }
      gap = std::max(gap, 1);
    }
    next = k + gap;
    return 0;
  }
};

// Inner solve of A' e = rT from e = 0 in type T, until every grid's residual norm is below
// its target, or the residual stagnates, or the cycle cap is reached.  rc holds R rT on entry.
//
// With a fixed check interval every check stops the stream and is evaluated at once.  With
// adaptive checks the stream never waits on the host: a check's norms are reduced into a
// pinned slot behind an event and the host keeps enqueuing cycles, evaluating each check after
// exactly kLag more cycles (waiting for its event then).  A stop decision therefore lands
// kLag cycles late; the cycles already enqueued only reduce the residual further and are
// counted.  The squared-residual partials are formed only by the cycles a
// check reads.
template <typename T>
int inner_solve(ism_ctx* c, const std::vector<double>& target, int& cycles, T** e_out) {
  T* cur = (T*)c->eA;
  T* spare = (T*)c->eB;
  const T* rhs = (const T*)c->rT;
  const int B = c->g.batch;
  Monitor mon(c, target, sizeof(T) == 4);
  if (c->cfg.check_every > 0) {
    for (int k = 0;;) {
      const bool due = k + 1 >= mon.next || cycles + 1 >= c->cfg.max_cycles;
      int rcode = run_cycle<T>(c, rhs, &cur, &spare, c->rc, due ? c->p_sq : nullptr, k == 0);
      if (rcode) return rcode;
      ++k;
      ++cycles;
      if (!due) continue;
      if ((rcode = finalize(c, c->p_sq, ism::SUM, 1.0, ISQ))) return rcode;
      rcode = mon.check(k, cycles);
      if (rcode < 0) return rcode;
      if (rcode == 1) break;
    }
    *e_out = cur;
    return ISM_OK;
  }
  while (c->pinned && c->chk_ev.size() < size_t(kChecks)) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->chk_ev.push_back(e);
  }
  struct Pending {
    int k, cycles, slot;
  };
  std::deque<Pending> pend;
  int slot = 0, gap = 1, sched = 1;  // next check after cycle `sched`
  for (int k = 0;;) {
    const bool due = k + 1 >= sched || cycles + 1 >= c->cfg.max_cycles;
    int rcode = run_cycle<T>(c, rhs, &cur, &spare, c->rc, due ? c->p_sq : nullptr, k == 0);
    if (rcode) return rcode;
    ++k;
    ++cycles;
    if (due) {
      // the check's norms are reduced straight into its read-back slot: the pinned host
      // slot through its device address, or the device slot
      double* dst = (c->pinned ? c->d_hchk : c->d_chk) + size_t(slot) * B;
      LAUNCH(c, ism::launch_finalize(c->p_sq, int(c->g.cplane), c->g.cplane, B, ism::SUM, 1.0,
                                     dst, 1, 0, c->fin, c->stream));
      if (c->pinned) HIPCHK(c, hipEventRecord(c->chk_ev[slot], c->stream));
      pend.push_back({k, cycles, slot});
      slot = (slot + 1) % kChecks;
      sched = k + gap;  // provisional, until this check's own evaluation reschedules
    }
    bool stop = false;
    while (!pend.empty()) {
      // a check is acted on exactly kLag cycles after it (or at the cycle cap), never earlier
      // even when its result is already in: the cycles a solve runs then do not depend on
      // host timing
      const Pending p = pend.front();
      if (k - p.k < kLag && cycles < c->cfg.max_cycles) break;
      if (c->pinned) {
        HIPCHK(c, hipEventSynchronize(c->chk_ev[p.slot]));
      } else {
        HIPCHK(c, hipMemcpyAsync(c->h_chk + size_t(p.slot) * B, c->d_chk + size_t(p.slot) * B,
                                 sizeof(double) * B, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
      }
      pend.pop_front();
      c->syncs++;
      rcode = mon.evaluate(p.k, p.cycles, c->h_chk + size_t(p.slot) * B);
      if (rcode < 0) return rcode;
      if (rcode == 1) {
        stop = true;
        break;
      }
      gap = std::max(1, mon.next - p.k);
      sched = std::max(mon.next, k + 1);
    }
    if (stop) break;
  }
  *e_out = cur;
  return ISM_OK;
}

// Geometry of ACM level l (spacing 2^l h).
Geo acm_level(const Geo& g, int l) {
  Geo gl = g;
  gl.nx = g.nx >> l;
  gl.ny = g.ny >> l;
  gl.plane = (long long)gl.nx * gl.ny;
  return gl;
}

// Inner solve by additive correction multigrid V(0,1) cycles (the comparison scheme): 2x2
// agglomeration of the residual down to spacing n h, exact solve of n times the 5-point
// operator there, then on the way up the piecewise-constant correction and one red-black
// sweep per level on 2^l A' e = r_l (Sec. 3.2, Sec. 4, Sec. 4.3.1).  FP64.  The level-0
// agglomeration at the start of a cycle also yields the residual norm of the previous one.
int acm_inner_solve(ism_ctx* c, const std::vector<double>& target, int& cycles, double** e_out) {
  const Geo& g = c->g;
  const int L = g.log2n, B = g.batch;
  hipStream_t s = c->stream;
  double* e0 = (double*)c->eA;
  double* sp0 = (double*)c->eB;
  const double* rhs = (const double*)c->rT;
  const long long count0 = (long long)(g.nx / 2) * (g.ny / 2);
  Monitor mon(c, target, false);
  for (int k = 0;;) {
    double* r1 = L == 1 ? c->rc : c->acm_r[1];
    LAUNCH(c, ism::launch_agglomerate(acm_level(g, 0), rhs, k == 0 ? nullptr : e0, 1.0, r1,
                                      c->acm_psq, s));
    if (k > 0 && (k >= mon.next || cycles >= c->cfg.max_cycles)) {
      LAUNCH(c, ism::launch_finalize(c->acm_psq, int(count0), count0, B, ism::SUM, 1.0,
                                     c->scal + size_t(ISQ) * B, 1, 0, c->fin, s));
      int rcode = mon.check(k, cycles);
      if (rcode < 0) return rcode;
      if (rcode == 1) break;
    }
    for (int l = 1; l < L; ++l)
      LAUNCH(c, ism::launch_agglomerate(acm_level(g, l), c->acm_r[l], nullptr, 1.0,
                                        l + 1 == L ? c->rc : c->acm_r[l + 1], nullptr, s));
    hipEvent_t ev = prof_start(c, ISM_KERNEL_COARSE);
    int rcode = coarse_solve(c, c->rc, c->E);
    if (rcode) return rcode;
    prof_stop(c, ISM_KERNEL_COARSE, ev);
    const double* above = c->E;
    for (int l = L - 1; l >= 1; --l) {
      LAUNCH(c, ism::launch_inject(acm_level(g, l), above, c->acm_ea[l], 1, s));
      ev = prof_start(c, ISM_KERNEL_SMOOTH);
      LAUNCH(c, ism::launch_rbgs<double>(acm_level(g, l), c->acm_r[l], c->acm_ea[l], c->acm_eb[l], s,
                                         std::ldexp(1.0, -l)));
      prof_stop(c, ISM_KERNEL_SMOOTH, ev);
      above = c->acm_eb[l];
    }
    LAUNCH(c, ism::launch_inject(acm_level(g, 0), above, e0, k == 0, s));
    ev = prof_start(c, ISM_KERNEL_SMOOTH);
    LAUNCH(c, ism::launch_rbgs<double>(acm_level(g, 0), rhs, e0, sp0, s, 1.0));
    prof_stop(c, ISM_KERNEL_SMOOTH, ev);
    std::swap(e0, sp0);
    ++k;
    ++cycles;
  }
  *e_out = e0;
  return ISM_OK;
}

// The MEAN_B slots: the mean of each right-hand side when A is singular (the compatibility
// projection b~ = b - mean b), else 0.
int mean_of_b(ism_ctx* c, const double* b) {
  if (!c->singular) {
    LAUNCH(c, ism::launch_fill(c->scal + size_t(MEAN_B) * c->g.batch, c->g.batch, 0.0, c->stream));
    return ISM_OK;
  }
  LAUNCH(c, ism::launch_tile_sum(c->g, b, c->p_sum, c->stream));
  return finalize(c, c->p_sum, ism::SUM, 1.0 / double(c->g.plane), MEAN_B);
}

// The coarse grid of a handle as a plane of its own (for the per-grid scalar kernels).
Geo coarse_geo(const Geo& g) {
  Geo gc = g;
  gc.nx = g.ncx;
  gc.ny = g.ncy;
  gc.plane = g.cplane;
  return gc;
}

// A device-checked iteration loop: iteration it (0, 1, ...) enqueues step(it, state, &part,
// &count), which leaves per-tile maxima of the residual of its incoming iterate in part
// (count per grid, grid k at k count), then one workgroup reduces them to the per-grid maxima
// m and tests them against tol on the device, recording the first iteration at which every
// grid is below it (the later steps then exit at once).  The host reads the state back once
// per batch of iterations.  *stop_it: that iteration, or max_iter when none was below tol by
// then (*converged false).
template <typename Step>
int device_checked_loop(ism_ctx* c, Step step, double* m, double tol, int max_iter,
                        const char* what, int* stop_it, bool* converged) {
  const int B = c->g.batch;
  double* state = c->scal + size_t(STOP) * B;
  double* at = c->scal + size_t(STOP_AT) * B;
  LAUNCH(c, ism::launch_fill(state, 1, 0.0, c->stream));
  int it = 0, batch = kBatchFirst;
  for (;;) {
    const int end = std::min(max_iter, it + batch - 1);
    for (; it <= end; ++it) {
      const double* part = nullptr;
      int count = 0;
      int rcode = step(it, state, &part, &count);
      if (rcode) return rcode;
      hipError_t err = hipSuccess;
      c->launches += ism::launch_max_stop(part, count, count, B, m, tol, it, state, at, c->fin,
                                          c->stream, &err);
      HIPCHK(c, err);
    }
    int rcode = read_scalars(c);
    if (rcode) return rcode;
    const double st = c->h_scal[size_t(STOP) * B], a = c->h_scal[size_t(STOP_AT) * B];
    if (st == 2.0) return set_err(c, ISM_ERR_NONFINITE, std::string("non-finite ") + what);
    if (st == 1.0) {
      *stop_it = int(a);
      *converged = true;
      return ISM_OK;
    }
    if (it > max_iter) {
      *stop_it = max_iter;
      *converged = false;
      return ISM_OK;
    }
    batch = std::min(2 * batch, kBatchMax);
  }
}

// Gauss-Seidel on every grid's A_c E = rc from E = 0, block-iterative (Sec. 4) or in
// multicolour order (Sec. 3.1) as the handle was created (ism_config.coarse_gs): iteration it
// forms the residual of its incoming iterate E_it (in t1 for even it, t2 for odd) and E_it+1,
// one launch for block GS, one per colour for multicolour GS; the loop stops at the first
// iterate whose residual max is below tol on every grid (or at max_iter).  The result stays
// in one of the t1 / t2 buffers (*E_out).  *syncs_per_iter: the synchronizations of one
// iteration (Sec. 4.3: one for block GS, one per colour).
int coarse_gs_loop(ism_ctx* c, const double* rc, double tol, int max_iter, double** E_out,
                   int* iters, bool* converged, int* syncs_per_iter) {
  const Geo& g = c->g;
  const bool mc = c->cfg.coarse_gs == ISM_COARSE_GS_MULTICOLOUR;
  const int B = g.batch, tiles = mc ? ism::coarse_mc_tiles(g) : ism::coarse_bgs_tiles(g);
  *syncs_per_iter = mc ? ism::coarse_mc_colours(g) : 1;
  hipStream_t s = c->stream;
  double* E[2] = {c->t1, c->t2};
  LAUNCH(c, ism::launch_fill(E[0], (long long)g.cplane * B, 0.0, s));
  double* m = c->scal + size_t(CMAX) * B;
  auto step = [&](int it, const double* stop, const double** part, int* count) {
    if (mc) {
      hipError_t err = hipSuccess;
      c->launches += ism::launch_coarse_mc(g, c->coef, rc, E[it & 1], E[(it + 1) & 1], c->p_max,
                                           s, stop, &err);
      HIPCHK(c, err);
    } else {
      LAUNCH(c, ism::launch_coarse_bgs(g, c->coef, rc, E[it & 1], E[(it + 1) & 1], c->p_max, s,
                                       stop));
    }
    *part = c->p_max;
    *count = tiles;
    return ISM_OK;
  };
  int it = 0;
  const int rcode = device_checked_loop(c, step, m, tol, max_iter, "coarse residual", &it, converged);
  if (rcode) return rcode;
  *E_out = E[it & 1];
  *iters = it;
  return ISM_OK;
}

// rc -= its mean, per grid (the compatibility projection of a singular coarse system).
int project_coarse(ism_ctx* c, double* rc) {
  const Geo& g = c->g;
  int rcode = finalize(c, rc, ism::SUM, 1.0 / double(g.cplane), MEAN_R);
  if (rcode) return rcode;
  LAUNCH(c, ism::launch_sub_scalar(coarse_geo(g), rc, c->scal + size_t(MEAN_R) * g.batch, 1, 0,
                                   c->stream));
  return ISM_OK;
}

// ISM_CYCLE_ONESHOT (Sec. 4.3.1): restrict once, block (or multicolour) GS on the coarse grid
// to coarse_tol, prolongate and add, then red-black sweeps until max |b~ - A x| < fine_tol.
// T = double iterates x itself; T = float (the paper's single precision, Sec. 4.2) iterates a
// correction e on A'e = fp32(r), r = h^2 b~ - A'x in FP64, from e = P E, and adds it to x at
// the end.
// Both stages are device-checked loops (one read-back per batch of iterations).
template <typename T>
int oneshot_solve(ism_ctx* c, const double* b, double* x, ism_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  c->launches = 0;
  c->syncs = 0;
  const Geo& g = c->g;
  const int B = g.batch;
  constexpr bool F64 = sizeof(T) == 8;
  hipStream_t s = c->stream;
  const double* mean = c->scal + size_t(MEAN_B) * B;
  int rcode;
  if ((rcode = mean_of_b(c, b))) return rcode;
  // r' = h^2 b~ - A'x and its tile sums, the coarse right-hand side (FP32 form: r' also as
  // the fine right-hand side, in T)
  Partials p0{nullptr, nullptr, c->p_bsq, c->p_bmax};
  LAUNCH(c, ism::launch_outer_residual<T>(g, b, x, mean, c->h2, F64 ? (T*)nullptr : (T*)c->rT,
                                          c->rc, p0, s));
  if ((rcode = finalize(c, c->p_bsq, ism::SUM, 1.0, BSQ))) return rcode;
  if ((rcode = finalize(c, c->p_bmax, ism::MAX, 1.0, BMAX))) return rcode;
  if (c->singular && (rcode = project_coarse(c, c->rc))) return rcode;
  double* E = nullptr;
  int ic = 0;
  bool cconv = false;
  const double h = c->h;
  int cper = 1;
  if ((rcode = coarse_gs_loop(c, c->rc, c->cfg.coarse_tol * h * h, c->cfg.max_cycles, &E, &ic,
                              &cconv, &cper)))
    return rcode;
  // the fine iterates: x and eA (FP64: x += P E, right-hand side b' = h^2 b~, the residual of
  // x = 0), or eA and eB (FP32: e = P E, right-hand side fp32(r'))
  T* buf[2];
  const T* rhs;
  if constexpr (F64) {
    LAUNCH(c, ism::launch_prolong<double>(g, E, x, 0, s));
    double* bp = (double*)c->rT;
    double* zero = (double*)c->eB;
    LAUNCH(c, ism::launch_fill(zero, (long long)g.plane * B, 0.0, s));
    Partials none{nullptr, nullptr, nullptr, nullptr};
    LAUNCH(c, ism::launch_outer_residual<double>(g, b, zero, mean, c->h2, bp, nullptr, none, s));
    buf[0] = x;
    buf[1] = (double*)c->eA;
    rhs = bp;
  } else {
    buf[0] = (T*)c->eA;
    buf[1] = (T*)c->eB;
    LAUNCH(c, ism::launch_prolong<T>(g, E, buf[0], 1, s));
    rhs = (const T*)c->rT;
  }
  // Iteration i checks iterate i, held in buf[i & 1].  Unfused: one sweep kernel forms the
  // residual maxima of its incoming iterate per tile and the next iterate.  Fused (16-byte
  // aligned iterates): iteration i >= 1 is one pass of the fused kernel with a zero coarse
  // correction, sweeping iterate i - 1 into iterate i and forming its residual maxima per
  // coarse tile (the same values, bit for bit); iteration 0 takes the unfused form for the
  // residual of the first iterate, and the sweep it also makes is made again by iteration 1.
  const int tiles = ism::rbgs_tiles(g);
  if (tiles > g.cplane) return set_err(c, ISM_ERR_UNSUPPORTED, "sweep tiles exceed the partials");
  const bool fused = c->cfg.fused && ((uintptr_t)buf[0] & 15) == 0;
  double* zeroE = c->E;
  if (fused) LAUNCH(c, ism::launch_fill(zeroE, (long long)g.cplane * B, 0.0, s));
  double* m = c->scal + size_t(RMAX) * B;
  auto step = [&](int i, const double* stop, const double** part, int* count) {
    if (!fused || i == 0) {
      hipEvent_t ev = prof_start(c, ISM_KERNEL_SMOOTH);
      LAUNCH(c, ism::launch_rbgs<T>(g, rhs, buf[i & 1], buf[(i + 1) & 1], s, T(1), c->p_max, stop));
      prof_stop(c, ISM_KERNEL_SMOOTH, ev);
      *count = tiles;
    } else {
      hipEvent_t ev = prof_start(c, ISM_KERNEL_CYCLE);
      LAUNCH(c, launch_fused<T>(c, rhs, buf[(i - 1) & 1], buf[i & 1], zeroE, c->rc, c->p_max, 1, 0,
                                stop, 1));
      prof_stop(c, ISM_KERNEL_CYCLE, ev);
      *count = int(g.cplane);
    }
    *part = c->p_max;
    return ISM_OK;
  };
  int fi = 0;
  bool fconv = false;
  if ((rcode = device_checked_loop(c, step, m, c->cfg.fine_tol * h * h, c->cfg.max_cycles,
                                   "value in b, x or the residual", &fi, &fconv)))
    return rcode;
  T* cur = buf[fi & 1];
  if constexpr (F64) {
    if (cur != x)
      HIPCHK(c, hipMemcpyAsync(x, cur, sizeof(double) * size_t(g.plane) * B, hipMemcpyDeviceToDevice, s));
  } else {
    LAUNCH(c, ism::launch_add_to<T>(g, x, cur, s));
  }
  // the reported norms: one residual pass over the result
  Partials pc{c->p_sq, c->p_max, nullptr, nullptr};
  LAUNCH(c, ism::launch_outer_residual<double>(g, b, x, mean, c->h2, (double*)nullptr, nullptr, pc, s));
  if ((rcode = finalize(c, c->p_sq, ism::SUM, 1.0, RSQ))) return rcode;
  if ((rcode = finalize(c, c->p_max, ism::MAX, 1.0, RMAX))) return rcode;
  if ((rcode = read_scalars(c))) return rcode;
  double rel_l2 = 0.0, rel_max = 0.0;
  for (int k = 0; k < B; ++k) {
    const double bn = std::sqrt(c->h_scal[size_t(BSQ) * B + k]), bm = c->h_scal[size_t(BMAX) * B + k];
    rel_l2 = std::max(rel_l2, std::sqrt(c->h_scal[size_t(RSQ) * B + k]) / (bn > 0.0 ? bn : 1.0));
    rel_max = std::max(rel_max, c->h_scal[size_t(RMAX) * B + k] / (bm > 0.0 ? bm : 1.0));
  }
  if (c->singular) {
    LAUNCH(c, ism::launch_tile_sum(g, x, c->p_sum, s));
    if ((rcode = finalize(c, c->p_sum, ism::SUM, 1.0 / double(g.plane), MEAN_X))) return rcode;
    LAUNCH(c, ism::launch_sub_scalar(g, x, c->scal + size_t(MEAN_X) * B, 1, 0, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  c->syncs++;
  prof_collect(c);
  const int status = (cconv && fconv) ? ISM_OK : ISM_NOT_CONVERGED;
  if (st) {
    st->status = status;
    st->outer_iters = 0;
    st->cycles = 1;
    st->sweeps = fi;
    st->launches = c->launches;
    st->host_syncs = c->syncs;
    st->rel_res_l2 = rel_l2;
    st->rel_res_max = rel_max;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st->coarse_iters = ic;
    st->fine_iters = fi;
    st->coarse_syncs = ic * cper;
  }
  return status;
}

// Geometry and scalars of a handle from a validated config.
void init_geometry(ism_ctx* c, const ism_config* cfg, hipStream_t stream) {
  c->cfg = *cfg;
  c->stream = stream;
  Geo& g = c->g;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.batch = cfg->batch;
  g.n = cfg->coarsen;
  g.log2n = 0;
  while ((1 << g.log2n) < g.n) ++g.log2n;
  g.ncx = (g.nx + g.n - 1) / g.n;  // the last tile short when n does not divide the axis
  g.ncy = (g.ny + g.n - 1) / g.n;
  c->padded = g.nx % g.n || g.ny % g.n;
  g.per_x = cfg->bc_x == ISM_BC_PERIODIC;
  g.per_y = cfg->bc_y == ISM_BC_PERIODIC;
  auto dir_lo = [](int bc) { return bc == ISM_BC_DIRICHLET || bc == ISM_BC_DIRICHLET_NEUMANN; };
  auto dir_hi = [](int bc) { return bc == ISM_BC_DIRICHLET || bc == ISM_BC_NEUMANN_DIRICHLET; };
  g.dmask = (dir_lo(cfg->bc_x) ? 1 : 0) | (dir_hi(cfg->bc_x) ? 2 : 0) |
            (dir_lo(cfg->bc_y) ? 4 : 0) | (dir_hi(cfg->bc_y) ? 8 : 0);
  c->singular = g.dmask == 0;
  g.plane = (long long)g.nx * g.ny;
  g.cplane = (long long)g.ncx * g.ncy;
  c->h = cfg->lx / cfg->nx;
  c->h2 = c->h * c->h;
  c->tsize = cfg->precision == ISM_PREC_MIXED ? 4 : 8;
}

// The device workspace of a handle (without the ACM levels), every buffer 256-byte aligned:
// the inner fine arrays rT, eA, eB; nine coarse-sized FP64 arrays; the per-grid scalars, the
// check slots and the reduction chunks; the coarse tables.  Returns its size in bytes; with
// a base address, also points the handle's buffers into it.
size_t layout_workspace(ism_ctx* c, char* base) {
  const Geo& g = c->g;
  auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t fine = align(size_t(g.plane) * g.batch * c->tsize);
  const size_t coarse = align(size_t(g.cplane) * g.batch * sizeof(double));
  const size_t scal = align(sizeof(double) * kSlots * g.batch);
  const size_t chk = align(sizeof(double) * kChecks * g.batch);
  const long long fin_count = std::max<long long>(g.cplane, (long long)(g.nx / 2) * (g.ny / 2));
  const size_t fin = align(sizeof(double) * g.batch * size_t(fin_count / 4096 + 2));
  const size_t vx = align(sizeof(double) * g.ncx * g.ncx), vy = align(sizeof(double) * g.ncy * g.ncy);
  const size_t lam = align(sizeof(double) * g.cplane), coef = align(sizeof(double) * 9 * g.cplane);
  const size_t fx = c->padded ? vx : 0, fy = c->padded ? vy : 0;
  const size_t itab = align(sizeof(double2) * size_t(g.nx + g.ny));
  const size_t total = 3 * fine + 9 * coarse + scal + chk + fin + vx + vy + lam + coef + fx + fy + itab;
  if (!base) return total;
  char* p = base;
  c->rT = p; p += fine;
  c->eA = p; p += fine;
  c->eB = p; p += fine;
  double** cbufs[9] = {&c->rc, &c->E, &c->t1, &c->t2, &c->p_sq, &c->p_max, &c->p_bsq, &c->p_bmax, &c->p_sum};
  for (double** q : cbufs) {
    *q = (double*)p;
    p += coarse;
  }
  c->scal = (double*)p; p += scal;
  c->d_chk = (double*)p; p += chk;
  c->fin = (double*)p; p += fin;
  c->Vx = (double*)p; p += vx;
  c->Vy = (double*)p; p += vy;
  c->invLam = (double*)p; p += lam;
  c->coef = (double*)p; p += coef;
  c->Fx = c->padded ? (double*)p : c->Vx; p += fx;
  c->Fy = c->padded ? (double*)p : c->Vy; p += fy;
  c->g.itab = p;
  return total;
}

// The coarse solve's tables of a padded grid, built on the host (the pencil of each axis
// that a tile size does not divide, the closed form of the other) and copied to the
// workspace; waits for the copies.
int upload_padded_tables(ism_ctx* c) {
  const Geo& g = c->g;
  const bool xlo = g.dmask & 1, xhi = g.dmask & 2, ylo = g.dmask & 4, yhi = g.dmask & 8;
  ism::AxisTable tx, ty;
  std::string why;
  if (!ism::coarse_axis_table(g.nx, g.n, g.ncx, g.per_x, xlo, xhi, tx, why) ||
      !ism::coarse_axis_table(g.ny, g.n, g.ncy, g.per_y, ylo, yhi, ty, why))
    return set_err(c, ISM_ERR_UNSUPPORTED, why);
  std::vector<double> inv(size_t(g.cplane));
  for (int l = 0; l < g.ncy; ++l)
    for (int k = 0; k < g.ncx; ++k) {
      const double lam = tx.k[k] * ty.m[l] + tx.m[k] * ty.k[l];
      inv[size_t(l) * g.ncx + k] = (c->singular && l == 0 && k == 0) ? 0.0 : 1.0 / lam;
    }
  const std::pair<double*, const std::vector<double>*> copies[] = {
      {c->Vx, &tx.V}, {c->Vy, &ty.V}, {c->Fx, &tx.F}, {c->Fy, &ty.F}, {c->invLam, &inv}};
  for (const auto& cp : copies) {
    const hipError_t e = hipMemcpyAsync(cp.first, cp.second->data(), sizeof(double) * cp.second->size(),
                                        hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return set_err(c, ISM_ERR_HIP, std::string("coarse tables: ") + hipGetErrorString(e));
  }
  const hipError_t e = hipStreamSynchronize(c->stream);  // the host tables go out of scope
  if (e != hipSuccess) return set_err(c, ISM_ERR_HIP, std::string("coarse tables: ") + hipGetErrorString(e));
  return ISM_OK;
}

// Enqueues what a workspace must hold before a solve: the interpolation tables, the coarse
// eigenbasis tables, the assembled coarse stencil (block Gauss-Seidel) and zeroed per-grid
// scalars.  No host wait, but for the host-built tables of a padded grid.
int init_device_state(ism_ctx* c) {
  const Geo& g = c->g;
  const int kind = c->cfg.coarse_stencil == ISM_COARSE_GMG5 ? 1 : c->cfg.coarse_stencil == ISM_COARSE_ACM ? 2 : 0;
  LAUNCH(c, ism::launch_interp_tables(g, (double2*)g.itab, c->stream));
  if (c->padded) {
    const int rcode = upload_padded_tables(c);
    if (rcode) return rcode;
  } else {
    LAUNCH(c, ism::launch_coarse_tables(g, kind, c->singular ? 1 : 0, c->Vx, c->Vy, c->invLam, c->stream));
  }
  LAUNCH(c, ism::launch_fill(c->scal, (long long)kSlots * g.batch, 0.0, c->stream));
  if (c->cfg.coarse_stencil != ISM_COARSE_ACM)
    LAUNCH(c, ism::launch_coarse_assemble(g, c->cfg.coarse_stencil == ISM_COARSE_GMG5, c->coef, c->stream));
  return ISM_OK;
}

template <typename T>
int solve_impl(ism_ctx* c, const double* b, double* x, ism_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  c->launches = 0;
  c->syncs = 0;
  const Geo& g = c->g;
  const int B = g.batch;
  hipStream_t s = c->stream;
  int rcode;
  if ((rcode = mean_of_b(c, b))) return rcode;

  std::vector<double> bnorm(B, 0.0), bmax(B, 0.0), den(B, 1.0), target(B);
  int cycles = 0, outer = 0, status = ISM_OK;
  double rel_l2 = 0.0, rel_max = 0.0;
  for (bool first = true;; first = false) {
    Partials p{c->p_sq, c->p_max, first ? c->p_bsq : nullptr, first ? c->p_bmax : nullptr};
    hipEvent_t ev = prof_start(c, ISM_KERNEL_OUTER);
    LAUNCH(c, ism::launch_outer_residual<T>(g, b, x, c->scal + size_t(MEAN_B) * B, c->h2, (T*)c->rT,
                                            c->rc, p, s));
    prof_stop(c, ISM_KERNEL_OUTER, ev);
    if ((rcode = finalize(c, c->p_sq, ism::SUM, 1.0, RSQ))) return rcode;
    if ((rcode = finalize(c, c->p_max, ism::MAX, 1.0, RMAX))) return rcode;
    if (first) {
      if ((rcode = finalize(c, c->p_bsq, ism::SUM, 1.0, BSQ))) return rcode;
      if ((rcode = finalize(c, c->p_bmax, ism::MAX, 1.0, BMAX))) return rcode;
    }
    if ((rcode = read_scalars(c))) return rcode;
    bool conv = true, finite = true;
    rel_l2 = rel_max = 0.0;
    for (int k = 0; k < B; ++k) {
      if (first) {
        bnorm[k] = std::sqrt(c->h_scal[size_t(BSQ) * B + k]);
        bmax[k] = c->h_scal[size_t(BMAX) * B + k];
        // a constant right-hand side has b~ = 0: the criterion becomes absolute
        den[k] = bnorm[k] > 0.0 ? bnorm[k] : 1.0;
      }
      const double rn = std::sqrt(c->h_scal[size_t(RSQ) * B + k]);
      const double rm = c->h_scal[size_t(RMAX) * B + k];
      finite = finite && std::isfinite(rn) && std::isfinite(bnorm[k]);
      rel_l2 = std::max(rel_l2, rn / den[k]);
      rel_max = std::max(rel_max, rm / (bmax[k] > 0.0 ? bmax[k] : 1.0));
      conv = conv && rn <= c->cfg.rtol * den[k];
      const bool fp64 = c->cfg.precision == ISM_PREC_FP64;
      const double inner = fp64 ? 0.0 : c->cfg.inner_rtol * rn;
      target[k] = std::max(inner, (fp64 ? kInnerMarginFP64 : kInnerMarginMixed) * c->cfg.rtol * den[k]);
    }
    if (!finite) {
      status = set_err(c, ISM_ERR_NONFINITE, "non-finite value in b, x or the residual");
      break;
    }
    if (conv) break;
    if (outer >= c->cfg.max_outer || cycles >= c->cfg.max_cycles) {
      status = ISM_NOT_CONVERGED;
      break;
    }
    ++outer;
    T* e = nullptr;
    if (c->cfg.coarse_stencil == ISM_COARSE_ACM) {
      double* e64 = nullptr;
      if ((rcode = acm_inner_solve(c, target, cycles, &e64))) return rcode;
      e = (T*)e64;  // ACM handles are FP64 (T = double)
    } else if ((rcode = inner_solve<T>(c, target, cycles, &e))) {
      return rcode;
    }
    LAUNCH(c, ism::launch_add_to<T>(g, x, e, s));
  }
  if (status >= 0 && c->singular) {
    LAUNCH(c, ism::launch_tile_sum(g, x, c->p_sum, s));
    if ((rcode = finalize(c, c->p_sum, ism::SUM, 1.0 / double(g.plane), MEAN_X))) return rcode;
    LAUNCH(c, ism::launch_sub_scalar(g, x, c->scal + size_t(MEAN_X) * B, 1, 0, s));
    // The reported norms are those of the returned x: removing the mean re-rounds every
    // entry, which moves a residual near the FP64 rounding floor.  One norms-only pass.
    Partials pn{c->p_sq, c->p_max, nullptr, nullptr};
    LAUNCH(c, ism::launch_outer_residual<double>(g, b, x, c->scal + size_t(MEAN_B) * B, c->h2,
                                                 (double*)nullptr, nullptr, pn, s));
    if ((rcode = finalize(c, c->p_sq, ism::SUM, 1.0, RSQ))) return rcode;
    if ((rcode = finalize(c, c->p_max, ism::MAX, 1.0, RMAX))) return rcode;
    if ((rcode = read_scalars(c))) return rcode;
    rel_l2 = rel_max = 0.0;
    for (int k = 0; k < B; ++k) {
      rel_l2 = std::max(rel_l2, std::sqrt(c->h_scal[size_t(RSQ) * B + k]) / den[k]);
      rel_max = std::max(rel_max, c->h_scal[size_t(RMAX) * B + k] / (bmax[k] > 0.0 ? bmax[k] : 1.0));
    }
  } else {
    HIPCHK(c, hipStreamSynchronize(s));
    c->syncs++;
    prof_collect(c);
  }
  if (st) {
    st->status = status;
    st->outer_iters = outer;
    st->cycles = cycles;
    st->sweeps = cycles * (c->cfg.coarse_stencil == ISM_COARSE_ACM ? 1 : c->cfg.nu);
    st->launches = c->launches;
    st->host_syncs = c->syncs;
    st->rel_res_l2 = rel_l2;
    st->rel_res_max = rel_max;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}


}  // namespace

// ================================================================== allocation-free solve
// A workspace for callers that cannot allocate: a static device array that every GPU the
// library runs on holds until the process ends.  In host code its name is only a stand-in,
// never a device address: each device holds its own copy, whose address is looked up once
// per device (with that device current) and used everywhere host code needs the memory.
constexpr size_t kStaticScratchBytes = size_t(ISM_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

// This device's copy of scratch (the current device must be dev).
int scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_err(nullptr, ISM_ERR_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(nullptr, ISM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (char*)p;
  }
  *out = g_scratch_dev[dev];
  return ISM_OK;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

int ism_config_init(ism_config* cfg, int32_t nx, int32_t ny, int32_t batch) {
  if (!cfg) return ISM_ERR_INVALID;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->nx = nx;
  cfg->ny = ny;
  cfg->batch = batch;
  cfg->bc_x = ISM_BC_NEUMANN;
  cfg->bc_y = ISM_BC_NEUMANN;
  cfg->coarsen = 16;
  cfg->lx = 1.0;
  cfg->ly = nx > 0 ? double(ny) / double(nx) : 1.0;
  cfg->precision = ISM_PREC_FP64;
  cfg->nu = 4;
  cfg->rtol = 1e-10;
  cfg->inner_rtol = 1e-3;
  cfg->max_cycles = 100000;
  cfg->max_outer = 50;
  cfg->check_every = 0;
  cfg->fused = 1;
  cfg->stall_window = 8;
  cfg->stall_drop = 0.02;
  cfg->cycling = ISM_CYCLE_REPEAT;
  cfg->coarse_tol = 1e-5;  // the paper's coarse and fine criteria (Sec. 4.3.1, Fig. 3)
  cfg->fine_tol = 1e-6;
  cfg->coarse_gs = ISM_COARSE_GS_BLOCK;
  return ISM_OK;
}

int ism_create(const ism_config* cfg, void* stream, ism_handle* out) {
  if (!out) return set_err(nullptr, ISM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  std::string why;
  int v = validate(cfg, why);
  if (v != ISM_OK) return set_err(nullptr, v, why);

  ism_ctx* c = new (std::nothrow) ism_ctx();
  if (!c) return set_err(nullptr, ISM_ERR_INVALID, "out of host memory");
  init_geometry(c, cfg, (hipStream_t)stream);
  const Geo& g = c->g;

  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) {
    delete c;
    return set_err(nullptr, ISM_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
  }
  c->bytes = layout_workspace(c, nullptr);
  he = hipMalloc((void**)&c->block, c->bytes);
  if (he != hipSuccess) {
    delete c;
    return set_err(nullptr, ISM_ERR_HIP, std::string("hipMalloc workspace: ") + hipGetErrorString(he));
  }
  layout_workspace(c, c->block);

  he = hipHostMalloc((void**)&c->h_scal, sizeof(double) * (kSlots + kChecks) * g.batch,
                     hipHostMallocDefault);
  c->h_chk = c->h_scal + size_t(kSlots) * g.batch;
  if (he != hipSuccess) {
    (void)hipFree(c->block);
    delete c;
    return set_err(nullptr, ISM_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(he));
  }
  {
    double* dh = nullptr;
    he = hipHostGetDevicePointer((void**)&dh, c->h_scal, 0);
    if (he != hipSuccess || !dh) {
      (void)hipHostFree(c->h_scal);
      (void)hipFree(c->block);
      delete c;
      return set_err(nullptr, ISM_ERR_HIP,
                     std::string("hipHostGetDevicePointer: ") + hipGetErrorString(he));
    }
    c->d_hchk = dh + size_t(kSlots) * g.batch;
  }

  auto align = [](size_t n) { return (n + 255) & ~size_t(255); };
  if (cfg->coarse_stencil == ISM_COARSE_ACM) {
    const int L = g.log2n;
    size_t total = align(sizeof(double) * size_t(g.nx / 2) * (g.ny / 2) * g.batch);
    for (int l = 1; l < L; ++l) total += 3 * align(sizeof(double) * size_t(g.nx >> l) * (g.ny >> l) * g.batch);
    he = hipMalloc(&c->acm_mem, total);
    if (he != hipSuccess) {
      (void)hipHostFree(c->h_scal);
      (void)hipFree(c->block);
      delete c;
      return set_err(nullptr, ISM_ERR_HIP, std::string("hipMalloc ACM levels: ") + hipGetErrorString(he));
    }
    char* q = (char*)c->acm_mem;
    c->acm_psq = (double*)q;
    q += align(sizeof(double) * size_t(g.nx / 2) * (g.ny / 2) * g.batch);
    c->acm_r.assign(L + 1, nullptr);
    c->acm_ea.assign(L + 1, nullptr);
    c->acm_eb.assign(L + 1, nullptr);
    for (int l = 1; l < L; ++l) {
      const size_t sz = align(sizeof(double) * size_t(g.nx >> l) * (g.ny >> l) * g.batch);
      c->acm_r[l] = (double*)q; q += sz;
      c->acm_ea[l] = (double*)q; q += sz;
      c->acm_eb[l] = (double*)q; q += sz;
    }
    c->bytes += total;
  }

  int rcode = init_device_state(c);
  if (rcode == ISM_OK) {
    he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) rcode = set_err(c, ISM_ERR_HIP, std::string("create: ") + hipGetErrorString(he));
  }
  if (rcode != ISM_OK) {
    const std::string msg = c->err;
    if (c->acm_mem) (void)hipFree(c->acm_mem);
    (void)hipHostFree(c->h_scal);
    (void)hipFree(c->block);
    delete c;
    return set_err(nullptr, rcode, msg);
  }
  *out = c;
  return ISM_OK;
}

int ism_destroy(ism_handle c) {
  if (!c) return ISM_OK;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->chk_ev) (void)hipEventDestroy(e);
  if (c->stage_tmp) (void)hipFree(c->stage_tmp);
  if (c->acm_mem) (void)hipFree(c->acm_mem);
  if (c->h_scal) (void)hipHostFree(c->h_scal);
  if (c->block) (void)hipFree(c->block);
  delete c;
  return ISM_OK;
}

int ism_workspace_bytes(ism_handle c, size_t* bytes) {
  if (!c || !bytes) return ISM_ERR_INVALID;
  *bytes = c->bytes + (c->stage_tmp ? size_t(c->g.plane) * c->g.batch * sizeof(double) : 0);
  return ISM_OK;
}

int ism_solve(ism_handle c, const double* b, double* x, ism_stats* st) {
  if (!c) return ISM_ERR_INVALID;
  if (!b || !x) return set_err(c, ISM_ERR_INVALID, "b and x must be device pointers");
  if (st) *st = ism_stats{};
  if (c->cfg.cycling == ISM_CYCLE_ONESHOT)
    return c->tsize == 4 ? oneshot_solve<float>(c, b, x, st) : oneshot_solve<double>(c, b, x, st);
  return c->tsize == 4 ? solve_impl<float>(c, b, x, st) : solve_impl<double>(c, b, x, st);
}

int ism_solve_static(const ism_config* cfg, const double* b, double* x, ism_stats* st,
                     void* stream) {
  if (st) *st = ism_stats{};
  std::string why;
  const int v = validate(cfg, why);
  if (v != ISM_OK) return set_err(nullptr, v, why);
  if (cfg->coarse_stencil == ISM_COARSE_ACM)
    return set_err(nullptr, ISM_ERR_UNSUPPORTED, "ism_solve_static: the ACM scheme needs level buffers; use ism_create");
  if (!b || !x) return set_err(nullptr, ISM_ERR_INVALID, "b and x must be device pointers");
  ism_ctx c;
  init_geometry(&c, cfg, (hipStream_t)stream);
  const size_t need = layout_workspace(&c, nullptr);
  if (need > kStaticScratchBytes)
    return set_err(nullptr, ISM_ERR_UNSUPPORTED,
                   "ism_solve_static: this grid needs " + std::to_string(need) +
                       " bytes of workspace, more than the " + std::to_string(kStaticScratchBytes) +
                       "-byte static scratch; use ism_create");
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return set_err(nullptr, ISM_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
  char* base = nullptr;
  int rcode = scratch_address(dev, &base);
  if (rcode) return rcode;
  layout_workspace(&c, base);
  c.bytes = need;
  c.pinned = false;
  c.h_mem.assign(size_t(kSlots + kChecks) * c.g.batch, 0.0);
  c.h_scal = c.h_mem.data();
  c.h_chk = c.h_scal + size_t(kSlots) * c.g.batch;
  rcode = init_device_state(&c);
  if (rcode == ISM_OK) {
    if (c.cfg.cycling == ISM_CYCLE_ONESHOT)
      rcode = c.tsize == 4 ? oneshot_solve<float>(&c, b, x, st) : oneshot_solve<double>(&c, b, x, st);
    else rcode = c.tsize == 4 ? solve_impl<float>(&c, b, x, st) : solve_impl<double>(&c, b, x, st);
  }
  if (rcode < 0) g_create_error = c.err;
  return rcode;
}

int ism_solve_adjoint(ism_handle c, const double* g, double* lam, ism_stats* st) {
  // A is symmetric (cell-centred 5-point operator with Neumann, Dirichlet or periodic
  // boundaries), and the mean projection is self-adjoint, so the adjoint solve is the
  // forward solve.
  return ism_solve(c, g, lam, st);
}

int ism_div(ism_handle c, const double* u, const double* v, double* b) {
  if (!c) return ISM_ERR_INVALID;
  if (!u || !v || !b) return set_err(c, ISM_ERR_INVALID, "NULL array");
  LAUNCH(c, ism::launch_div(c->g, u, v, c->h, b, c->stream));
  return ISM_OK;
}

int ism_grad(ism_handle c, const double* p, double* gu, double* gv) {
  if (!c) return ISM_ERR_INVALID;
  if (!p || !gu || !gv) return set_err(c, ISM_ERR_INVALID, "NULL array");
  LAUNCH(c, ism::launch_grad(c->g, p, c->h, gu, gv, c->stream));
  return ISM_OK;
}

int ism_div_adjoint(ism_handle c, const double* lam, double* gu, double* gv) {
  if (!c) return ISM_ERR_INVALID;
  if (!lam || !gu || !gv) return set_err(c, ISM_ERR_INVALID, "NULL array");
  LAUNCH(c, ism::launch_div_adjoint(c->g, lam, c->h, gu, gv, c->stream));
  return ISM_OK;
}

int ism_grad_adjoint(ism_handle c, const double* gu, const double* gv, double* p) {
  if (!c) return ISM_ERR_INVALID;
  if (!gu || !gv || !p) return set_err(c, ISM_ERR_INVALID, "NULL array");
  LAUNCH(c, ism::launch_grad_adjoint(c->g, gu, gv, c->h, p, c->stream));
  return ISM_OK;
}

}  // extern "C"

namespace {

template <typename T>
int smooth_impl(ism_ctx* c, const T* rhs, T* e, int nsweeps) {
  T* tmp = (T*)scratch_fine(c);
  if (!tmp) return set_err(c, ISM_ERR_HIP, "hipMalloc of the stage scratch failed");
  T* cur = e;
  T* spare = tmp;
  for (int k = 0; k < nsweeps; ++k) {
    LAUNCH(c, ism::launch_rbgs<T>(c->g, rhs, cur, spare, c->stream));
    std::swap(cur, spare);
  }
  if (cur != e)
    HIPCHK(c, hipMemcpyAsync(e, cur, sizeof(T) * size_t(c->g.plane) * c->g.batch,
                             hipMemcpyDeviceToDevice, c->stream));
  return ISM_OK;
}

template <typename T>
int cycle_impl(ism_ctx* c, const T* rhs, T* e, double* rc, int zero_e, double* sumsq) {
  if ((reinterpret_cast<uintptr_t>(rhs) | reinterpret_cast<uintptr_t>(e)) % 16)
    return set_err(c, ISM_ERR_INVALID, "rhs and e must be 16-byte aligned");
  if (c->cfg.fused && c->cfg.nu > ism::fused_max_nu<T>())
    return set_err(c, ISM_ERR_UNSUPPORTED, "nu exceeds the fused kernel's limit for this dtype");
  T* tmp = (T*)scratch_fine(c);
  if (!tmp) return set_err(c, ISM_ERR_HIP, "hipMalloc of the stage scratch failed");
  T* cur = e;
  T* spare = tmp;
  int rcode = run_cycle<T>(c, rhs, &cur, &spare, rc, sumsq ? c->p_sq : nullptr, zero_e);
  if (rcode) return rcode;
  if (cur != e)
    HIPCHK(c, hipMemcpyAsync(e, cur, sizeof(T) * size_t(c->g.plane) * c->g.batch,
                             hipMemcpyDeviceToDevice, c->stream));
  if (sumsq)
    LAUNCH(c, ism::launch_finalize(c->p_sq, int(c->g.cplane), c->g.cplane, c->g.batch, ism::SUM, 1.0,
                                   sumsq, 1, 0, c->fin, c->stream));
  return ISM_OK;
}

}  // namespace

extern "C" {

int ism_smooth(ism_handle c, int32_t dtype, const void* rhs, void* e, int32_t nsweeps) {
  if (!c) return ISM_ERR_INVALID;
  if (!rhs || !e || nsweeps < 0) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  if (dtype == ISM_F32) return smooth_impl<float>(c, (const float*)rhs, (float*)e, nsweeps);
  if (dtype == ISM_F64) return smooth_impl<double>(c, (const double*)rhs, (double*)e, nsweeps);
  return set_err(c, ISM_ERR_INVALID, "dtype must be ISM_F32 or ISM_F64");
}

int ism_restrict(ism_handle c, int32_t dtype, const void* rhs, const void* e, double* rc, double* sumsq) {
  if (!c) return ISM_ERR_INVALID;
  if (!rhs || !e || !rc) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  double* psq = sumsq ? c->p_sq : nullptr;
  if (dtype == ISM_F32)
    LAUNCH(c, ism::launch_restrict<float>(c->g, (const float*)rhs, (const float*)e, rc, psq, c->stream));
  else if (dtype == ISM_F64)
    LAUNCH(c, ism::launch_restrict<double>(c->g, (const double*)rhs, (const double*)e, rc, psq, c->stream));
  else
    return set_err(c, ISM_ERR_INVALID, "dtype must be ISM_F32 or ISM_F64");
  if (sumsq)
    LAUNCH(c, ism::launch_finalize(c->p_sq, int(c->g.cplane), c->g.cplane, c->g.batch, ism::SUM, 1.0,
                                   sumsq, 1, 0, c->fin, c->stream));
  return ISM_OK;
}

int ism_prolong(ism_handle c, int32_t dtype, const double* E, void* e) {
  if (!c) return ISM_ERR_INVALID;
  if (!E || !e) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  if (dtype == ISM_F32) LAUNCH(c, ism::launch_prolong<float>(c->g, E, (float*)e, 0, c->stream));
  else if (dtype == ISM_F64) LAUNCH(c, ism::launch_prolong<double>(c->g, E, (double*)e, 0, c->stream));
  else return set_err(c, ISM_ERR_INVALID, "dtype must be ISM_F32 or ISM_F64");
  return ISM_OK;
}

int ism_coarse_solve(ism_handle c, const double* rc, double* E) {
  if (!c) return ISM_ERR_INVALID;
  if (!rc || !E) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  return coarse_solve(c, rc, E);
}

int ism_cycle(ism_handle c, int32_t dtype, const void* rhs, void* e, double* rc, int32_t zero_e,
              double* sumsq) {
  if (!c) return ISM_ERR_INVALID;
  if (c->cfg.coarse_stencil == ISM_COARSE_ACM)
    return set_err(c, ISM_ERR_UNSUPPORTED, "ism_cycle is the two-level cycle; an ACM handle has none");
  if (!rhs || !e || !rc) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  if (dtype == ISM_F32) return cycle_impl<float>(c, (const float*)rhs, (float*)e, rc, zero_e, sumsq);
  if (dtype == ISM_F64) return cycle_impl<double>(c, (const double*)rhs, (double*)e, rc, zero_e, sumsq);
  return set_err(c, ISM_ERR_INVALID, "dtype must be ISM_F32 or ISM_F64");
}

int ism_predict(ism_handle c, const double* u, const double* v, const double* p, double dt,
                double eta, const double* walls, double* us, double* vs) {
  if (!c) return ISM_ERR_INVALID;
  if (!u || !v || !p || !us || !vs) return set_err(c, ISM_ERR_INVALID, "NULL array");
  if (us == u || us == v || vs == u || vs == v)
    return set_err(c, ISM_ERR_INVALID, "the predicted faces must not alias the input faces");
  if (!std::isfinite(dt) || !std::isfinite(eta) || eta < 0.0)
    return set_err(c, ISM_ERR_INVALID, "dt must be finite and eta finite and >= 0");
  const double rest[4] = {0.0, 0.0, 0.0, 0.0};
  LAUNCH(c, ism::launch_predict(c->g, u, v, p, c->h, dt, eta, walls ? walls : rest, us, vs, c->stream));
  return ISM_OK;
}

int ism_correct(ism_handle c, const double* x, double* u, double* v, double* p) {
  if (!c) return ISM_ERR_INVALID;
  if (!x || !u || !v || !p) return set_err(c, ISM_ERR_INVALID, "NULL array");
  LAUNCH(c, ism::launch_correct(c->g, x, c->h, u, v, p, c->stream));
  return ISM_OK;
}

int ism_coarse_gs(ism_handle c, const double* rc, double* E, double tol, int32_t max_iter,
                  int32_t* iters) {
  if (!c) return ISM_ERR_INVALID;
  if (!rc || !E || !iters || !(tol >= 0.0) || max_iter < 0)
    return set_err(c, ISM_ERR_INVALID, "bad arguments");
  if (c->cfg.coarse_stencil == ISM_COARSE_ACM)
    return set_err(c, ISM_ERR_UNSUPPORTED, "no 9-point coarse stencil on an ACM handle");
  const size_t bytes = sizeof(double) * size_t(c->g.cplane) * c->g.batch;
  HIPCHK(c, hipMemcpyAsync(c->rc, rc, bytes, hipMemcpyDeviceToDevice, c->stream));
  int rcode;
  if (c->singular && (rcode = project_coarse(c, c->rc))) return rcode;
  double* out = nullptr;
  int it = 0;
  bool conv = false;
  int per = 1;
  if ((rcode = coarse_gs_loop(c, c->rc, tol, max_iter, &out, &it, &conv, &per))) return rcode;
  HIPCHK(c, hipMemcpyAsync(E, out, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *iters = it;
  return conv ? ISM_OK : ISM_NOT_CONVERGED;
}

int ism_coarse_stencil(ism_handle c, double* coef) {
  if (!c) return ISM_ERR_INVALID;
  if (!coef) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  LAUNCH(c, ism::launch_coarse_assemble(c->g, c->cfg.coarse_stencil == ISM_COARSE_GMG5, coef, c->stream));
  return ISM_OK;
}

int ism_outer_residual(ism_handle c, const double* b, const double* x, double* r) {
  if (!c) return ISM_ERR_INVALID;
  if (!b || !x || !r) return set_err(c, ISM_ERR_INVALID, "bad arguments");
  int rcode = mean_of_b(c, b);
  if (rcode) return rcode;
  Partials p{nullptr, nullptr, nullptr, nullptr};
  LAUNCH(c, ism::launch_outer_residual<double>(c->g, b, x, c->scal + size_t(MEAN_B) * c->g.batch, c->h2,
                                               r, nullptr, p, c->stream));
  return ISM_OK;
}

int ism_profile(ism_handle c, int32_t enable) {
  if (!c) return ISM_ERR_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  for (int k = 0; k < ISM_KERNEL_CLASSES; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  if (enable < 0) return set_err(c, ISM_ERR_INVALID, "enable must be >= 0");
  for (int k = 0; k < ISM_KERNEL_CLASSES; ++k) c->prof_seen[k] = 0;
  c->prof = enable != 0;
  c->prof_every = enable > 0 ? enable : 1;
  return ISM_OK;
}

int ism_profile_read(ism_handle c, int32_t kind, double* total_ms, int64_t* launches) {
  if (!c) return ISM_ERR_INVALID;
  if (kind < 0 || kind >= ISM_KERNEL_CLASSES || !total_ms || !launches)
    return set_err(c, ISM_ERR_INVALID, "bad kernel class or NULL output");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  *total_ms = c->prof_ms[kind];
  *launches = c->prof_n[kind];
  return ISM_OK;
}

const char* ism_status_string(int status) {
  switch (status) {
    case ISM_OK: return "ok";
    case ISM_NOT_CONVERGED: return "not converged";
    case ISM_ERR_INVALID: return "invalid argument";
    case ISM_ERR_UNSUPPORTED: return "unsupported configuration";
    case ISM_ERR_HIP: return "HIP runtime error";
    case ISM_ERR_NONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

const char* ism_last_error(ism_handle c) { return c ? c->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
