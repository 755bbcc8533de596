// HAMLET library for gfx950: plan set-up, pass orchestration and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hamlet.h"
#include "common.hpp"
#include "fft.hpp"
#include "analysis.hpp"
#include "flat.hpp"
#include "passes.hpp"
#include "galaxies.hpp"
#include "hmc.hpp"
#include "nuts.hpp"
#include "workspace.hpp"

using namespace hamlet;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static hamlet_status fail(hamlet_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(HAMLET_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK()                                                                            \
  do {                                                                                            \
    hipError_t e_ = hipGetLastError();                                                            \
    if (e_ != hipSuccess) return fail(HAMLET_EDEVICE, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// The plan
// ---------------------------------------------------------------------------
struct hamlet_plan;

// A shared launch: up to kMaxBatch plans of one grid size and precision,
// each with its mode for this launch, on the stream of the first plan.
struct Batch {
  hipStream_t stream = nullptr;
  int count = 0;
  hamlet_plan* plan[kMaxBatch] = {};
  int8_t mode[kMaxBatch] = {};
  double plane_scale = 1.0;   // kXGrad: factor on the kz = 0 plane of the gradient
  bool chain = false;         // first steps: trajectories of chains (momenta drawn here, start kept)
  // the plans' modes, momenta and cached gradients are chain states, which
  // the FP32 path stores in complex64 (FP64 plans ignore it)
  bool chain_state = false;
};

// Launch sequences and workspace layout, one instantiation per (precision, N).
struct Ops {
  hamlet_status (*eval)(const Batch&);       // one evaluation, per-plan modes
  hamlet_status (*start)(const Batch&);      // trajectory start: step, momenta, K0, saved state
  hamlet_status (*first)(const Batch&);      // first half kick and drift, inverse pass 1
  hamlet_status (*end)(const Batch&);        // trajectory end: K1, Metropolis test, restore, sum
  hamlet_status (*leap_out)(const Batch&);   // Psi of a leapfrog end point to the caller
  size_t (*bytes)(int n_gal, int n_hist);    // workspace size
  void (*locate)(hamlet_plan*);              // host copies of the workspace addresses it needs
  hamlet_status (*field)(const Batch&, void*);    // the velocity field of the plan's modes, to the caller
  hamlet_status (*density)(const Batch&, void*);  // the density contrast of the plan's modes, to the caller
  hamlet_status (*stats)(const Batch&, double*);  // delta, v_r and their squares added to running sums
  hamlet_status (*nuts_start)(const Batch&);      // NUTS: momenta r0 (st.p, st.pd, st.ps) and K0
  hamlet_status (*kin1)(const Batch&);            // kinetic energy after a trajectory's last step -> K1
};

struct hamlet_plan {
  int device = 0;                  // the HIP device the plan was created on
  int n = 0, prec = 0, n_gal = 0, sample_d = 1, sample_s = 1, sample_c = 0, n_hist = 0;
  double box = 0, om = 0, h = 0, f = 0, sigma_v = 0, hist_w = 5.0, minv_d = 0;
  double minv_u8 = 0, minv_phi = 0, minv_eta = 0;
  hipStream_t stream = nullptr;
  hipEvent_t order_ev = nullptr;   // orders shared launches against this plan's stream
  char* base = nullptr;            // the workspace (one allocation)
  size_t bytes = 0;
  StateDev st{};                   // what the current call works on
  // workspace addresses used by the host
  PlanConst* consts = nullptr;
  ChainScalars* cs = nullptr;
  double *var = nullptr, *mvar = nullptr, *hist = nullptr, *mom_part = nullptr, *wtab = nullptr;
  void* tw = nullptr;
  double *rhat = nullptr, *mu = nullptr, *smu = nullptr, *cz = nullptr, *scz = nullptr;
  int *count = nullptr, *off = nullptr, *most = nullptr;
  double2* gcache = nullptr;
  double2* pm = nullptr;
  float2* qc = nullptr;            // a chain's complex64 modes (FP32 plans), else nullptr
  double *gd = nullptr, *qd0 = nullptr, *pd = nullptr, *ps = nullptr, *eps_slot = nullptr, *dz = nullptr;
  bool pooled = false;             // workspace from the stream-ordered pool
  int n_prior_part = 0, n_like_part = 0, n_kin_part = 0;
  bool chain_ready = false;        // chain state and cached gradient valid (resume)
  struct NutsMem* nuts = nullptr;  // buffers of the No-U-Turn sampler (first hamlet_nuts_run)
  const Ops* ops = nullptr;
  // event timing of one kernel kind (hamlet_profile_start / stop)
  int prof_kind = -1;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pool;
  size_t prof_used = 0;
  bool prof_failed = false;
  size_t modes_count() const { return (size_t)n * n * (n / 2); }
  int n_small() const { return sample_c ? kSmallMax : 1; }   // s, and u8, phi, eta when sampled
};

// Bracket one launch of kernel kind `kind` with events when it is armed on
// the first plan of the batch (events go to the batch's stream).
static void prof_before(const Batch& b, int kind) {
  hamlet_plan* pl = b.plan[0];
  if (pl->prof_kind != kind) return;
  if (pl->prof_used == pl->prof_pool.size()) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      pl->prof_failed = true;
      pl->prof_kind = -1;
      return;
    }
    pl->prof_pool.emplace_back(e0, e1);
  }
  if (hipEventRecord(pl->prof_pool[pl->prof_used].first, b.stream) != hipSuccess) pl->prof_failed = true;
}
static void prof_after(const Batch& b, int kind) {
  hamlet_plan* pl = b.plan[0];
  if (pl->prof_kind != kind) return;
  if (hipEventRecord(pl->prof_pool[pl->prof_used].second, b.stream) != hipSuccess) pl->prof_failed = true;
  ++pl->prof_used;
}
#define TIMED(b, kind, ...)   \
  do {                        \
    prof_before(b, kind);     \
    __VA_ARGS__;              \
    prof_after(b, kind);      \
  } while (0)

static inline unsigned blocks_for(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Argument table of a batch; `force` >= kXSkip replaces every plan's mode.
constexpr int kOwnModes = -100;
static Launch launch_table(const Batch& b, int force = kOwnModes) {
  Launch L;
  for (int i = 0; i < kMaxBatch; ++i) {
    const bool in = i < b.count;
    const hamlet_plan* p = b.plan[in ? i : 0];
    L.base[i] = p->base;
    L.n_gal[i] = p->n_gal;
    L.mode[i] = in ? (force == kOwnModes ? b.mode[i] : force) : kXSkip;
    L.st[i] = p->st;
  }
  return L;
}

// Largest catalogue among the plans of a batch that take part.
static int batch_max_gal(const Batch& b) {
  int m = 0;
  for (int i = 0; i < b.count; ++i)
    if (b.mode[i] != kXSkip) m = std::max(m, b.plan[i]->n_gal);
  return m;
}

static bool batch_has(const Batch& b, int mode) {
  for (int i = 0; i < b.count; ++i)
    if (b.mode[i] == mode) return true;
  return false;
}

// Chain states in complex64: the FP32 path's chains (kS32<T> is true only
// for float, so no such variant of the FP64 kernels is built).
template <typename T> constexpr bool kS32 = sizeof(T) == 4;
template <typename T> static bool chain_f32(const Batch& b) { return kS32<T> && b.chain_state; }

// The x passes of an evaluation (gradient, middle or last leapfrog step).
template <typename T, int N, bool S32>
static void x_passes(const Batch& b, const Launch& sel, dim3 g_xy) {
  using TH = PassThreads<T, N>;
  hipStream_t st = b.stream;
  if (batch_has(b, kXGrad))
    TIMED(b, HAMLET_K_FWD_X, (k_x_pass<T, N, kXGrad, TH::X, false, S32><<<g_xy, TH::X, 0, st>>>(sel, b.plane_scale)));
  if (batch_has(b, kXMid))
    TIMED(b, HAMLET_K_FWD_X, (k_x_pass<T, N, kXMid, TH::X, false, S32><<<g_xy, TH::X, 0, st>>>(sel, 1.0)));
  if (batch_has(b, kXLast))
    TIMED(b, HAMLET_K_FWD_X, (k_x_pass<T, N, kXLast, TH::X, false, S32><<<g_xy, TH::X, 0, st>>>(sel, 1.0)));
}

// One log-posterior-and-gradient evaluation of every plan of the batch:
// bin, inverse passes with the gather, likelihood, final sums (Psi,
// dPsi/ds), forward passes with the scatter, and the x pass (gradient, or
// the fused leapfrog update and the next evaluation's inverse pass 1).
template <typename T, int N>
static hamlet_status eval_impl(const Batch& b) {
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  using SL = XSlabs<N>;
  if (b.count <= 0) return HAMLET_OK;
  hipStream_t st = b.stream;
  const Launch sel = launch_table(b);
  const unsigned nb = (unsigned)b.count;
  const int ng = batch_max_gal(b);
  if (ng > 0) {
    constexpr unsigned tiles = (N * N + kScanTile - 1) / kScanTile;
    const dim3 g_gal(blocks_for(ng, kGalThreads), 1, nb);
    prof_before(b, HAMLET_K_BIN);
    // points are counted here only before a plain gradient; inside a
    // trajectory the drifting kernels binned them already
    if (batch_has(b, kXGrad)) {
      Batch grad = b;
      for (int i = 0; i < b.count; ++i)
        if (grad.mode[i] != kXGrad) grad.mode[i] = kXSkip;
      k_bin_count<T, N><<<g_gal, kGalThreads, 0, st>>>(launch_table(grad));
    }
    k_bin_scan<T, N><<<dim3(tiles, 1, nb), kScanTile, 0, st>>>(sel);
    k_bin_place<T, N><<<g_gal, kGalThreads, 0, st>>>(sel);
    k_bin_rank<T, N><<<g_gal, kGalThreads, 0, st>>>(sel);
    prof_after(b, HAMLET_K_BIN);
    LAUNCH_CHECK();
  }
  const dim3 g_xy(S::CHUNKS, N, nb);
  const dim3 g_xy_slab(S::CHUNKS, SL::SIZE, nb), g_z_slab(N / S::P, SL::SIZE, nb), g_zg_slab(N / S::PG, SL::SIZE, nb);
  if (batch_has(b, kXGrad)) {
    if (chain_f32<T>(b))
      TIMED(b, HAMLET_K_INV_X, (k_inv_x<T, N, TH::XY, kS32<T>><<<g_xy, TH::XY, 0, st>>>(sel)));
    else
      TIMED(b, HAMLET_K_INV_X, (k_inv_x<T, N, TH::XY><<<g_xy, TH::XY, 0, st>>>(sel)));
  }
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    TIMED(b, HAMLET_K_INV_Y, (k_inv_y<T, N, TH::XY><<<g_xy_slab, TH::XY, 0, st>>>(sel, x0)));
    TIMED(b, HAMLET_K_INV_Z, (k_inv_z_gather<T, N, TH::ZG><<<g_zg_slab, TH::ZG, 0, st>>>(sel, x0)));
  }
  LAUNCH_CHECK();
  if (ng > 0) {
    TIMED(b, HAMLET_K_LIKE, (k_like<T, N><<<dim3(blocks_for(ng, kLikeThreads), 1, nb), kLikeThreads, 0, st>>>(sel)));
    LAUNCH_CHECK();
  }
  // plans without points still need their final sums (prior only)
  Batch empty = b;
  bool any_empty = false;
  for (int i = 0; i < b.count; ++i) {
    if (b.plan[i]->n_gal > 0) empty.mode[i] = kXSkip;
    any_empty = any_empty || empty.mode[i] != kXSkip;
  }
  if (any_empty) k_finalize<T, N><<<dim3(1, 1, nb), 256, 0, st>>>(launch_table(empty));
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    TIMED(b, HAMLET_K_FWD_Z, (k_fwd_z_scatter<T, N, TH::ZS><<<g_z_slab, TH::ZS, 0, st>>>(sel, x0)));
    TIMED(b, HAMLET_K_FWD_Y, (k_fwd_y<T, N, TH::XY><<<g_xy_slab, TH::XY, 0, st>>>(sel, x0)));
  }
  if (chain_f32<T>(b))
    x_passes<T, N, kS32<T>>(b, sel, g_xy);
  else
    x_passes<T, N, false>(b, sel, g_xy);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// The velocity field of one plan's modes (st.q) on every grid node: the
// inverse passes of an evaluation with every row kept, the last one writing
// the real field instead of gathering.
template <typename T, int N>
static hamlet_status field_impl(const Batch& b, void* out) {
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  using SL = XSlabs<N>;
  hipStream_t st = b.stream;
  const Launch sel = launch_table(b);
  const unsigned nb = (unsigned)b.count;
  k_inv_x<T, N, TH::XY><<<dim3(S::CHUNKS, N, nb), TH::XY, 0, st>>>(sel);
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    k_inv_y_all<T, N, TH::XY><<<dim3(S::CHUNKS, SL::SIZE, nb), TH::XY, 0, st>>>(sel, x0);
    k_inv_z_field<T, N, TH::ZG><<<dim3(N / S::PG, SL::SIZE, nb), TH::ZG, 0, st>>>(sel, x0, (T*)out);
  }
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// The density contrast of one plan's modes on every grid node: the same
// passes with q / N^3 for the velocity multiplier, the third array written.
template <typename T, int N>
static hamlet_status density_impl(const Batch& b, void* out) {
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  using SL = XSlabs<N>;
  hipStream_t st = b.stream;
  const Launch sel = launch_table(b);
  const unsigned nb = (unsigned)b.count;
  k_inv_x_density<T, N, TH::XY><<<dim3(S::CHUNKS, N, nb), TH::XY, 0, st>>>(sel);
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    k_inv_y_all<T, N, TH::XY><<<dim3(S::CHUNKS, SL::SIZE, nb), TH::XY, 0, st>>>(sel, x0);
    k_inv_z_field<T, N, TH::ZG, true><<<dim3(N / S::PG, SL::SIZE, nb), TH::ZG, 0, st>>>(sel, x0, (T*)out);
  }
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// One state's delta and radial velocity added to the caller's running sums
// acc = [sum delta, sum delta^2, sum v_r, sum v_r^2] (N^3 each): the passes
// of the velocity field, then those of the density contrast, each ending in
// a z pass that adds instead of storing.
template <typename T, int N>
static hamlet_status stats_impl(const Batch& b, double* acc) {
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  using SL = XSlabs<N>;
  constexpr size_t kGrid = (size_t)N * N * N;
  hipStream_t st = b.stream;
  const Launch sel = launch_table(b);
  const unsigned nb = (unsigned)b.count;
  k_inv_x<T, N, TH::XY><<<dim3(S::CHUNKS, N, nb), TH::XY, 0, st>>>(sel);
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    k_inv_y_all<T, N, TH::XY><<<dim3(S::CHUNKS, SL::SIZE, nb), TH::XY, 0, st>>>(sel, x0);
    k_inv_z_acc<T, N, TH::ZG, false><<<dim3(N / S::PG, SL::SIZE, nb), TH::ZG, 0, st>>>(sel, x0, acc + 2 * kGrid);
  }
  k_inv_x_density<T, N, TH::XY><<<dim3(S::CHUNKS, N, nb), TH::XY, 0, st>>>(sel);
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    k_inv_y_all<T, N, TH::XY><<<dim3(S::CHUNKS, SL::SIZE, nb), TH::XY, 0, st>>>(sel, x0);
    k_inv_z_acc<T, N, TH::ZG, true><<<dim3(N / S::PG, SL::SIZE, nb), TH::ZG, 0, st>>>(sel, x0, acc);
  }
  LAUNCH_CHECK();
  return HAMLET_OK;
}

static int batch_gal_or_one(const Batch& b) {
  int m = 1;
  for (int i = 0; i < b.count; ++i) m = std::max(m, b.plan[i]->n_gal);
  return m;
}

// Start of a trajectory of every plan of the batch: the iteration's step,
// fresh momenta of the distances and s, their saved values and their part of
// K0 (the mode momenta, their part of K0 and the saved modes come with the
// first step).
template <typename T, int N>
static hamlet_status start_impl(const Batch& b) {
  if (b.count <= 0) return HAMLET_OK;
  const Launch sel = launch_table(b, 0);
  const unsigned nb = (unsigned)b.count;
  k_iter_begin<T, N><<<dim3(1, 1, nb), 64, 0, b.stream>>>(sel);
  k_momenta_small<T, N><<<dim3(FixedLayout<N, sizeof(T)>::N_KIN_SMALL, 1, nb), kEltThreads, 0, b.stream>>>(sel);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// First step of a trajectory: half kick from the cached gradient and drift
// of every coordinate, then inverse pass 1 of the new modes.
template <typename T, int N>
static hamlet_status first_impl(const Batch& b) {
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  if (b.count <= 0) return HAMLET_OK;
  const Launch sel = launch_table(b, kXFirst);
  const unsigned nb = (unsigned)b.count;
  k_small_kick_drift<T, N><<<dim3(blocks_for(batch_gal_or_one(b), kEltThreads), 1, nb), kEltThreads, 0, b.stream>>>(
      sel);
  if (b.chain) {
    // a chain's trajectory: the pass also draws the mode momenta, keeps the
    // start point and sums the mode part of K0, which is completed here
    if (chain_f32<T>(b))
      TIMED(b, HAMLET_K_FWD_X, (k_x_pass<T, N, kXFirst, TH::X, true, kS32<T>>
                                <<<dim3(S::CHUNKS, N, nb), TH::X, 0, b.stream>>>(sel, 1.0)));
    else
      TIMED(b, HAMLET_K_FWD_X,
            (k_x_pass<T, N, kXFirst, TH::X, true><<<dim3(S::CHUNKS, N, nb), TH::X, 0, b.stream>>>(sel, 1.0)));
    k_kinetic_final<T, N><<<dim3(1, 1, nb), 256, 0, b.stream>>>(sel, 0);
  } else {
    TIMED(b, HAMLET_K_FWD_X,
          (k_x_pass<T, N, kXFirst, TH::X><<<dim3(S::CHUNKS, N, nb), TH::X, 0, b.stream>>>(sel, 1.0)));
  }
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// End of a trajectory: K1, Metropolis-Hastings test and step adaptation,
// restore on rejection, running sum of the post-warm-up samples.
template <typename T, int N>
static hamlet_status end_impl(const Batch& b) {
  if (b.count <= 0) return HAMLET_OK;
  const Launch sel = launch_table(b, 0);
  const unsigned nb = (unsigned)b.count;
  const size_t nm = (size_t)N * N * (N / 2);
  // K1 of the plans whose trajectory had steps (its last x pass summed the
  // mode part); a trajectory without steps keeps K1 = K0
  if (batch_has(b, kXLast)) {
    Batch moved = b;
    for (int i = 0; i < b.count; ++i)
      if (moved.mode[i] != kXLast) moved.mode[i] = kXSkip;
    const Launch kin = launch_table(moved);
    k_kinetic_small<T, N><<<dim3(FixedLayout<N, sizeof(T)>::N_KIN_SMALL, 1, nb), kEltThreads, 0, b.stream>>>(kin);
    k_kinetic_final<T, N><<<dim3(1, 1, nb), 256, 0, b.stream>>>(kin, 1);
  }
  k_accept<T, N><<<dim3(1, 1, nb), 64, 0, b.stream>>>(sel);
  const dim3 g_rest(blocks_for(std::max(nm, (size_t)batch_gal_or_one(b)), kEltThreads), 1, nb);
  if (chain_f32<T>(b))
    k_restore_accumulate<T, N, kS32<T>><<<g_rest, kEltThreads, 0, b.stream>>>(sel);
  else
    k_restore_accumulate<T, N><<<g_rest, kEltThreads, 0, b.stream>>>(sel);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// Start of a NUTS iteration: momenta r0 ~ N(0, M) of every coordinate into
// the state's momenta (st.p, st.pd, st.ps) and K0 = K(r0) into the chain
// scalars.
template <typename T, int N>
static hamlet_status nuts_start_impl(const Batch& b) {
  if (b.count <= 0) return HAMLET_OK;
  const Launch sel = launch_table(b, 0);
  const unsigned nb = (unsigned)b.count;
  using F = FixedLayout<N, sizeof(T)>;
  k_nuts_momenta<T, N><<<dim3(F::N_PRIOR, 1, nb), kEltThreads, 0, b.stream>>>(sel);
  k_momenta_small<T, N><<<dim3(F::N_KIN_SMALL, 1, nb), kEltThreads, 0, b.stream>>>(sel);
  k_kinetic_final<T, N><<<dim3(1, 1, nb), 256, 0, b.stream>>>(sel, 0);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// K1 after a trajectory's last step: the mode part summed by its x pass,
// the distances and s here.
template <typename T, int N>
static hamlet_status kin1_impl(const Batch& b) {
  if (b.count <= 0) return HAMLET_OK;
  const Launch sel = launch_table(b, 0);
  const unsigned nb = (unsigned)b.count;
  k_kinetic_small<T, N><<<dim3(FixedLayout<N, sizeof(T)>::N_KIN_SMALL, 1, nb), kEltThreads, 0, b.stream>>>(sel);
  k_kinetic_final<T, N><<<dim3(1, 1, nb), 256, 0, b.stream>>>(sel, 1);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

template <typename T, int N>
static hamlet_status leap_out_impl(const Batch& b) {
  if (b.count <= 0) return HAMLET_OK;
  k_leap_out<T, N><<<dim3(1, 1, (unsigned)b.count), 64, 0, b.stream>>>(launch_table(b, 0));
  LAUNCH_CHECK();
  return HAMLET_OK;
}

template <typename T, int N> static size_t bytes_impl(int n_gal, int n_hist) {
  return workspace_bytes<N, sizeof(T)>(n_gal, n_hist);
}

template <typename T, int N> static void locate_impl(hamlet_plan* pl) {
  using F = FixedLayout<N, sizeof(T)>;
  const Ws<T, N> w(pl->base, pl->n_gal);
  pl->consts = w.template at<PlanConst>(F::consts);
  pl->cs = w.template at<ChainScalars>(F::chain);
  pl->var = w.var_n2();
  pl->mvar = w.mvar();
  pl->mom_part = w.template at<double>(F::mom_part);
  pl->wtab = w.template at<double>(F::wtab);
  pl->hist = w.hist(pl->n_gal);
  pl->tw = w.tw();
  pl->rhat = w.rhat(); pl->mu = w.mu(); pl->smu = w.smu(); pl->cz = w.cz(); pl->scz = w.scz();
  pl->count = w.count();
  pl->off = w.off();
  pl->most = w.most();
  pl->gcache = w.gcache();
  pl->pm = w.pm();
  pl->qc = sizeof(T) == 4 ? w.qc() : nullptr;
  pl->gd = w.gd(); pl->qd0 = w.qd0(); pl->pd = w.pd(); pl->ps = w.ps(); pl->eps_slot = w.eps_slot();
  pl->dz = w.dz();
  pl->n_prior_part = F::N_PRIOR;
  pl->n_like_part = pl->n_gal > 0 ? (int)blocks_for(pl->n_gal, kLikeThreads) : 0;
  pl->n_kin_part = F::N_KIN;
}

template <typename T, int N> struct OpsFor {
  static constexpr Ops ops{eval_impl<T, N>,      start_impl<T, N>, first_impl<T, N>,  end_impl<T, N>,
                           leap_out_impl<T, N>,   bytes_impl<T, N>, locate_impl<T, N>, field_impl<T, N>,
                           density_impl<T, N>,    stats_impl<T, N>, nuts_start_impl<T, N>, kin1_impl<T, N>};
};

template <typename T, int N> static const Ops* ops_if_built() {
  if constexpr (has_grid(N)) return &OpsFor<T, N>::ops;
  else return nullptr;
}

template <typename T> static const Ops* pick_ops(int n) {
  switch (n) {
    case 16: return ops_if_built<T, 16>();
    case 32: return ops_if_built<T, 32>();
    case 64: return ops_if_built<T, 64>();
    case 128: return ops_if_built<T, 128>();
    case 256: return ops_if_built<T, 256>();
    case 512: return ops_if_built<T, 512>();
    case 1024: return ops_if_built<T, 1024>();
    default: return nullptr;
  }
}

// ---------------------------------------------------------------------------
// Host-side set-up
// ---------------------------------------------------------------------------
static hamlet_status check_desc(const hamlet_plan_desc* d) {
  if (!d) return fail(HAMLET_EINVAL, "desc is NULL");
  const int n = d->n_grid;
  if ((n != 16 && n != 32 && n != 64 && n != 128 && n != 256 && n != 512 && n != 1024) || !pick_ops<float>(n))
    return fail(HAMLET_EUNSUPPORTED, "n_grid %d: built for 16, 32, 64, 128, 256, 512, 1024", n);
  if (d->precision != HAMLET_FP64 && d->precision != HAMLET_FP32_FP64E)
    return fail(HAMLET_EINVAL, "precision %d", d->precision);
  if (!(d->box > 0) || !std::isfinite(d->box)) return fail(HAMLET_EINVAL, "box must be positive");
  if (!(d->omega_m > 0 && d->omega_m <= 1.0)) return fail(HAMLET_EINVAL, "omega_m must be in (0, 1]");
  if (!(d->h > 0) || !std::isfinite(d->h)) return fail(HAMLET_EINVAL, "h must be positive");
  if (!std::isfinite(d->f_growth)) return fail(HAMLET_EINVAL, "f_growth must be finite");
  if (!(d->sigma_v > 0) || !std::isfinite(d->sigma_v)) return fail(HAMLET_EINVAL, "sigma_v must be positive");
  const int64_t npk = 3 * (int64_t)(n / 2) * (n / 2) + 1;
  if (!d->pk_n2 || d->n_pk != npk) return fail(HAMLET_EINVAL, "pk_n2 needs %lld entries", (long long)npk);
  for (int64_t j = 0; j < npk; ++j)
    if (!(d->pk_n2[j] >= 0) || !std::isfinite(d->pk_n2[j])) return fail(HAMLET_EINVAL, "pk_n2[%lld] invalid", (long long)j);
  return HAMLET_OK;
}

static hamlet_status check_catalog(const hamlet_catalog* c) {
  if (!c) return fail(HAMLET_EINVAL, "catalog is NULL");
  if (c->n < 0 || c->n > (int64_t)(1 << 28)) return fail(HAMLET_EINVAL, "catalog size %lld", (long long)c->n);
  if (c->n == 0) return HAMLET_OK;
  if (!c->rhat || !c->mu || !c->sigma_mu || !c->cz || !c->sigma_cz) return fail(HAMLET_EINVAL, "catalog array is NULL");
  for (int64_t i = 0; i < c->n; ++i) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(c->rhat[3 * i + a])) return fail(HAMLET_EINVAL, "rhat[%lld] not finite", (long long)i);
    if (!std::isfinite(c->mu[i]) || !std::isfinite(c->cz[i])) return fail(HAMLET_EINVAL, "point %lld: mu/cz not finite", (long long)i);
    if (!(c->sigma_mu[i] > 0) || !std::isfinite(c->sigma_mu[i])) return fail(HAMLET_EINVAL, "point %lld: sigma_mu must be > 0", (long long)i);
    if (!(c->sigma_cz[i] >= 0) || !std::isfinite(c->sigma_cz[i])) return fail(HAMLET_EINVAL, "point %lld: sigma_cz must be >= 0", (long long)i);
  }
  return HAMLET_OK;
}

// Redshift distance of eq:e:dz by composite Simpson (2000 intervals).
static double redshift_distance(double z, double om) {
  const int m = 2000;
  const double hstep = z / m;
  double acc = 0.0;
  for (int j = 0; j <= m; ++j) {
    const double zz = hstep * j;
    const double coef = (j == 0 || j == m) ? 1.0 : (j % 2 ? 4.0 : 2.0);
    acc += coef / std::sqrt(om * (1.0 + zz) * (1.0 + zz) * (1.0 + zz) + (1.0 - om));
  }
  return (kC / kH0) * (hstep / 3.0) * acc;
}

// Number of distance-prior bins (eq:D): width w on [0, max d_z + 15).  d_z
// grows with z, so the largest redshift distance is that of the largest cz.
static int distance_prior_bins(const hamlet_catalog* c, double om, double w) {
  double top = 0.0;
  if (c->n > 0) {
    double zmax = c->cz[0];
    for (int64_t i = 1; i < c->n; ++i) zmax = std::max(zmax, c->cz[i]);
    top = std::max(0.0, redshift_distance(zmax / kC, om));
  }
  return (int)std::ceil((top + 15.0) / w);
}

// Host values an upload reads from; they must outlive the upload (the
// caller synchronises, or keeps them until the plan is done).
struct Staging {
  std::vector<double> var;
  std::vector<double> twd;
  std::vector<float> twf;
  PlanConst pc{};
};

// Enqueues the plan's set-up on its stream: tables, twiddles, catalogue,
// distance prior, constants.  Reads the catalogue arrays and `sg` until the
// stream reaches the end of the set-up.
// The x pass's tile width of a plan's grid and precision, in whose tiles
// sigma^2 is laid out (the schedule's W).
template <typename T> static int tile_width_of(int n) {
  switch (n) {
    case 16: return Sched<T, 16>::W;
    case 32: return Sched<T, 32>::W;
    case 64: return Sched<T, 64>::W;
    case 128: return Sched<T, 128>::W;
    case 256: return Sched<T, 256>::W;
    case 512: return Sched<T, 512>::W;
    default: return Sched<T, 1024>::W;
  }
}
static int scheduled_tile_width(int prec, int n) {
  return prec == HAMLET_FP64 ? tile_width_of<double>(n) : tile_width_of<float>(n);
}

static hamlet_status upload(hamlet_plan* pl, const hamlet_plan_desc* d, const hamlet_catalog* c, Staging& sg) {
  const int n = pl->n;
  const size_t npk = 3 * (size_t)(n / 2) * (n / 2) + 1;
  const double kf = 2.0 * M_PI / pl->box;
  const double n3 = (double)n * n * n;
  const double vol = pl->box * pl->box * pl->box;
  std::vector<double>& var = sg.var;
  var.resize(npk);
  for (size_t j = 0; j < npk; ++j) var[j] = n3 * n3 / vol * d->pk_n2[j];
  // Twiddles exp(-2 pi i m / N), computed in long double and rounded once.
  std::vector<double>& twd = sg.twd;
  std::vector<float>& twf = sg.twf;
  twd.resize(2 * n);
  twf.resize(2 * n);
  for (int m = 0; m < n; ++m) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * m / n;
    twd[2 * m] = (double)cosl(ang);
    twd[2 * m + 1] = (double)sinl(ang);
    twf[2 * m] = (float)cosl(ang);
    twf[2 * m + 1] = (float)sinl(ang);
  }
  hipStream_t st = pl->stream;
  HIP_TRY(hipMemcpyAsync(pl->var, var.data(), npk * 8, hipMemcpyHostToDevice, st));
  const int w = scheduled_tile_width(pl->prec, n);
  k_fill_mode_var<<<blocks_for(pl->modes_count(), kEltThreads), kEltThreads, 0, st>>>(pl->mvar, pl->var, n, w);
  LAUNCH_CHECK();
  if (pl->prec == HAMLET_FP64)
    HIP_TRY(hipMemcpyAsync(pl->tw, twd.data(), twd.size() * 8, hipMemcpyHostToDevice, st));
  else
    HIP_TRY(hipMemcpyAsync(pl->tw, twf.data(), twf.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(pl->hist, 0, (size_t)pl->n_hist * 8, st));
  if (c->n > 0) {
    HIP_TRY(hipMemcpyAsync(pl->rhat, c->rhat, 3 * c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->mu, c->mu, c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->smu, c->sigma_mu, c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->cz, c->cz, c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->scz, c->sigma_cz, c->n * 8, hipMemcpyHostToDevice, st));
    k_dist_prior_count<<<blocks_for(c->n, kGalThreads), kGalThreads, 0, st>>>(pl->cz, pl->n_gal, pl->om, pl->hist_w,
                                                                               pl->n_hist, pl->dz, pl->hist);
    LAUNCH_CHECK();
  }
  k_dist_prior_norm<<<blocks_for(pl->n_hist, kGalThreads), kGalThreads, 0, st>>>(pl->hist, pl->n_hist, pl->n_gal,
                                                                                 pl->hist_w);
  LAUNCH_CHECK();
  HIP_TRY(hipMemsetAsync(pl->count, 0, (size_t)n * n * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(pl->off, 0, ((size_t)n * n + 1) * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(pl->most, 0, 2 * sizeof(int), st));   // most crowded column, likelihood ticket
  PlanConst& pc = sg.pc;
  pc.n_gal = pl->n_gal;
  pc.n_hist = pl->n_hist;
  pc.sample_d = pl->sample_d;
  pc.sample_s = pl->sample_s;
  pc.n_prior_part = pl->n_prior_part;
  pc.n_like_part = pl->n_like_part;
  pc.n_kin_part = pl->n_kin_part;
  pc.om = pl->om;
  pc.h = pl->h;
  pc.box = pl->box;
  pc.spacing = pl->box / pl->n;
  pc.dmax = kC / (3.0 * pl->om * kH0);
  pc.hist_w = pl->hist_w;
  pc.minv_d = pl->minv_d;
  pc.psd = kH0 / pl->sigma_v;
  pc.kfac0 = kH0 * pl->f / ((double)pl->n * pl->n * pl->n * kf);
  pc.sample_c = pl->sample_c;
  pc.minv_u8 = pl->minv_u8;
  pc.minv_phi = pl->minv_phi;
  pc.minv_eta = pl->minv_eta;
  pc.d_modes = std::pow((double)(pl->n - 1), 3.0) - 1.0;
  HIP_TRY(hipMemcpyAsync(pl->consts, &pc, sizeof(pc), hipMemcpyHostToDevice, st));
  return HAMLET_OK;
}

static void fill_plan_scalars(hamlet_plan* pl, const hamlet_plan_desc* d, const hamlet_catalog* cat, int n_hist) {
  const int64_t n_gal = cat->n;
  pl->n = d->n_grid;
  pl->prec = d->precision;
  pl->box = d->box;
  pl->om = d->omega_m;
  pl->h = d->h;
  pl->f = d->f_growth;
  pl->sigma_v = d->sigma_v;
  pl->hist_w = d->hist_width > 0 ? d->hist_width : 5.0;
  pl->sample_d = d->sample_distances ? 1 : 0;
  pl->sample_s = d->sample_sigma_nl ? 1 : 0;
  pl->minv_d = pl->sample_d ? (pl->sigma_v / kH0) * (pl->sigma_v / kH0) : 0.0;
  pl->n_gal = (int)n_gal;
  pl->n_hist = n_hist;
  // u8 = sigma_8 / sigma_8,fid, phi = f / f_fid and eta = h / h_fid:
  // inverse masses 1 / (2 D) (the prior's curvature in u8 at u8 = 1, D real
  // mode coordinates), 1 / n, and the inverse curvature of the distance
  // modulus terms in eta at eta = 1, 1 / sum_i (5 / ln 10)^2 / sigma_mu,i^2
  pl->sample_c = d->sample_cosmology ? 1 : 0;
  const double dof = std::pow((double)(pl->n - 1), 3.0) - 1.0;
  pl->minv_u8 = pl->sample_c ? 1.0 / (2.0 * dof) : 0.0;
  pl->minv_phi = pl->sample_c ? 1.0 / (double)std::max<int64_t>(n_gal, 1) : 0.0;
  const double c5 = (5.0 / std::log(10.0)) * (5.0 / std::log(10.0));
  double curv = 0.0;
  for (int64_t i = 0; i < n_gal; ++i) curv += c5 / (cat->sigma_mu[i] * cat->sigma_mu[i]);
  pl->minv_eta = pl->sample_c ? (n_gal > 0 ? 1.0 / curv : 1.0) : 0.0;
}

// Upper bound of the histogram bin count for the footprint query: the
// redshift distance of cz is below c z / H0 (1 + z), take max cz unknown ->
// use a generous fixed bound.
static const int kFootprintHistBins = 4096;

extern "C" hamlet_status hamlet_plan_footprint_bytes(const hamlet_plan_desc* desc, int64_t n_gal, size_t* bytes) {
  hamlet_status st = check_desc(desc);
  if (st != HAMLET_OK) return st;
  if (!bytes) return fail(HAMLET_EINVAL, "bytes is NULL");
  if (n_gal < 0) return fail(HAMLET_EINVAL, "n_gal < 0");
  if (n_gal > (int64_t)(1 << 28)) return fail(HAMLET_EINVAL, "n_gal %lld", (long long)n_gal);
  const Ops* ops = desc->precision == HAMLET_FP64 ? pick_ops<double>(desc->n_grid) : pick_ops<float>(desc->n_grid);
  *bytes = ops->bytes((int)n_gal, kFootprintHistBins);
  return HAMLET_OK;
}

// Validates, allocates (from the stream-ordered pool when `pooled`) and
// enqueues the set-up of a plan on `stream`, without waiting for it.
static hamlet_status plan_make(const hamlet_plan_desc* desc, const hamlet_catalog* cat, hipStream_t stream,
                               bool pooled, Staging& sg, hamlet_plan** out) {
  if (!out) return fail(HAMLET_EINVAL, "out is NULL");
  *out = nullptr;
  hamlet_status st = check_desc(desc);
  if (st != HAMLET_OK) return st;
  st = check_catalog(cat);
  if (st != HAMLET_OK) return st;
  const double w = desc->hist_width > 0 ? desc->hist_width : 5.0;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(HAMLET_EDEVICE, "hipGetDevice failed");
  hamlet_plan* pl = new hamlet_plan();
  pl->device = device;
  fill_plan_scalars(pl, desc, cat, distance_prior_bins(cat, desc->omega_m, w));
  pl->stream = stream;
  pl->pooled = pooled;
  pl->ops = pl->prec == HAMLET_FP64 ? pick_ops<double>(pl->n) : pick_ops<float>(pl->n);
  if (hipEventCreateWithFlags(&pl->order_ev, hipEventDisableTiming) != hipSuccess) {
    delete pl;
    return fail(HAMLET_EDEVICE, "hipEventCreateWithFlags failed");
  }
  pl->bytes = pl->ops->bytes(pl->n_gal, pl->n_hist);
  const hipError_t e = pooled ? hipMallocAsync((void**)&pl->base, pl->bytes, stream)
                              : hipMalloc((void**)&pl->base, pl->bytes);
  if (e != hipSuccess) {
    (void)hipEventDestroy(pl->order_ev);
    const size_t bytes = pl->bytes;
    delete pl;
    return fail(HAMLET_ENOMEM, "allocation of %zu bytes failed", bytes);
  }
  pl->ops->locate(pl);
  st = upload(pl, desc, cat, sg);
  if (st != HAMLET_OK) {
    (void)hipStreamSynchronize(stream);
    (void)(pooled ? hipFreeAsync(pl->base, stream) : hipFree(pl->base));
    (void)hipEventDestroy(pl->order_ev);
    delete pl;
    return st;
  }
  *out = pl;
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_plan_create(const hamlet_plan_desc* desc, const hamlet_catalog* cat, void* stream,
                                            hamlet_plan** out) {
  Staging sg;
  hamlet_status st = plan_make(desc, cat, (hipStream_t)stream, false, sg, out);
  if (st != HAMLET_OK) return st;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
    hamlet_plan* pl = *out;
    *out = nullptr;
    (void)hipFree(pl->base);
    (void)hipEventDestroy(pl->order_ev);
    delete pl;
    return fail(HAMLET_EDEVICE, "plan set-up failed on the device");
  }
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// Device memory of a plan's No-U-Turn chain: the two ends of the trajectory
// (coordinates, momenta, gradient each), pools of kept coordinates (tree
// candidates and the first leaves of subtrees) and kept momenta, the dot
// products' partials and the values read back after each step.  A "set" is
// one state-shaped allocation: modes | distances | small coordinates.
// ---------------------------------------------------------------------------
struct NutsSet {
  double2* modes = nullptr;
  double* dist = nullptr;
  double* small = nullptr;
};

struct NutsMem {
  int depth = 0;                  // most doublings the pools serve
  size_t set_bytes = 0;
  char* base = nullptr;
  NutsSet end[2][3];              // [side: 0 = minus, 1 = plus][0 coordinates, 1 momenta, 2 gradient]
  std::vector<NutsSet> theta, mom;   // pools
  double* part = nullptr;         // dot partials: (depth + 1) slots x kNutsDotBlocks x 2
  double* back = nullptr;         // device: Psi, K0, K1, then 2 per dot slot
  double* host = nullptr;         // pinned copy of `back`
  size_t back_count = 0;
};

static size_t nuts_set_bytes(const hamlet_plan* pl) {
  return align256(16 * pl->modes_count()) + align256(8 * (size_t)std::max(pl->n_gal, 1)) + 256;
}

static NutsSet nuts_set_at(char* p, const hamlet_plan* pl) {
  NutsSet s;
  s.modes = (double2*)p;
  p += align256(16 * pl->modes_count());
  s.dist = (double*)p;
  p += align256(8 * (size_t)std::max(pl->n_gal, 1));
  s.small = (double*)p;
  return s;
}

static void nuts_free(hamlet_plan* pl) {
  if (!pl->nuts) return;
  if (pl->nuts->base) (void)hipFree(pl->nuts->base);
  if (pl->nuts->host) (void)hipHostFree(pl->nuts->host);
  delete pl->nuts;
  pl->nuts = nullptr;
}

extern "C" hamlet_status hamlet_plan_destroy(hamlet_plan* pl) {
  if (!pl) return HAMLET_OK;
  hipError_t e1 = hipStreamSynchronize(pl->stream);
  nuts_free(pl);
  for (auto& ev : pl->prof_pool) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  hipError_t e2 = pl->pooled ? hipFreeAsync(pl->base, pl->stream) : hipFree(pl->base);
  (void)hipEventDestroy(pl->order_ev);
  delete pl;
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(HAMLET_EDEVICE, "plan destroy: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  return HAMLET_OK;
}


// ---------------------------------------------------------------------------
// Batching: plans of one grid size and precision share launches
// ---------------------------------------------------------------------------
static hamlet_status check_plans(hamlet_plan* const* plans, int32_t n_plans) {
  if (!plans || n_plans <= 0) return fail(HAMLET_EINVAL, "need at least one plan");
  for (int j = 0; j < n_plans; ++j) {
    if (!plans[j]) return fail(HAMLET_EINVAL, "plans[%d] is NULL", j);
    for (int k = 0; k < j; ++k)
      if (plans[k] == plans[j]) return fail(HAMLET_EINVAL, "plans[%d] and plans[%d] are the same plan", k, j);
  }
  return HAMLET_OK;
}

// Plan indices grouped by (N, precision, extra key) in call order, at most
// kMaxBatch per group.
static std::vector<std::vector<int>> group_plans(hamlet_plan* const* plans, int32_t n_plans,
                                                 const int32_t* extra = nullptr) {
  std::vector<std::vector<int>> groups;
  for (int j = 0; j < n_plans; ++j) {
    const hamlet_plan* p = plans[j];
    int found = -1;
    for (int g = (int)groups.size() - 1; g >= 0; --g) {
      const int k = groups[g][0];
      const hamlet_plan* q = plans[k];
      if (q->n == p->n && q->prec == p->prec && (!extra || extra[k] == extra[j])) {
        if ((int)groups[g].size() < kMaxBatch) found = g;
        break;
      }
    }
    if (found < 0) {
      groups.emplace_back();
      found = (int)groups.size() - 1;
    }
    groups[found].push_back(j);
  }
  return groups;
}

// Side streams of a stream (per device): created on first use and kept for
// the life of the process, so that no call waits for a stream to drain
// before destroying it.  Default priority, non-blocking.
static hipStream_t side_stream(hipStream_t main, int k) {
  static std::mutex mu;
  static std::map<std::tuple<int, hipStream_t, int>, hipStream_t> sides;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, main, k);
  auto it = sides.find(key);
  if (it != sides.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  sides.emplace(key, s);
  return s;
}

// The stream each group of one call runs on.  Groups are independent (no
// plan is in two of them), so when several groups share their first plan's
// stream, every group after the first on it runs on a side stream of that
// stream, and the groups' launches can run side by side (a bandwidth-bound
// 256^3 group leaves room for the small launches of a 64^3 one).  Without a
// side stream the group runs on the shared stream, in call order.
static std::vector<hipStream_t> group_streams(hamlet_plan* const* plans, const std::vector<std::vector<int>>& groups) {
  std::vector<hipStream_t> out;
  std::map<hipStream_t, int> used;
  for (const std::vector<int>& g : groups) {
    hipStream_t s = plans[g[0]]->stream;
    const int k = used[s]++;
    hipStream_t side = k > 0 ? side_stream(s, k) : nullptr;
    out.push_back(side ? side : s);
  }
  return out;
}

// A group's launches go to its stream `run` (see group_streams); every
// plan's stream is ordered before (join) and after (release) them with
// events.
static hamlet_status streams_join(hamlet_plan* const* plans, const std::vector<int>& g, hipStream_t run) {
  for (int j : g) {
    hamlet_plan* p = plans[j];
    if (p->stream == run) continue;
    HIP_TRY(hipEventRecord(p->order_ev, p->stream));
    HIP_TRY(hipStreamWaitEvent(run, p->order_ev, 0));
  }
  return HAMLET_OK;
}

static hamlet_status streams_release(hamlet_plan* const* plans, const std::vector<int>& g, hipStream_t run) {
  hamlet_plan* p0 = plans[g[0]];
  bool recorded = false;
  for (int j : g) {
    hamlet_plan* p = plans[j];
    if (p->stream == run) continue;
    if (!recorded) {
      HIP_TRY(hipEventRecord(p0->order_ev, run));
      recorded = true;
    }
    HIP_TRY(hipStreamWaitEvent(p->stream, p0->order_ev, 0));
  }
  return HAMLET_OK;
}

static Batch make_batch(hamlet_plan* const* plans, const std::vector<int>& g, int mode, hipStream_t run) {
  Batch b;
  b.stream = run;
  b.count = (int)g.size();
  for (int i = 0; i < b.count; ++i) {
    b.plan[i] = plans[g[i]];
    b.mode[i] = (int8_t)mode;
  }
  return b;
}

static void batch_add(Batch& b, hamlet_plan* pl, int mode) {
  b.plan[b.count] = pl;
  b.mode[b.count] = (int8_t)mode;
  ++b.count;
}

static void batch_set_modes(Batch& b, int mode) {
  for (int i = 0; i < b.count; ++i) b.mode[i] = (int8_t)mode;
}

// ---------------------------------------------------------------------------
// Chains advanced one leapfrog step (one evaluation) per tick
// ---------------------------------------------------------------------------
// A chain's schedule: one plain gradient at the start point (unless resumed
// with a valid cached gradient), then per iteration a trajectory of L
// evaluations (eq:hamilton, kick-drift-kick): the tick of its first step
// also refreshes the momenta and does the first half kick and drift; the
// tick of its last step ends with the Metropolis-Hastings test (Section
// 3.2).  Chains of one group at different points of their schedules share
// the tick's launches.
struct ChainRun {
  hamlet_plan* pl = nullptr;
  int L = 0;             // leapfrog steps per trajectory
  int todo = 0;          // iterations to run
  int iter = 0;          // iterations done
  int step = 0;          // evaluations done in the current trajectory
  bool need_grad = false;
  bool active() const { return need_grad || iter < todo; }
};

// The modes of an FP32 plan's chain into its complex64 state, and back
// (only the retained modes are written back).
static hamlet_status chain_modes_in(const hamlet_plan* pl, const double2* q, hipStream_t s) {
  const size_t nm = pl->modes_count();
  k_modes_narrow<<<blocks_for(nm, kEltThreads), kEltThreads, 0, s>>>(q, pl->qc, nm);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

static hamlet_status chain_modes_out(const hamlet_plan* pl, double2* q, hipStream_t s) {
  k_modes_widen<<<blocks_for(pl->modes_count(), kEltThreads), kEltThreads, 0, s>>>(pl->qc, q, pl->n);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

static hamlet_status tick_group(hipStream_t stream, const std::vector<ChainRun*>& runs) {
  Batch start, first, eval, end;
  start.stream = first.stream = eval.stream = end.stream = stream;
  first.chain = true;
  start.chain_state = first.chain_state = eval.chain_state = end.chain_state = true;
  const Ops* ops = nullptr;
  for (ChainRun* r : runs) {
    if (!r->active()) continue;
    ops = r->pl->ops;
    if (r->need_grad) {
      batch_add(eval, r->pl, kXGrad);
      continue;
    }
    const bool ending = r->L == 0 || r->step + 1 == r->L;
    if (r->step == 0) {
      batch_add(start, r->pl, 0);
      if (r->L > 0) batch_add(first, r->pl, kXFirst);
    }
    if (r->L > 0) batch_add(eval, r->pl, ending ? kXLast : kXMid);
    if (ending) batch_add(end, r->pl, r->L > 0 ? kXLast : kXGrad);
  }
  if (!ops) return HAMLET_OK;
  hamlet_status s = ops->start(start);
  if (s == HAMLET_OK) s = ops->first(first);
  if (s == HAMLET_OK) s = ops->eval(eval);
  if (s == HAMLET_OK) s = ops->end(end);
  if (s != HAMLET_OK) return s;
  for (ChainRun* r : runs) {
    if (!r->active()) continue;
    if (r->need_grad) {
      r->need_grad = false;
    } else if (r->L == 0 || r->step + 1 == r->L) {
      r->step = 0;
      ++r->iter;
    } else {
      ++r->step;
    }
  }
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// Entry points
// ---------------------------------------------------------------------------
static hamlet_status logpost_grad_impl(hamlet_plan* const* plans, int32_t n_plans, const void* const* q_modes,
                                       const double* const* q_dist, const double* const* q_snl,
                                       void* const* g_modes, double* const* g_dist, double* const* g_snl,
                                       double* const* psi, double plane_scale) {
  hamlet_status st = check_plans(plans, n_plans);
  if (st != HAMLET_OK) return st;
  if (!q_modes || !q_snl || !g_modes || !g_snl || !psi) return fail(HAMLET_EINVAL, "NULL argument array");
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    if (!q_modes[j] || !g_modes[j] || !q_snl[j] || !g_snl[j] || !psi[j])
      return fail(HAMLET_EINVAL, "plan %d: NULL buffer", j);
    if (pl->n_gal > 0 && (!q_dist || !g_dist || !q_dist[j] || !g_dist[j]))
      return fail(HAMLET_EINVAL, "plan %d: NULL distance buffer", j);
  }
  const std::vector<std::vector<int>> groups = group_plans(plans, n_plans);
  const std::vector<hipStream_t> runs = group_streams(plans, groups);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int>& g = groups[gi];
    if ((st = streams_join(plans, g, runs[gi])) != HAMLET_OK) return st;
    Batch b = make_batch(plans, g, kXGrad, runs[gi]);
    b.plane_scale = plane_scale;
    for (int j : g) {
      hamlet_plan* pl = plans[j];
      StateDev sd{};
      sd.q = (double2*)q_modes[j];
      sd.qd = pl->n_gal ? (double*)q_dist[j] : pl->qd0;
      sd.qs = (double*)q_snl[j];
      sd.g = (double2*)g_modes[j];
      sd.gd = pl->n_gal ? g_dist[j] : pl->gd;
      sd.gs = g_snl[j];
      sd.psi = psi[j];
      pl->st = sd;
    }
    if ((st = b.plan[0]->ops->eval(b)) != HAMLET_OK) return st;
    if ((st = streams_release(plans, g, runs[gi])) != HAMLET_OK) return st;
  }
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_logpost_grad(hamlet_plan* const* plans, int32_t n_plans,
                                             const void* const* q_modes, const double* const* q_dist,
                                             const double* const* q_snl, void* const* g_modes,
                                             double* const* g_dist, double* const* g_snl, double* const* psi) {
  return logpost_grad_impl(plans, n_plans, q_modes, q_dist, q_snl, g_modes, g_dist, g_snl, psi, 1.0);
}

extern "C" hamlet_status hamlet_logpost_grad_entries(hamlet_plan* const* plans, int32_t n_plans,
                                                     const void* const* q_modes, const double* const* q_dist,
                                                     const double* const* q_snl, void* const* g_modes,
                                                     double* const* g_dist, double* const* g_snl,
                                                     double* const* psi) {
  return logpost_grad_impl(plans, n_plans, q_modes, q_dist, q_snl, g_modes, g_dist, g_snl, psi, 0.5);
}

extern "C" hamlet_status hamlet_leapfrog(hamlet_plan* const* plans, int32_t n_plans, const double* eps,
                                         const int32_t* n_steps, void* const* q_modes, double* const* q_dist,
                                         double* const* q_snl, void* const* p_modes, double* const* p_dist,
                                         double* const* p_snl, double* const* psi) {
  hamlet_status st = check_plans(plans, n_plans);
  if (st != HAMLET_OK) return st;
  if (!eps || !n_steps || !q_modes || !q_snl || !p_modes || !p_snl || !psi)
    return fail(HAMLET_EINVAL, "NULL argument array");
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    if (n_steps[j] < 0) return fail(HAMLET_EINVAL, "plan %d: n_steps < 0", j);
    if (!std::isfinite(eps[j])) return fail(HAMLET_EINVAL, "plan %d: eps not finite", j);
    if (!q_modes[j] || !p_modes[j] || !q_snl[j] || !p_snl[j] || !psi[j])
      return fail(HAMLET_EINVAL, "plan %d: NULL buffer", j);
    if (pl->n_gal > 0 && (!q_dist || !p_dist || !q_dist[j] || !p_dist[j]))
      return fail(HAMLET_EINVAL, "plan %d: NULL distance buffer", j);
  }
  const std::vector<std::vector<int>> groups = group_plans(plans, n_plans, n_steps);
  const std::vector<hipStream_t> runs = group_streams(plans, groups);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int>& g = groups[gi];
    if ((st = streams_join(plans, g, runs[gi])) != HAMLET_OK) return st;
    Batch b = make_batch(plans, g, kXGrad, runs[gi]);
    for (int j : g) {
      hamlet_plan* pl = plans[j];
      StateDev sd{};
      sd.q = (double2*)q_modes[j];
      sd.qd = pl->n_gal ? q_dist[j] : pl->qd0;
      sd.qs = q_snl[j];
      sd.p = (double2*)p_modes[j];
      sd.pd = pl->n_gal ? p_dist[j] : pl->pd;
      sd.ps = p_snl[j];
      sd.g = pl->gcache;
      sd.gd = pl->gd;
      sd.gs = &pl->cs->gs[0];
      sd.psi = &pl->cs->psi;
      sd.eps = pl->eps_slot;
      sd.psi_out = psi[j];
      pl->st = sd;
      k_set_scalar<<<1, 64, 0, b.stream>>>(pl->eps_slot, eps[j]);
      LAUNCH_CHECK();
      pl->chain_ready = false;   // the cached gradient now belongs to this call
    }
    const Ops* ops = b.plan[0]->ops;
    const int steps = n_steps[g[0]];
    if ((st = ops->eval(b)) != HAMLET_OK) return st;   // gradient at the start point
    if (steps > 0) {
      if ((st = ops->first(b)) != HAMLET_OK) return st;
      for (int k = 1; k <= steps; ++k) {
        batch_set_modes(b, k < steps ? kXMid : kXLast);
        if ((st = ops->eval(b)) != HAMLET_OK) return st;
      }
    }
    if ((st = ops->leap_out(b)) != HAMLET_OK) return st;
    if ((st = streams_release(plans, g, runs[gi])) != HAMLET_OK) return st;
  }
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_hmc_run(hamlet_plan* const* plans, int32_t n_plans, const hamlet_hmc_opts* o,
                                        void* const* q_modes, double* const* q_dist, double* const* q_snl,
                                        void* const* mode_sum, double* const* dh, int32_t* const* accepted,
                                        double* eps_out) {
  hamlet_status st = check_plans(plans, n_plans);
  if (st != HAMLET_OK) return st;
  if (!o) return fail(HAMLET_EINVAL, "opts is NULL");
  if (o->n_iter < 0 || o->n_leapfrog < 0 || o->warmup < 0)
    return fail(HAMLET_EINVAL, "n_iter/n_leapfrog/warmup out of range");
  if (!(o->eps0 > 0) || !std::isfinite(o->eps0)) return fail(HAMLET_EINVAL, "eps0 must be positive");
  if (!(o->target_accept > 0 && o->target_accept < 1)) return fail(HAMLET_EINVAL, "target_accept must be in (0,1)");
  if (!q_modes || !q_snl) return fail(HAMLET_EINVAL, "NULL argument array");
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    if (!q_modes[j] || !q_snl[j]) return fail(HAMLET_EINVAL, "plan %d: NULL buffer", j);
    if (pl->n_gal > 0 && (!q_dist || !q_dist[j])) return fail(HAMLET_EINVAL, "plan %d: NULL distance buffer", j);
  }
  const std::vector<std::vector<int>> groups = group_plans(plans, n_plans);
  const std::vector<hipStream_t> gstream = group_streams(plans, groups);
  std::vector<ChainRun> runs(n_plans);
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int>& g = groups[gi];
    if ((st = streams_join(plans, g, gstream[gi])) != HAMLET_OK) return st;
    hipStream_t s0 = gstream[gi];
    for (int j : g) {
      hamlet_plan* pl = plans[j];
      StateDev sd{};
      sd.q = (double2*)q_modes[j];
      if (pl->qc) {
        // the FP32 path's chain runs on complex64 modes
        if ((st = chain_modes_in(pl, (const double2*)q_modes[j], s0)) != HAMLET_OK) return st;
        sd.q = (double2*)pl->qc;
      }
      sd.qd = pl->n_gal ? q_dist[j] : pl->qd0;
      sd.qs = q_snl[j];
      sd.p = pl->pm;
      sd.pd = pl->pd;
      sd.ps = pl->ps;
      sd.g = pl->gcache;
      sd.gd = pl->gd;
      sd.gs = &pl->cs->gs[0];
      sd.psi = &pl->cs->psi;
      sd.eps = &pl->cs->eps_it;
      sd.dh = dh ? dh[j] : nullptr;
      sd.acc = accepted ? accepted[j] : nullptr;
      sd.msum = mode_sum ? (double2*)mode_sum[j] : nullptr;
      pl->st = sd;
      ChainRun& r = runs[j];
      r.pl = pl;
      r.L = o->n_leapfrog;
      r.todo = o->n_iter;
      r.need_grad = !(o->resume && pl->chain_ready);
      if (r.need_grad) {
        const uint64_t seed = o->seeds ? o->seeds[j] : o->seed + (uint64_t)j;
        k_chain_init<<<1, 1, 0, s0>>>(pl->cs, o->eps0, o->target_accept, seed, o->warmup, o->jitter_eps);
        LAUNCH_CHECK();
      }
    }
  }
  std::vector<std::vector<ChainRun*>> group_runs(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi)
    for (int j : groups[gi]) group_runs[gi].push_back(&runs[j]);
  for (;;) {
    bool any = false;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      bool act = false;
      for (ChainRun* r : group_runs[gi]) act = act || r->active();
      if (!act) continue;
      any = true;
      if ((st = tick_group(gstream[gi], group_runs[gi])) != HAMLET_OK) return st;
    }
    if (!any) break;
  }
  for (int j = 0; j < n_plans; ++j) plans[j]->chain_ready = true;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int>& g = groups[gi];
    for (int j : g)
      if (plans[j]->qc && (st = chain_modes_out(plans[j], (double2*)q_modes[j], gstream[gi])) != HAMLET_OK) return st;
    if (eps_out) {
      hipStream_t s0 = gstream[gi];
      for (int j : g) HIP_TRY(hipMemcpyAsync(&eps_out[j], &plans[j]->cs->eps, sizeof(double), hipMemcpyDeviceToHost, s0));
      HIP_TRY(hipStreamSynchronize(s0));
    }
    if ((st = streams_release(plans, g, gstream[gi])) != HAMLET_OK) return st;
  }
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// The No-U-Turn sampler (Section 3.3: Hoffman & Gelman's efficient NUTS with
// slice variable and dual averaging)
//
// The host builds each chain's tree in the order of the recursive algorithm
// (a stack of completed first halves per height replaces the recursion); the
// device does every leapfrog step (the fused passes, one step per tick, in
// shared launches across chains), the kinetic energies and the dot products
// of the no-U-turn tests.  The trajectory's two ends are advanced in place;
// a leaf that the tree still needs later (a subtree's first leaf, a
// candidate sample) is written out by the first pass of the next step from
// that end, which reads it anyway.  Every decision takes its uniform from the
// counter-based stream: direction of doubling j, merge of a subtree's halves,
// move to a new subtree's sample, slice variable.
// ---------------------------------------------------------------------------
constexpr double kNutsDeltaMax = 1000.0;
constexpr int kNutsMaxDepth = 12;

static double host_uniform(uint64_t seed, int iteration, uint32_t purpose, uint64_t index) {
  const Philox4 w = draw_words(seed, (uint32_t)iteration, purpose, index);
  return uniform53(w.v[0], w.v[1]);
}

static hamlet_status nuts_alloc(hamlet_plan* pl, int depth) {
  if (pl->nuts && pl->nuts->depth >= depth) return HAMLET_OK;
  HIP_TRY(hipStreamSynchronize(pl->stream));
  nuts_free(pl);
  std::unique_ptr<NutsMem> m(new NutsMem());
  m->depth = depth;
  m->set_bytes = nuts_set_bytes(pl);
  const int n_theta = 2 * depth + 4, n_mom = depth + 2;
  const size_t sets = 6 + (size_t)n_theta + (size_t)n_mom;
  const size_t part_bytes = align256(8 * 2 * (size_t)kNutsDotBlocks * (depth + 1));
  m->back_count = 3 + 2 * (size_t)(depth + 1);
  const size_t total = sets * m->set_bytes + part_bytes + align256(8 * m->back_count);
  if (hipMalloc((void**)&m->base, total) != hipSuccess) return fail(HAMLET_ENOMEM, "NUTS buffers: %zu bytes", total);
  if (hipHostMalloc((void**)&m->host, 8 * m->back_count, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(m->base);
    return fail(HAMLET_ENOMEM, "NUTS read-back buffer");
  }
  char* p = m->base;
  for (int side = 0; side < 2; ++side)
    for (int k = 0; k < 3; ++k, p += m->set_bytes) m->end[side][k] = nuts_set_at(p, pl);
  for (int k = 0; k < n_theta; ++k, p += m->set_bytes) m->theta.push_back(nuts_set_at(p, pl));
  for (int k = 0; k < n_mom; ++k, p += m->set_bytes) m->mom.push_back(nuts_set_at(p, pl));
  m->part = (double*)p;
  p += part_bytes;
  m->back = (double*)p;
  if (hipMemsetAsync(m->base, 0, sets * m->set_bytes, pl->stream) != hipSuccess) {
    (void)hipFree(m->base);
    (void)hipHostFree(m->host);
    return fail(HAMLET_EDEVICE, "NUTS buffers: clear failed");
  }
  pl->nuts = m.release();
  return HAMLET_OK;
}

// A reference to a kept state: the chain's own state (the start of the
// iteration), the current state of one end, or a pool set.
enum NRefKind : int8_t { kRefNone = 0, kRefStart = 1, kRefEnd = 2, kRefPool = 3 };
struct NRef {
  int8_t kind = kRefNone;
  int idx = 0;
};

// A completed subtree: its sample, counts, subtree test, acceptance sums and
// where its sample's leaf sits (doubling, position).
struct NutsNode {
  NRef cand;
  int n = 0, s = 1, n_alpha = 0, wj = -1, wt = 0;
  double alpha = 0.0;
};

struct NutsChain {
  hamlet_plan* pl = nullptr;
  double2* q = nullptr;           // the chain's state (caller's buffers)
  double* qd = nullptr;
  double* qs = nullptr;
  double2* msum = nullptr;
  int32_t *o_depth = nullptr, *o_leaves = nullptr, *o_where = nullptr;
  double* o_alpha = nullptr;
  uint64_t seed = 0;
  int n_iter = 0, warmup = 0, max_depth = 10;
  // dual averaging (Hoffman & Gelman) of the step
  double eps = 0.0, target = 0.65, da_mu = 0.0, da_hbar = 0.0, da_leb = 0.0, da_m = 0.0;
  // the iteration
  int it = 0, phase = 0;          // phase 0: start of an iteration, 1: building the tree
  double h0 = 0.0, ln_u = 0.0;
  int n_top = 1, j = 0, v = 1, t = 0, leaves = 0, n_alpha = 0;
  double alpha = 0.0;
  NRef sample;
  int swj = -1, swt = 0;
  NutsNode stack[kNutsMaxDepth];            // completed first halves, by height
  NRef first_q[kNutsMaxDepth + 1], first_p[kNutsMaxDepth + 1];   // first leaf of the node being built, by height
  std::vector<int> rc_theta, rc_mom;        // reference counts of the pool sets
  bool done() const { return it >= n_iter; }
};

static void nref_release(NutsChain& c, NRef& r, bool mom) {
  if (r.kind == kRefPool) --(mom ? c.rc_mom : c.rc_theta)[r.idx];
  r = NRef{};
}

static void nref_copy(NutsChain& c, NRef& dst, const NRef& src, bool mom) {
  nref_release(c, dst, mom);
  dst = src;
  if (dst.kind == kRefPool) ++(mom ? c.rc_mom : c.rc_theta)[dst.idx];
}

static int nuts_pool_take(std::vector<int>& rc) {
  for (size_t k = 0; k < rc.size(); ++k)
    if (rc[k] == 0) return (int)k;
  return -1;
}

// Every reference to the current state of end `side` is moved to a pool set
// (into which the next step from that end writes the state); returns the
// pool sets (-1: none needed) for the coordinates and the momenta.
static hamlet_status nuts_keep_end(NutsChain& c, int side, int* theta, int* mom) {
  *theta = *mom = -1;
  auto move = [&](NRef& r, bool is_mom, int* slot) -> hamlet_status {
    if (r.kind != kRefEnd || r.idx != side) return HAMLET_OK;
    std::vector<int>& rc = is_mom ? c.rc_mom : c.rc_theta;
    if (*slot < 0) {
      *slot = nuts_pool_take(rc);
      if (*slot < 0) return fail(HAMLET_EDEVICE, "NUTS %s pool exhausted", is_mom ? "momentum" : "state");
    }
    r.kind = kRefPool;
    r.idx = *slot;
    ++rc[*slot];
    return HAMLET_OK;
  };
  hamlet_status st = move(c.sample, false, theta);
  for (int h = 0; h < kNutsMaxDepth && st == HAMLET_OK; ++h) st = move(c.stack[h].cand, false, theta);
  for (int h = 0; h <= kNutsMaxDepth && st == HAMLET_OK; ++h) {
    st = move(c.first_q[h], false, theta);
    if (st == HAMLET_OK) st = move(c.first_p[h], true, mom);
  }
  return st;
}

static void nuts_clear_doubling(NutsChain& c) {
  for (int h = 0; h < kNutsMaxDepth; ++h) {
    nref_release(c, c.stack[h].cand, false);
    c.stack[h] = NutsNode{};
  }
  for (int h = 0; h <= kNutsMaxDepth; ++h) {
    nref_release(c, c.first_q[h], false);
    nref_release(c, c.first_p[h], true);
  }
}

static void nuts_new_doubling(NutsChain& c) {
  nuts_clear_doubling(c);
  c.v = host_uniform(c.seed, c.it, kPurposeNutsDir, (uint64_t)c.j) <= 0.5 ? -1 : 1;
  c.t = 0;
}

static hamlet_status copy_async(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0 || dst == src) return HAMLET_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
  return HAMLET_OK;
}

// Copies the coordinates (modes, distances, s) of one state to another.
static hamlet_status copy_state(const hamlet_plan* pl, double2* dq, double* dd, double* ds, const double2* sq,
                                const double* sd, const double* ss, hipStream_t st) {
  hamlet_status r = copy_async(dq, sq, 16 * pl->modes_count(), st);
  if (r == HAMLET_OK && pl->n_gal > 0) r = copy_async(dd, sd, 8 * (size_t)pl->n_gal, st);
  if (r == HAMLET_OK) r = copy_async(ds, ss, 8 * (size_t)pl->n_small(), st);
  return r;
}

static hamlet_status copy_set(const hamlet_plan* pl, const NutsSet& d, const NutsSet& s, hipStream_t st) {
  return copy_state(pl, d.modes, d.dist, d.small, s.modes, s.dist, s.small, st);
}

// The coordinates a reference points to.
static NutsSet nuts_ref_set(const NutsChain& c, const NRef& r) {
  const NutsMem* m = c.pl->nuts;
  if (r.kind == kRefEnd) return m->end[r.idx][0];
  if (r.kind == kRefPool) return m->theta[r.idx];
  NutsSet s;
  s.modes = c.q;
  s.dist = c.pl->n_gal ? c.qd : m->end[0][0].dist;
  s.small = c.qs;
  return s;
}

template <int N> static void nuts_dot_launch(const NutsDotArgs& a, hipStream_t st) {
  if constexpr (has_grid(N)) k_nuts_dot<N><<<kNutsDotBlocks, kEltThreads, 0, st>>>(a);
}

static hamlet_status nuts_dot(const hamlet_plan* pl, const NutsSet& qa, const NutsSet& qb, const NutsSet& ra,
                              const NutsSet& rb, int slot, hipStream_t st) {
  NutsDotArgs a;
  a.qa = qa.modes; a.qb = qb.modes; a.ra = ra.modes; a.rb = rb.modes;
  a.da = qa.dist; a.db = qb.dist; a.pda = ra.dist; a.pdb = rb.dist;
  a.sa = qa.small; a.sb = qb.small; a.psa = ra.small; a.psb = rb.small;
  a.n_gal = pl->n_gal;
  a.use_d = pl->sample_d && pl->n_gal > 0;
  a.use_s = pl->sample_s;
  a.use_c = pl->sample_c;
  a.part = pl->nuts->part + (size_t)slot * 2 * kNutsDotBlocks;
  a.out = pl->nuts->back + 3 + 2 * slot;
  switch (pl->n) {
    case 16: nuts_dot_launch<16>(a, st); break;
    case 32: nuts_dot_launch<32>(a, st); break;
    case 64: nuts_dot_launch<64>(a, st); break;
    case 128: nuts_dot_launch<128>(a, st); break;
    case 256: nuts_dot_launch<256>(a, st); break;
    case 512: nuts_dot_launch<512>(a, st); break;
    case 1024: nuts_dot_launch<1024>(a, st); break;
    default: return fail(HAMLET_EUNSUPPORTED, "grid size %d", pl->n);
  }
  k_nuts_dot_final<<<1, 256, 0, st>>>(a.part, kNutsDotBlocks, a.out);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// Enqueues one tick of a group's chains: the start of an iteration (the
// gradient at the chain's state, both ends set to it, momenta, K0) or one
// leapfrog step from the end being extended (K1, and the dot products of
// the no-U-turn tests that end at the new leaf); then the read-back.
static hamlet_status nuts_enqueue(hipStream_t st, const std::vector<NutsChain*>& chains) {
  Batch first, eval, start, kin;
  first.stream = eval.stream = start.stream = kin.stream = st;
  const Ops* ops = nullptr;
  hamlet_status r = HAMLET_OK;
  for (NutsChain* c : chains) {
    if (c->done()) continue;
    hamlet_plan* pl = c->pl;
    NutsMem* m = pl->nuts;
    ops = pl->ops;
    StateDev sd{};
    sd.psi = &pl->cs->psi;
    sd.eps = pl->eps_slot;
    if (c->phase == 0) {
      k_set_chain_iter<<<1, 64, 0, st>>>(pl->cs, c->it);
      const NutsSet& e = m->end[0][0];
      if ((r = copy_state(pl, e.modes, e.dist, e.small, c->q, c->qd, c->qs, st)) != HAMLET_OK) return r;
      sd.q = e.modes; sd.qd = e.dist; sd.qs = e.small;
      sd.p = m->end[0][1].modes; sd.pd = m->end[0][1].dist; sd.ps = m->end[0][1].small;
      sd.g = m->end[0][2].modes; sd.gd = m->end[0][2].dist; sd.gs = m->end[0][2].small;
      pl->st = sd;
      batch_add(eval, pl, kXGrad);
      batch_add(start, pl, 0);
    } else {
      const int side = c->v < 0 ? 0 : 1;
      if (c->t == 0) k_set_scalar<<<1, 64, 0, st>>>(pl->eps_slot, (double)c->v * c->eps);
      int kt = -1, kp = -1;
      if ((r = nuts_keep_end(*c, side, &kt, &kp)) != HAMLET_OK) return r;
      const NutsSet *E = m->end[side];
      sd.q = E[0].modes; sd.qd = E[0].dist; sd.qs = E[0].small;
      sd.p = E[1].modes; sd.pd = E[1].dist; sd.ps = E[1].small;
      sd.g = E[2].modes; sd.gd = E[2].dist; sd.gs = E[2].small;
      if (kt >= 0) {
        sd.sv_q = m->theta[kt].modes; sd.sv_qd = m->theta[kt].dist; sd.sv_qs = m->theta[kt].small;
      }
      if (kp >= 0) {
        sd.sv_p = m->mom[kp].modes; sd.sv_pd = m->mom[kp].dist; sd.sv_ps = m->mom[kp].small;
      }
      pl->st = sd;
      batch_add(first, pl, kXFirst);
      batch_add(eval, pl, kXLast);
      batch_add(kin, pl, 0);
    }
  }
  if (!ops) return HAMLET_OK;
  if ((r = ops->first(first)) != HAMLET_OK) return r;
  if ((r = ops->eval(eval)) != HAMLET_OK) return r;
  // both ends of a new trajectory start at the chain's state, with its gradient
  for (NutsChain* c : chains) {
    if (c->done() || c->phase != 0) continue;
    const NutsMem* m = c->pl->nuts;
    if ((r = copy_set(c->pl, m->end[1][0], m->end[0][0], st)) != HAMLET_OK) return r;
    if ((r = copy_set(c->pl, m->end[1][2], m->end[0][2], st)) != HAMLET_OK) return r;
  }
  if ((r = ops->nuts_start(start)) != HAMLET_OK) return r;
  if ((r = ops->kin1(kin)) != HAMLET_OK) return r;
  for (NutsChain* c : chains) {
    if (c->done()) continue;
    hamlet_plan* pl = c->pl;
    NutsMem* m = pl->nuts;
    if (c->phase == 0) {
      if ((r = copy_set(pl, m->end[1][1], m->end[0][1], st)) != HAMLET_OK) return r;
    } else {
      const int side = c->v < 0 ? 0 : 1;
      // the nodes of height h >= 1 that the new leaf completes: their first
      // leaf (kept in the pools) against the leaf, now the end's state
      for (int h = 1; h <= c->j && ((c->t + 1) & ((1 << h) - 1)) == 0; ++h) {
        const NRef& fq = c->first_q[h];
        const NRef& fp = c->first_p[h];
        if (fq.kind != kRefPool || fp.kind != kRefPool) return fail(HAMLET_EDEVICE, "NUTS: first leaf not kept");
        if ((r = nuts_dot(pl, m->theta[fq.idx], m->end[side][0], m->mom[fp.idx], m->end[side][1], h - 1, st)) !=
            HAMLET_OK)
          return r;
      }
      // the doubling's last leaf: the test over the whole trajectory
      if (c->t + 1 == (1 << c->j)) {
        if ((r = nuts_dot(pl, m->end[0][0], m->end[1][0], m->end[0][1], m->end[1][1], m->depth, st)) != HAMLET_OK)
          return r;
      }
    }
    k_nuts_collect<<<1, 64, 0, st>>>(pl->cs, m->back);
    HIP_TRY(hipMemcpyAsync(m->host, m->back, 8 * m->back_count, hipMemcpyDeviceToHost, st));
  }
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// End of an iteration: the sample becomes the chain's state (and enters the
// running sum past warm-up), the outputs are recorded, the step is adapted.
static hamlet_status nuts_end_iteration(NutsChain& c, hipStream_t st) {
  hamlet_plan* pl = c.pl;
  if (c.sample.kind != kRefStart) {
    const NutsSet s = nuts_ref_set(c, c.sample);
    hamlet_status r = copy_state(pl, c.q, c.qd, c.qs, s.modes, s.dist, s.small, st);
    if (r != HAMLET_OK) return r;
  }
  if (c.msum && c.it >= c.warmup) {
    const size_t nm = pl->modes_count();
    k_add_modes<<<(unsigned)std::min<size_t>(blocks_for(nm, kEltThreads), 4096), kEltThreads, 0, st>>>(c.msum, c.q, nm);
    LAUNCH_CHECK();
  }
  const double stat = c.alpha / (double)c.n_alpha;
  if (c.o_depth) c.o_depth[c.it] = c.j;
  if (c.o_leaves) c.o_leaves[c.it] = c.leaves;
  if (c.o_where) {
    c.o_where[2 * c.it] = c.swj;
    c.o_where[2 * c.it + 1] = c.swt;
  }
  if (c.o_alpha) c.o_alpha[c.it] = stat;
  if (c.it < c.warmup) {
    // Hoffman & Gelman's dual averaging (gamma 0.05, t0 10, kappa 0.75)
    c.da_m += 1.0;
    const double m = c.da_m;
    const double eta = 1.0 / (m + 10.0);
    c.da_hbar = (1.0 - eta) * c.da_hbar + eta * (c.target - stat);
    const double log_eps = c.da_mu - std::sqrt(m) / 0.05 * c.da_hbar;
    const double wgt = std::pow(m, -0.75);
    c.da_leb = wgt * log_eps + (1.0 - wgt) * c.da_leb;
    c.eps = c.it == c.warmup - 1 ? std::exp(c.da_leb) : std::exp(log_eps);
  }
  nuts_clear_doubling(c);
  nref_release(c, c.sample, false);
  ++c.it;
  c.phase = 0;
  return HAMLET_OK;
}

// The read-back of a leaf: slice and divergence tests, the merges of the
// subtrees it completes (with their no-U-turn tests), and at the end of a
// doubling the move to its sample and the test over the whole trajectory.
static hamlet_status nuts_leaf(NutsChain& c, const double* back, hipStream_t st) {
  const int j = c.j, t = c.t, v = c.v, side = v < 0 ? 0 : 1;
  double H = back[0] + back[2];
  if (!std::isfinite(H)) H = HUGE_VAL;
  ++c.leaves;
  NutsNode cur;
  cur.cand.kind = kRefEnd;
  cur.cand.idx = side;
  cur.n = c.ln_u <= -H ? 1 : 0;
  cur.s = c.ln_u < kNutsDeltaMax - H ? 1 : 0;
  cur.alpha = std::isfinite(H) ? std::min(1.0, std::exp(c.h0 - H)) : 0.0;
  cur.n_alpha = 1;
  cur.wj = j;
  cur.wt = t;
  // the first leaf of the nodes that start here (heights 1 .. trailing zeros of t)
  if (j >= 1 && (t & 1) == 0) {
    int hf = j;
    if (t != 0) {
      hf = 0;
      while (((t >> hf) & 1) == 0) ++hf;
    }
    NRef eq, ep;
    eq.kind = ep.kind = kRefEnd;
    eq.idx = ep.idx = side;
    for (int h = 1; h <= hf && h <= j; ++h) {
      nref_copy(c, c.first_q[h], eq, false);
      nref_copy(c, c.first_p[h], ep, true);
    }
  }
  int h = 0;
  bool pushed = false, failed = cur.s == 0;
  while (!failed && h < j) {
    const int k = t >> h;
    if ((k & 1) == 0) {             // a first half: it waits for its sibling
      c.stack[h] = cur;
      pushed = true;
      break;
    }
    NutsNode left = c.stack[h];
    c.stack[h] = NutsNode{};
    const double u = host_uniform(c.seed, c.it, kPurposeNutsMerge,
                                  ((uint64_t)(j * 16 + h + 1) << 32) | (uint64_t)(k >> 1));
    const bool right = cur.n > 0 && u * (double)(left.n + cur.n) <= (double)cur.n;
    NutsNode mg = left;
    if (right) {
      nref_release(c, mg.cand, false);
      mg.cand = cur.cand;
      mg.wj = cur.wj;
      mg.wt = cur.wt;
    } else {
      nref_release(c, cur.cand, false);
    }
    mg.n = left.n + cur.n;
    mg.alpha = left.alpha + cur.alpha;
    mg.n_alpha = left.n_alpha + cur.n_alpha;
    const double* d = back + 3 + 2 * h;
    const int ok = ((double)v * d[0] >= 0.0 && (double)v * d[1] >= 0.0) ? 1 : 0;
    mg.s = cur.s * ok;
    nref_release(c, c.first_q[h + 1], false);
    nref_release(c, c.first_p[h + 1], true);
    cur = mg;
    ++h;
    failed = cur.s == 0;
  }
  if (pushed) {
    ++c.t;
    return HAMLET_OK;
  }
  if (failed) {
    // the recursion returns from here: a second half adds its sums to its
    // first half's, a first half returns alone
    for (; h < j; ++h) {
      if (((t >> h) & 1) != 0) {
        cur.alpha = c.stack[h].alpha + cur.alpha;
        cur.n_alpha = c.stack[h].n_alpha + cur.n_alpha;
      }
    }
  }
  // the doubling is done: move to its sample with probability min(1, n'/n)
  if (!failed && cur.n > 0 &&
      host_uniform(c.seed, c.it, kPurposeNutsTop, (uint64_t)j) * (double)c.n_top <= (double)cur.n) {
    nref_release(c, c.sample, false);
    c.sample = cur.cand;
    cur.cand = NRef{};
    c.swj = cur.wj;
    c.swt = cur.wt;
  }
  nref_release(c, cur.cand, false);
  c.n_top += cur.n;
  c.alpha += cur.alpha;
  c.n_alpha += cur.n_alpha;
  int s_top = 0;
  if (!failed) {
    const double* d = back + 3 + 2 * c.pl->nuts->depth;
    s_top = (d[0] >= 0.0 && d[1] >= 0.0) ? 1 : 0;
  }
  ++c.j;
  if (s_top && c.j < c.max_depth) {
    nuts_new_doubling(c);
    return HAMLET_OK;
  }
  return nuts_end_iteration(c, st);
}

static hamlet_status nuts_finish(hipStream_t st, const std::vector<NutsChain*>& chains) {
  HIP_TRY(hipStreamSynchronize(st));
  for (NutsChain* c : chains) {
    if (c->done()) continue;
    const double* back = c->pl->nuts->host;
    if (c->phase == 0) {
      // H0 = Psi + K(r0); slice variable ln u = ln U - H0
      c->h0 = back[0] + back[1];
      c->ln_u = std::log(host_uniform(c->seed, c->it, kPurposeAccept, 0)) - c->h0;
      c->n_top = 1;
      c->j = 0;
      c->leaves = 0;
      c->alpha = 0.0;
      c->n_alpha = 0;
      c->sample = NRef{};
      c->sample.kind = kRefStart;
      c->swj = -1;
      c->swt = 0;
      c->phase = 1;
      nuts_new_doubling(*c);
    } else {
      hamlet_status r = nuts_leaf(*c, back, st);
      if (r != HAMLET_OK) return r;
    }
  }
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_nuts_run(hamlet_plan* const* plans, int32_t n_plans, const hamlet_nuts_opts* o,
                                         void* const* q_modes, double* const* q_dist, double* const* q_snl,
                                         void* const* mode_sum, int32_t* const* depth, int32_t* const* n_leapfrog,
                                         int32_t* const* leaf, double* const* accept_stat, double* eps_out) {
  hamlet_status st = check_plans(plans, n_plans);
  if (st != HAMLET_OK) return st;
  if (!o) return fail(HAMLET_EINVAL, "opts is NULL");
  if (o->n_iter < 0 || o->warmup < 0) return fail(HAMLET_EINVAL, "n_iter/warmup out of range");
  if (o->max_depth < 1 || o->max_depth > kNutsMaxDepth)
    return fail(HAMLET_EINVAL, "max_depth %d outside [1, %d]", (int)o->max_depth, kNutsMaxDepth);
  if (!(o->eps0 > 0) || !std::isfinite(o->eps0)) return fail(HAMLET_EINVAL, "eps0 must be positive");
  if (!(o->target_accept > 0 && o->target_accept < 1)) return fail(HAMLET_EINVAL, "target_accept must be in (0,1)");
  if (!q_modes || !q_snl) return fail(HAMLET_EINVAL, "NULL argument array");
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    if (!q_modes[j] || !q_snl[j]) return fail(HAMLET_EINVAL, "plan %d: NULL buffer", j);
    if (pl->n_gal > 0 && (!q_dist || !q_dist[j])) return fail(HAMLET_EINVAL, "plan %d: NULL distance buffer", j);
  }
  for (int j = 0; j < n_plans; ++j)
    if ((st = nuts_alloc(plans[j], o->max_depth)) != HAMLET_OK) return st;
  const std::vector<std::vector<int>> groups = group_plans(plans, n_plans);
  const std::vector<hipStream_t> gstream = group_streams(plans, groups);
  std::vector<NutsChain> chains(n_plans);
  std::vector<std::vector<NutsChain*>> gch(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    if ((st = streams_join(plans, groups[gi], gstream[gi])) != HAMLET_OK) return st;
    for (int j : groups[gi]) {
      hamlet_plan* pl = plans[j];
      NutsChain& c = chains[j];
      c.pl = pl;
      c.q = (double2*)q_modes[j];
      c.qd = pl->n_gal ? q_dist[j] : nullptr;
      c.qs = q_snl[j];
      c.msum = mode_sum ? (double2*)mode_sum[j] : nullptr;
      c.o_depth = depth ? depth[j] : nullptr;
      c.o_leaves = n_leapfrog ? n_leapfrog[j] : nullptr;
      c.o_where = leaf ? leaf[j] : nullptr;
      c.o_alpha = accept_stat ? accept_stat[j] : nullptr;
      c.seed = o->seeds ? o->seeds[j] : o->seed + (uint64_t)j;
      c.n_iter = o->n_iter;
      c.warmup = o->warmup;
      c.max_depth = o->max_depth;
      c.eps = o->eps0;
      c.target = o->target_accept;
      c.da_mu = std::log(10.0 * o->eps0);
      c.rc_theta.assign(pl->nuts->theta.size(), 0);
      c.rc_mom.assign(pl->nuts->mom.size(), 0);
      // the chain scalars carry the key for the device's momentum draws
      k_chain_init<<<1, 1, 0, gstream[gi]>>>(pl->cs, o->eps0, o->target_accept, c.seed, 0, 0);
      LAUNCH_CHECK();
      pl->chain_ready = false;
      gch[gi].push_back(&c);
    }
  }
  for (;;) {
    bool any = false;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      bool act = false;
      for (NutsChain* c : gch[gi]) act = act || !c->done();
      if (!act) continue;
      any = true;
      if ((st = nuts_enqueue(gstream[gi], gch[gi])) != HAMLET_OK) return st;
    }
    if (!any) break;
    for (size_t gi = 0; gi < groups.size(); ++gi)
      if ((st = nuts_finish(gstream[gi], gch[gi])) != HAMLET_OK) return st;
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    HIP_TRY(hipStreamSynchronize(gstream[gi]));
    if ((st = streams_release(plans, groups[gi], gstream[gi])) != HAMLET_OK) return st;
  }
  if (eps_out)
    for (int j = 0; j < n_plans; ++j) eps_out[j] = chains[j].eps;
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// The paper's flat parameter vector
// ---------------------------------------------------------------------------
extern "C" hamlet_status hamlet_flat_size(const hamlet_plan* plan, int64_t* n_flat) {
  if (!plan || !n_flat) return fail(HAMLET_EINVAL, "NULL argument");
  *n_flat = 2 * flat_modes(plan->n) + plan->n_gal + plan->n_small();
  return HAMLET_OK;
}

static unsigned flat_blocks(const hamlet_plan* pl) {
  return blocks_for(std::max(pl->modes_count(), (size_t)pl->n_gal + pl->n_small()), 256);
}

extern "C" hamlet_status hamlet_pack_flat(hamlet_plan* plan, const void* modes, const double* dist,
                                          const double* snl, double* flat) {
  if (!plan || !modes || !snl || !flat) return fail(HAMLET_EINVAL, "NULL argument");
  if (plan->n_gal > 0 && !dist) return fail(HAMLET_EINVAL, "NULL distance buffer");
  k_pack_flat<<<flat_blocks(plan), 256, 0, plan->stream>>>((const double2*)modes, dist, snl, flat, plan->n,
                                                           plan->n_gal, plan->n_small());
  LAUNCH_CHECK();
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_unpack_flat(hamlet_plan* plan, const double* flat, void* modes, double* dist,
                                            double* snl) {
  if (!plan || !flat || !modes || !snl) return fail(HAMLET_EINVAL, "NULL argument");
  if (plan->n_gal > 0 && !dist) return fail(HAMLET_EINVAL, "NULL distance buffer");
  k_unpack_flat<<<flat_blocks(plan), 256, 0, plan->stream>>>(flat, (double2*)modes, dist, snl, plan->n,
                                                             plan->n_gal, plan->n_small());
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// The velocity field of a state (eq:vel-field)
// ---------------------------------------------------------------------------
extern "C" hamlet_status hamlet_velocity_field(hamlet_plan* plan, const void* modes, void* out) {
  if (!plan || !modes || !out) return fail(HAMLET_EINVAL, "NULL argument");
  Batch b;
  b.stream = plan->stream;
  b.count = 1;
  b.plan[0] = plan;
  b.mode[0] = kXGrad;
  StateDev sd{};
  sd.q = (double2*)modes;
  plan->st = sd;
  return plan->ops->field(b, out);
}

extern "C" hamlet_status hamlet_density_field(hamlet_plan* plan, const void* modes, void* out) {
  if (!plan || !modes || !out) return fail(HAMLET_EINVAL, "NULL argument");
  Batch b;
  b.stream = plan->stream;
  b.count = 1;
  b.plan[0] = plan;
  b.mode[0] = kXGrad;
  StateDev sd{};
  sd.q = (double2*)modes;
  plan->st = sd;
  return plan->ops->density(b, out);
}

extern "C" hamlet_status hamlet_field_stats_accumulate(hamlet_plan* plan, const void* modes, double* acc) {
  if (!plan || !modes || !acc) return fail(HAMLET_EINVAL, "NULL argument");
  Batch b;
  b.stream = plan->stream;
  b.count = 1;
  b.plan[0] = plan;
  b.mode[0] = kXGrad;
  StateDev sd{};
  sd.q = (double2*)modes;
  plan->st = sd;
  return plan->ops->stats(b, acc);
}

// ---------------------------------------------------------------------------
// Statistics of two fields in spherical shells (Section 5, correlation
// coefficients)
// ---------------------------------------------------------------------------
// Scratch of the allocation-free variant: a file-scope device array, one
// copy per device, held until the process ends.  In host code `scratch`
// names a host-side stand-in, not a device address: the array's address on
// each device is looked up once, with that device current, and only that
// address reaches kernels.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

static hamlet_status static_scratch(int device, double** out) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return HAMLET_OK;
  }
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != device) HIP_TRY(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) return fail(HAMLET_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  addr[device] = static_cast<double*>(p);
  *out = static_cast<double*>(p);
  return HAMLET_OK;
}

// Both sweeps of the shell statistics, with their partial sums in `part`
// (hipMallocAsync on the plan's stream when `fixed` is false, else the
// device's static scratch).
static hamlet_status shell_stats_run(hamlet_plan* plan, const double* a, const double* b, double width,
                                     int32_t n_shells, double* out, bool fixed) {
  if (!plan || (n_shells > 0 && (!a || !out))) return fail(HAMLET_EINVAL, "NULL argument");
  if (n_shells < 0 || n_shells > kShellMax)
    return fail(HAMLET_EINVAL, "n_shells %d outside [0, %d]", (int)n_shells, kShellMax);
  if (!(width > 0.0) || !std::isfinite(width)) return fail(HAMLET_EINVAL, "shell width %g is not positive", width);
  if (n_shells == 0) return HAMLET_OK;
  const ShellGeom g{plan->box / plan->n, width, plan->n, (int)n_shells};
  // one partial per shell and x plane
  const size_t bytes = (size_t)n_shells * plan->n * kShellValues * sizeof(double);
  double* part = nullptr;
  if (fixed) {
    if (bytes > kStaticScratchBytes)
      return fail(HAMLET_EINVAL,
                  "shell partials need %zu bytes (%d shells x %d planes), the static scratch holds %zu: "
                  "use fewer shells, or hamlet_shell_stats",
                  bytes, (int)n_shells, plan->n, kStaticScratchBytes);
    hamlet_status st = static_scratch(plan->device, &part);
    if (st != HAMLET_OK) return st;
  } else if (hipMallocAsync((void**)&part, bytes, plan->stream) != hipSuccess) {
    return fail(HAMLET_ENOMEM, "shell partials: %zu bytes", bytes);
  }
  // the means, then the centred sums (both sweeps reuse the partials; every
  // partial the finish stage reads is written by the part stage before it)
  const dim3 grid(plan->n, n_shells);
  k_shell_part<false><<<grid, kShellThreads, 0, plan->stream>>>(a, b, g, out, part);
  k_shell_finish<false><<<n_shells, kShellFinishThreads, 0, plan->stream>>>(part, g, out);
  k_shell_part<true><<<grid, kShellThreads, 0, plan->stream>>>(a, b, g, out, part);
  k_shell_finish<true><<<n_shells, kShellFinishThreads, 0, plan->stream>>>(part, g, out);
  const hipError_t le = hipGetLastError();
  if (!fixed) HIP_TRY(hipFreeAsync(part, plan->stream));
  if (le != hipSuccess) return fail(HAMLET_EDEVICE, "kernel launch: %s", hipGetErrorString(le));
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_shell_stats(hamlet_plan* plan, const double* a, const double* b, double width,
                                            int32_t n_shells, double* out) {
  return shell_stats_run(plan, a, b, width, n_shells, out, false);
}

extern "C" hamlet_status hamlet_shell_stats_static(hamlet_plan* plan, const double* a, const double* b, double width,
                                                   int32_t n_shells, double* out) {
  return shell_stats_run(plan, a, b, width, n_shells, out, true);
}

// ---------------------------------------------------------------------------
// Sphere moments of the velocity field (Section 5, monopole and dipole)
// ---------------------------------------------------------------------------
template <int N>
static void moments_pass(const hamlet_plan* pl, const double2* modes, const MomentRadii& rad, double kf,
                         double mono_scale, double dip_scale, double* part) {
  if constexpr (has_grid(N)) {
    constexpr int kN2 = 3 * (N / 2) * (N / 2) + 1;
    k_sphere_window<N><<<blocks_for((size_t)kN2 * kMomentsRadiiPerPass, 256), 256, 0, pl->stream>>>(rad, kf, pl->wtab);
    k_sphere_moments<N><<<kMomentsBlocks, 256, 0, pl->stream>>>(modes, rad, pl->wtab, mono_scale, dip_scale, part);
  }
}

extern "C" hamlet_status hamlet_sphere_moments(hamlet_plan* plan, const void* modes, const double* radii,
                                               int32_t n_radii, double* out) {
  if (!plan || !modes || (n_radii > 0 && (!radii || !out))) return fail(HAMLET_EINVAL, "NULL argument");
  if (n_radii < 0 || n_radii > kMomentsMaxRadii)
    return fail(HAMLET_EINVAL, "n_radii %d outside [0, %d]", (int)n_radii, kMomentsMaxRadii);
  for (int j = 0; j < n_radii; ++j)
    if (!(radii[j] > 0.0) || !std::isfinite(radii[j]))
      return fail(HAMLET_EINVAL, "radius %d (%g) is not positive and finite", j, radii[j]);
  if (n_radii == 0) return HAMLET_OK;
  const double kf = 2.0 * M_PI / plan->box;
  const double n3 = (double)plan->n * plan->n * plan->n;
  const double mono_scale = plan->f / n3;             // f / N^3
  const double dip_scale = kH0 * plan->f / (n3 * kf);  // H0 f / (N^3 k_f)
  for (int j0 = 0; j0 < n_radii; j0 += kMomentsRadiiPerPass) {
    MomentRadii rad{};
    rad.count = std::min(kMomentsRadiiPerPass, n_radii - j0);
    for (int j = 0; j < rad.count; ++j) rad.r[j] = radii[j0 + j];
    double* part = plan->mom_part + (size_t)(j0 / kMomentsRadiiPerPass) * kMomentsBlocks * kMomentsPassValues;
    const double2* q = (const double2*)modes;
    switch (plan->n) {
      case 16: moments_pass<16>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      case 32: moments_pass<32>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      case 64: moments_pass<64>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      case 128: moments_pass<128>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      case 256: moments_pass<256>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      case 512: moments_pass<512>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      case 1024: moments_pass<1024>(plan, q, rad, kf, mono_scale, dip_scale, part); break;
      default: return fail(HAMLET_EUNSUPPORTED, "grid size %d", plan->n);
    }
  }
  k_sphere_moments_sum<<<4 * n_radii, 256, 0, plan->stream>>>(plan->mom_part, out);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// Serving: continuous batching of independent jobs
// ---------------------------------------------------------------------------
struct Job {
  int64_t id = 0;
  int state = 0;                   // 0 queued, 1 running, 2 last tick enqueued, 3 done on the device,
                                   // -1 failed at admission
  // the request; uploads read from it, so it lives as long as the job
  hamlet_plan_desc desc{};
  std::vector<double> pk, rhat, mu, smu, cz, scz, q_modes, q_dist;
  double q_snl = 1.0;
  hamlet_hmc_opts opts{};
  Staging sg;
  size_t state_bytes = 0, bytes = 0;
  // once admitted
  hamlet_plan* plan = nullptr;
  char* mem = nullptr;             // chain state: q, mode sum, distances, s, dH, accept flags
  double2 *q = nullptr, *msum = nullptr;
  double *qd = nullptr, *qs = nullptr, *dh = nullptr;
  int32_t* acc = nullptr;
  ChainRun run;
  hipEvent_t done = nullptr;
  hamlet_catalog catalog() const {
    hamlet_catalog c;
    c.n = (int64_t)mu.size();
    c.rhat = rhat.data(); c.mu = mu.data(); c.sigma_mu = smu.data(); c.cz = cz.data(); c.sigma_cz = scz.data();
    return c;
  }
};

constexpr int kServerSides = 4;   // side streams a server tick uses at most

struct hamlet_server {
  size_t budget = 0, in_use = 0;
  int max_running = 0, ahead = 2;
  hipStream_t stream = nullptr;
  hipStream_t copy = nullptr;      // result copies, off the tick stream
  std::vector<hipEvent_t> tick_ev;
  // the groups of a tick after the first run on side streams of `stream`
  // (see group_streams), forked and joined with these events
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;   // one per side stream
  int64_t ticks = 0, next_id = 1;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  std::deque<Job*> queue;
  std::vector<Job*> running;       // state 1
};

// Chain state of a job: q and the mode sum (N^3 / 2 complex each), distances,
// s, dH and accept flags (n_iter each).
static size_t job_state_bytes(int n, int64_t n_gal, int n_iter) {
  const size_t nm = (size_t)n * n * (n / 2);
  return 2 * align256(16 * nm) + align256(8 * (size_t)std::max<int64_t>(n_gal, 1)) + 256 +
         align256(8 * (size_t)std::max(n_iter, 1)) + align256(4 * (size_t)std::max(n_iter, 1));
}

static hamlet_status check_opts(const hamlet_hmc_opts* o) {
  if (!o) return fail(HAMLET_EINVAL, "opts is NULL");
  if (o->n_iter < 0 || o->n_leapfrog < 0 || o->warmup < 0)
    return fail(HAMLET_EINVAL, "n_iter/n_leapfrog/warmup out of range");
  if (!(o->eps0 > 0) || !std::isfinite(o->eps0)) return fail(HAMLET_EINVAL, "eps0 must be positive");
  if (!(o->target_accept > 0 && o->target_accept < 1)) return fail(HAMLET_EINVAL, "target_accept must be in (0,1)");
  return HAMLET_OK;
}

static void job_release(hamlet_server* sv, Job* j) {
  if (j->plan) {
    hamlet_plan* pl = j->plan;
    (void)hipFreeAsync(pl->base, sv->stream);
    for (auto& ev : pl->prof_pool) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
    (void)hipEventDestroy(pl->order_ev);
    delete pl;
    j->plan = nullptr;
  }
  if (j->mem) (void)hipFreeAsync(j->mem, sv->stream);
  j->mem = nullptr;
  if (j->done) (void)hipEventDestroy(j->done);
  j->done = nullptr;
  if (j->state >= 1) sv->in_use -= j->bytes;
  j->state = j->state >= 1 ? 4 : j->state;   // released
}

extern "C" hamlet_status hamlet_server_create(const hamlet_server_desc* desc, void* stream, hamlet_server** out) {
  if (!out) return fail(HAMLET_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(HAMLET_EINVAL, "desc is NULL");
  if (desc->hbm_budget == 0) return fail(HAMLET_EINVAL, "hbm_budget is 0");
  std::unique_ptr<hamlet_server> sv(new hamlet_server());
  sv->budget = desc->hbm_budget;
  sv->max_running = desc->max_running;
  sv->ahead = desc->ticks_ahead > 0 ? desc->ticks_ahead : 2;
  sv->stream = (hipStream_t)stream;
  HIP_TRY(hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking));
  sv->tick_ev.resize(sv->ahead, nullptr);
  for (hipEvent_t& e : sv->tick_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&sv->fork_ev, hipEventDisableTiming));
  sv->join_ev.resize(kServerSides, nullptr);
  for (hipEvent_t& e : sv->join_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  *out = sv.release();
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_server_destroy(hamlet_server* sv) {
  if (!sv) return HAMLET_OK;
  hipError_t e = hipStreamSynchronize(sv->stream);
  for (auto& kv : sv->jobs) job_release(sv, kv.second.get());
  if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);
  for (hipEvent_t ev : sv->tick_ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : sv->join_ev) (void)hipEventDestroy(ev);
  if (sv->fork_ev) (void)hipEventDestroy(sv->fork_ev);
  (void)hipStreamDestroy(sv->copy);
  delete sv;
  if (e != hipSuccess) return fail(HAMLET_EDEVICE, "server destroy: %s", hipGetErrorString(e));
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_server_submit(hamlet_server* sv, const hamlet_plan_desc* desc,
                                              const hamlet_catalog* cat, const hamlet_hmc_opts* opts,
                                              const double* q_modes, const double* q_dist, double q_snl,
                                              int64_t* job_id) {
  if (!sv || !job_id) return fail(HAMLET_EINVAL, "NULL argument");
  hamlet_status st = check_desc(desc);
  if (st == HAMLET_OK) st = check_catalog(cat);
  if (st == HAMLET_OK) st = check_opts(opts);
  if (st != HAMLET_OK) return st;
  if (!std::isfinite(q_snl)) return fail(HAMLET_EINVAL, "q_snl not finite");
  std::unique_ptr<Job> j(new Job());
  j->desc = *desc;
  j->pk.assign(desc->pk_n2, desc->pk_n2 + desc->n_pk);
  j->desc.pk_n2 = j->pk.data();
  const int64_t n = cat->n;
  if (n > 0) {
    j->rhat.assign(cat->rhat, cat->rhat + 3 * n);
    j->mu.assign(cat->mu, cat->mu + n);
    j->smu.assign(cat->sigma_mu, cat->sigma_mu + n);
    j->cz.assign(cat->cz, cat->cz + n);
    j->scz.assign(cat->sigma_cz, cat->sigma_cz + n);
  }
  const size_t nm = (size_t)desc->n_grid * desc->n_grid * (desc->n_grid / 2);
  if (q_modes) j->q_modes.assign(q_modes, q_modes + 2 * nm);
  if (q_dist && n > 0) j->q_dist.assign(q_dist, q_dist + n);
  j->q_snl = q_snl;
  j->opts = *opts;
  const Ops* ops = desc->precision == HAMLET_FP64 ? pick_ops<double>(desc->n_grid) : pick_ops<float>(desc->n_grid);
  const double w = desc->hist_width > 0 ? desc->hist_width : 5.0;
  const hamlet_catalog c = j->catalog();
  j->state_bytes = job_state_bytes(desc->n_grid, n, opts->n_iter);
  j->bytes = ops->bytes((int)n, distance_prior_bins(&c, desc->omega_m, w)) + j->state_bytes;
  if (j->bytes > sv->budget)
    return fail(HAMLET_ENOMEM, "job needs %zu device bytes, budget %zu", j->bytes, sv->budget);
  j->id = sv->next_id++;
  *job_id = j->id;
  sv->queue.push_back(j.get());
  sv->jobs[j->id] = std::move(j);
  return HAMLET_OK;
}

// Creates the job's plan and chain state on the server's stream and
// initialises its chain; it runs from the next tick on.
static hamlet_status job_admit(hamlet_server* sv, Job* j) {
  const hamlet_catalog c = j->catalog();
  hamlet_status st = plan_make(&j->desc, &c, sv->stream, true, j->sg, &j->plan);
  if (st != HAMLET_OK) return st;
  hamlet_plan* pl = j->plan;
  const size_t nm = pl->modes_count();
  if (hipMallocAsync((void**)&j->mem, j->state_bytes, sv->stream) != hipSuccess) {
    j->mem = nullptr;
    return fail(HAMLET_ENOMEM, "allocation of %zu bytes failed", j->state_bytes);
  }
  char* m = j->mem;
  j->q = (double2*)m;                 m += align256(16 * nm);
  j->msum = (double2*)m;              m += align256(16 * nm);
  j->qd = (double*)m;                 m += align256(8 * (size_t)std::max(pl->n_gal, 1));
  j->qs = (double*)m;                 m += 256;
  j->dh = (double*)m;                 m += align256(8 * (size_t)std::max(j->opts.n_iter, 1));
  j->acc = (int32_t*)m;
  hipStream_t s = sv->stream;
  if (!j->q_modes.empty())
    HIP_TRY(hipMemcpyAsync(j->q, j->q_modes.data(), 16 * nm, hipMemcpyHostToDevice, s));
  else
    HIP_TRY(hipMemsetAsync(j->q, 0, 16 * nm, s));
  HIP_TRY(hipMemsetAsync(j->msum, 0, 16 * nm, s));
  if (pl->n_gal > 0) {
    if (!j->q_dist.empty())
      HIP_TRY(hipMemcpyAsync(j->qd, j->q_dist.data(), 8 * (size_t)pl->n_gal, hipMemcpyHostToDevice, s));
    else
      HIP_TRY(hipMemcpyAsync(j->qd, pl->dz, 8 * (size_t)pl->n_gal, hipMemcpyDeviceToDevice, s));
  }
  k_set_small<<<1, 64, 0, s>>>(j->qs, j->q_snl, pl->n_small());
  k_chain_init<<<1, 1, 0, s>>>(pl->cs, j->opts.eps0, j->opts.target_accept, j->opts.seed, j->opts.warmup,
                               j->opts.jitter_eps);
  LAUNCH_CHECK();
  StateDev sd{};
  sd.q = j->q;
  if (pl->qc) {
    // the FP32 path's chain runs on complex64 modes (back into j->q when done)
    hamlet_status cs = chain_modes_in(pl, j->q, s);
    if (cs != HAMLET_OK) return cs;
    sd.q = (double2*)pl->qc;
  }
  sd.qd = pl->n_gal ? j->qd : pl->qd0;
  sd.qs = j->qs;
  sd.p = pl->pm;
  sd.pd = pl->pd;
  sd.ps = pl->ps;
  sd.g = pl->gcache;
  sd.gd = pl->gd;
  sd.gs = &pl->cs->gs[0];
  sd.psi = &pl->cs->psi;
  sd.eps = &pl->cs->eps_it;
  sd.dh = j->dh;
  sd.acc = j->acc;
  sd.msum = j->msum;
  pl->st = sd;
  j->run.pl = pl;
  j->run.L = j->opts.n_leapfrog;
  j->run.todo = j->opts.n_iter;
  j->run.need_grad = true;
  HIP_TRY(hipEventCreateWithFlags(&j->done, hipEventDisableTiming));
  return HAMLET_OK;
}

static int job_poll(Job* j) {
  if (j->state == 2 && hipEventQuery(j->done) == hipSuccess) j->state = 3;
  return j->state;
}

static void server_stats(hamlet_server* sv, hamlet_server_stats* out) {
  if (!out) return;
  out->queued = (int32_t)sv->queue.size();
  out->running = 0;
  out->finished = 0;
  for (auto& kv : sv->jobs) {
    const int s = job_poll(kv.second.get());
    if (s == 1 || s == 2) ++out->running;
    if (s == 3) ++out->finished;
  }
  out->ticks = sv->ticks;
  out->bytes_in_use = sv->in_use;
}

extern "C" hamlet_status hamlet_server_tick(hamlet_server* sv, hamlet_server_stats* stats) {
  if (!sv) return fail(HAMLET_EINVAL, "server is NULL");
  hamlet_status st;
  // keep at most `ahead` ticks queued on the device
  if (sv->ticks >= sv->ahead) HIP_TRY(hipEventSynchronize(sv->tick_ev[sv->ticks % sv->ahead]));
  // admission in arrival order, by device footprint
  while (!sv->queue.empty()) {
    Job* j = sv->queue.front();
    if (sv->max_running > 0 && (int)sv->running.size() >= sv->max_running) break;
    if (sv->in_use + j->bytes > sv->budget) break;
    sv->queue.pop_front();
    j->state = 1;
    sv->in_use += j->bytes;
    if ((st = job_admit(sv, j)) != HAMLET_OK) {
      const std::string msg = g_last_error;
      job_release(sv, j);
      j->state = -1;
      return fail(st, "job %lld not admitted: %s", (long long)j->id, msg.c_str());
    }
    sv->running.push_back(j);
  }
  // one leapfrog step of every running job; jobs of one grid size and
  // precision share launches, up to kMaxBatch per launch, and the groups
  // after the first run side by side on side streams of the server's stream
  std::vector<bool> taken(sv->running.size(), false);
  std::vector<std::vector<ChainRun*>> groups;
  for (size_t a = 0; a < sv->running.size(); ++a) {
    if (taken[a]) continue;
    std::vector<ChainRun*> group;
    const hamlet_plan* p0 = sv->running[a]->plan;
    for (size_t b = a; b < sv->running.size() && (int)group.size() < kMaxBatch; ++b) {
      const hamlet_plan* pb = sv->running[b]->plan;
      if (taken[b] || pb->n != p0->n || pb->prec != p0->prec) continue;
      taken[b] = true;
      group.push_back(&sv->running[b]->run);
    }
    groups.push_back(std::move(group));
  }
  hipStream_t side[kServerSides] = {};
  if (groups.size() > 1) HIP_TRY(hipEventRecord(sv->fork_ev, sv->stream));
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    hipStream_t run = sv->stream;
    if (gi > 0) {
      const int k = (int)((gi - 1) % kServerSides);
      if (!side[k]) {
        side[k] = side_stream(sv->stream, k + 1);
        if (side[k]) HIP_TRY(hipStreamWaitEvent(side[k], sv->fork_ev, 0));
      }
      if (side[k]) run = side[k];
    }
    if ((st = tick_group(run, groups[gi])) != HAMLET_OK) return st;
  }
  for (int k = 0; k < kServerSides; ++k) {
    if (!side[k]) continue;
    HIP_TRY(hipEventRecord(sv->join_ev[k], side[k]));
    HIP_TRY(hipStreamWaitEvent(sv->stream, sv->join_ev[k], 0));
  }
  // jobs whose last iteration was in this tick leave
  std::vector<Job*> still;
  for (Job* j : sv->running) {
    if (j->run.active()) {
      still.push_back(j);
      continue;
    }
    if (j->plan->qc && (st = chain_modes_out(j->plan, j->q, sv->stream)) != HAMLET_OK) return st;
    HIP_TRY(hipEventRecord(j->done, sv->stream));
    j->state = 2;
  }
  sv->running.swap(still);
  HIP_TRY(hipEventRecord(sv->tick_ev[sv->ticks % sv->ahead], sv->stream));
  ++sv->ticks;
  server_stats(sv, stats);
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_server_job_state(hamlet_server* sv, int64_t job_id, int32_t* state) {
  if (!sv || !state) return fail(HAMLET_EINVAL, "NULL argument");
  auto it = sv->jobs.find(job_id);
  if (it == sv->jobs.end()) return fail(HAMLET_EINVAL, "no job %lld", (long long)job_id);
  const int s = job_poll(it->second.get());
  *state = s < 0 ? -1 : (s == 3 ? 2 : (s == 0 ? 0 : 1));
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_server_take(hamlet_server* sv, int64_t job_id, double* mode_sum, double* q_modes,
                                            double* q_dist, double* q_snl, double* dh, int32_t* accepted,
                                            double* eps) {
  if (!sv) return fail(HAMLET_EINVAL, "server is NULL");
  auto it = sv->jobs.find(job_id);
  if (it == sv->jobs.end()) return fail(HAMLET_EINVAL, "no job %lld", (long long)job_id);
  Job* j = it->second.get();
  if (j->state < 2) return fail(HAMLET_EINVAL, "job %lld has not finished", (long long)job_id);
  HIP_TRY(hipEventSynchronize(j->done));
  const hamlet_plan* pl = j->plan;
  const size_t nm = pl->modes_count();
  hipStream_t c = sv->copy;
  if (mode_sum) HIP_TRY(hipMemcpyAsync(mode_sum, j->msum, 16 * nm, hipMemcpyDeviceToHost, c));
  if (q_modes) HIP_TRY(hipMemcpyAsync(q_modes, j->q, 16 * nm, hipMemcpyDeviceToHost, c));
  if (q_dist && pl->n_gal > 0)
    HIP_TRY(hipMemcpyAsync(q_dist, j->qd, 8 * (size_t)pl->n_gal, hipMemcpyDeviceToHost, c));
  if (q_snl) HIP_TRY(hipMemcpyAsync(q_snl, j->qs, 8, hipMemcpyDeviceToHost, c));
  if (dh && j->opts.n_iter > 0)
    HIP_TRY(hipMemcpyAsync(dh, j->dh, 8 * (size_t)j->opts.n_iter, hipMemcpyDeviceToHost, c));
  if (accepted && j->opts.n_iter > 0)
    HIP_TRY(hipMemcpyAsync(accepted, j->acc, 4 * (size_t)j->opts.n_iter, hipMemcpyDeviceToHost, c));
  if (eps) HIP_TRY(hipMemcpyAsync(eps, &pl->cs->eps, 8, hipMemcpyDeviceToHost, c));
  HIP_TRY(hipStreamSynchronize(c));
  job_release(sv, j);
  sv->jobs.erase(it);
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_profile_start(hamlet_plan* pl, int32_t kernel) {
  if (!pl) return fail(HAMLET_EINVAL, "plan is NULL");
  if (kernel < 0 || kernel >= HAMLET_K_COUNT) return fail(HAMLET_EINVAL, "kernel kind %d", kernel);
  pl->prof_kind = kernel;
  pl->prof_used = 0;
  pl->prof_failed = false;
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_profile_stop(hamlet_plan* pl, double* total_ms, int64_t* launches) {
  if (!pl || !total_ms || !launches) return fail(HAMLET_EINVAL, "NULL argument");
  pl->prof_kind = -1;
  HIP_TRY(hipStreamSynchronize(pl->stream));
  double sum = 0.0;
  for (size_t i = 0; i < pl->prof_used; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pl->prof_pool[i].first, pl->prof_pool[i].second));
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)pl->prof_used;
  pl->prof_used = 0;
  if (pl->prof_failed) return fail(HAMLET_EDEVICE, "event creation or record failed while profiling");
  return HAMLET_OK;
}

template <typename T, int N> static void schedule_of(hamlet_schedule* o) {
  using SC = Sched<T, N>;
  o->threads_xy = SC::XY;
  o->threads_x = SC::X;
  o->threads_gather = SC::ZG;
  o->threads_scatter = SC::ZS;
  o->tile_width = SC::W;
  o->pencils_scatter = SC::PZ;
  o->pencils_gather = SC::PG;
  o->radix_plan = SC::RADIX < radix_plans(N) ? SC::RADIX : 0;
  const RadixPlan rp = radix_plan(N, SC::RADIX);
  for (int i = 0; i < 3; ++i) o->radix[i] = rp.r[i];
}

template <typename T> static bool schedule_for(int n, hamlet_schedule* o) {
  switch (n) {
    case 16: schedule_of<T, 16>(o); break;
    case 32: schedule_of<T, 32>(o); break;
    case 64: schedule_of<T, 64>(o); break;
    case 128: schedule_of<T, 128>(o); break;
    case 256: schedule_of<T, 256>(o); break;
    case 512: schedule_of<T, 512>(o); break;
    case 1024: schedule_of<T, 1024>(o); break;
    default: return false;
  }
  return pick_ops<T>(n) != nullptr;
}

extern "C" hamlet_status hamlet_schedule_get(int32_t precision, int32_t n_grid, hamlet_schedule* out) {
  if (!out) return fail(HAMLET_EINVAL, "NULL argument");
  bool ok;
  if (precision == HAMLET_FP64) ok = schedule_for<double>(n_grid, out);
  else if (precision == HAMLET_FP32_FP64E) ok = schedule_for<float>(n_grid, out);
  else return fail(HAMLET_EINVAL, "precision %d", precision);
  if (!ok) return fail(HAMLET_EUNSUPPORTED, "n_grid %d: not built into this library", n_grid);
  return HAMLET_OK;
}

extern "C" const char* hamlet_last_error(void) { return g_last_error.c_str(); }
