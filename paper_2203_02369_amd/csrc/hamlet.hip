// HAMLET library for gfx950: plan set-up, pass orchestration and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hamlet.h"
#include "common.hpp"
#include "fft.hpp"
#include "passes.hpp"
#include "galaxies.hpp"
#include "hmc.hpp"

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
struct Workspace {
  char* base = nullptr;
  size_t used = 0;
  size_t cap = 0;
  template <typename X> X* take(size_t count) {
    const size_t bytes = ((count * sizeof(X)) + 255) & ~size_t(255);
    X* p = base ? reinterpret_cast<X*>(base + used) : nullptr;
    used += bytes;
    return p;
  }
};

struct hamlet_plan;

// What one evaluation does besides Psi and the gradient.  Plain gradient:
// x_mode = kXGrad, the gradient goes to g.  Inside a leapfrog trajectory the
// inverse pass 1 was already done by the previous evaluation's x pass, and
// the leapfrog update of every coordinate is fused in (x_mode kXMid or
// kXLast; the gradient of a kXLast evaluation goes to g as the cache).
struct EvalMode {
  int x_mode = kXGrad;
  double plane_scale = 1.0;   // kXGrad: factor on the kz = 0 plane of the gradient
  double2* p_modes = nullptr;
  double* p_dist = nullptr;
  double* p_snl = nullptr;
  const double* eps = nullptr;
};

typedef hamlet_status (*eval_fn)(hamlet_plan*, double2*, double*, double*, double2*, double*, double*, double*,
                                 const EvalMode&);
typedef hamlet_status (*first_fn)(hamlet_plan*, double2*, double2*, const double*);

struct hamlet_plan {
  int n = 0, prec = 0, n_gal = 0, sample_d = 1, sample_s = 1, n_hist = 0;
  double box = 0, om = 0, h = 0, f = 0, sigma_v = 0, hist_w = 5.0, minv_d = 0;
  hipStream_t stream = nullptr;
  Workspace ws;
  // tables
  double *var = nullptr, *mvar = nullptr, *hist = nullptr;
  void* tw = nullptr;
  // catalogue
  double *rhat = nullptr, *mu = nullptr, *smu = nullptr, *cz = nullptr, *scz = nullptr;
  // binning
  int *count = nullptr, *off = nullptr, *cursor = nullptr, *key = nullptr, *cellz = nullptr, *slot = nullptr,
      *iz = nullptr, *bsum = nullptr;
  double* frac = nullptr;
  void *rx = nullptr, *ry = nullptr, *rz = nullptr, *tx = nullptr, *ty = nullptr, *tz = nullptr;
  // spectral intermediates and galaxy partials (precision T)
  void *a = nullptr, *b = nullptr, *v0 = nullptr, *v1 = nullptr, *v2 = nullptr, *part = nullptr, *gsort = nullptr;
  double *prior_part = nullptr, *like_part = nullptr, *kin_part = nullptr;
  int n_prior_part = 0, n_like_part = 0, n_kin_part = 0;
  // chain state
  ChainScalars* cs = nullptr;
  double2 *gcache = nullptr, *q0 = nullptr, *g0 = nullptr, *pm = nullptr;
  double *gd = nullptr, *gd0 = nullptr, *qd0 = nullptr, *pd = nullptr, *qs0 = nullptr, *ps = nullptr;
  double* eps_slot = nullptr;
  eval_fn eval = nullptr;
  first_fn first = nullptr;
  // event timing of one kernel kind (hamlet_profile_start / stop)
  int prof_kind = -1;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pool;
  size_t prof_used = 0;
  bool prof_failed = false;
  size_t modes_count() const { return (size_t)n * n * (n / 2); }
};

// Bracket one launch of kernel kind `kind` with events when it is armed.
static void prof_before(hamlet_plan* pl, int kind) {
  if (pl->prof_kind != kind) return;
  if (pl->prof_used == pl->prof_pool.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      pl->prof_failed = true;
      pl->prof_kind = -1;
      return;
    }
    pl->prof_pool.emplace_back(a, b);
  }
  if (hipEventRecord(pl->prof_pool[pl->prof_used].first, pl->stream) != hipSuccess) pl->prof_failed = true;
}
static void prof_after(hamlet_plan* pl, int kind) {
  if (pl->prof_kind != kind) return;
  if (hipEventRecord(pl->prof_pool[pl->prof_used].second, pl->stream) != hipSuccess) pl->prof_failed = true;
  ++pl->prof_used;
}
#define TIMED(pl, kind, ...)   \
  do {                         \
    prof_before(pl, kind);     \
    __VA_ARGS__;               \
    prof_after(pl, kind);      \
  } while (0)

template <typename T> static Binned<T> binned_view(hamlet_plan* pl) {
  Binned<T> b;
  b.off = pl->off;
  b.rx = (const T*)pl->rx; b.ry = (const T*)pl->ry; b.rz = (const T*)pl->rz;
  b.tx = (const T*)pl->tx; b.ty = (const T*)pl->ty; b.tz = (const T*)pl->tz;
  b.iz = pl->iz;
  return b;
}

static Catalogue catalogue_view(hamlet_plan* pl) {
  Catalogue c;
  c.n = pl->n_gal; c.rhat = pl->rhat; c.mu = pl->mu; c.sigma_mu = pl->smu; c.cz = pl->cz; c.sigma_cz = pl->scz;
  c.hist = pl->hist; c.n_hist = pl->n_hist; c.hist_w = pl->hist_w;
  return c;
}

static Cosmo cosmo_view(hamlet_plan* pl) {
  Cosmo c;
  c.om = pl->om; c.h = pl->h; c.box = pl->box; c.spacing = pl->box / pl->n;
  c.dmax = kC / (3.0 * pl->om * kH0);
  return c;
}

static ModeTables tables_view(hamlet_plan* pl) {
  ModeTables t;
  t.var = pl->mvar;
  t.kfac0 = kH0 * pl->f / ((double)pl->n * pl->n * pl->n * (2.0 * M_PI / pl->box));
  return t;
}

static inline unsigned blocks_for(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// One log-posterior-and-gradient evaluation: bin, inverse passes with the
// gather, likelihood, final sums (Psi, dPsi/ds), forward passes with the
// scatter, and the x pass (gradient, or the fused leapfrog update and the
// next evaluation's inverse pass 1).
template <typename T, int N>
static hamlet_status eval_impl(hamlet_plan* pl, double2* q, double* qd, double* qs, double2* g, double* gd,
                               double* gs, double* psi, const EvalMode& em) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  hipStream_t st = pl->stream;
  const int n = pl->n_gal;
  const Catalogue cat = catalogue_view(pl);
  const Cosmo cm = cosmo_view(pl);
  const ModeTables tab = tables_view(pl);
  const C* tw = (const C*)pl->tw;
  const Binned<T> bins = binned_view<T>(pl);
  const bool leap = em.x_mode != kXGrad;
  LeapUpdate lf_d, lf_s;
  if (leap) {
    const double kick = em.x_mode == kXMid ? 1.0 : 0.5;
    const int drift = em.x_mode == kXMid ? 1 : 0;
    if (pl->sample_d) {
      lf_d.p = em.p_dist; lf_d.eps = em.eps; lf_d.kick = kick; lf_d.drift = drift; lf_d.minv = pl->minv_d;
    }
    if (pl->sample_s) {
      lf_s.p = em.p_snl; lf_s.eps = em.eps; lf_s.kick = kick; lf_s.drift = drift; lf_s.minv = 1.0;
    }
  }
  if (n > 0) {
    prof_before(pl, HAMLET_K_BIN);
    k_bin_count<T><<<blocks_for(n, kGalThreads), kGalThreads, 0, st>>>(qd, cat, cm, N, pl->count, pl->key,
                                                                        pl->cellz, pl->frac);
    constexpr int tiles = (N * N + kScanTile - 1) / kScanTile;
    k_bin_scan_tiles<<<tiles, kScanTile, 0, st>>>(pl->count, pl->off, pl->bsum, N * N);
    k_bin_scan_add<<<tiles, kScanTile, 0, st>>>(pl->count, pl->off, pl->cursor, pl->bsum, N * N);
    k_bin_place<<<blocks_for(n, kGalThreads), kGalThreads, 0, st>>>(pl->key, pl->cursor, pl->slot, n);
    k_bin_sort<T><<<blocks_for((size_t)N * N, kGalThreads), kGalThreads, 0, st>>>(
        pl->off, pl->slot, pl->cellz, pl->frac, cat, N * N, (T*)pl->rx, (T*)pl->ry, (T*)pl->rz, (T*)pl->tx,
        (T*)pl->ty, (T*)pl->tz, pl->iz, pl->slot);
    prof_after(pl, HAMLET_K_BIN);
    LAUNCH_CHECK();
  }
  const dim3 gs_xy(S::CHUNKS, N);
  if (!leap)
    TIMED(pl, HAMLET_K_INV_X,
          k_inv_x<T, N, TH::XY><<<gs_xy, TH::XY, 0, st>>>(q, tab, tw, (C*)pl->a, (C*)pl->b, pl->prior_part));
  using SL = XSlabs<N>;
  const dim3 gs_xy_slab(S::CHUNKS, SL::SIZE), gs_z_slab(N / S::P, SL::SIZE);
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    TIMED(pl, HAMLET_K_INV_Y,
          k_inv_y<T, N, TH::XY><<<gs_xy_slab, TH::XY, 0, st>>>((const C*)pl->a, (const C*)pl->b, tw, (C*)pl->v0,
                                                                (C*)pl->v1, (C*)pl->v2, x0));
    TIMED(pl, HAMLET_K_INV_Z,
          k_inv_z_gather<T, N, TH::Z><<<gs_z_slab, TH::Z, 0, st>>>((const C*)pl->v0, (const C*)pl->v1,
                                                                    (const C*)pl->v2, tw, bins, (C*)pl->part, x0));
  }
  LAUNCH_CHECK();
  if (n > 0) {
    LikeOut lo;
    lo.g_dist = gd;
    lo.part = pl->like_part;
    TIMED(pl, HAMLET_K_LIKE,
          k_like<T><<<blocks_for(n, kGalThreads), kGalThreads, 0, st>>>((const C*)pl->part, pl->slot, pl->frac,
                                                                         qd, qs, cat, cm, (T*)pl->gsort, lo, lf_d));
    LAUNCH_CHECK();
  }
  k_finalize<<<1, 256, 0, st>>>(pl->prior_part, pl->n_prior_part, pl->like_part, n > 0 ? pl->n_like_part : 0, psi,
                                gs, qs, lf_s);
  for (int sl = 0; sl < SL::COUNT; ++sl) {
    const int x0 = sl * SL::SIZE;
    TIMED(pl, HAMLET_K_FWD_Z,
          k_fwd_z_scatter<T, N, TH::Z><<<gs_z_slab, TH::Z, 0, st>>>((const T*)pl->gsort, bins, tw, (C*)pl->v0,
                                                                     (C*)pl->v1, (C*)pl->v2, x0));
    TIMED(pl, HAMLET_K_FWD_Y,
          k_fwd_y<T, N, TH::XY><<<gs_xy_slab, TH::XY, 0, st>>>((const C*)pl->v0, (const C*)pl->v1,
                                                                (const C*)pl->v2, tw, (C*)pl->a, (C*)pl->b, x0));
  }
  const C* s1 = (const C*)pl->a;
  const C* s2 = (const C*)pl->b;
  if (em.x_mode == kXGrad) {
    TIMED(pl, HAMLET_K_FWD_X,
          (k_x_pass<T, N, kXGrad, TH::X><<<gs_xy, TH::X, 0, st>>>(s1, s2, q, nullptr, g, tab, tw, nullptr, nullptr,
                                                                    nullptr, nullptr, em.plane_scale)));
  } else if (em.x_mode == kXMid) {
    // S1, S2 live in a, b and are read by the same tile that writes the next
    // A, B: the x pass writes them to v0, v1 and the plan swaps the roles.
    TIMED(pl, HAMLET_K_FWD_X,
          (k_x_pass<T, N, kXMid, TH::X><<<gs_xy, TH::X, 0, st>>>(s1, s2, q, em.p_modes, nullptr, tab, tw, em.eps,
                                                                   (C*)pl->v0, (C*)pl->v1, pl->prior_part, 1.0)));
    std::swap(pl->a, pl->v0);
    std::swap(pl->b, pl->v1);
  } else {
    TIMED(pl, HAMLET_K_FWD_X,
          (k_x_pass<T, N, kXLast, TH::X><<<gs_xy, TH::X, 0, st>>>(s1, s2, q, em.p_modes, g, tab, tw, em.eps, nullptr,
                                                                    nullptr, nullptr, 1.0)));
  }
  LAUNCH_CHECK();
  return HAMLET_OK;
}

// First step of a trajectory: half kick from the cached gradient and drift
// of every coordinate, then inverse pass 1 of the new modes.
template <typename T, int N>
static hamlet_status first_impl(hamlet_plan* pl, double2* q, double2* p_modes, const double* eps) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using TH = PassThreads<T, N>;
  const dim3 gs_xy(S::CHUNKS, N);
  TIMED(pl, HAMLET_K_FWD_X,
        (k_x_pass<T, N, kXFirst, TH::X><<<gs_xy, TH::X, 0, pl->stream>>>(
            nullptr, nullptr, q, p_modes, pl->gcache, tables_view(pl), (const C*)pl->tw, eps, (C*)pl->a, (C*)pl->b,
            pl->prior_part, 1.0)));
  LAUNCH_CHECK();
  return HAMLET_OK;
}

template <typename T> static eval_fn pick_eval(int n) {
  switch (n) {
    case 16: return eval_impl<T, 16>;
    case 32: return eval_impl<T, 32>;
    case 64: return eval_impl<T, 64>;
    case 128: return eval_impl<T, 128>;
    case 256: return eval_impl<T, 256>;
    default: return nullptr;
  }
}

template <typename T> static first_fn pick_first(int n) {
  switch (n) {
    case 16: return first_impl<T, 16>;
    case 32: return first_impl<T, 32>;
    case 64: return first_impl<T, 64>;
    case 128: return first_impl<T, 128>;
    case 256: return first_impl<T, 256>;
    default: return nullptr;
  }
}

// Workspace layout; with ws.base == nullptr only the size is computed.
static void carve(hamlet_plan* pl) {
  Workspace& ws = pl->ws;
  ws.used = 0;
  const int n = pl->n;
  const size_t nm = pl->modes_count();
  const size_t npk = 3 * (size_t)(n / 2) * (n / 2) + 1;
  const size_t real = pl->prec == HAMLET_FP64 ? 8 : 4;
  const size_t ng = std::max(pl->n_gal, 1);
  pl->var = ws.take<double>(npk);
  pl->mvar = ws.take<double>(nm);
  pl->hist = ws.take<double>(std::max(pl->n_hist, 1));
  pl->tw = ws.take<char>(2 * real * n);
  pl->rhat = ws.take<double>(3 * ng);
  pl->mu = ws.take<double>(ng);
  pl->smu = ws.take<double>(ng);
  pl->cz = ws.take<double>(ng);
  pl->scz = ws.take<double>(ng);
  pl->count = ws.take<int>((size_t)n * n);
  pl->off = ws.take<int>((size_t)n * n + 1);
  pl->cursor = ws.take<int>((size_t)n * n);
  pl->bsum = ws.take<int>(((size_t)n * n + kScanTile - 1) / kScanTile);
  pl->key = ws.take<int>(ng);
  pl->cellz = ws.take<int>(ng);
  pl->slot = ws.take<int>(ng);
  pl->iz = ws.take<int>(ng);
  pl->frac = ws.take<double>(3 * ng);
  pl->rx = ws.take<char>(real * ng);
  pl->ry = ws.take<char>(real * ng);
  pl->rz = ws.take<char>(real * ng);
  pl->tx = ws.take<char>(real * ng);
  pl->ty = ws.take<char>(real * ng);
  pl->tz = ws.take<char>(real * ng);
  pl->gsort = ws.take<char>(real * ng);
  pl->part = ws.take<char>(2 * real * 4 * ng);
  pl->a = ws.take<char>(2 * real * nm);
  pl->b = ws.take<char>(2 * real * nm);
  pl->v0 = ws.take<char>(2 * real * nm);
  pl->v1 = ws.take<char>(2 * real * nm);
  pl->v2 = ws.take<char>(2 * real * nm);
  const int chunks = (n / 2) / (pl->prec == HAMLET_FP64 ? std::min(8, n / 2) : std::min(16, n / 2));
  pl->n_prior_part = n * chunks;
  pl->prior_part = ws.take<double>(pl->n_prior_part);
  pl->n_like_part = (int)blocks_for(ng, kGalThreads);
  pl->like_part = ws.take<double>(3 * (size_t)pl->n_like_part);
  pl->n_kin_part = 1024;
  pl->kin_part = ws.take<double>(pl->n_kin_part);
  pl->cs = ws.take<ChainScalars>(1);
  pl->gcache = ws.take<double2>(nm);
  pl->q0 = ws.take<double2>(nm);
  pl->g0 = ws.take<double2>(nm);
  pl->pm = ws.take<double2>(nm);
  pl->gd = ws.take<double>(ng);
  pl->gd0 = ws.take<double>(ng);
  pl->qd0 = ws.take<double>(ng);
  pl->pd = ws.take<double>(ng);
  pl->qs0 = ws.take<double>(1);
  pl->ps = ws.take<double>(1);
  pl->eps_slot = ws.take<double>(1);
}

// ---------------------------------------------------------------------------
// Host-side set-up
// ---------------------------------------------------------------------------
static hamlet_status check_desc(const hamlet_plan_desc* d) {
  if (!d) return fail(HAMLET_EINVAL, "desc is NULL");
  const int n = d->n_grid;
  if (n != 16 && n != 32 && n != 64 && n != 128 && n != 256)
    return fail(HAMLET_EUNSUPPORTED, "n_grid %d: built for 16, 32, 64, 128, 256", n);
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

// Distance prior (eq:D): density histogram of the redshift distances, bins
// of width w on [0, max d_z + 15), one pseudo-count per bin.
static std::vector<double> distance_histogram(const hamlet_catalog* c, double om, double w) {
  std::vector<double> dz(c->n);
  double top = 0.0;
  for (int64_t i = 0; i < c->n; ++i) {
    dz[i] = redshift_distance(c->cz[i] / kC, om);
    top = std::max(top, dz[i]);
  }
  const int nb = (int)std::ceil((top + 15.0) / w);
  std::vector<double> cnt(nb, 0.0);
  for (int64_t i = 0; i < c->n; ++i) {
    long long b = (long long)std::floor(dz[i] / w);
    b = std::min<long long>(std::max<long long>(b, 0), nb - 1);
    cnt[b] += 1.0;
  }
  for (int b = 0; b < nb; ++b) cnt[b] = (cnt[b] + 1.0) / ((double)(c->n + nb) * w);
  return cnt;
}

static hamlet_status upload(hamlet_plan* pl, const hamlet_plan_desc* d, const hamlet_catalog* c,
                            const std::vector<double>& hist) {
  const int n = pl->n;
  const size_t npk = 3 * (size_t)(n / 2) * (n / 2) + 1;
  const double kf = 2.0 * M_PI / pl->box;
  const double n3 = (double)n * n * n;
  const double vol = pl->box * pl->box * pl->box;
  std::vector<double> var(npk);
  for (size_t j = 0; j < npk; ++j) var[j] = n3 * n3 / vol * d->pk_n2[j];
  (void)kf;
  // Twiddles exp(-2 pi i m / N), computed in long double and rounded once.
  std::vector<double> twd(2 * n);
  std::vector<float> twf(2 * n);
  for (int m = 0; m < n; ++m) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * m / n;
    twd[2 * m] = (double)cosl(ang);
    twd[2 * m + 1] = (double)sinl(ang);
    twf[2 * m] = (float)cosl(ang);
    twf[2 * m + 1] = (float)sinl(ang);
  }
  hipStream_t st = pl->stream;
  HIP_TRY(hipMemcpyAsync(pl->var, var.data(), npk * 8, hipMemcpyHostToDevice, st));
  k_fill_mode_var<<<blocks_for(pl->modes_count(), kEltThreads), kEltThreads, 0, st>>>(pl->mvar, pl->var, n);
  LAUNCH_CHECK();
  if (pl->prec == HAMLET_FP64)
    HIP_TRY(hipMemcpyAsync(pl->tw, twd.data(), twd.size() * 8, hipMemcpyHostToDevice, st));
  else
    HIP_TRY(hipMemcpyAsync(pl->tw, twf.data(), twf.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(pl->hist, hist.data(), hist.size() * 8, hipMemcpyHostToDevice, st));
  if (c->n > 0) {
    HIP_TRY(hipMemcpyAsync(pl->rhat, c->rhat, 3 * c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->mu, c->mu, c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->smu, c->sigma_mu, c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->cz, c->cz, c->n * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pl->scz, c->sigma_cz, c->n * 8, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemsetAsync(pl->count, 0, (size_t)n * n * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(pl->off, 0, ((size_t)n * n + 1) * sizeof(int), st));
  HIP_TRY(hipStreamSynchronize(st));
  return HAMLET_OK;
}

static void fill_plan_scalars(hamlet_plan* pl, const hamlet_plan_desc* d, int64_t n_gal, int n_hist) {
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
  hamlet_plan tmp;
  fill_plan_scalars(&tmp, desc, n_gal, kFootprintHistBins);
  carve(&tmp);
  *bytes = tmp.ws.used;
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_plan_create(const hamlet_plan_desc* desc, const hamlet_catalog* cat, void* stream,
                                            hamlet_plan** out) {
  if (!out) return fail(HAMLET_EINVAL, "out is NULL");
  *out = nullptr;
  hamlet_status st = check_desc(desc);
  if (st != HAMLET_OK) return st;
  st = check_catalog(cat);
  if (st != HAMLET_OK) return st;
  const double w = desc->hist_width > 0 ? desc->hist_width : 5.0;
  std::vector<double> hist = distance_histogram(cat, desc->omega_m, w);
  hamlet_plan* pl = new hamlet_plan();
  fill_plan_scalars(pl, desc, cat->n, (int)hist.size());
  pl->stream = (hipStream_t)stream;
  pl->eval = pl->prec == HAMLET_FP64 ? pick_eval<double>(pl->n) : pick_eval<float>(pl->n);
  pl->first = pl->prec == HAMLET_FP64 ? pick_first<double>(pl->n) : pick_first<float>(pl->n);
  carve(pl);
  const size_t bytes = pl->ws.used;
  if (hipMalloc((void**)&pl->ws.base, bytes) != hipSuccess) {
    delete pl;
    return fail(HAMLET_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  pl->ws.cap = bytes;
  carve(pl);
  st = upload(pl, desc, cat, hist);
  if (st != HAMLET_OK) {
    (void)hipFree(pl->ws.base);
    delete pl;
    return st;
  }
  *out = pl;
  return HAMLET_OK;
}

extern "C" hamlet_status hamlet_plan_destroy(hamlet_plan* pl) {
  if (!pl) return HAMLET_OK;
  hipError_t e1 = hipStreamSynchronize(pl->stream);
  for (auto& ev : pl->prof_pool) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  hipError_t e2 = hipFree(pl->ws.base);
  delete pl;
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(HAMLET_EDEVICE, "plan destroy: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  return HAMLET_OK;
}

// ---------------------------------------------------------------------------
// Leapfrog and chain orchestration
// ---------------------------------------------------------------------------
// Kick-drift-kick trajectory (eq:hamilton, Section 3.3) of `steps` steps from
// a state whose gradient is cached in (pl->gcache, pl->gd, cs->gs); leaves
// the end point's gradient there and its Psi in cs->psi.  Consecutive half
// kicks are merged and every update is fused into the evaluation kernels.
static hamlet_status trajectory(hamlet_plan* pl, int steps, const double* eps, double2* q, double* qd, double* qs,
                                double2* pmodes, double* pd, double* ps) {
  if (steps <= 0) return HAMLET_OK;
  double* psi = &pl->cs->psi;
  double* gs = &pl->cs->gs;
  k_small_kick_drift<<<blocks_for(std::max(pl->n_gal, 1), kEltThreads), kEltThreads, 0, pl->stream>>>(
      qd, pd, pl->gd, qs, ps, gs, pl->n_gal, pl->sample_d, pl->sample_s, pl->minv_d, eps);
  LAUNCH_CHECK();
  hamlet_status st = pl->first(pl, q, pmodes, eps);
  if (st != HAMLET_OK) return st;
  EvalMode em;
  em.p_modes = pmodes;
  em.p_dist = pd;
  em.p_snl = ps;
  em.eps = eps;
  for (int k = 1; k <= steps; ++k) {
    em.x_mode = k < steps ? kXMid : kXLast;
    st = pl->eval(pl, q, qd, qs, pl->gcache, pl->gd, gs, psi, em);
    if (st != HAMLET_OK) return st;
  }
  return HAMLET_OK;
}

static hamlet_status kinetic(hamlet_plan* pl, const double2* pmodes, const double* pd, const double* ps,
                             double* out) {
  k_kinetic_modes<<<pl->n_kin_part, kEltThreads, 0, pl->stream>>>(pmodes, tables_view(pl), pl->n, pl->kin_part);
  k_kinetic_final<<<1, 256, 0, pl->stream>>>(pl->kin_part, pl->n_kin_part, pd, pl->n_gal, ps, pl->minv_d,
                                              pl->sample_s ? 1.0 : 0.0, out);
  LAUNCH_CHECK();
  return HAMLET_OK;
}

static hamlet_status check_plans(hamlet_plan* const* plans, int32_t n_plans) {
  if (!plans || n_plans <= 0) return fail(HAMLET_EINVAL, "need at least one plan");
  for (int j = 0; j < n_plans; ++j)
    if (!plans[j]) return fail(HAMLET_EINVAL, "plans[%d] is NULL", j);
  return HAMLET_OK;
}

static hamlet_status logpost_grad_impl(hamlet_plan* const* plans, int32_t n_plans, const void* const* q_modes,
                                       const double* const* q_dist, const double* const* q_snl,
                                       void* const* g_modes, double* const* g_dist, double* const* g_snl,
                                       double* const* psi, double plane_scale) {
  EvalMode em;
  em.plane_scale = plane_scale;
  hamlet_status st = check_plans(plans, n_plans);
  if (st != HAMLET_OK) return st;
  if (!q_modes || !q_snl || !g_modes || !g_snl || !psi) return fail(HAMLET_EINVAL, "NULL argument array");
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    if (!q_modes[j] || !g_modes[j] || !q_snl[j] || !g_snl[j] || !psi[j])
      return fail(HAMLET_EINVAL, "plan %d: NULL buffer", j);
    if (pl->n_gal > 0 && (!q_dist || !g_dist || !q_dist[j] || !g_dist[j]))
      return fail(HAMLET_EINVAL, "plan %d: NULL distance buffer", j);
    st = pl->eval(pl, (double2*)q_modes[j], pl->n_gal ? (double*)q_dist[j] : nullptr, (double*)q_snl[j],
                  (double2*)g_modes[j], pl->n_gal ? g_dist[j] : nullptr, g_snl[j], psi[j], em);
    if (st != HAMLET_OK) return st;
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
    double* qd = pl->n_gal ? q_dist[j] : pl->qd0;
    double* pd = pl->n_gal ? p_dist[j] : pl->pd;
    k_set_scalar<<<1, 1, 0, pl->stream>>>(pl->eps_slot, eps[j]);
    st = pl->eval(pl, (double2*)q_modes[j], qd, q_snl[j], pl->gcache, pl->gd, &pl->cs->gs, &pl->cs->psi, EvalMode());
    if (st != HAMLET_OK) return st;
    st = trajectory(pl, n_steps[j], pl->eps_slot, (double2*)q_modes[j], qd, q_snl[j], (double2*)p_modes[j], pd,
                    p_snl[j]);
    if (st != HAMLET_OK) return st;
    HIP_TRY(hipMemcpyAsync(psi[j], &pl->cs->psi, sizeof(double), hipMemcpyDeviceToDevice, pl->stream));
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
  if (o->n_iter < 0 || o->n_leapfrog < 0 || o->warmup < 0 || o->warmup > o->n_iter)
    return fail(HAMLET_EINVAL, "n_iter/n_leapfrog/warmup out of range");
  if (!(o->eps0 > 0) || !std::isfinite(o->eps0)) return fail(HAMLET_EINVAL, "eps0 must be positive");
  if (!(o->target_accept > 0 && o->target_accept < 1)) return fail(HAMLET_EINVAL, "target_accept must be in (0,1)");
  if (!q_modes || !q_snl) return fail(HAMLET_EINVAL, "NULL argument array");
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    if (!q_modes[j] || !q_snl[j]) return fail(HAMLET_EINVAL, "plan %d: NULL buffer", j);
    if (pl->n_gal > 0 && (!q_dist || !q_dist[j])) return fail(HAMLET_EINVAL, "plan %d: NULL distance buffer", j);
  }
  // Initial gradient of every chain.
  for (int j = 0; j < n_plans; ++j) {
    hamlet_plan* pl = plans[j];
    double* qd = pl->n_gal ? q_dist[j] : pl->qd0;
    k_chain_init<<<1, 1, 0, pl->stream>>>(pl->cs, o->eps0, o->target_accept);
    st = pl->eval(pl, (double2*)q_modes[j], qd, q_snl[j], pl->gcache, pl->gd, &pl->cs->gs, &pl->cs->psi, EvalMode());
    if (st != HAMLET_OK) return st;
  }
  for (int it = 0; it < o->n_iter; ++it) {
    for (int j = 0; j < n_plans; ++j) {
      hamlet_plan* pl = plans[j];
      hipStream_t s = pl->stream;
      const size_t nm = pl->modes_count();
      double2* q = (double2*)q_modes[j];
      double* qd = pl->n_gal ? q_dist[j] : pl->qd0;
      const int ng1 = std::max(pl->n_gal, 1);
      k_iter_begin<<<1, 1, 0, s>>>(pl->cs, o->seed, (uint32_t)it, o->jitter_eps);
      k_momenta_modes<<<blocks_for(nm, kEltThreads), kEltThreads, 0, s>>>(pl->pm, tables_view(pl), pl->n, o->seed,
                                                                           (uint32_t)it);
      k_momenta_small<<<blocks_for(ng1, kEltThreads), kEltThreads, 0, s>>>(
          pl->pd, pl->ps, pl->n_gal, kH0 / pl->sigma_v, pl->sample_d, pl->sample_s, o->seed, (uint32_t)it);
      LAUNCH_CHECK();
      st = kinetic(pl, pl->pm, pl->pd, pl->ps, &pl->cs->kin0);
      if (st != HAMLET_OK) return st;
      HIP_TRY(hipMemcpyAsync(pl->q0, q, nm * sizeof(double2), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(pl->g0, pl->gcache, nm * sizeof(double2), hipMemcpyDeviceToDevice, s));
      if (pl->n_gal > 0) {
        HIP_TRY(hipMemcpyAsync(pl->qd0, qd, pl->n_gal * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(pl->gd0, pl->gd, pl->n_gal * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
      HIP_TRY(hipMemcpyAsync(pl->qs0, q_snl[j], sizeof(double), hipMemcpyDeviceToDevice, s));
      st = trajectory(pl, o->n_leapfrog, &pl->cs->eps_it, q, qd, q_snl[j], pl->pm, pl->pd, pl->ps);
      if (st != HAMLET_OK) return st;
      st = kinetic(pl, pl->pm, pl->pd, pl->ps, &pl->cs->kin1);
      if (st != HAMLET_OK) return st;
      k_accept<<<1, 1, 0, s>>>(pl->cs, o->seed, (uint32_t)it, o->warmup, dh ? dh[j] : nullptr,
                               accepted ? accepted[j] : nullptr);
      k_restore_modes<<<blocks_for(nm, kEltThreads), kEltThreads, 0, s>>>(pl->cs, q, pl->q0, pl->gcache, pl->g0,
                                                                           nm);
      k_restore_small<<<blocks_for(ng1, kEltThreads), kEltThreads, 0, s>>>(pl->cs, qd, pl->qd0, pl->gd, pl->gd0,
                                                                           q_snl[j], pl->qs0, pl->n_gal);
      if (it >= o->warmup && mode_sum && mode_sum[j])
        k_accumulate<<<blocks_for(nm, kEltThreads), kEltThreads, 0, s>>>((double2*)mode_sum[j], q, nm);
      LAUNCH_CHECK();
    }
  }
  if (eps_out) {
    for (int j = 0; j < n_plans; ++j) {
      hamlet_plan* pl = plans[j];
      HIP_TRY(hipMemcpyAsync(&eps_out[j], &pl->cs->eps, sizeof(double), hipMemcpyDeviceToHost, pl->stream));
      HIP_TRY(hipStreamSynchronize(pl->stream));
    }
  }
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

extern "C" const char* hamlet_last_error(void) { return g_last_error.c_str(); }
