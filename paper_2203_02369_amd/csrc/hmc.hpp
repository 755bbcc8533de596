// Hamiltonian Monte Carlo kernels (Section 3), all in FP64.
//
// Mass matrix eq:M_ab per real coordinate: M^-1 = sigma_k^2 / 2 for each of
// Re and Im of a retained mode, sigma_v^2 / H0^2 for a distance, 1 for
// s = sigma_NL / 100 km/s.  Momenta of the kz = 0 plane keep the Hermitian
// pairing of the modes (a mirror entry holds the conjugate of its partner).
#pragma once

#include "common.hpp"
#include "galaxies.hpp"
#include "passes.hpp"
#include "random.hpp"
#include "workspace.hpp"

namespace hamlet {

constexpr int kEltThreads = 256;

// Mode coordinates of flat index g of the [kx][ky][kz < N/2] layout.
struct ModeIdx { int x, y, kz, sx, sy; };
__device__ __forceinline__ ModeIdx mode_idx(size_t g, int n) {
  const int h = n / 2;
  ModeIdx m;
  m.kz = (int)(g % h);
  const size_t r = g / h;
  m.y = (int)(r % n);
  m.x = (int)(r / n);
  m.sx = signed_freq(m.x, n);
  m.sy = signed_freq(m.y, n);
  return m;
}

// sigma_k^2 per mode from the n^2-indexed table (plan set-up only), in the
// x-pass tile order (var_ofs, tile width w).
__global__ void __launch_bounds__(kEltThreads)
k_fill_mode_var(double* __restrict__ mvar, const double* __restrict__ var_n2, int n, int w) {
  const size_t total = (size_t)n * n * (n / 2);
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const ModeIdx m = mode_idx(g, n);
  mvar[var_ofs(n, w, m.x, m.y, m.kz)] =
      retained(m.sx, m.sy, m.kz, n) ? var_n2[m.sx * m.sx + m.sy * m.sy + m.kz * m.kz] : 0.0;
}


template <typename T, int N> __device__ __forceinline__ ChainScalars* chain(const Ws<T, N>& w) { return w.chain(); }

__global__ void k_set_scalar(double* dst, double v) {
  if (threadIdx.x == 0) dst[0] = v;
}

// The small coordinates of a start state: s, then u8 = phi = 1 (the
// fiducial cosmology) when they are sampled.
__global__ void k_set_small(double* dst, double s, int ns) {
  if (threadIdx.x == 0) dst[0] = s;
  if (threadIdx.x > 0 && threadIdx.x < ns) dst[threadIdx.x] = 1.0;
}

__global__ void k_chain_init(ChainScalars* cs, double eps0, double target, uint64_t seed, int warmup, int jitter) {
  cs->eps = eps0;
  cs->eps_it = eps0;
  cs->da_mu = log(10.0 * eps0);
  cs->da_hbar = 0.0;
  cs->da_log_eps_bar = 0.0;
  cs->da_m = 0.0;
  cs->target = target;
  cs->seed = seed;
  cs->iter = 0;
  cs->warmup = warmup;
  cs->jitter = jitter;
  cs->accept = 0;
  cs->post = 0;
}

// ---------------------------------------------------------------------------
// Kinetic energy K = (1/2) p^T M^-1 p: per stored mode (w_k / 8) sigma^2 |p|^2
// (w_k = 1 on kz = 0 where both Hermitian partners are stored, else 2), per
// distance (1/2) M_d^-1 p_d^2, and (1/2) M_s^-1 p_s^2.  The mode terms are
// block partials of the x pass that starts (K0) or ends (K1) a trajectory;
// the distance and s terms are N_KIN_SMALL block partials after them; one
// block sums all of them in order into kin0 or kin1.
// ---------------------------------------------------------------------------
template <typename T, int N> __device__ __forceinline__ double* kin_small(const Ws<T, N>& w) {
  return w.kin_part() + Ws<T, N>::F::N_PRIOR;
}

// Distance and s terms of the kinetic energy, one partial per block.
template <typename T, int N>
__device__ __forceinline__ void kinetic_small_part(const Pick<T, N>& k, CSum acc, double* red) {
  const PlanConst& pc = k.w.pc();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (pc.sample_s) {
      const double ps = k.st.ps[0];
      acc.add(0.5 * ps * ps);
    }
    if (pc.sample_c) {
      acc.add(0.5 * pc.minv_u8 * k.st.ps[1] * k.st.ps[1]);
      acc.add(0.5 * pc.minv_phi * k.st.ps[2] * k.st.ps[2]);
      acc.add(0.5 * pc.minv_eta * k.st.ps[3] * k.st.ps[3]);
    }
  }
  const double s = block_csum(acc, red);
  if (threadIdx.x == 0) kin_small(k.w)[blockIdx.x] = s;
}

// Momentum refresh of the distances and s (grid: N_KIN_SMALL blocks), the
// saved start point of the small variables, and their part of K0.
template <typename T, int N>
__global__ void __launch_bounds__(kEltThreads) k_momenta_small(Launch L) {
  __shared__ double red[2 * (kEltThreads / 64)];
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const PlanConst& pc = k.w.pc();
  const ChainScalars* cs = chain(k.w);
  const uint64_t seed = cs->seed;
  const uint32_t iteration = (uint32_t)cs->iter;
  CSum acc;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.n_gal; i += gridDim.x * blockDim.x) {
    const double pv = pc.sample_d ? pc.psd * normal_pair(draw_words(seed, iteration, kPurposeDist, i)).x : 0.0;
    k.st.pd[i] = pv;
    k.w.qd0()[i] = k.st.qd[i];
    k.w.gd0()[i] = k.w.gd()[i];
    acc.add(0.5 * pc.minv_d * pv * pv);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    k.st.ps[0] = pc.sample_s ? normal_pair(draw_words(seed, iteration, kPurposeSnl, 0)).x : 0.0;
    k.w.qs0()[0] = k.st.qs[0];
    if (pc.sample_c) {
      // (u8, phi) from one pair, eta from the first of the next: p ~ N(0, M),
      // M = 1 / minv
      const double2 z = normal_pair(draw_words(seed, iteration, kPurposeCosmo, 0));
      const double2 z2 = normal_pair(draw_words(seed, iteration, kPurposeCosmo, 1));
      k.st.ps[1] = z.x / sqrt(pc.minv_u8);
      k.st.ps[2] = z.y / sqrt(pc.minv_phi);
      k.st.ps[3] = z2.x / sqrt(pc.minv_eta);
      for (int j = 1; j < kSmallMax; ++j) k.w.qs0()[j] = k.st.qs[j];
    }
  }
  kinetic_small_part(k, acc, red);
}

// Distance and s terms of K1 (grid: N_KIN_SMALL blocks).
template <typename T, int N>
__global__ void __launch_bounds__(kEltThreads) k_kinetic_small(Launch L) {
  __shared__ double red[2 * (kEltThreads / 64)];
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const double minv = k.w.pc().minv_d;
  const double* __restrict__ pd = k.st.pd;
  CSum acc;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k.n_gal; i += gridDim.x * blockDim.x)
    acc.add(0.5 * minv * pd[i] * pd[i]);
  kinetic_small_part(k, acc, red);
}

template <typename T, int N>
__global__ void __launch_bounds__(256) k_kinetic_final(Launch L, int which) {
  __shared__ double red[2 * 4];
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const PlanConst& pc = k.w.pc();
  const double* __restrict__ kin = k.w.kin_part();
  CSum acc;
  for (int i = threadIdx.x; i < pc.n_kin_part; i += blockDim.x) acc.add(kin[i]);
  const double a = block_csum(acc, red);
  if (threadIdx.x == 0) {
    ChainScalars* cs = chain(k.w);
    if (which) cs->kin1 = a;
    else cs->kin0 = a;
  }
}

// First half kick (from the cached gradient) and drift of the distances and
// of s: p -= (eps/2) g, q += eps M^-1 p; then the binning of the drifted
// points for the next evaluation.
template <typename T, int N>
__global__ void __launch_bounds__(kEltThreads) k_small_kick_drift(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const StateDev& st = k.st;
  const PlanConst& pc = k.w.pc();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double e = st.eps[0];
  if (i < k.n_gal) {
    if (st.sv_qd) st.sv_qd[i] = st.qd[i];
    if (st.sv_pd) st.sv_pd[i] = st.pd[i];
    if (pc.sample_d) {
      const double pv = st.pd[i] - 0.5 * e * st.gd[i];
      st.pd[i] = pv;
      st.qd[i] += e * pc.minv_d * pv;
    }
    bin_point(i, st.qd[i], catalogue(k.w, k.n_gal), cosmo(k.w), N, bin_out(k.w));
  }
  if (i == 0) {
    const int ns = pc.sample_c ? kSmallMax : 1;
    for (int j = 0; j < ns; ++j) {
      if (st.sv_qs) st.sv_qs[j] = st.qs[j];
      if (st.sv_ps) st.sv_ps[j] = st.ps[j];
    }
    const double minv[kSmallMax] = {1.0, pc.minv_u8, pc.minv_phi, pc.minv_eta};
    for (int j = 0; j < ns; ++j) {
      if (j == 0 && !pc.sample_s) continue;
      const double pv = st.ps[j] - 0.5 * e * st.gs[j];
      st.ps[j] = pv;
      st.qs[j] += e * minv[j] * pv;
    }
  }
}

// Start of an iteration: the (optionally jittered) step, and the state's
// Psi / dPsi/ds saved for a possible rejection.
template <typename T, int N>
__global__ void k_iter_begin(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip || threadIdx.x != 0) return;
  ChainScalars* cs = chain(k.w);
  double e = cs->eps;
  if (cs->jitter) {
    const Philox4 w = draw_words(cs->seed, (uint32_t)cs->iter, kPurposeJitter, 0);
    e = e * (0.9 + 0.2 * uniform53(w.v[0], w.v[1]));
  }
  cs->eps_it = e;
  cs->psi_saved = cs->psi;
  for (int j = 0; j < kSmallMax; ++j) cs->gs_saved[j] = cs->gs[j];
  // set by the trajectory; equal (no change of H) when it has no steps
  cs->kin0 = 0.0;
  cs->kin1 = 0.0;
}

// Metropolis-Hastings test of the end point (Section 3.2) and dual
// averaging of the step (Hoffman & Gelman) during warm-up; advances the
// chain's iteration counter.
template <typename T, int N>
__global__ void k_accept(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip || threadIdx.x != 0) return;
  ChainScalars* cs = chain(k.w);
  const int it = cs->iter;
  double dh = (cs->kin1 + cs->psi) - (cs->kin0 + cs->psi_saved);
  if (!isfinite(dh)) dh = __builtin_inf();
  const Philox4 w = draw_words(cs->seed, (uint32_t)it, kPurposeAccept, 0);
  const double u = uniform53(w.v[0], w.v[1]);
  const int acc = log(u) < -dh ? 1 : 0;
  cs->accept = acc;
  cs->post = it >= cs->warmup ? 1 : 0;
  if (k.st.dh) k.st.dh[it] = dh;
  if (k.st.acc) k.st.acc[it] = acc;
  if (it < cs->warmup) {
    const double alpha = !isfinite(dh) ? 0.0 : (dh <= 0.0 ? 1.0 : exp(-dh));
    cs->da_m += 1.0;
    const double m = cs->da_m;
    const double eta = 1.0 / (m + 10.0);
    cs->da_hbar = (1.0 - eta) * cs->da_hbar + eta * (cs->target - alpha);
    const double log_eps = cs->da_mu - sqrt(m) / 0.05 * cs->da_hbar;
    const double wgt = pow(m, -0.75);
    cs->da_log_eps_bar = wgt * log_eps + (1.0 - wgt) * cs->da_log_eps_bar;
    cs->eps = (it == cs->warmup - 1) ? exp(cs->da_log_eps_bar) : exp(log_eps);
  }
  if (!acc) {
    cs->psi = cs->psi_saved;
    for (int j = 0; j < kSmallMax; ++j) cs->gs[j] = cs->gs_saved[j];
  }
  cs->iter = it + 1;
}

// After the test: on rejection restore the saved state and its cached
// gradient; past warm-up add the (possibly restored) modes to the running
// sum of samples (FP64).  S32: the chain state is stored in complex64.
template <typename T, int N, bool S32 = false>
__global__ void __launch_bounds__(kEltThreads) k_restore_accumulate(Launch L) {
  using Q = typename StateElt<S32>::type;
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const size_t total = (size_t)N * N * (N / 2);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const ChainScalars* cs = chain(k.w);
  const int rejected = !cs->accept;
  Q* sq = reinterpret_cast<Q*>(k.st.q);
  if (i < total) {
    double2 q = make_double2(0.0, 0.0);
    if (rejected) {
      const Q q0 = ld_stream(&reinterpret_cast<const Q*>(k.w.q0())[i]);
      st_stream(&sq[i], q0);
      st_stream(&reinterpret_cast<Q*>(k.w.gcache())[i], ld_stream(&reinterpret_cast<const Q*>(k.w.g0())[i]));
      q = widen(q0);
    } else if (cs->post && k.st.msum) {
      q = widen(ld_stream(&sq[i]));
    }
    if (cs->post && k.st.msum) {
      double2 a = ld_stream(&k.st.msum[i]);
      a.x += q.x;
      a.y += q.y;
      st_stream(&k.st.msum[i], a);
    }
  }
  if (rejected) {
    if (i < (size_t)k.n_gal) {
      k.st.qd[i] = k.w.qd0()[i];
      k.w.gd()[i] = k.w.gd0()[i];
    }
    if (i == 0) {
      const int ns = k.w.pc().sample_c ? kSmallMax : 1;
      for (int j = 0; j < ns; ++j) k.st.qs[j] = k.w.qs0()[j];
    }
  }
}

// A chain's modes into and out of the complex64 state of the FP32 path's
// chains: every entry rounded in, only the retained modes written back (the
// caller's other entries keep their values).
__global__ void __launch_bounds__(kEltThreads) k_modes_narrow(const double2* __restrict__ in, float2* __restrict__ out,
                                                              size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = narrow<float2>(in[i]);
}

__global__ void __launch_bounds__(kEltThreads) k_modes_widen(const float2* __restrict__ in, double2* __restrict__ out,
                                                             int n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int hz = n / 2;
  if (i >= (size_t)n * n * hz) return;
  const int kz = (int)(i % hz), y = (int)((i / hz) % n), x = (int)(i / ((size_t)hz * n));
  if (retained(signed_freq(x, n), signed_freq(y, n), kz, n)) out[i] = widen(in[i]);
}

// End of a leapfrog call: Psi of the end point to the caller's slot.
template <typename T, int N>
__global__ void k_leap_out(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip || threadIdx.x != 0) return;
  k.st.psi_out[0] = chain(k.w)->psi;
}

}  // namespace hamlet
