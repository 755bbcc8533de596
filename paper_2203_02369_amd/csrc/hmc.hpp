// Hamiltonian Monte Carlo kernels (Section 3), all in FP64.
//
// Mass matrix eq:M_ab per real coordinate: M^-1 = sigma_k^2 / 2 for each of
// Re and Im of a retained mode, sigma_v^2 / H0^2 for a distance, 1 for
// s = sigma_NL / 100 km/s.  Momenta of the kz = 0 plane keep the Hermitian
// pairing of the modes (a mirror entry holds the conjugate of its partner).
#pragma once

#include "common.hpp"
#include "passes.hpp"

namespace hamlet {

constexpr int kEltThreads = 256;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), counter (idx lo, idx hi, iteration,
// purpose), key (seed lo, seed hi).
// ---------------------------------------------------------------------------
struct Philox4 { uint32_t v[4]; };

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0; c1 = lo1; c2 = hi0 ^ c3 ^ k1; c3 = lo0;
  }
  Philox4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3; return o;
}

enum Purpose : uint32_t { kPurposeModes = 0, kPurposeDist = 1, kPurposeSnl = 2, kPurposeAccept = 3, kPurposeJitter = 4 };

__device__ __forceinline__ Philox4 draw_words(uint64_t seed, uint32_t iteration, uint32_t purpose, uint64_t index) {
  return philox4x32_10((uint32_t)index, (uint32_t)(index >> 32), iteration, purpose,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ((x >> 11) + 1) 2^-53 in (0, 1], x = (hi << 32) | lo.
__device__ __forceinline__ double uniform53(uint32_t lo, uint32_t hi) {
  const uint64_t x = ((uint64_t)hi << 32) | lo;
  return ((double)(x >> 11) + 1.0) * 0x1.0p-53;
}

// Box-Muller on the two uniforms of one Philox output.
__device__ __forceinline__ double2 normal_pair(const Philox4& w) {
  const double u1 = uniform53(w.v[0], w.v[1]);
  const double u2 = uniform53(w.v[2], w.v[3]);
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  double sn, cs;
  sincos(ang, &sn, &cs);
  return make_double2(rad * cs, rad * sn);
}

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

// kz = 0 entries whose canonical Hermitian partner is (-kx, -ky, 0):
// canonical half = ny > 0, or ny = 0 and nx > 0.
__device__ __forceinline__ bool is_mirror(const ModeIdx& m) {
  return m.kz == 0 && (m.sy < 0 || (m.sy == 0 && m.sx < 0));
}

// sigma_k^2 per mode from the n^2-indexed table (plan set-up only).
__global__ void __launch_bounds__(kEltThreads)
k_fill_mode_var(double* __restrict__ mvar, const double* __restrict__ var_n2, int n) {
  const size_t total = (size_t)n * n * (n / 2);
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const ModeIdx m = mode_idx(g, n);
  mvar[g] = retained(m.sx, m.sy, m.kz, n) ? var_n2[m.sx * m.sx + m.sy * m.sy + m.kz * m.kz] : 0.0;
}

// ---------------------------------------------------------------------------
// Momentum refresh p ~ N(0, M).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kEltThreads)
k_momenta_modes(double2* __restrict__ p, ModeTables tab, int n, uint64_t seed, uint32_t iteration) {
  const size_t total = (size_t)n * n * (n / 2);
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const ModeIdx m = mode_idx(g, n);
  double2 out = make_double2(0.0, 0.0);
  if (retained(m.sx, m.sy, m.kz, n)) {
    const bool mir = is_mirror(m);
    size_t src = g;
    if (mir) src = ((size_t)((n - m.x) & (n - 1)) * n + ((n - m.y) & (n - 1))) * (n / 2);
    const double2 z = normal_pair(draw_words(seed, iteration, kPurposeModes, src));
    const double sc = sqrt(2.0 * inv_or_zero(tab.var[g]));
    out = make_double2(sc * z.x, mir ? -sc * z.y : sc * z.y);
  }
  p[g] = out;
}

__global__ void __launch_bounds__(kEltThreads)
k_momenta_small(double* __restrict__ p_dist, double* __restrict__ p_snl, int n_gal, double inv_sqrt_minv_d,
                int sample_d, int sample_s, uint64_t seed, uint32_t iteration) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_gal) {
    p_dist[i] = sample_d ? inv_sqrt_minv_d * normal_pair(draw_words(seed, iteration, kPurposeDist, i)).x : 0.0;
  }
  if (i == 0) p_snl[0] = sample_s ? normal_pair(draw_words(seed, iteration, kPurposeSnl, 0)).x : 0.0;
}

// ---------------------------------------------------------------------------
// Kinetic energy K = (1/2) p^T M^-1 p: per stored mode (w_k / 8) sigma^2 |p|^2
// (w_k = 1 on kz = 0 where both Hermitian partners are stored, else 2).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kEltThreads)
k_kinetic_modes(const double2* __restrict__ p, ModeTables tab, int n, double* __restrict__ part) {
  __shared__ double red[kEltThreads / 64];
  const size_t total = (size_t)n * n * (n / 2);
  double acc = 0.0;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
    const ModeIdx m = mode_idx(g, n);
    if (retained(m.sx, m.sy, m.kz, n)) {
      const double2 v = p[g];
      acc += (m.kz == 0 ? 0.125 : 0.25) * tab.var[g] * (v.x * v.x + v.y * v.y);
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sums the mode partials and adds (1/2) M_d^-1 sum p_d^2 + (1/2) M_s^-1 p_s^2.
__global__ void __launch_bounds__(256)
k_kinetic_final(const double* __restrict__ part, int n_part, const double* __restrict__ p_dist, int n_gal,
                const double* __restrict__ p_snl, double minv_d, double minv_s, double* __restrict__ out) {
  __shared__ double red[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n_part; i += blockDim.x) a += part[i];
  for (int i = threadIdx.x; i < n_gal; i += blockDim.x) b += p_dist[i] * p_dist[i];
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) out[0] = a + 0.5 * minv_d * b + 0.5 * minv_s * p_snl[0] * p_snl[0];
}

// First half kick (from the cached gradient) and drift of the distances and
// of s: p -= (eps/2) g, q += eps M^-1 p.
__global__ void __launch_bounds__(kEltThreads)
k_small_kick_drift(double* __restrict__ q_dist, double* __restrict__ p_dist, const double* __restrict__ g_dist,
                   double* __restrict__ q_snl, double* __restrict__ p_snl, const double* __restrict__ g_snl,
                   int n_gal, int sample_d, int sample_s, double minv_d, const double* __restrict__ eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double e = eps[0];
  if (i < n_gal && sample_d) {
    const double pv = p_dist[i] - 0.5 * e * g_dist[i];
    p_dist[i] = pv;
    q_dist[i] += e * minv_d * pv;
  }
  if (i == 0 && sample_s) {
    const double pv = p_snl[0] - 0.5 * e * g_snl[0];
    p_snl[0] = pv;
    q_snl[0] += e * pv;
  }
}

// ---------------------------------------------------------------------------
// Chain scalars kept on the device so a whole run is enqueued without a
// host round trip.
// ---------------------------------------------------------------------------
struct ChainScalars {
  double eps;          // step size of the chain (adapted during warm-up)
  double eps_it;       // step of the current iteration (jittered)
  double da_mu, da_hbar, da_log_eps_bar, da_m;
  double psi, gs;              // Psi and dPsi/ds at the current state
  double psi_saved, gs_saved;  // at the start of the trajectory
  double kin0, kin1;
  double target;
  int accept;
};

__global__ void k_set_scalar(double* dst, double v) { dst[0] = v; }

__global__ void k_chain_init(ChainScalars* cs, double eps0, double target) {
  cs->eps = eps0;
  cs->eps_it = eps0;
  cs->da_mu = log(10.0 * eps0);
  cs->da_hbar = 0.0;
  cs->da_log_eps_bar = 0.0;
  cs->da_m = 0.0;
  cs->target = target;
  cs->accept = 0;
}

// Start of an iteration: the (optionally jittered) step, and the state's
// Psi / dPsi/ds saved for a possible rejection.
__global__ void k_iter_begin(ChainScalars* cs, uint64_t seed, uint32_t iteration, int jitter) {
  double e = cs->eps;
  if (jitter) {
    const Philox4 w = draw_words(seed, iteration, kPurposeJitter, 0);
    e = e * (0.9 + 0.2 * uniform53(w.v[0], w.v[1]));
  }
  cs->eps_it = e;
  cs->psi_saved = cs->psi;
  cs->gs_saved = cs->gs;
}

// Metropolis-Hastings test of the end point (Section 3.2) and dual
// averaging of the step (Hoffman & Gelman) during warm-up.
__global__ void k_accept(ChainScalars* cs, uint64_t seed, uint32_t iteration, int warmup,
                         double* __restrict__ dh_out, int32_t* __restrict__ acc_out) {
  double dh = (cs->kin1 + cs->psi) - (cs->kin0 + cs->psi_saved);
  if (!isfinite(dh)) dh = __builtin_inf();
  const Philox4 w = draw_words(seed, iteration, kPurposeAccept, 0);
  const double u = uniform53(w.v[0], w.v[1]);
  const int acc = log(u) < -dh ? 1 : 0;
  cs->accept = acc;
  if (dh_out) dh_out[iteration] = dh;
  if (acc_out) acc_out[iteration] = acc;
  if ((int)iteration < warmup) {
    const double alpha = !isfinite(dh) ? 0.0 : (dh <= 0.0 ? 1.0 : exp(-dh));
    cs->da_m += 1.0;
    const double m = cs->da_m;
    const double eta = 1.0 / (m + 10.0);
    cs->da_hbar = (1.0 - eta) * cs->da_hbar + eta * (cs->target - alpha);
    const double log_eps = cs->da_mu - sqrt(m) / 0.05 * cs->da_hbar;
    const double wgt = pow(m, -0.75);
    cs->da_log_eps_bar = wgt * log_eps + (1.0 - wgt) * cs->da_log_eps_bar;
    cs->eps = ((int)iteration == warmup - 1) ? exp(cs->da_log_eps_bar) : exp(log_eps);
  }
  if (!acc) {
    cs->psi = cs->psi_saved;
    cs->gs = cs->gs_saved;
  }
}

// On rejection restore the saved state and its cached gradient.
__global__ void __launch_bounds__(kEltThreads)
k_restore_modes(const ChainScalars* __restrict__ cs, double2* __restrict__ q, const double2* __restrict__ q0,
                double2* __restrict__ g, const double2* __restrict__ g0, size_t total) {
  if (cs->accept) return;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  q[i] = q0[i];
  g[i] = g0[i];
}

__global__ void __launch_bounds__(kEltThreads)
k_restore_small(const ChainScalars* __restrict__ cs, double* __restrict__ qd, const double* __restrict__ qd0,
                double* __restrict__ gd, const double* __restrict__ gd0, double* __restrict__ qs,
                const double* __restrict__ qs0, int n_gal) {
  if (cs->accept) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_gal) { qd[i] = qd0[i]; gd[i] = gd0[i]; }
  if (i == 0) qs[0] = qs0[0];
}

__global__ void __launch_bounds__(kEltThreads)
k_accumulate(double2* __restrict__ sum, const double2* __restrict__ q, size_t total) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double2 a = sum[i];
  const double2 b = q[i];
  a.x += b.x;
  a.y += b.y;
  sum[i] = a;
}

__global__ void k_copy_gs(const ChainScalars* cs, double* out_eps) { out_eps[0] = cs->eps; }

}  // namespace hamlet
