// Kernels of the No-U-Turn sampler (Section 3.3; Hoffman & Gelman's NUTS):
// fresh momenta at the start of an iteration, the dot products of the
// no-U-turn test, the running sum of samples, and the values the host reads
// after each leapfrog step.  The tree itself is built by the host; every
// leapfrog step is the fused passes of an evaluation (passes.hpp).
#pragma once

#include "common.hpp"
#include "galaxies.hpp"
#include "hmc.hpp"
#include "passes.hpp"
#include "random.hpp"
#include "workspace.hpp"

namespace hamlet {

// Momenta r0 ~ N(0, M) of the modes (eq:M_ab: variance 2 / sigma_k^2 per real
// part), from the same stream and with the same mirror rule as the first x
// pass of an HMC trajectory, into st.p; the mode part of K0 as block
// partials kin_part[block] (N_PRIOR blocks of N W modes each).  The chain's
// key and iteration come from its chain scalars.
template <typename T, int N>
__global__ void __launch_bounds__(kEltThreads) k_nuts_momenta(Launch L) {
  using F = FixedLayout<N, sizeof(T)>;
  __shared__ double red[2 * (kEltThreads / 64)];
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const ChainScalars* cs = k.w.chain();
  const uint64_t seed = cs->seed;
  const uint32_t iteration = (uint32_t)cs->iter;
  const double* __restrict__ var = k.w.mvar();
  constexpr size_t per = F::NM / F::N_PRIOR;
  const size_t g0 = (size_t)blockIdx.x * per;
  CSum kin;
  for (size_t g = g0 + threadIdx.x; g < g0 + per; g += blockDim.x) {
    const ModeIdx m = mode_idx(g, N);
    double2 p = make_double2(0.0, 0.0);
    if (retained(m.sx, m.sy, m.kz, N)) {
      const double v = var[var_ofs(N, F::W, m.x, m.y, m.kz)];
      const bool mirror = m.kz == 0 && (m.sy < 0 || (m.sy == 0 && m.sx < 0));
      const size_t src = mirror ? gofs<N>((N - m.x) & (N - 1), (N - m.y) & (N - 1), 0) : g;
      const double2 z = normal_pair(draw_words(seed, iteration, kPurposeModes, src));
      const double sc = sqrt(2.0 * inv_or_zero(v));
      p = make_double2(sc * z.x, mirror ? -sc * z.y : sc * z.y);
      kin.add((m.kz == 0 ? 0.125 : 0.25) * v * (p.x * p.x + p.y * p.y));
    }
    st_stream(&k.st.p[g], p);
  }
  const double s = block_csum(kin, red);
  if (threadIdx.x == 0) k.w.kin_part()[blockIdx.x] = s;
}

// The dot products of the no-U-turn test over the independent real
// coordinates of a state (pair-weighted on the kz = 0 plane, distances and
// s when they are sampled): (b - a) . ra and (b - a) . rb for coordinates a,
// b and momenta ra, rb.  Block partials, then one block sums them in order.
struct NutsDotArgs {
  const double2 *qa, *qb, *ra, *rb;
  const double *da, *db, *pda, *pdb;
  const double *sa, *sb, *psa, *psb;
  int n_gal, use_d, use_s, use_c;   // use_c: u8 and phi (small[1], small[2])
  double* part;      // 2 per block
  double* out;       // 2 results
};

constexpr int kNutsDotBlocks = 256;

template <int N>
__global__ void __launch_bounds__(kEltThreads) k_nuts_dot(NutsDotArgs a) {
  __shared__ double red[2 * 2 * (kEltThreads / 64)];
  constexpr size_t NM = (size_t)N * N * (N / 2);
  CSum acc[2];
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < NM; g += (size_t)gridDim.x * blockDim.x) {
    const double w = (g % (N / 2)) == 0 ? 0.5 : 1.0;
    const double2 qa = ld_stream(&a.qa[g]), qb = ld_stream(&a.qb[g]);
    const double2 ra = ld_stream(&a.ra[g]), rb = ld_stream(&a.rb[g]);
    const double dx = qb.x - qa.x, dy = qb.y - qa.y;
    acc[0].add(w * (dx * ra.x + dy * ra.y));
    acc[1].add(w * (dx * rb.x + dy * rb.y));
  }
  if (a.use_d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n_gal; i += gridDim.x * blockDim.x) {
      const double d = a.db[i] - a.da[i];
      acc[0].add(d * a.pda[i]);
      acc[1].add(d * a.pdb[i]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = a.use_s ? 0 : 1; j < (a.use_c ? kSmallMax : 1); ++j) {
      const double d = a.sb[j] - a.sa[j];
      acc[0].add(d * a.psa[j]);
      acc[1].add(d * a.psb[j]);
    }
  }
  block_csums<2>(acc, red);
  if (threadIdx.x == 0) {
    a.part[2 * blockIdx.x] = acc[0].value();
    a.part[2 * blockIdx.x + 1] = acc[1].value();
  }
}

__global__ void __launch_bounds__(256) k_nuts_dot_final(const double* __restrict__ part, int blocks, double* out) {
  __shared__ double red[2 * 2 * 4];
  CSum acc[2];
  for (int b = threadIdx.x; b < blocks; b += blockDim.x) {
    acc[0].add(part[2 * b]);
    acc[1].add(part[2 * b + 1]);
  }
  block_csums<2>(acc, red);
  if (threadIdx.x == 0) {
    out[0] = acc[0].value();
    out[1] = acc[1].value();
  }
}

// What the host reads after a step: Psi, K0, K1 of the chain scalars.
__global__ void k_nuts_collect(const ChainScalars* cs, double* out) {
  if (threadIdx.x == 0) {
    out[0] = cs->psi;
    out[1] = cs->kin0;
    out[2] = cs->kin1;
  }
}

__global__ void k_set_chain_iter(ChainScalars* cs, int iteration) {
  if (threadIdx.x == 0) cs->iter = iteration;
}

// sum += q over the stored modes (the Monte-Carlo mean of eq:int_mc).
__global__ void __launch_bounds__(kEltThreads) k_add_modes(double2* __restrict__ sum, const double2* __restrict__ q,
                                                           size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double2 a = ld_stream(&sum[i]);
    const double2 b = ld_stream(&q[i]);
    a.x += b.x;
    a.y += b.y;
    st_stream(&sum[i], a);
  }
}

}  // namespace hamlet
