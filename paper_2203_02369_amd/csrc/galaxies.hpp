// Per-galaxy kernels: CIC binning and the likelihood of Section 2.
#pragma once

#include "common.hpp"
#include "passes.hpp"

namespace hamlet {

// Block sizes: one thread per point.  The binning kernels run in blocks of
// one wave, spread over more compute units; the likelihood kernel in blocks
// of four (its partial sums are per block, and its last block sums them all:
// smaller blocks made launches that carry several plans slower).
constexpr int kGalThreads = 64;
constexpr int kLikeThreads = 256;

// Catalogue and distance-prior data on the device (by galaxy id).
struct Catalogue {
  int n;
  const double* rhat;      // 3 n, (x, y, z) per galaxy
  const double* mu;        // observed distance modulus
  const double* sigma_mu;
  const double* cz;        // observed redshift times c, km/s
  const double* sigma_cz;  // km/s
  const double* hist;      // distance-prior density per bin (eq:D)
  int n_hist;
  double hist_w;           // bin width, Mpc/h
};

struct Cosmo {
  double om, h;            // Omega_0, little h (for mu; times eta when sampled)
  double box, spacing;     // L, L / N
  double dmax;             // c / (3 Omega_0 H0): domain of zbar(d)
  int sample_c;            // eta = h / h_fid is the fourth small coordinate
};

// Optional leapfrog update of a block of coordinates right after their
// gradient is known: p -= kick * eps * g, then (drift) q += eps * minv * p.
struct LeapUpdate {
  double* p = nullptr;       // momenta (nullptr: no update)
  const double* eps = nullptr;
  double kick = 0.0;         // 1 for merged half kicks, 0.5 for the last half kick
  int drift = 0;
  double minv = 0.0;         // inverse mass
};

// A distance in the domain of the posterior: zbar(d) real and d > 0.
__device__ __forceinline__ bool dist_ok(double d, const Cosmo& cm) { return d > 0.0 && d < cm.dmax; }

// ---------------------------------------------------------------------------
// Binning.  Positions x = o + d rhat with o = (L/2)(1,1,1) in FP64 without
// contraction, so the lower CIC node floor(x / Delta) is bit-identical to a
// plain FP64 evaluation.  Invalid distances are replaced by 1 Mpc/h for the
// geometry (their Psi is +inf anyway), which keeps every index in range.
// ---------------------------------------------------------------------------
// Where binning writes: the bucket counts and, per point, its bucket,
// lower z node and fractional offsets.
struct BinOut {
  int* count;
  int* key;
  int* cell_z;
  double* frac;
};

// Bins point i at distance d.  The next evaluation's binning is known as soon
// as a drift has moved the distances, so the drifting kernels (the
// likelihood inside a trajectory, the first kick and drift) bin their points
// right away and the counting kernel runs only before a plain gradient.
__device__ __forceinline__ void bin_point(int i, double d, const Catalogue& cat, const Cosmo& cm, int n_grid,
                                          const BinOut& bo) {
#pragma clang fp contract(off)
  if (!dist_ok(d, cm)) d = 1.0;
  const double half = 0.5 * cm.box;
  int cell[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double prod = d * cat.rhat[3 * i + a];
    const double xa = half + prod;
    const double s = xa / cm.spacing;
    const double fl = floor(s);
    bo.frac[3 * i + a] = s - fl;
    long long c = (long long)fl % n_grid;
    if (c < 0) c += n_grid;
    cell[a] = (int)c;
  }
  const int k = cell[0] * n_grid + cell[1];
  bo.key[i] = k;
  bo.cell_z[i] = cell[2];
  atomicAdd(&bo.count[k], 1);
}

__device__ __forceinline__ void bin_count_body(const double* __restrict__ dist, Catalogue cat, Cosmo cm, int n_grid,
                                               BinOut bo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cat.n) return;
  bin_point(i, dist[i], cat, cm, n_grid, bo);
}

// Exclusive scan of the N^2 bucket counts over tiles of 1024 counts, in one
// kernel: every block adds up the counts before its tile itself (the early
// tiles are read by many blocks: a few hundred KB in all at 256^3, from the
// caches), scans its tile and primes the placement cursors; the last block,
// which has read every count, writes the total and the largest count of any
// column.  No block waits for another, and integer sums do not depend on
// their order.  The placement clears the counts afterwards (each point its
// own column), so nothing here changes what another block reads.
constexpr int kScanTile = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum, int* total) {
  // inclusive scan within the wave
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      const int t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    *total = run;
  }
  __syncthreads();
  return x - v + wsum[wid];
}

__device__ __forceinline__ void
bin_scan_body(const int* __restrict__ count, int* __restrict__ off, int* __restrict__ cursor, int* __restrict__ most,
              int nkeys) {
  __shared__ int wsum[kScanTile / 64];
  __shared__ int wred[2][kScanTile / 64];
  __shared__ int total;
  const int t0 = blockIdx.x * kScanTile;
  // the counts before this tile, and the largest count up to its end
  // (16-byte loads, eight in flight per thread: t0 is a multiple of 1024)
  int s = 0, m = 0;
  const int4* c4 = reinterpret_cast<const int4*>(count);
#pragma unroll 8
  for (int j = threadIdx.x; j < t0 / 4; j += blockDim.x) {
    const int4 v = c4[j];
    s += (v.x + v.y) + (v.z + v.w);
    m = max(m, max(max(v.x, v.y), max(v.z, v.w)));
  }
  const int k = t0 + threadIdx.x;
  const int c = k < nkeys ? count[k] : 0;
  m = max(m, c);
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    m = max(m, __shfl_xor(m, o, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  if (lane == 0) {
    wred[0][wid] = s;
    wred[1][wid] = m;
  }
  __syncthreads();
  int base = 0, mx = 0;
  for (int w = 0; w < nw; ++w) {
    base += wred[0][w];
    mx = max(mx, wred[1][w]);
  }
  const int ex = block_exclusive_scan(c, wsum, &total);
  if (k < nkeys) {
    off[k] = base + ex;
    cursor[k] = base + ex;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    off[nkeys] = base + total;
    most[0] = mx;
  }
}

__device__ __forceinline__ void
bin_place_body(const int* __restrict__ key, int* __restrict__ cursor, int* __restrict__ slot_gid,
               int* __restrict__ count, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int kk = key[i];
  const int s = atomicAdd(&cursor[kk], 1);
  slot_gid[s] = i;
  count[kk] = 0;   // cleared for the next evaluation's counting
}

// Final position of each point in its column: the members of a column are
// ordered by (z cell, galaxy id), so the z passes find the points of one z
// cell as a contiguous run, and the order does not depend on the racy
// placement.  One thread per point: its rank is a count over its column.
// Writes the binned records used by the z passes and the likelihood.
template <typename T>
__device__ __forceinline__ void
bin_rank_body(const int* __restrict__ off, const int* __restrict__ key, const int* __restrict__ placed,
              const int* __restrict__ cell_z, const double* __restrict__ frac, Catalogue cat, int* __restrict__ bpos,
              T* __restrict__ rx, T* __restrict__ ry, T* __restrict__ rz, T* __restrict__ tx, T* __restrict__ ty,
              T* __restrict__ tz, int* __restrict__ iz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cat.n) return;
  const int k = key[i], z = cell_z[i];
  // the point's own record, loaded before the walk so that it arrives meanwhile
  const T r0 = (T)cat.rhat[3 * i + 0], r1 = (T)cat.rhat[3 * i + 1], r2 = (T)cat.rhat[3 * i + 2];
  const T f0 = (T)frac[3 * i + 0], f1 = (T)frac[3 * i + 1], f2 = (T)frac[3 * i + 2];
  const int s0 = off[k], s1 = off[k + 1];
  // members four at a time: their ids, then their z cells, each group of
  // loads in flight together
  constexpr int U = 4;
  int rank = 0;
  for (int s = s0; s < s1; s += U) {
    int j[U], zj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = s + u < s1 ? placed[s + u] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) zj[u] = j[u] >= 0 ? cell_z[j[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; ++u) rank += (j[u] >= 0 && (zj[u] < z || (zj[u] == z && j[u] < i))) ? 1 : 0;
  }
  const int pos = s0 + rank;
  bpos[i] = pos;
  rx[pos] = r0;
  ry[pos] = r1;
  rz[pos] = r2;
  tx[pos] = f0;
  ty[pos] = f1;
  tz[pos] = f2;
  iz[pos] = z;
}

// ---------------------------------------------------------------------------
// Likelihood (eqn:lmu, eq:vrobs, eqn:lvr, eq:kappa, eq:D) per galaxy, in
// galaxy order (so the per-galaxy arrays are read coalesced and the block
// partials do not depend on the binning); the gather's partials and the
// scatter's input sit at the galaxy's binned index.  Combines the four
// column partials of the gather into
//   u  = sum_col wx wy Pc
//   u' = sum_col (dwx wy rx + wx dwy ry) Pc + wx wy rz Qc / Delta,
// then, in FP64,
//   Psi_i = (mu_i - mu(d))^2 / 2 sigma_mu^2 + r^2 / 2 kappa^2 + ln kappa - ln N(d),
//   g_i = dPsi/du = -r / kappa^2,  dPsi/dd_i,  dPsi_i/ds,
// with r = v_obs(d) - u.  Block partials (Psi, dPsi/ds, invalid count) are
// written for a deterministic final sum.
// ---------------------------------------------------------------------------
// Binning of the next evaluation, done by the likelihood kernel inside a
// trajectory (after the drift of the distances) when `rebin` is set.  Passed
// by value: a pointer to a local copy would put it in scratch memory.
struct BinNext {
  BinOut out;
  int n_grid;
  bool rebin;
};

// Values per block of the likelihood's partial sums: Psi, dPsi/ds, invalid
// distances, a slice of the prior partials, sum g_i u_i (for dPsi/dphi),
// sum dmu_i / sigma_mu,i^2 (for dPsi/deta).
constexpr int kLikeVals = 8;

struct LikeOut {
  double* g_dist;     // dPsi/dd by galaxy id (n)
  double* part;       // kLikeVals per block (see above)
  const double* prior_part;   // prior partials of the x pass
  int n_prior;
  int n_blocks;               // this plan's blocks (ceil(n / block size)); block b sums slice b
};

template <typename T>
__device__ __forceinline__ void
like_body(const cplx_t<T>* __restrict__ part, const int* __restrict__ bpos, const double* __restrict__ frac,
          double* __restrict__ dist, const double* snl_q, Catalogue cat, Cosmo cm, T* __restrict__ gsort,
          LikeOut out, LeapUpdate lf, BinNext next) {
  __shared__ double red[2 * 6 * (kLikeThreads / 64)];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double psi = 0.0, dps = 0.0, bad = 0.0, gu = 0.0, dmw = 0.0;
  if (i < cat.n) {
    const int s = bpos[i];
    const double tx = frac[3 * i], ty = frac[3 * i + 1];
    const double rx = cat.rhat[3 * i], ry = cat.rhat[3 * i + 1], rz = cat.rhat[3 * i + 2];
    const double inv_d = 1.0 / cm.spacing;
    double u = 0.0, du = 0.0;
#pragma unroll
    for (int corner = 0; corner < 4; ++corner) {
      const int ox = corner >> 1, oy = corner & 1;
      const double wx = ox ? tx : 1.0 - tx, wy = oy ? ty : 1.0 - ty;
      const double dwx = ox ? inv_d : -inv_d, dwy = oy ? inv_d : -inv_d;
      const cplx_t<T> pq = part[4 * (size_t)s + corner];
      const double pc = (double)pq.x, qc = (double)pq.y;
      u += wx * wy * pc;
      du += (dwx * wy * rx + wx * dwy * ry) * pc + wx * wy * rz * qc * inv_d;
    }
    double d = dist[i];
    const bool ok_d = dist_ok(d, cm);
    if (!ok_d) d = 1.0;
    const double sv = snl_q[0];
    const double a3 = 3.0 * cm.om * kH0 / kC;
    const double root = sqrt(1.0 - a3 * d);
    const double zb = (2.0 / (3.0 * cm.om)) * (1.0 - root);
    const double zbp = (kH0 / kC) / root;
    const double opz = 1.0 + zb;
    const double scz = cat.sigma_cz[i];
    const double snl = kSigmaNlUnit * sv;
    const double kappa2 = snl * snl + scz * scz / (opz * opz);
    // h = eta h_fid when sampled: d_L / h in Mpc
    const double hh = cm.sample_c ? cm.h * snl_q[3] : cm.h;
    const double mu_d = 5.0 * log10(d * opz / hh) + 25.0;
    const double mup = (5.0 / log(10.0)) * (opz + d * zbp) / (d * opz);
    const double smu = cat.sigma_mu[i];
    const double dmu = cat.mu[i] - mu_d;
    const double czi = cat.cz[i];
    const double vobs = kC * (czi / kC - zb) / opz;
    const double vobsp = -kC * zbp * (1.0 + czi / kC) / (opz * opz);
    const double r = vobs - u;
    // distance prior: histogram bin of d
    const double bf = floor(d / cat.hist_w);
    const bool ok_h = bf >= 0.0 && bf < (double)cat.n_hist;
    const double lnN = ok_h ? log(cat.hist[(int)bf]) : 0.0;
    psi = dmu * dmu / (2.0 * smu * smu) + r * r / (2.0 * kappa2) + 0.5 * log(kappa2) - lnN;
    const double dk2 = 0.5 / kappa2 - 0.5 * r * r / (kappa2 * kappa2);
    const double dkappa2_dd = -2.0 * scz * scz * zbp / (opz * opz * opz);
    const double gd = -dmu * mup / (smu * smu) + (r / kappa2) * (vobsp - du) + dk2 * dkappa2_dd;
    dps = dk2 * 2.0 * kSigmaNlUnit * kSigmaNlUnit * sv;
    out.g_dist[i] = gd;
    gsort[s] = (T)(-r / kappa2);
    gu = (-r / kappa2) * u;   // u is linear in the growth rate: dPsi/dphi = sum g u / phi
    dmw = dmu / (smu * smu);  // mu(d) moves by -5 log10 eta: dPsi/deta = sum dmw 5 / (eta ln 10)
    if (lf.p) {
      const double e = lf.eps[0];
      const double pv = lf.p[i] - lf.kick * e * gd;
      lf.p[i] = pv;
      if (lf.drift) dist[i] = dist[i] + e * lf.minv * pv;
    }
    if (next.rebin) bin_point(i, dist[i], cat, cm, next.n_grid, next.out);
    bad = (ok_d && ok_h) ? 0.0 : 1.0;
  }
  // this block's slice of the prior partials
  const int per = (out.n_prior + out.n_blocks - 1) / out.n_blocks;
  const int lo = blockIdx.x * per, hi = min(out.n_prior, lo + per);
  CSum sums[6];
  sums[0].add(psi);
  sums[1].add(dps);
  sums[2].add(bad);
  for (int j = lo + threadIdx.x; j < hi; j += blockDim.x) sums[3].add(out.prior_part[j]);
  sums[4].add(gu);
  sums[5].add(dmw);
  block_csums(sums, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < 6; ++v) out.part[kLikeVals * blockIdx.x + v] = sums[v].value();
  }
}

// The small coordinates at the final sums: where they are, their momenta and
// gradient, and the leapfrog update of them once the gradient is known.
struct SmallState {
  double* q;            // s, and u8, phi, eta when sampled
  double* p;            // momenta, or nullptr: no update
  double* g;            // dPsi/d(s, u8, phi, eta) out
  double* cosmo_eval;   // u8 and phi of this evaluation, kept for the adjoint pass
  const double* eps;
  double kick;          // 1 for merged half kicks, 0.5 for the last half kick
  int drift;
  int sample_s, sample_c;
  double minv_u8, minv_phi, minv_eta, d_modes;
};

// Final deterministic sums (compensated): Psi = prior + sum of galaxy terms
// (+inf when a distance left the domain or Psi is not finite); dPsi/ds.
// With u8, phi and eta sampled the prior is E / u8^2 + D ln u8 (E the
// fiducial prior energy, D real mode coordinates), dPsi/du8 = -2 E / u8^3 +
// D / u8, dPsi/dphi = sum g_i u_i / phi, dPsi/deta = sum (dmu_i /
// sigma_mu,i^2) 5 / (eta ln 10), and Psi = +inf unless u8, phi, eta > 0.
__device__ __forceinline__ void
finalize_body(const double* __restrict__ prior_part, int n_prior, const double* __restrict__ like_part, int n_like,
              double* __restrict__ psi_out, const SmallState& sm) {
  __shared__ double red[2 * 6 * 4];   // blocks of up to 256 threads
  CSum sums[6];                       // prior, galaxy terms, dPsi/ds, invalid, sum g u, sum dmu / sigma^2
  for (int i = threadIdx.x; i < n_prior; i += blockDim.x) sums[0].add(prior_part[i]);
  for (int i = threadIdx.x; i < n_like; i += blockDim.x) {
    const double* lp = like_part + (size_t)kLikeVals * i;
    sums[1].add(lp[0]);
    sums[0].add(lp[3]);
    sums[2].add(lp[1]);
    sums[3].add(lp[2]);
    sums[4].add(lp[4]);
    sums[5].add(lp[5]);
  }
  block_csums(sums, red);
  if (threadIdx.x != 0) return;
  const double e = sums[0].value();
  double psi;
  bool ok = sums[3].value() == 0.0;
  double g[kSmallMax] = {sums[2].value(), 0.0, 0.0, 0.0};
  if (sm.sample_c) {
    const double u8 = sm.q[1], phi = sm.q[2], eta = sm.q[3];
    ok = ok && u8 > 0.0 && phi > 0.0 && eta > 0.0;
    psi = e / (u8 * u8) + sm.d_modes * log(u8) + sums[1].value();
    g[1] = -2.0 * e / (u8 * u8 * u8) + sm.d_modes / u8;
    g[2] = sums[4].value() / phi;
    g[3] = sums[5].value() * 5.0 / (eta * log(10.0));
    sm.cosmo_eval[0] = u8;
    sm.cosmo_eval[1] = phi;
  } else {
    CSum tot = sums[0];
    tot.add(sums[1].s, sums[1].c);
    psi = tot.value();
  }
  psi_out[0] = ok && isfinite(psi) ? psi : __builtin_inf();
  const int ns = sm.sample_c ? kSmallMax : 1;
  for (int k = 0; k < ns; ++k)
    if (sm.g) sm.g[k] = g[k];
  if (sm.p) {
    const double eps = sm.eps[0];
    const double minv[kSmallMax] = {1.0, sm.minv_u8, sm.minv_phi, sm.minv_eta};
    for (int k = 0; k < ns; ++k) {
      if (k == 0 && !sm.sample_s) continue;
      const double pv = sm.p[k] - sm.kick * eps * g[k];
      sm.p[k] = pv;
      if (sm.drift) sm.q[k] = sm.q[k] + eps * minv[k] * pv;
    }
  }
}

// ---------------------------------------------------------------------------
// Distance prior (eq:D), built at plan set-up: the redshift distance of
// eq:e:dz of every point (composite Simpson with 2000 intervals, summed in
// order, no contraction), then a density histogram with bins of width w on
// [0, nb w), negative distances in the first bin and one pseudo-count per
// bin: N(b) = (count_b + 1) / ((n + nb) w).  Counts are exact (whole numbers
// in FP64), so the histogram does not depend on the order of the atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double redshift_distance(double z, double om) {
#pragma clang fp contract(off)
  const int m = 2000;
  const double hstep = z / m;
  double acc = 0.0;
  for (int j = 0; j <= m; ++j) {
    const double zz = hstep * j;
    const double coef = (j == 0 || j == m) ? 1.0 : (j % 2 ? 4.0 : 2.0);
    acc += coef / sqrt(om * (1.0 + zz) * (1.0 + zz) * (1.0 + zz) + (1.0 - om));
  }
  return (kC / kH0) * (hstep / 3.0) * acc;
}

__global__ void __launch_bounds__(kGalThreads)
k_dist_prior_count(const double* __restrict__ cz, int n, double om, double w, int nb, double* __restrict__ dz,
                   double* __restrict__ hist) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = redshift_distance(cz[i] / kC, om);
  dz[i] = d;
  long long b = (long long)floor(d / w);
  b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
  atomicAdd(&hist[b], 1.0);
}

__global__ void __launch_bounds__(kGalThreads)
k_dist_prior_norm(double* __restrict__ hist, int nb, int n, double w) {
#pragma clang fp contract(off)
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  hist[b] = (hist[b] + 1.0) / ((double)(n + nb) * w);
}

// ---------------------------------------------------------------------------
// Shared launches: blockIdx.z selects the plan; galaxy grids cover the
// largest catalogue of the batch and each plan ignores blocks past its own.
// ---------------------------------------------------------------------------
template <typename T, int N> __device__ __forceinline__ Catalogue catalogue(const Ws<T, N>& w, int n_gal) {
  const PlanConst& pc = w.pc();
  Catalogue c;
  c.n = n_gal;
  c.rhat = w.rhat(); c.mu = w.mu(); c.sigma_mu = w.smu(); c.cz = w.cz(); c.sigma_cz = w.scz();
  c.hist = w.hist(n_gal);
  c.n_hist = pc.n_hist;
  c.hist_w = pc.hist_w;
  return c;
}

template <typename T, int N> __device__ __forceinline__ Cosmo cosmo(const Ws<T, N>& w) {
  const PlanConst& pc = w.pc();
  Cosmo c;
  c.om = pc.om; c.h = pc.h; c.box = pc.box; c.spacing = pc.spacing; c.dmax = pc.dmax;
  c.sample_c = pc.sample_c;
  return c;
}

template <typename T, int N> __device__ __forceinline__ BinOut bin_out(const Ws<T, N>& w) {
  return BinOut{w.count(), w.key(), w.cellz(), w.frac()};
}

template <typename T, int N>
__global__ void __launch_bounds__(kGalThreads) k_bin_count(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  bin_count_body(k.st.qd, catalogue(k.w, k.n_gal), cosmo(k.w), N, bin_out(k.w));
}

template <typename T, int N>
__global__ void __launch_bounds__(kScanTile) k_bin_scan(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  bin_scan_body(k.w.count(), k.w.off(), k.w.cursor(), k.w.most(), N * N);
}

template <typename T, int N>
__global__ void __launch_bounds__(kGalThreads) k_bin_place(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  bin_place_body(k.w.key(), k.w.cursor(), k.w.slot(), k.w.count(), k.n_gal);
}

template <typename T, int N>
__global__ void __launch_bounds__(kGalThreads) k_bin_rank(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  bin_rank_body<T>(k.w.off(), k.w.key(), k.w.slot(), k.w.cellz(), k.w.frac(), catalogue(k.w, k.n_gal), k.w.bpos(),
                   k.w.rx(), k.w.ry(), k.w.rz(), k.w.tx(), k.w.ty(), k.w.tz(), k.w.iz());
}

// Leapfrog update fused into the galaxy kernels: merged kicks with a drift
// inside a trajectory (kXMid), a last half kick (kXLast), none for a plain
// gradient (kXGrad).
__device__ __forceinline__ LeapUpdate leap_update(int x_mode, int sample, double* p, const double* eps, double minv) {
  LeapUpdate lf;
  if (x_mode == kXGrad || !sample) return lf;
  lf.p = p;
  lf.eps = eps;
  lf.kick = x_mode == kXMid ? 1.0 : 0.5;
  lf.drift = x_mode == kXMid ? 1 : 0;
  lf.minv = minv;
  return lf;
}

// The small coordinates of a plan in an evaluation of mode k.mode: kicked
// (merged half kicks and a drift inside a trajectory, a last half kick at
// its end) unless it is a plain gradient.
template <typename T, int N> __device__ __forceinline__ SmallState small_state(const Pick<T, N>& k) {
  const PlanConst& pc = k.w.pc();
  SmallState sm;
  sm.q = k.st.qs;
  sm.g = k.st.gs;
  sm.cosmo_eval = k.w.cosmo_eval();
  sm.eps = k.st.eps;
  sm.sample_s = pc.sample_s;
  sm.sample_c = pc.sample_c;
  sm.minv_u8 = pc.minv_u8;
  sm.minv_phi = pc.minv_phi;
  sm.minv_eta = pc.minv_eta;
  sm.d_modes = pc.d_modes;
  const bool update = k.mode != kXGrad && (pc.sample_s || pc.sample_c);
  sm.p = update ? k.st.ps : nullptr;
  sm.kick = k.mode == kXMid ? 1.0 : 0.5;
  sm.drift = k.mode == kXMid ? 1 : 0;
  return sm;
}

template <typename T, int N>
__global__ void __launch_bounds__(kLikeThreads) k_like(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  if ((int)(blockIdx.x * blockDim.x) >= k.n_gal) return;   // whole block past this catalogue
  const PlanConst& pc = k.w.pc();
  LikeOut lo;
  lo.g_dist = k.st.gd;
  lo.part = k.w.like_part();
  lo.prior_part = k.w.prior_part();
  lo.n_prior = pc.n_prior_part;
  lo.n_blocks = pc.n_like_part;
  like_body<T>(k.w.part(), k.w.bpos(), k.w.frac(), k.st.qd, k.st.qs, catalogue(k.w, k.n_gal), cosmo(k.w),
               k.w.gsort(), lo, leap_update(k.mode, pc.sample_d, k.st.pd, k.st.eps, pc.minv_d),
               BinNext{bin_out(k.w), N, k.mode == kXMid});
  // The plan's last block to finish completes the evaluation: it sums every
  // block's partials in block order (the final sums) and resets the ticket.
  __shared__ int last;
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(k.w.ticket(), 1) == pc.n_like_part - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  finalize_body(k.w.prior_part(), 0, k.w.like_part(), pc.n_like_part, k.st.psi, small_state(k));
  if (threadIdx.x == 0) *k.w.ticket() = 0;
}

// The final sums of a plan with no points (the likelihood kernel does them
// for the others).
template <typename T, int N>
__global__ void __launch_bounds__(256) k_finalize(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  const PlanConst& pc = k.w.pc();
  finalize_body(k.w.prior_part(), pc.n_prior_part, k.w.like_part(), pc.n_like_part, k.st.psi, small_state(k));
}

}  // namespace hamlet
