// Monopole and dipole moments of the linear velocity field in spheres about
// the observer (Section 5, monopole and dipole): for a ball of radius R
// centred on o = (L/2)(1, 1, 1),
//   M(R) = ball mean of -div v / H0   (= f times the mean density contrast),
//   D(R) = ball mean of v             (the bulk velocity, km/s),
// of the band-limited field of the modes.  A plane wave exp(i k.x) averages
// to exp(i k.o) W(|k| R) over the ball, W(y) = 3 (sin y - y cos y) / y^3, and
// exp(i k.o) = (-1)^(nx + ny + nz) at this observer, so with the velocity
// multiplier i H0 f k / k^2 and the pair weight w (1 on the kz = 0 plane,
// whose Hermitian partners are both stored, 2 elsewhere):
//   M(R)   = sum_stored w (-1)^(n) (f / N^3) Re q_k W(|k| R),
//   D_c(R) = sum_stored w (-1)^(n) (-H0 f / (N^3 k_f)) (n_c / n^2) Im q_k W(|k| R).
// One pass over the stored modes handles kMomentsRadiiPerPass radii (their
// sums stay in registers); every block writes its partial sums, and a second
// kernel adds them in block order, so the result does not depend on timing.
// FP64 throughout: the modes are the FP64 masters in both precisions.
//
// Also: the last inverse pass of the field maps in a form that adds a state's
// density contrast or radial velocity, and its square, to running sums; and
// the statistics of two fields in spherical shells about the observer.
#pragma once

#include "common.hpp"
#include "passes.hpp"
#include "workspace.hpp"

namespace hamlet {

struct MomentRadii {
  double r[kMomentsRadiiPerPass];
  int count;
};

// Coefficient m of the Taylor series of the window,
// W(y) = sum_m (-1)^m 3 (2m + 2) y^(2m) / (2m + 3)!.
__host__ __device__ constexpr double tophat_coefficient(int m) {
  double fact = 1.0;
  for (int i = 2; i <= 2 * m + 3; ++i) fact *= i;
  return (m % 2 ? -3.0 : 3.0) * (2 * m + 2) / fact;
}

// W(y); below |y| = 1/2, where sin y - y cos y cancels, the series to m = 7
// (the first term left out is below 1e-17 there).
__device__ __forceinline__ double tophat_window(double y) {
  if (fabs(y) < 0.5) {
    const double y2 = y * y;
    double acc = tophat_coefficient(7);
#pragma unroll
    for (int m = 6; m >= 0; --m) acc = acc * y2 + tophat_coefficient(m);
    return acc;
  }
  double s, c;
  sincos(y, &s, &c);
  return 3.0 * (s - y * c) / (y * y * y);
}

// One pass: partial sums of (M, Dx, Dy, Dz) for each radius of rad, per
// block, into part[block * kMomentsPassValues + 4 j + c].
template <int N>
__global__ void __launch_bounds__(256)
k_sphere_moments(const double2* __restrict__ modes, MomentRadii rad, double kf, double mono_scale,
                 double dip_scale, double* __restrict__ part) {
  __shared__ double red[kMomentsPassValues * (256 / 64)];
  constexpr int H = N / 2;
  constexpr size_t total = (size_t)N * N * H;
  double acc[kMomentsPassValues];
#pragma unroll
  for (int i = 0; i < kMomentsPassValues; ++i) acc[i] = 0.0;
  for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
    const int kz = (int)(g % H), y = (int)((g / H) % N), x = (int)(g / ((size_t)H * N));
    const int sx = signed_freq(x, N), sy = signed_freq(y, N);
    if (!retained(sx, sy, kz, N)) continue;
    const double2 q = modes[g];
    const int n2 = sx * sx + sy * sy + kz * kz;
    const double w = (kz == 0 ? 1.0 : 2.0) * (((sx + sy + kz) & 1) ? -1.0 : 1.0);
    const double a = w * mono_scale * q.x;
    const double b = -w * dip_scale * q.y / (double)n2;
    const double kmag = kf * sqrt((double)n2);
#pragma unroll
    for (int j = 0; j < kMomentsRadiiPerPass; ++j) {
      if (j < rad.count) {
        const double wr = tophat_window(kmag * rad.r[j]);
        acc[4 * j + 0] += a * wr;
        acc[4 * j + 1] += b * sx * wr;
        acc[4 * j + 2] += b * sy * wr;
        acc[4 * j + 3] += b * kz * wr;
      }
    }
  }
  block_sums<kMomentsPassValues>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kMomentsPassValues; ++i) part[(size_t)blockIdx.x * kMomentsPassValues + i] = acc[i];
  }
}

// out[t] = the sum over the blocks of a pass of value t, in a fixed order:
// one block per output value, t = 4 j + c over all radii of the call.
__global__ void __launch_bounds__(256) k_sphere_moments_sum(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256 / 64];
  const int t = blockIdx.x;
  const int pass = t / kMomentsPassValues, i = t % kMomentsPassValues;
  const double* p = part + (size_t)pass * kMomentsBlocks * kMomentsPassValues + i;
  double s[1] = {0.0};
  for (int b = threadIdx.x; b < kMomentsBlocks; b += blockDim.x) s[0] += p[(size_t)b * kMomentsPassValues];
  block_sums<1>(s, red);
  if (threadIdx.x == 0) out[t] = s[0];
}

// ---------------------------------------------------------------------------
// Inverse pass 3 adding a state's field to running sums on every node, for
// the chain's mean and scatter maps: DENSITY, delta (the third array of the
// density passes); otherwise the radial velocity v_r = v . r / |r| about the observer
// o = (L/2)(1, 1, 1), which sits on node N/2 of each axis (v_r = 0 there).
// acc[g] += value and acc[N^3 + g] += value^2, g = (x N + y) N + z; every
// node belongs to one thread, so the updates need no atomics.
template <typename T, int N, int NT, bool DENSITY>
__device__ __forceinline__ void
inv_z_acc_body(const cplx_t<T>* __restrict__ vx, const cplx_t<T>* __restrict__ vy, const cplx_t<T>* __restrict__ vz,
               const cplx_t<T>* __restrict__ tw, double* __restrict__ acc, int x0) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Pen;
  constexpr int P = S::PG, F = S::FG;
  constexpr size_t kGrid = (size_t)N * N * N;
  __shared__ C buf[LAY::size(F)];
  __shared__ C twl[N];
  const int x = x0 + blockIdx.y, y0 = blockIdx.x * P;
  load_twiddles<T, N, NT>(twl, tw);
  z_tile_spectra<T, N, NT, P, !DENSITY>(vx, vy, vz, x, y0, (1u << P) - 1u, buf);
  __syncthreads();
  lds_fft<T, N, F, LAY, NT, +1>(buf, twl);
  auto comp = [&](int p, int c, int z) {
    const C v = buf[LAY::idx(z, zslot_f(p, c))];
    return (double)(zslot_part(p, c) ? v.y : v.x);
  };
  for (int idx = threadIdx.x; idx < P * N; idx += NT) {
    const int z = idx % N, p = idx / N;
    double val;
    if constexpr (DENSITY) {
      val = comp(p, 2, z);
    } else {
      const int rx = x - N / 2, ry = y0 + p - N / 2, rz = z - N / 2;
      const int r2 = rx * rx + ry * ry + rz * rz;
      const double dot = rx * comp(p, 0, z) + ry * comp(p, 1, z) + rz * comp(p, 2, z);
      val = r2 > 0 ? dot / sqrt((double)r2) : 0.0;
    }
    const size_t g = ((size_t)x * N + (y0 + p)) * N + z;
    acc[g] += val;
    acc[kGrid + g] += val * val;
  }
}

template <typename T, int N, int NT, bool DENSITY>
__global__ void __launch_bounds__(NT) k_inv_z_acc(Launch L, int x0, double* acc) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  inv_z_acc_body<T, N, NT, DENSITY>(k.w.v0(), k.w.v1(), k.w.v2(), k.w.tw(), acc, x0);
}

// ---------------------------------------------------------------------------
// Statistics in spherical shells about the observer (Section 5, correlation
// coefficients): shell s holds the nodes at distance |r| in
// [s w, (s + 1) w), r = (j - N/2) h per axis (the observer is node N/2),
// h = L / N.  Per shell: the node count, mean and scatter (population
// standard deviation) of fields a and b over its nodes, and their Pearson
// correlation coefficient.  Two sweeps, as the definitions read: the means,
// then the sums of the centred products (no cancellation for a field whose
// scatter is small against its mean).  Each sweep has two stages, both in
// fixed order: each block sums the nodes of a 4 x 8 x 16 tile per shell that
// the tile reaches (a few consecutive shells, the range found from the
// tile's nearest and farthest node), and one block per shell adds those
// partials in block order.
// ---------------------------------------------------------------------------
constexpr int kShellTX = 4, kShellTY = 8, kShellTZ = 16;
constexpr int kShellThreads = 256;
constexpr int kShellFinishThreads = 1024;
constexpr int kShellsPerReduce = 1;   // shells a block reduces together (4 measured slower)
constexpr int kShellNodes = kShellTX * kShellTY * kShellTZ;
constexpr int kShellValues = 3;   // sweep 1: count, sum a, sum b; sweep 2: sum da^2, sum db^2, sum da db
constexpr int kShellOut = 6;
constexpr int kShellMax = 4096;

struct ShellGeom {
  double h, width;   // node spacing, shell width (Mpc/h)
  int n, n_shells;
  int slots;         // partials stored per block (most shells a tile reaches)
};

__host__ __device__ inline int shell_index(int r2, const ShellGeom& g) {
  return (int)floor(sqrt((double)r2) * g.h / g.width);
}

// Shells [lo, hi] (hi clamped to the last shell) that tile (bx, by, bz)
// reaches: the squared distance of its nearest and farthest node, per axis.
__host__ __device__ inline int2 shell_range(int bx, int by, int bz, const ShellGeom& g) {
  const int half = g.n / 2;
  int dmin = 0, dmax = 0;
  const int start[3] = {bx * kShellTX, by * kShellTY, bz * kShellTZ};
  const int len[3] = {kShellTX, kShellTY, kShellTZ};
  for (int a = 0; a < 3; ++a) {
    const int lo = start[a] - half, hi = start[a] + len[a] - 1 - half;
    const int alo = lo < 0 ? -lo : lo, ahi = hi < 0 ? -hi : hi;
    const int mn = (lo <= 0 && hi >= 0) ? 0 : (alo < ahi ? alo : ahi), mx = alo > ahi ? alo : ahi;
    dmin += mn * mn;
    dmax += mx * mx;
  }
  const int s1 = shell_index(dmax, g);
  return make_int2(shell_index(dmin, g), s1 < g.n_shells - 1 ? s1 : g.n_shells - 1);
}

// Stage 1 of a sweep: grid (N / 16, N / 8, N / 4) = (tile z, y, x), z
// fastest, so that blocks dispatched together read neighbouring pieces of the
// same rows; part[(block * slots + s - lo) * 3 + v], block = (bx ny + by) nz + bz.  Sweep 2 (CENTRED) reads the means
// of shell s from out[s * 6 + 1] and out[s * 6 + 3].
template <bool CENTRED>
__global__ void __launch_bounds__(kShellThreads)
k_shell_part(const double* __restrict__ a, const double* __restrict__ b, ShellGeom g, const double* __restrict__ out,
             double* __restrict__ part) {
  constexpr int V = kShellValues * kShellsPerReduce;
  __shared__ double red[V * (kShellThreads / 64)];
  const int bx = blockIdx.z, by = blockIdx.y, bz = blockIdx.x;
  const int2 range = shell_range(bx, by, bz, g);
  if (range.x > range.y) return;   // block-uniform: every node lies beyond the last shell
  const size_t blk = ((size_t)bx * gridDim.y + by) * gridDim.x + bz;
  constexpr int K = kShellNodes / kShellThreads;
  double va[K], vb[K];
  int sh[K];
  const int half = g.n / 2;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + k * kShellThreads;
    const int x = bx * kShellTX + i / (kShellTY * kShellTZ);
    const int y = by * kShellTY + (i / kShellTZ) % kShellTY;
    const int z = bz * kShellTZ + i % kShellTZ;
    const size_t node = ((size_t)x * g.n + y) * g.n + z;
    const int rx = x - half, ry = y - half, rz = z - half;
    sh[k] = shell_index(rx * rx + ry * ry + rz * rz, g);
    va[k] = a[node];
    vb[k] = b ? b[node] : 0.0;
  }
  const int last = min(range.y, range.x + g.slots - 1);
  for (int s0 = range.x; s0 <= last; s0 += kShellsPerReduce) {
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
#pragma unroll
    for (int j = 0; j < kShellsPerReduce; ++j) {
      const int s = s0 + j;
      if (s > last) break;
      double ma = 0.0, mb = 0.0;
      if constexpr (CENTRED) {
        ma = out[(size_t)s * kShellOut + 1];
        mb = out[(size_t)s * kShellOut + 3];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (sh[k] == s) {
          if constexpr (CENTRED) {
            const double da = va[k] - ma, db = vb[k] - mb;
            acc[3 * j + 0] += da * da;
            acc[3 * j + 1] += db * db;
            acc[3 * j + 2] += da * db;
          } else {
            acc[3 * j + 0] += 1.0;
            acc[3 * j + 1] += va[k];
            acc[3 * j + 2] += vb[k];
          }
        }
      }
    }
    block_sums<V>(acc, red);
    if (threadIdx.x == 0) {
      for (int j = 0; j < kShellsPerReduce && s0 + j <= last; ++j) {
#pragma unroll
        for (int v = 0; v < kShellValues; ++v)
          part[(blk * g.slots + (s0 + j - range.x)) * kShellValues + v] = acc[3 * j + v];
      }
    }
  }
}

// Stage 2 of a sweep: one block per shell.  out[s * 6 + ...] = count,
// mean a, scatter a, mean b, scatter b, correlation; sweep 1 writes the
// count and the means, sweep 2 the rest.  NaN where undefined: an empty
// shell, or a field constant over it (its correlation).
template <bool CENTRED>
__global__ void __launch_bounds__(kShellFinishThreads)
k_shell_finish(const double* __restrict__ part, ShellGeom g, double* __restrict__ out) {
  __shared__ double red[kShellValues * (kShellFinishThreads / 64)];
  const int s = blockIdx.x;
  const int nbx = g.n / kShellTX, nby = g.n / kShellTY, nbz = g.n / kShellTZ;
  const int blocks = nbx * nby * nbz;
  double acc[kShellValues] = {0.0, 0.0, 0.0};
  for (int blk = threadIdx.x; blk < blocks; blk += kShellFinishThreads) {
    const int bz = blk % nbz, by = (blk / nbz) % nby, bx = blk / (nbz * nby);
    const int2 range = shell_range(bx, by, bz, g);
    if (s < range.x || s > range.y || s - range.x >= g.slots) continue;
    const double* p = part + ((size_t)blk * g.slots + (s - range.x)) * kShellValues;
#pragma unroll
    for (int v = 0; v < kShellValues; ++v) acc[v] += p[v];
  }
  block_sums<kShellValues>(acc, red);
  if (threadIdx.x == 0) {
    const double nan = __builtin_nan("");
    double* o = out + (size_t)s * kShellOut;
    if constexpr (!CENTRED) {
      const double n = acc[0];
      o[0] = n;
      o[1] = n > 0.0 ? acc[1] / n : nan;
      o[3] = n > 0.0 ? acc[2] / n : nan;
    } else {
      const double n = o[0];
      if (n > 0.0) {
        const double va = acc[0] / n, vb = acc[1] / n;
        o[2] = sqrt(va);
        o[4] = sqrt(vb);
        o[5] = (va > 0.0 && vb > 0.0) ? (acc[2] / n) / sqrt(va * vb) : nan;
      } else {
        o[2] = o[4] = o[5] = nan;
      }
    }
  }
}

}  // namespace hamlet
