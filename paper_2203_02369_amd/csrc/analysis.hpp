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
// W depends on a mode only through |n|^2, so each pass first tabulates
// W(k_f sqrt(n^2) R) for its radii over the 3 (N/2)^2 + 1 values of n^2 (the
// same expression the modes would evaluate, so the same values), and the
// pass over the modes reads the table instead of evaluating two FP64
// transcendentals per mode and radius.
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

// The window of a pass: wtab[n2 * kMomentsRadiiPerPass + j] = W(k_f sqrt(n2)
// R_j) for n2 = 0 .. 3 (N/2)^2 (zero for the radii past rad.count).
template <int N>
__global__ void __launch_bounds__(256) k_sphere_window(MomentRadii rad, double kf, double* __restrict__ wtab) {
  constexpr int kN2 = 3 * (N / 2) * (N / 2) + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kN2 * kMomentsRadiiPerPass) return;
  const int n2 = i / kMomentsRadiiPerPass, j = i % kMomentsRadiiPerPass;
  const double kmag = kf * sqrt((double)n2);
  wtab[i] = j < rad.count ? tophat_window(kmag * rad.r[j]) : 0.0;
}

// One pass: partial sums of (M, Dx, Dy, Dz) for each radius of rad, per
// block, into part[block * kMomentsPassValues + 4 j + c].
template <int N>
__global__ void __launch_bounds__(256)
k_sphere_moments(const double2* __restrict__ modes, MomentRadii rad, const double* __restrict__ wtab,
                 double mono_scale, double dip_scale, double* __restrict__ part) {
  static_assert(kMomentsRadiiPerPass % 2 == 0, "the window is read in pairs");
  __shared__ double red[kMomentsPassValues * (256 / 64)];
  constexpr int H = N / 2;
  constexpr size_t total = (size_t)N * N * H;
  double acc[kMomentsPassValues];
#pragma unroll
  for (int i = 0; i < kMomentsPassValues; ++i) acc[i] = 0.0;
  // U modes per loop turn: per mode its index, whether it is retained, |n|^2
  // and the loads of the mode and its window, all before any arithmetic on
  // them.  U = 1 measured fastest (0.18 ms per 16-radius call at 256^3;
  // U = 2: 0.21, and the same loop without the per-mode arrays, skipping
  // excluded modes before their loads: 0.25).
  constexpr int U = 1;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t g0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < total; g0 += U * stride) {
    double2 q[U];
    double wn[U][kMomentsRadiiPerPass];
    int n2[U], sx[U], sy[U], kz[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t g = g0 + u * stride;
      kz[u] = (int)(g % H);
      sy[u] = signed_freq((int)((g / H) % N), N);
      sx[u] = signed_freq((int)(g / ((size_t)H * N)), N);
      ok[u] = g < total && retained(sx[u], sy[u], kz[u], N);
      n2[u] = sx[u] * sx[u] + sy[u] * sy[u] + kz[u] * kz[u];
      if (ok[u]) {
        q[u] = modes[g];
        const double2* wp = reinterpret_cast<const double2*>(wtab + (size_t)n2[u] * kMomentsRadiiPerPass);
#pragma unroll
        for (int j = 0; j < kMomentsRadiiPerPass / 2; ++j) {
          const double2 v = wp[j];
          wn[u][2 * j] = v.x;
          wn[u][2 * j + 1] = v.y;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      const double w = (kz[u] == 0 ? 1.0 : 2.0) * (((sx[u] + sy[u] + kz[u]) & 1) ? -1.0 : 1.0);
      const double a = w * mono_scale * q[u].x;
      const double b = -w * dip_scale * q[u].y / (double)n2[u];
#pragma unroll
      for (int j = 0; j < kMomentsRadiiPerPass; ++j) {
        if (j < rad.count) {
          const double wr = wn[u][j];
          acc[4 * j + 0] += a * wr;
          acc[4 * j + 1] += b * sx[u] * wr;
          acc[4 * j + 2] += b * sy[u] * wr;
          acc[4 * j + 3] += b * kz[u] * wr;
        }
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
// scatter is small against its mean).
//
// Each sweep runs shell by shell.  Block (x, s) adds the nodes of shell s
// in the plane x: in a row y within reach, the nodes that can lie in the
// shell form at most two runs of z (|r_z| between bounds found from the
// shell's radii, widened by a node on each side), and each candidate counts
// only if shell_index puts it in s, so every node is assigned exactly as
// node by node.  Groups of 16 lanes take the rows in turn and walk the runs
// 16 nodes at a time (128-byte pieces of a row), each lane summing in
// order; one block sum at the end.  The finish adds the N plane partials of
// a shell in x order, so reruns are bit-identical.
// ---------------------------------------------------------------------------
constexpr int kShellThreads = 256;
constexpr int kShellGroup = 16;          // lanes that walk one row
constexpr int kShellFinishThreads = 256;
constexpr int kShellValues = 3;   // sweep 1: count, sum a, sum b; sweep 2: sum da^2, sum db^2, sum da db
constexpr int kShellOut = 6;
constexpr int kShellMax = 4096;

struct ShellGeom {
  double h, width;   // node spacing, shell width (Mpc/h)
  int n, n_shells;
};

__host__ __device__ inline int shell_index(int r2, const ShellGeom& g) {
  return (int)floor(sqrt((double)r2) * g.h / g.width);
}

// Squared radii (in nodes^2) that bound shell s, widened by 2 for the
// rounding of shell_index at the shell's faces: every node of the shell has
// r2 in [lo, hi].
__device__ __forceinline__ double2 shell_r2_bounds(int s, const ShellGeom& g) {
  const double c = g.width / g.h;
  const double r0 = s * c, r1 = (s + 1) * c;
  return make_double2(r0 * r0 - 2.0, r1 * r1 + 2.0);
}

// Per plane x, shell s: partial sums into part[(s N + x) 3 + v].  Sweep 2
// (CENTRED) reads the means of shell s from out[s * 6 + 1] and out[s * 6 + 3].
template <bool CENTRED>
__global__ void __launch_bounds__(kShellThreads)
k_shell_part(const double* __restrict__ a, const double* __restrict__ b, ShellGeom g, const double* __restrict__ out,
             double* __restrict__ part) {
  __shared__ double red[kShellValues * (kShellThreads / 64)];
  const int x = blockIdx.x, s = blockIdx.y, n = g.n, half = n / 2;
  const int rx = x - half;
  const double2 bd = shell_r2_bounds(s, g);
  double ma = 0.0, mb = 0.0;
  if constexpr (CENTRED) {
    ma = out[(size_t)s * kShellOut + 1];
    mb = out[(size_t)s * kShellOut + 3];
  }
  double acc[kShellValues] = {0.0, 0.0, 0.0};
  const double reach = bd.y - (double)rx * rx;   // ry^2 + rz^2 at most this
  if (reach >= 0.0) {
    const double ry_reach = sqrt(reach);   // (compared before any conversion: a wide shell can reach far)
    const int ry_max = ry_reach >= half ? half : min((int)floor(ry_reach) + 1, half);
    const int group = threadIdx.x / kShellGroup, lane = threadIdx.x % kShellGroup;
    constexpr int kGroups = kShellThreads / kShellGroup;
    for (int ry = -ry_max + group; ry <= min(ry_max, half - 1); ry += kGroups) {
      const int rho2 = rx * rx + ry * ry;
      const double hi = bd.y - rho2;
      if (hi < 0.0) continue;
      const double lo = bd.x - rho2, slo = lo <= 0.0 ? 0.0 : sqrt(lo), shi = sqrt(hi);
      if (slo > half + 1) continue;   // the shell starts beyond this row's nodes
      const int a0 = max(0, (int)floor(slo) - 1);
      const int a1 = shi >= half ? half : (int)ceil(shi) + 1;
      const size_t row = ((size_t)x * n + (ry + half)) * n + half;   // node of r_z = 0
      // the runs r_z in [-a1, -a0] and [a0, a1] (one run when a0 = 0),
      // clipped to the grid's r_z in [-N/2, N/2 - 1]
      for (int run = 0; run < 2; ++run) {
        int z0, z1;
        if (run == 0) {
          z0 = -min(a1, half);
          z1 = a0 == 0 ? min(a1, half - 1) : -a0;
        } else {
          if (a0 == 0) break;
          z0 = a0;
          z1 = min(a1, half - 1);
        }
        for (int rz = z0 + lane; rz <= z1; rz += kShellGroup) {
          if (shell_index(rho2 + rz * rz, g) != s) continue;
          const size_t node = row + rz;
          const double va = a[node], vb = b ? b[node] : 0.0;
          if constexpr (CENTRED) {
            const double da = va - ma, db = vb - mb;
            acc[0] += da * da;
            acc[1] += db * db;
            acc[2] += da * db;
          } else {
            acc[0] += 1.0;
            acc[1] += va;
            acc[2] += vb;
          }
        }
      }
    }
  }
  block_sums<kShellValues>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < kShellValues; ++v) part[((size_t)s * n + x) * kShellValues + v] = acc[v];
  }
}

// Stage 2 of a sweep: one block per shell adds its N plane partials in x
// order.  out[s * 6 + ...] = count, mean a, scatter a, mean b, scatter b,
// correlation; sweep 1 writes the count and the means, sweep 2 the rest.
// NaN where undefined: an empty shell, or a field constant over it (its
// correlation).
template <bool CENTRED>
__global__ void __launch_bounds__(kShellFinishThreads)
k_shell_finish(const double* __restrict__ part, ShellGeom g, double* __restrict__ out) {
  __shared__ double red[kShellValues * (kShellFinishThreads / 64)];
  const int s = blockIdx.x;
  double acc[kShellValues] = {0.0, 0.0, 0.0};
  for (int x = threadIdx.x; x < g.n; x += kShellFinishThreads) {
    const double* p = part + ((size_t)s * g.n + x) * kShellValues;
#pragma unroll
    for (int v = 0; v < kShellValues; ++v) acc[v] += p[v];
  }
  block_sums<kShellValues>(acc, red);
  if (threadIdx.x == 0) {
    const double nan = __builtin_nan("");
    double* o = out + (size_t)s * kShellOut;
    if constexpr (!CENTRED) {
      const double cnt = acc[0];
      o[0] = cnt;
      o[1] = cnt > 0.0 ? acc[1] / cnt : nan;
      o[3] = cnt > 0.0 ? acc[2] / cnt : nan;
    } else {
      const double cnt = o[0];
      if (cnt > 0.0) {
        const double va = acc[0] / cnt, vb = acc[1] / cnt;
        o[2] = sqrt(va);
        o[4] = sqrt(vb);
        o[5] = (va > 0.0 && vb > 0.0) ? (acc[2] / cnt) / sqrt(va * vb) : nan;
      } else {
        o[2] = o[4] = o[5] = nan;
      }
    }
  }
}

}  // namespace hamlet
