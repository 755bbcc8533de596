// The six batched FFT passes of one log-posterior-and-gradient evaluation.
//
// Layouts (row-major, last index fastest):
//   modes, gradient, momenta   double2 [kx][ky][kz], kz in [0, N/2)
//   spectral intermediates     cplx<T> [i][j][kz],   kz in [0, N/2)
// The kz = N/2 plane carries only excluded (Nyquist) modes and is never
// stored.  After a pass along an axis that axis index is a real-space one.
//
// Velocity (eq:vel-field): v_c = N^-3 sum_k m_c(k) dhat_k e^{+i k.x}, with
// m_c / N^3 = i kfac(k) n_c, kfac = H0 f / (N^3 k_f n^2), n_c the signed
// integer wave number and k_f = 2 pi / L.  Since n_y, n_z are constant
// along an x pencil and n_z along a y pencil, only two spectral arrays
// leave the first pass: A = IFFT_x(i kfac dhat), B = IFFT_x(n_x i kfac dhat);
// then V_x = IFFT_y(B), V_y = IFFT_y(n_y A), V_z' = IFFT_y(A), and n_z is
// applied to V_z' in the last (z, complex-to-real) pass.  The adjoint runs
// the same factorisation backwards:
//   S1 = n_y FFT_y(Gy) + FFT_y(n_z Gz),  S2 = FFT_y(Gx),
//   sum_c n_c Ghat_c = FFT_x(S1) + n_x FFT_x(S2),
// and the mode gradient (complex convention dPsi/dRe + i dPsi/dIm) is
//   G = 2 dhat / sigma_k^2 - 2 i kfac sum_c n_c Ghat_c      (eq:prior-k + adjoint).
#pragma once

#include "common.hpp"
#include "fft.hpp"

namespace hamlet {

constexpr int kPassThreads = 256;

// Chunk of contiguous kz columns per strided-pass tile, pencils per z tile.
template <typename T, int N> struct PassShape {
  static constexpr int W = (sizeof(T) == 4 ? 16 : 8) < N / 2 ? (sizeof(T) == 4 ? 16 : 8) : N / 2;
  static constexpr int P = (sizeof(T) == 4 ? 16 : 8) < N ? (sizeof(T) == 4 ? 16 : 8) : N;
  static constexpr int H = N / 2;
  static constexpr int CHUNKS = H / W;
  static constexpr int ELEMS = N * W;
  static constexpr int EPT = (ELEMS + kPassThreads - 1) / kPassThreads;
};

// Tables indexed by n^2 = nx^2 + ny^2 + nz^2 (0 .. 3 (N/2)^2).
struct ModeTables {
  const double* kfac;      // H0 f / (N^3 k_f n^2), 0 at n^2 = 0
  const double* inv_var;   // 1 / sigma_k^2, 0 where P = 0
  const double* var;       // sigma_k^2 = N^6 P / V
};

// Deterministic block sum of a double (wave64 shuffles, then LDS).
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;   // valid in thread 0
}

// ---------------------------------------------------------------------------
// Inverse pass 1 (along x): multiplier, prior energy, two spectral outputs.
// Tile: fixed ky, kz chunk [z0, z0 + W), all kx.  Grid (N, CHUNKS).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kPassThreads)
k_inv_x(const double2* __restrict__ modes, ModeTables tab, const cplx_t<T>* __restrict__ tw,
        cplx_t<T>* __restrict__ outA, cplx_t<T>* __restrict__ outB, double* __restrict__ prior_part) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  constexpr int W = S::W, H = S::H;
  __shared__ C tile[S::ELEMS];
  __shared__ C twl[N];
  __shared__ double red[kPassThreads / 64];
  load_twiddles<T, N, kPassThreads>(twl, tw);
  const int y = blockIdx.x, z0 = blockIdx.y * W;
  const int sy = signed_freq(y, N);
  double2 ain[S::EPT];
  double prior = 0.0;
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    ain[e] = make_double2(0.0, 0.0);
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W, kz = z0 + w;
      const int sx = signed_freq(x, N);
      const double2 q = modes[((size_t)x * N + y) * H + kz];
      if (retained(sx, sy, kz, N)) {
        const int n2 = sx * sx + sy * sy + kz * kz;
        const double wk = kz == 0 ? 0.5 : 1.0;
        prior += wk * (q.x * q.x + q.y * q.y) * tab.inv_var[n2];
        const double kf = tab.kfac[n2];
        ain[e] = make_double2(-kf * q.y, kf * q.x);   // i kfac q
      }
      tile[x * W + w] = cconvert<C>(ain[e]);
    }
  }
  const double ps = block_sum(prior, red);
  if (threadIdx.x == 0) prior_part[blockIdx.y * gridDim.x + blockIdx.x] = ps;
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, +1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W;
      outA[((size_t)x * N + y) * H + z0 + w] = tile[x * W + w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W;
      const double sx = (double)signed_freq(x, N);
      tile[x * W + w] = cconvert<C>(make_double2(sx * ain[e].x, sx * ain[e].y));
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, +1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W;
      outB[((size_t)x * N + y) * H + z0 + w] = tile[x * W + w];
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse pass 2 (along y).  Tile: fixed x, kz chunk, all ky.  Grid (N, CHUNKS).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kPassThreads)
k_inv_y(const cplx_t<T>* __restrict__ inA, const cplx_t<T>* __restrict__ inB, const cplx_t<T>* __restrict__ tw,
        cplx_t<T>* __restrict__ vx, cplx_t<T>* __restrict__ vy, cplx_t<T>* __restrict__ vz) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  constexpr int W = S::W, H = S::H;
  __shared__ C tile[S::ELEMS];
  __shared__ C twl[N];
  load_twiddles<T, N, kPassThreads>(twl, tw);
  const int x = blockIdx.x, z0 = blockIdx.y * W;
  C a[S::EPT];
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      const size_t g = ((size_t)x * N + y) * H + z0 + w;
      a[e] = inA[g];
      tile[y * W + w] = inB[g];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, +1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      vx[((size_t)x * N + y) * H + z0 + w] = tile[y * W + w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      tile[y * W + w] = cscale(a[e], (T)signed_freq(y, N));
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, +1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      vy[((size_t)x * N + y) * H + z0 + w] = tile[y * W + w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      tile[y * W + w] = a[e];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, +1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      vz[((size_t)x * N + y) * H + z0 + w] = tile[y * W + w];
    }
  }
}

// Galaxies binned by CIC column (ix, iy) of their lower corner, in sorted
// order s; bucket key = ix * N + iy, members off[key] .. off[key + 1].
template <typename T> struct Binned {
  const int* off;          // N^2 + 1
  const T* rx; const T* ry; const T* rz;   // rhat
  const T* tx; const T* ty; const T* tz;   // fractional offsets in the cell
  const int* iz;           // lower z node
};

// Transform slot of the real pencil of component c of pencil p in a z tile:
// pairs of pencils (2m, 2m+1) fill three complex transforms
//   3m   : (vx_2m,   vy_2m)      3m+1 : (vz_2m, vz_2m+1)      3m+2 : (vx_2m+1, vy_2m+1)
// and the real pencil is the real (slot 0) or imaginary (slot 1) part.
__device__ __forceinline__ int zslot_f(int p, int c) {
  const int m = p >> 1, odd = p & 1;
  return c == 2 ? 3 * m + 1 : 3 * m + (odd ? 2 : 0);
}
__device__ __forceinline__ int zslot_part(int p, int c) {
  return c == 0 ? 0 : (c == 1 ? 1 : (p & 1));
}
template <typename C> __device__ __forceinline__ decltype(C{}.x) part_of(C v, int slot) { return slot ? v.y : v.x; }

// ---------------------------------------------------------------------------
// Inverse pass 3 (along z, complex-to-real) fused with the CIC gather.
// Tile: fixed x, pencils y0 .. y0 + P.  Grid (N, N / P).
// Writes, for every galaxy whose CIC stencil touches a pencil of the tile,
// the column partials of its projected velocity (eqn:lvr):
//   Pc = sum_c rhat_c [(1 - tz) v_c(z0) + tz v_c(z1)],  Qc = sum_c rhat_c [v_c(z1) - v_c(z0)]
// into part[4 s + corner], corner = 2 (x - ix) + (y - iy).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kPassThreads)
k_inv_z_gather(const cplx_t<T>* __restrict__ vx, const cplx_t<T>* __restrict__ vy, const cplx_t<T>* __restrict__ vz,
               const cplx_t<T>* __restrict__ tw, Binned<T> bins, cplx_t<T>* __restrict__ part) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  constexpr int P = S::P, H = S::H, F = 3 * P / 2;
  __shared__ C buf[F * N];
  __shared__ C twl[N];
  load_twiddles<T, N, kPassThreads>(twl, tw);
  const int x = blockIdx.x, y0 = blockIdx.y * P;
  // Build Z = A + i B with A, B the Hermitian half spectra of the two real
  // pencils of each transform (Nyquist entry zero, DC entries real).
  for (int idx = threadIdx.x; idx < F * H; idx += kPassThreads) {
    const int k = idx % H, f = idx / H;
    const int m = f / 3, r = f % 3;
    C av, bv;
    if (r == 1) {
      const size_t g0 = ((size_t)x * N + y0 + 2 * m) * H + k;
      av = cscale(vz[g0], (T)k);
      bv = cscale(vz[g0 + H], (T)k);
    } else {
      const size_t g = ((size_t)x * N + y0 + 2 * m + (r == 2 ? 1 : 0)) * H + k;
      av = vx[g];
      bv = vy[g];
    }
    C* row = buf + f * N;
    if (k == 0) {
      row[0] = cmake<C>(av.x, bv.x);
      row[H] = cmake<C>((T)0, (T)0);
    } else {
      row[k] = cmake<C>(av.x - bv.y, av.y + bv.x);          // A + i B
      row[N - k] = cmake<C>(av.x + bv.y, bv.x - av.y);      // conj(A) + i conj(B)
    }
  }
  __syncthreads();
  lds_fft<T, N, F, 1, N, true, kPassThreads, +1>(buf, twl);
  // Gather: one thread per (pencil, corner), bucket members in sorted order.
  if (threadIdx.x < 4 * P) {
    const int p = threadIdx.x >> 2, corner = threadIdx.x & 3;
    const int ox = corner >> 1, oy = corner & 1;
    const int y = y0 + p;
    const int key = ((x - ox + N) & (N - 1)) * N + ((y - oy + N) & (N - 1));
    const int s0 = bins.off[key], s1 = bins.off[key + 1];
    const C* fx = buf + zslot_f(p, 0) * N;
    const C* fy = buf + zslot_f(p, 1) * N;
    const C* fz = buf + zslot_f(p, 2) * N;
    const int sz = zslot_part(p, 2);
    for (int s = s0; s < s1; ++s) {
      const int z0 = bins.iz[s], z1 = (z0 + 1) & (N - 1);
      const T tz = bins.tz[s];
      const T rx = bins.rx[s], ry = bins.ry[s], rz = bins.rz[s];
      const T ax0 = fx[z0].x, ax1 = fx[z1].x;
      const T ay0 = fy[z0].y, ay1 = fy[z1].y;
      const T az0 = part_of(fz[z0], sz), az1 = part_of(fz[z1], sz);
      const T omt = (T)1 - tz;
      const T pc = rx * (omt * ax0 + tz * ax1) + ry * (omt * ay0 + tz * ay1) + rz * (omt * az0 + tz * az1);
      const T qc = rx * (ax1 - ax0) + ry * (ay1 - ay0) + rz * (az1 - az0);
      part[4 * (size_t)s + corner] = cmake<C>(pc, qc);
    }
  }
}

// ---------------------------------------------------------------------------
// Forward pass 1 (along z, real-to-complex) fused with the CIC scatter-add:
// each pencil of the tile is built in LDS from the galaxies whose stencil
// touches it, one thread per pencil adding contributions in a fixed order
// (corner, then sorted index), so the result is deterministic.
//   G_c(x_j) = sum_i g_i rhat_ic W_i(x_j)  (adjoint of the gather)
// Outputs Gx, Gy and n_z Gz on kz in [0, N/2).  Grid (N, N / P).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kPassThreads)
k_fwd_z_scatter(const T* __restrict__ gsort, Binned<T> bins, const cplx_t<T>* __restrict__ tw,
                cplx_t<T>* __restrict__ gx, cplx_t<T>* __restrict__ gy, cplx_t<T>* __restrict__ gz) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  constexpr int P = S::P, H = S::H, F = 3 * P / 2;
  __shared__ C buf[F * N];
  __shared__ C twl[N];
  load_twiddles<T, N, kPassThreads>(twl, tw);
  for (int i = threadIdx.x; i < F * N; i += kPassThreads) buf[i] = cmake<C>((T)0, (T)0);
  __syncthreads();
  const int x = blockIdx.x, y0 = blockIdx.y * P;
  if (threadIdx.x < P) {
    const int p = threadIdx.x, y = y0 + p;
    T* rowx = reinterpret_cast<T*>(buf + zslot_f(p, 0) * N) + zslot_part(p, 0);
    T* rowy = reinterpret_cast<T*>(buf + zslot_f(p, 1) * N) + zslot_part(p, 1);
    T* rowz = reinterpret_cast<T*>(buf + zslot_f(p, 2) * N) + zslot_part(p, 2);
    for (int corner = 0; corner < 4; ++corner) {
      const int ox = corner >> 1, oy = corner & 1;
      const int key = ((x - ox + N) & (N - 1)) * N + ((y - oy + N) & (N - 1));
      const int s0 = bins.off[key], s1 = bins.off[key + 1];
      for (int s = s0; s < s1; ++s) {
        const T tx = bins.tx[s], ty = bins.ty[s], tz = bins.tz[s];
        const T wxy = (ox ? tx : (T)1 - tx) * (oy ? ty : (T)1 - ty);
        const T gw = gsort[s] * wxy;
        const int z0 = bins.iz[s], z1 = (z0 + 1) & (N - 1);
        const T w0 = (T)1 - tz, w1 = tz;
        const T cx = gw * bins.rx[s], cy = gw * bins.ry[s], cz = gw * bins.rz[s];
        rowx[2 * z0] += cx * w0; rowx[2 * z1] += cx * w1;
        rowy[2 * z0] += cy * w0; rowy[2 * z1] += cy * w1;
        rowz[2 * z0] += cz * w0; rowz[2 * z1] += cz * w1;
      }
    }
  }
  __syncthreads();
  lds_fft<T, N, F, 1, N, true, kPassThreads, -1>(buf, twl);
  // Split each transform Z of a + i b into the half spectra
  //   A_k = (Z_k + conj Z_{N-k}) / 2,   B_k = (Z_k - conj Z_{N-k}) / (2 i).
  for (int idx = threadIdx.x; idx < F * H; idx += kPassThreads) {
    const int k = idx % H, f = idx / H;
    const int m = f / 3, r = f % 3;
    const C* row = buf + f * N;
    const C zk = row[k];
    const C zm = row[(N - k) & (N - 1)];
    const T half = (T)0.5;
    const C av = cmake<C>(half * (zk.x + zm.x), half * (zk.y - zm.y));
    const C bv = cmake<C>(half * (zk.y + zm.y), half * (zm.x - zk.x));
    if (r == 1) {
      const size_t g0 = ((size_t)x * N + y0 + 2 * m) * H + k;
      gz[g0] = cscale(av, (T)k);
      gz[g0 + H] = cscale(bv, (T)k);
    } else {
      const size_t g = ((size_t)x * N + y0 + 2 * m + (r == 2 ? 1 : 0)) * H + k;
      gx[g] = av;
      gy[g] = bv;
    }
  }
}

// ---------------------------------------------------------------------------
// Forward pass 2 (along y): S1 = n_y FFT_y(Gy) + FFT_y(n_z Gz), S2 = FFT_y(Gx).
// Tile: fixed x, kz chunk, all ky.  Grid (N, CHUNKS).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kPassThreads)
k_fwd_y(const cplx_t<T>* __restrict__ gx, const cplx_t<T>* __restrict__ gy, const cplx_t<T>* __restrict__ gz,
        const cplx_t<T>* __restrict__ tw, cplx_t<T>* __restrict__ s1, cplx_t<T>* __restrict__ s2) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  constexpr int W = S::W, H = S::H;
  __shared__ C tile[S::ELEMS];
  __shared__ C twl[N];
  load_twiddles<T, N, kPassThreads>(twl, tw);
  const int x = blockIdx.x, z0 = blockIdx.y * W;
  C acc[S::EPT];
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      tile[y * W + w] = gy[((size_t)x * N + y) * H + z0 + w];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, -1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      acc[e] = cscale(tile[y * W + w], (T)signed_freq(y, N));
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      tile[y * W + w] = gz[((size_t)x * N + y) * H + z0 + w];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, -1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      s1[((size_t)x * N + y) * H + z0 + w] = cadd(acc[e], tile[y * W + w]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      tile[y * W + w] = gx[((size_t)x * N + y) * H + z0 + w];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, -1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, y = idx / W;
      s2[((size_t)x * N + y) * H + z0 + w] = tile[y * W + w];
    }
  }
}

// ---------------------------------------------------------------------------
// Forward pass 3 (along x) with the adjoint multiply and the prior gradient:
//   G = 2 dhat / sigma^2 - 2 i kfac (FFT_x(S1) + n_x FFT_x(S2)),  0 on
//   excluded modes.  Tile: fixed ky, kz chunk, all kx.  Grid (N, CHUNKS).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ void __launch_bounds__(kPassThreads)
k_fwd_x_grad(const cplx_t<T>* __restrict__ s1, const cplx_t<T>* __restrict__ s2, const double2* __restrict__ modes,
             ModeTables tab, const cplx_t<T>* __restrict__ tw, double2* __restrict__ grad) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  constexpr int W = S::W, H = S::H;
  __shared__ C tile[S::ELEMS];
  __shared__ C twl[N];
  load_twiddles<T, N, kPassThreads>(twl, tw);
  const int y = blockIdx.x, z0 = blockIdx.y * W;
  const int sy = signed_freq(y, N);
  C acc[S::EPT];
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W;
      tile[x * W + w] = s2[((size_t)x * N + y) * H + z0 + w];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, -1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W;
      acc[e] = cscale(tile[x * W + w], (T)signed_freq(x, N));
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W;
      tile[x * W + w] = s1[((size_t)x * N + y) * H + z0 + w];
    }
  }
  __syncthreads();
  lds_fft<T, N, W, W, 1, false, kPassThreads, -1>(tile, twl);
#pragma unroll
  for (int e = 0; e < S::EPT; ++e) {
    const int idx = threadIdx.x + e * kPassThreads;
    if (idx < S::ELEMS) {
      const int w = idx % W, x = idx / W, kz = z0 + w;
      const int sx = signed_freq(x, N);
      const size_t g = ((size_t)x * N + y) * H + kz;
      double2 out = make_double2(0.0, 0.0);
      if (retained(sx, sy, kz, N)) {
        const int n2 = sx * sx + sy * sy + kz * kz;
        const C tv = cadd(acc[e], tile[x * W + w]);
        const double2 q = modes[g];
        const double iv2 = 2.0 * tab.inv_var[n2], kf2 = 2.0 * tab.kfac[n2];
        // -2 i kfac t = (2 kfac t.y, -2 kfac t.x)
        out = make_double2(iv2 * q.x + kf2 * (double)tv.y, iv2 * q.y - kf2 * (double)tv.x);
      }
      grad[g] = out;
    }
  }
}

}  // namespace hamlet
