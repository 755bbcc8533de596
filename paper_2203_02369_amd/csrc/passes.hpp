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
//
// Strided passes (x, y) work on tiles of W consecutive kz columns times all
// N entries along the axis; the grid is (N/2 / W chunks, N rows) with the
// chunk index fastest, so the blocks that run together read whole 1 KB
// (FP32) rows of the array.  z passes work on P consecutive pencils.
#pragma once

#include "common.hpp"
#include "fft.hpp"
#include "random.hpp"
#include "workspace.hpp"

namespace hamlet {

// Threads per block of each pass kind: the schedule of the grid size and
// real type (schedule.hpp; the autotuner's choice where it has one).
template <typename T, int N> struct PassThreads {
  static constexpr int XY = Sched<T, N>::XY;   // k_inv_x, k_inv_y, k_fwd_y
  static constexpr int X = Sched<T, N>::X;     // k_x_pass
  static constexpr int ZG = Sched<T, N>::ZG;   // k_inv_z_gather
  static constexpr int ZS = Sched<T, N>::ZS;   // k_fwd_z_scatter
};

// The y and z passes of each direction may run slab by slab in x so that the
// arrays handed from one to the other stay in the memory-side cache; at
// 256^3 smaller launches cost more than that saves, so one slab is used.
template <int N> struct XSlabs {
  static constexpr int COUNT = 1;
  static constexpr int SIZE = N / COUNT;
};

template <typename T, int N> struct PassShape {
  using C = cplx_t<T>;
  static constexpr int W = Sched<T, N>::W;                  // kz columns per strided tile
  static constexpr int P = Sched<T, N>::PZ;                 // pencils per z tile (scatter)
  static constexpr int PG = Sched<T, N>::PG;                // pencils per z tile (gather)
  static constexpr int FG = 3 * PG / 2;
  static constexpr int H = N / 2;
  static constexpr int CHUNKS = H / W;
  static constexpr int ELEMS = N * W;
  static constexpr int F = 3 * P / 2;                       // complex transforms per z tile
  // pencils per round of the scatter's dense path (its LDS buffer holds
  // 3 PC / 2 transforms)
  static constexpr int PCMAX = 4;
  static constexpr int PC = PCMAX < P ? PCMAX : P;
  using Row = RowLayout<C, W>;
  using Pen = PencilLayout<N>;
};

// Per-mode constants.  sigma_k^2 = N^6 P(|k|) / V is stored per mode in
// FP64 (0 on excluded modes), so every pass reads it coalesced instead of
// gathering from a table indexed by n^2, in the order of the x-pass tiles
// (see var_ofs): a tile's values are contiguous.  The multiplier factor
// kfac = H0 f / (N^3 k_f n^2) is computed from n^2.
struct ModeTables {
  const double* var;       // sigma_k^2 per mode, [ky][kz / W][kx][kz % W]
  double kfac0;            // H0 f / (N^3 k_f) of the state now (the inverse pass)
  double kfac_adj;         // the same at the point whose gradient the adjoint pass takes
  double inv_a;            // 1 / u8^2 there (the prior of the modes scales with u8^2)
};
__device__ __forceinline__ double mode_kfac(double kfac0, int n2) { return n2 > 0 ? kfac0 / (double)n2 : 0.0; }
__device__ __forceinline__ double inv_or_zero(double v) { return v > 0.0 ? 1.0 / v : 0.0; }

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

// K block sums at once, each in the same order as block_sum (so with the
// same result) but with one pair of barriers; red holds K * (waves per
// block) doubles.  Results valid in thread 0.
template <int K> __device__ __forceinline__ void block_sums(double (&v)[K], double* red) {
#pragma unroll
  for (int j = 0; j < K; ++j)
    for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_down(v[j], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) red[j * nw + wid] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += red[j * nw + i];
      v[j] = s;
    }
  }
}

// Neumaier's compensated summation: a running sum s and the rounding errors
// c of its additions, each recovered exactly as the two-sum error of the
// operands, so that the value s + c carries the sum to about one rounding
// whatever the number and spread of the terms.  Every FP64 sum of the
// Hamiltonian (the log-posterior, its derivative in s, the kinetic energy)
// runs in it: block partials per thread, across the block, and over the
// blocks' partials.
struct CSum {
  double s, c;
  __device__ __forceinline__ CSum() : s(0.0), c(0.0) {}
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  // adds another compensated sum
  __device__ __forceinline__ void add(double s2, double c2) {
    const double t = s + s2;
    c += (fabs(s) >= fabs(s2) ? (s - t) + s2 : (s2 - t) + s) + c2;
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

// K compensated block sums in a fixed order (wave64 shuffles, then the waves
// in order in thread 0); red holds 2 K (waves per block) doubles.  Results
// valid in thread 0.
template <int K> __device__ __forceinline__ void block_csums(CSum (&v)[K], double* red) {
#pragma unroll
  for (int j = 0; j < K; ++j)
    for (int off = 32; off > 0; off >>= 1) {
      const double s2 = __shfl_down(v[j].s, off, 64), c2 = __shfl_down(v[j].c, off, 64);
      v[j].add(s2, c2);
    }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      red[2 * (j * nw + wid)] = v[j].s;
      red[2 * (j * nw + wid) + 1] = v[j].c;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      CSum t;
      for (int i = 0; i < nw; ++i) t.add(red[2 * (j * nw + i)], red[2 * (j * nw + i) + 1]);
      v[j] = t;
    }
  }
}

// One compensated block sum; the value is valid in thread 0.
__device__ __forceinline__ double block_csum(CSum v, double* red) {
  CSum a[1] = {v};
  block_csums<1>(a, red);
  return a[0].value();
}

// Visit this thread's elements (a = index along the FFT axis, w = column)
// of a strided tile.
template <typename T, int N, int NT, typename Fn>
__device__ __forceinline__ void tile_elems(Fn&& fn) {
  using S = PassShape<T, N>;
  constexpr int EPT = (S::ELEMS + NT - 1) / NT;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (S::ELEMS % NT == 0 || idx < S::ELEMS) fn(e, idx / S::W, idx % S::W);
  }
}
template <typename T, int N, int NT> constexpr int elems_per_thread() { return (PassShape<T, N>::ELEMS + NT - 1) / NT; }

// K consecutive columns of a strided tile moved as one 16-byte access (K = 2
// for 8-byte complex elements, 1 for 16-byte ones).
template <typename T> struct ColVec {
  using C = cplx_t<T>;
  static constexpr int K = sizeof(C) == 8 ? 2 : 1;
  struct alignas(16) V { C v[K]; };
};

// Visit this thread's groups of K columns (w a multiple of K).
template <typename T, int N, int NT, typename Fn>
__device__ __forceinline__ void tile_vecs(Fn&& fn) {
  using S = PassShape<T, N>;
  constexpr int K = ColVec<T>::K, WK = S::W / K, NV = S::ELEMS / K;
  constexpr int VPT = (NV + NT - 1) / NT;
#pragma unroll
  for (int e = 0; e < VPT; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (NV % NT == 0 || idx < NV) fn(e, idx / WK, K * (idx % WK));
  }
}
template <typename T, int N, int NT> constexpr int vecs_per_thread() {
  return (PassShape<T, N>::ELEMS / ColVec<T>::K + NT - 1) / NT;
}

// Global <-> LDS moves of one group of K columns of row a.
template <typename T, typename LAY>
__device__ __forceinline__ void vec_to_lds(cplx_t<T>* tile, int a, int w, const typename ColVec<T>::V& v) {
#pragma unroll
  for (int j = 0; j < ColVec<T>::K; ++j) tile[LAY::idx(a, w + j)] = v.v[j];
}
template <typename T, typename LAY>
__device__ __forceinline__ typename ColVec<T>::V vec_from_lds(const cplx_t<T>* tile, int a, int w) {
  typename ColVec<T>::V v;
#pragma unroll
  for (int j = 0; j < ColVec<T>::K; ++j) v.v[j] = tile[LAY::idx(a, w + j)];
  return v;
}
template <typename T> __device__ __forceinline__ typename ColVec<T>::V vec_load(const cplx_t<T>* p) {
  return ld_stream(reinterpret_cast<const typename ColVec<T>::V*>(p));
}
template <typename T> __device__ __forceinline__ void vec_store(cplx_t<T>* p, const typename ColVec<T>::V& v) {
  *reinterpret_cast<typename ColVec<T>::V*>(p) = v;
}

// The strided tile (kz chunk, row) of this block in the x and y passes.
// Where a chunk's row is shorter than a 128-byte line (W complex values in
// under 128 bytes: the 512^3 grid), two neighbouring chunks share every
// line, while the hardware deals consecutive workgroups to the eight XCDs in
// turn, each with its own L2.  The blocks are then renumbered so that the
// two chunks of each line run on one XCD: in every group of 16 workgroups,
// ids 8h + j (XCD j) take chunk slot 2j + h.  Identity otherwise.
template <typename T, int N> __device__ __forceinline__ int2 strided_tile() {
  using S = PassShape<T, N>;
  unsigned id = blockIdx.x + S::CHUNKS * blockIdx.y;
  if constexpr (S::W * sizeof(cplx_t<T>) < 128 && S::CHUNKS % 2 == 0) {
    static_assert((S::CHUNKS * N) % 16 == 0, "whole groups of 16 workgroups");
    id = (id & ~15u) | ((id & 7u) << 1) | ((id >> 3) & 1u);
  }
  return make_int2((int)(id % S::CHUNKS), (int)(id / S::CHUNKS));
}

// Global offset of (i, j, kz) in an [N][N][N/2] array.
template <int N> __device__ __forceinline__ size_t gofs(int i, int j, int kz) {
  return ((size_t)i * N + j) * (N / 2) + kz;
}

// Pencils in reach of the points.  A real-space pencil (x, y) (after the x
// and y transforms) takes part in the gather and the scatter only when a
// point's CIC stencil reaches it: one of the columns (x - ox, y - oy),
// ox, oy in {0, 1}, holds a point.  Elsewhere the velocity pencils are never
// read and the scattered field is zero, so the passes on either side skip
// those pencils' rows: the inverse y pass does not store them, the gather
// does not load them, the scatter does not store them and the forward y
// pass reads them as zero.  Every pass derives the flag from the same bucket
// offsets (off, N^2 + 1 entries) of the evaluation.
//
// PencilProbe loads the bucket bounds of the four stencil columns of pencil
// (x, y) together; the flag is taken later, so the loads can overlap other
// work.
template <int N> struct PencilProbe {
  int b[8];
  __device__ __forceinline__ void load(const int* off, int x, int y) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = ((x - (c >> 1) + N) & (N - 1)) * N + ((y - (c & 1) + N) & (N - 1));
      b[2 * c] = off[k];
      b[2 * c + 1] = off[k + 1];
    }
  }
  __device__ __forceinline__ bool touched() const {
    return (b[1] > b[0]) | (b[3] > b[2]) | (b[5] > b[4]) | (b[7] > b[6]);
  }
};

// The flags of the pencils (x, y), y in [0, N), into LDS (visible after the
// caller's next barrier).
template <int N, int NT> __device__ __forceinline__ void plane_flags(const int* off, int x, bool* touched) {
  for (int y = threadIdx.x; y < N; y += NT) {
    PencilProbe<N> pr;
    pr.load(off, x, y);
    touched[y] = pr.touched();
  }
}

// Bit e: the row of this thread's e-th column group (tile_vecs order) is
// flagged.
template <typename T, int N, int NT> __device__ __forceinline__ unsigned row_bits(const bool* touched) {
  static_assert(vecs_per_thread<T, N, NT>() <= 32, "one bit per column group");
  unsigned m = 0;
  tile_vecs<T, N, NT>([&](int e, int y, int) { m |= touched[y] ? 1u << e : 0u; });
  return m;
}

// Offset of mode (kx, ky, kz) in the per-mode sigma_k^2 array, laid out as
// the x-pass tiles [ky][kz / W][kx][kz % W]: element e of a tile is at
// tile * N W + e, so a wave reads whole cache lines (a row of W values
// alone is half a line in the FP64 path, whose tiles are 8 columns wide).
__host__ __device__ inline size_t var_ofs(int n, int w, int kx, int ky, int kz) {
  return (((size_t)ky * (n / 2 / w) + kz / w) * n + kx) * w + kz % w;
}

// ---------------------------------------------------------------------------
// Inverse pass 1 (along x): multiplier, prior energy, two spectral outputs.
// Tile: fixed ky, kz chunk, all kx.
// ---------------------------------------------------------------------------
// DENSITY: A = q / N^3 (the density contrast's spectrum) instead of the
// velocity multiplier's i kfac q.
template <typename T, int N, int NT, bool DENSITY = false, typename Q = double2>
__device__ __forceinline__ void
inv_x_body(const Q* __restrict__ modes, ModeTables tab, const cplx_t<T>* __restrict__ tw,
        cplx_t<T>* __restrict__ outA, cplx_t<T>* __restrict__ outB, double* __restrict__ prior_part) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Row;
  __shared__ C tile[LAY::size(N)];
  __shared__ C twl[N];
  __shared__ double red[2 * (NT / 64)];
  load_twiddles<T, N, NT>(twl, tw);
  const int2 tl = strided_tile<T, N>();
  const int y = tl.y, z0 = tl.x * S::W;
  const int sy = signed_freq(y, N);
  CSum prior;
  // i kfac q (and n_x times it), zero on excluded modes
  auto ain = [&](int x, int w, double scale_x) {
    const int kz = z0 + w, sx = signed_freq(x, N);
    if (!retained(sx, sy, kz, N)) return make_double2(0.0, 0.0);
    const double2 q = widen(modes[gofs<N>(x, y, kz)]);
    if constexpr (DENSITY) {
      const double sc = (scale_x != 0.0 ? scale_x * sx : 1.0) / ((double)N * N * N);
      return make_double2(sc * q.x, sc * q.y);
    }
    const double kf = mode_kfac(tab.kfac0, sx * sx + sy * sy + kz * kz) * (scale_x != 0.0 ? scale_x * sx : 1.0);
    return make_double2(-kf * q.y, kf * q.x);
  };
  tile_elems<T, N, NT>([&](int, int x, int w) {
    const int kz = z0 + w, sx = signed_freq(x, N);
    if (retained(sx, sy, kz, N)) {
      const size_t g = gofs<N>(x, y, kz);
      const double2 q = widen(modes[g]);
      prior.add((kz == 0 ? 0.5 : 1.0) * (q.x * q.x + q.y * q.y) * inv_or_zero(tab.var[var_ofs(N, S::W, x, y, kz)]));
    }
    tile[LAY::idx(x, w)] = cconvert<C>(ain(x, w, 0.0));
  });
  const double ps = block_csum(prior, red);
  if (threadIdx.x == 0) prior_part[blockIdx.y * gridDim.x + blockIdx.x] = ps;
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
  tile_elems<T, N, NT>([&](int, int x, int w) { outA[gofs<N>(x, y, z0 + w)] = tile[LAY::idx(x, w)]; });
  __syncthreads();
  tile_elems<T, N, NT>([&](int, int x, int w) { tile[LAY::idx(x, w)] = cconvert<C>(ain(x, w, 1.0)); });
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
  tile_elems<T, N, NT>([&](int, int x, int w) { outB[gofs<N>(x, y, z0 + w)] = tile[LAY::idx(x, w)]; });
}

// ---------------------------------------------------------------------------
// Inverse pass 2 (along y).  Tile: fixed x, kz chunk, all ky.
// ---------------------------------------------------------------------------
// ALL: every row is stored (the whole field is wanted; off is not read).
template <typename T, int N, int NT, bool ALL = false>
__device__ __forceinline__ void
inv_y_body(const cplx_t<T>* __restrict__ inA, const cplx_t<T>* __restrict__ inB, const cplx_t<T>* __restrict__ tw,
        cplx_t<T>* __restrict__ vx, cplx_t<T>* __restrict__ vy, cplx_t<T>* __restrict__ vz, const int* __restrict__ off,
        int x0) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Row;
  using CV = ColVec<T>;
  __shared__ C tile[LAY::size(N)];
  __shared__ C twl[N];
  __shared__ bool touched[N];   // rows stored (see PencilProbe)
  const int2 tl = strided_tile<T, N>();
  const int x = x0 + tl.y, z0 = tl.x * S::W;
  // the flags are needed only at the first store: their loads go first,
  // and they are taken once the tile is in
  constexpr int PP = (N + NT - 1) / NT;   // pencils per thread
  PencilProbe<N> probe[PP];
#pragma unroll
  for (int i = 0; i < PP; ++i)
    if (!ALL && threadIdx.x + i * NT < N) probe[i].load(off, x, threadIdx.x + i * NT);
  TwiddleStage<T, N, NT> tws;
  tws.load(tw);
  tile_vecs<T, N, NT>([&](int, int y, int w) { vec_to_lds<T, LAY>(tile, y, w, vec_load<T>(&inB[gofs<N>(x, y, z0 + w)])); });
  tws.store(twl);
#pragma unroll
  for (int i = 0; i < PP; ++i)
    if (!ALL && threadIdx.x + i * NT < N) touched[threadIdx.x + i * NT] = probe[i].touched();
  __syncthreads();
  const unsigned rows = ALL ? ~0u : row_bits<T, N, NT>(touched);
  lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
  tile_vecs<T, N, NT>([&](int e, int y, int w) {
    if ((rows >> e) & 1u) vec_store<T>(&vx[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY>(tile, y, w));
  });
  __syncthreads();
  // A is read once and kept in registers for its second transform
  typename CV::V ra[vecs_per_thread<T, N, NT>()];
  tile_vecs<T, N, NT>([&](int e, int y, int w) {
    ra[e] = vec_load<T>(&inA[gofs<N>(x, y, z0 + w)]);
    const T ny = (T)signed_freq(y, N);
#pragma unroll
    for (int j = 0; j < CV::K; ++j) tile[LAY::idx(y, w + j)] = cscale(ra[e].v[j], ny);
  });
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
  tile_vecs<T, N, NT>([&](int e, int y, int w) {
    if ((rows >> e) & 1u) vec_store<T>(&vy[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY>(tile, y, w));
  });
  __syncthreads();
  tile_vecs<T, N, NT>([&](int e, int y, int w) { vec_to_lds<T, LAY>(tile, y, w, ra[e]); });
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
  tile_vecs<T, N, NT>([&](int e, int y, int w) {
    if ((rows >> e) & 1u) vec_store<T>(&vz[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY>(tile, y, w));
  });
}

// Galaxies binned by CIC column (ix, iy) of their lower corner, in sorted
// order s; bucket key = ix * N + iy, members off[key] .. off[key + 1].
template <typename T> struct Binned {
  const int* off;          // N^2 + 1
  const T* rx; const T* ry; const T* rz;   // rhat
  const T* tx; const T* ty; const T* tz;   // fractional offsets in the cell
  const int* iz;           // lower z node
  const int* most;         // most points in one column
};

// Transform slot of the real pencil of component c of pencil p in a z tile:
// pairs of pencils (2m, 2m+1) fill three complex transforms
//   3m   : (vx_2m,   vy_2m)      3m+1 : (vz_2m, vz_2m+1)      3m+2 : (vx_2m+1, vy_2m+1)
// and the real pencil is the real (part 0) or imaginary (part 1) part.
__device__ __forceinline__ int zslot_f(int p, int c) {
  const int m = p >> 1, odd = p & 1;
  return c == 2 ? 3 * m + 1 : 3 * m + (odd ? 2 : 0);
}
__device__ __forceinline__ int zslot_part(int p, int c) {
  return c == 0 ? 0 : (c == 1 ? 1 : (p & 1));
}

// The spectra of a z tile, loaded into registers (load) and then written
// into LDS (put; a barrier must follow): for each transform f of the tile (P
// pencils from y0), Z = A + i B with A, B the Hermitian half spectra of its
// two real pencils (Nyquist entry zero, DC entries real).  Pencils whose bit
// in tp is clear are taken as zero and not loaded.  Splitting the two lets a
// pass issue the next tile's loads before it transforms the current one.
// NZ: the third array carries n_z (velocity component z); without it the
// third array is taken as it is (a scalar field).
template <typename T, int N, int NT, int P, bool NZ = true> struct ZSpectra {
  using C = cplx_t<T>;
  using LAY = typename PassShape<T, N>::Pen;
  static constexpr int H = N / 2, F = 3 * P / 2;
  // FP32: two consecutive kz per thread (16-byte loads); FP64: one
  static constexpr int KT = sizeof(C) == 8 ? 2 : 1;
  static constexpr int HK = H / KT, IT = (F * HK + NT - 1) / NT;
  struct alignas(16) CK { C v[KT]; };
  CK av[IT], bv[IT];

  // Real pencils of transform f: pa in the real part, pb in the imaginary
  // part, from vx / vy (f = 3m, 3m + 2) or n_z vz (f = 3m + 1).
  __device__ __forceinline__ static bool sources(int f, int& pa, int& pb) {
    const int m = f / 3, r = f % 3;
    pa = 2 * m + (r == 2 ? 1 : 0);
    pb = r == 1 ? 2 * m + 1 : pa;
    return r == 1;
  }

  // Every load of a thread is issued before any wait.
  __device__ __forceinline__ void load(const C* __restrict__ vx, const C* __restrict__ vy,
                                       const C* __restrict__ vz, int x, int y0, unsigned tp) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
#pragma unroll
      for (int j = 0; j < KT; ++j) av[it].v[j] = bv[it].v[j] = cmake<C>((T)0, (T)0);
      if (idx < F * HK) {
        const int k = KT * (idx % HK), f = idx / HK;
        int pa, pb;
        const bool zc = sources(f, pa, pb);
        if ((tp >> pa) & 1u) av[it] = ld_stream(reinterpret_cast<const CK*>(&(zc ? vz : vx)[gofs<N>(x, y0 + pa, k)]));
        if ((tp >> pb) & 1u) bv[it] = ld_stream(reinterpret_cast<const CK*>(&(zc ? vz : vy)[gofs<N>(x, y0 + pb, k)]));
      }
    }
  }

  __device__ __forceinline__ void put(C* buf) const {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < F * HK) {
        const int k0 = KT * (idx % HK), f = idx / HK;
        int pa, pb;
        const bool zc = sources(f, pa, pb);
#pragma unroll
        for (int j = 0; j < KT; ++j) {
          const int k = k0 + j;
          C av_ = av[it].v[j], bv_ = bv[it].v[j];
          if (zc && NZ) {
            av_ = cscale(av_, (T)k);
            bv_ = cscale(bv_, (T)k);
          }
          if (k == 0) {
            buf[LAY::idx(0, f)] = cmake<C>(av_.x, bv_.x);
            buf[LAY::idx(H, f)] = cmake<C>((T)0, (T)0);
          } else {
            buf[LAY::idx(k, f)] = cmake<C>(av_.x - bv_.y, av_.y + bv_.x);        // A + i B
            buf[LAY::idx(N - k, f)] = cmake<C>(av_.x + bv_.y, bv_.x - av_.y);    // conj(A) + i conj(B)
          }
        }
      }
    }
  }
};

template <typename T, int N, int NT, int P, bool NZ = true>
__device__ __forceinline__ void
z_tile_spectra(const cplx_t<T>* __restrict__ vx, const cplx_t<T>* __restrict__ vy, const cplx_t<T>* __restrict__ vz,
               int x, int y0, unsigned tp, cplx_t<T>* buf) {
  ZSpectra<T, N, NT, P, NZ> sp;
  sp.load(vx, vy, vz, x, y0, tp);
  sp.put(buf);
}

// ---------------------------------------------------------------------------
// Inverse pass 3 (along z, complex-to-real) fused with the CIC gather.
// Tile: fixed x, pencils y0 .. y0 + P (P = PassShape::PG).  Grid (N / P, N).
// Writes, for every galaxy whose CIC stencil touches a pencil of the tile,
// the column partials of its projected velocity (eqn:lvr):
//   Pc = sum_c rhat_c [(1 - tz) v_c(z0) + tz v_c(z1)],  Qc = sum_c rhat_c [v_c(z1) - v_c(z0)]
// into part[4 s + corner], corner = 2 (x - ix) + (y - iy).
// ---------------------------------------------------------------------------
template <typename T, int N, int NT>
__device__ __forceinline__ void
inv_z_gather_body(const cplx_t<T>* __restrict__ vx, const cplx_t<T>* __restrict__ vy, const cplx_t<T>* __restrict__ vz,
               const cplx_t<T>* __restrict__ tw, Binned<T> bins, cplx_t<T>* __restrict__ part, int x0) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Pen;
  constexpr int P = S::PG, F = S::FG;
  __shared__ C buf[LAY::size(F)];
  __shared__ C twl[N];
  const int x = x0 + blockIdx.y, y0 = blockIdx.x * P;
  // Gather: (pencil, corner, lane) per thread; lane strides the bucket.  The
  // column range is loaded first, and (FP32) the first point before the
  // transform, so that their latency overlaps the field loads and the FFT;
  // the FP64 path loads its points after the transform, which keeps its
  // registers, and occupancy, where they were.
  constexpr int LANES = NT / (4 * P);
  const int t = threadIdx.x;
  const int pc = t % (4 * P), lane = t / (4 * P);
  const int p = pc >> 2, corner = pc & 3;
  const int ox = corner >> 1, oy = corner & 1;
  const int y = y0 + p;
  const int key = ((x - ox + N) & (N - 1)) * N + ((y - oy + N) & (N - 1));
  const int s0 = bins.off[key], s1 = bins.off[key + 1];
  load_twiddles<T, N, NT>(twl, tw);
  // Pencils of the tile in reach of a point (see PencilProbe).  Every
  // wave holds every (pencil, corner) in its lanes, so a ballot gives each
  // wave the whole tile's flags.  The inverse y pass stored only these
  // pencils; the others are transformed as zero and never read.
  static_assert(64 % (4 * P) == 0 && NT % 64 == 0, "a wave covers the tile's stencil columns");
  const unsigned long long occ = __ballot(s1 > s0);
  unsigned tp = 0;
#pragma unroll
  for (int q = 0; q < P; ++q) tp |= ((occ >> (4 * q)) & 0xFull) ? 1u << q : 0u;
  if (tp == 0) return;   // block-uniform: no point reaches the tile
  z_tile_spectra<T, N, NT, P>(vx, vy, vz, x, y0, tp, buf);
  __syncthreads();
  constexpr bool kEarly = sizeof(T) == 4;
  int s = s0 + lane;
  int pz = 0;
  T ptz = 0, prx = 0, pry = 0, prz = 0;
  auto load_point = [&](int i) {
    pz = bins.iz[i];
    ptz = bins.tz[i];
    prx = bins.rx[i];
    pry = bins.ry[i];
    prz = bins.rz[i];
  };
  if (kEarly && s < s1) load_point(s);
  lds_fft<T, N, F, LAY, NT, +1>(buf, twl);
  const int fxy = zslot_f(p, 0), fz = zslot_f(p, 2), sz = zslot_part(p, 2);
  for (; s < s1; s += LANES) {
    if (!kEarly) load_point(s);
    const int z0 = pz, z1 = (z0 + 1) & (N - 1);
    const T tz = ptz, rx = prx, ry = pry, rz = prz;
    const C a0 = buf[LAY::idx(z0, fxy)], a1 = buf[LAY::idx(z1, fxy)];
    const C c0 = buf[LAY::idx(z0, fz)], c1 = buf[LAY::idx(z1, fz)];
    const T az0 = sz ? c0.y : c0.x, az1 = sz ? c1.y : c1.x;
    const T omt = (T)1 - tz;
    const T pcv = rx * (omt * a0.x + tz * a1.x) + ry * (omt * a0.y + tz * a1.y) + rz * (omt * az0 + tz * az1);
    const T qcv = rx * (a1.x - a0.x) + ry * (a1.y - a0.y) + rz * (az1 - az0);
    part[4 * (size_t)s + corner] = cmake<C>(pcv, qcv);
    if (kEarly && s + LANES < s1) load_point(s + LANES);
  }
}

// ---------------------------------------------------------------------------
// Inverse pass 3 writing the velocity field itself: the transform of the
// gather's tile (every pencil), then out[c][x][y][z] = v_c at node (x, y, z),
// c = x, y, z.  Used to hand a state's field to the caller, not inside an
// evaluation.
// ---------------------------------------------------------------------------
// DENSITY: the third array is the density spectrum (no n_z), and only it is
// written: out[x][y][z].
template <typename T, int N, int NT, bool DENSITY = false>
__device__ __forceinline__ void
inv_z_field_body(const cplx_t<T>* __restrict__ vx, const cplx_t<T>* __restrict__ vy, const cplx_t<T>* __restrict__ vz,
                 const cplx_t<T>* __restrict__ tw, T* __restrict__ out, int x0) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Pen;
  constexpr int P = S::PG, F = S::FG;
  __shared__ C buf[LAY::size(F)];
  __shared__ C twl[N];
  const int x = x0 + blockIdx.y, y0 = blockIdx.x * P;
  load_twiddles<T, N, NT>(twl, tw);
  z_tile_spectra<T, N, NT, P, !DENSITY>(vx, vy, vz, x, y0, (1u << P) - 1u, buf);
  __syncthreads();
  lds_fft<T, N, F, LAY, NT, +1>(buf, twl);
  // (pencil, component, z) with z fastest: each row of N values is one
  // contiguous store
  constexpr int NC = DENSITY ? 1 : 3;
  for (int idx = threadIdx.x; idx < P * NC * N; idx += NT) {
    const int z = idx % N, pc = idx / N;
    const int p = pc / NC, c = DENSITY ? 2 : pc % 3;
    const C v = buf[LAY::idx(z, zslot_f(p, c))];
    out[(((size_t)(DENSITY ? 0 : c) * N + x) * N + (y0 + p)) * N + z] = zslot_part(p, c) ? v.y : v.x;
  }
}

// First index in [lo, hi) of the ascending z cells `iz` with iz[s] >= v.
template <typename I>
__device__ __forceinline__ int lower_bound_cell(const I* iz, int lo, int hi, int v) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int)iz[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The binned points of the stencil columns of a z tile (columns x and x - 1,
// rows y0 - 1 .. y0 + P - 1) are at most four contiguous ranges of the
// binned arrays: rows max(y0 - 1, 0) .. y0 + P - 1 of each column index, and
// row N - 1 when y0 = 0.  A tile stages them in LDS when they fit.
template <typename T, int CAP> struct ZStage {
  T g[CAP], tx[CAP], ty[CAP], tz[CAP], r[3][CAP];
  int16_t iz[CAP];
  int start[4], at[4], count;   // range start in the binned arrays, its index in the stage
};

// Index in the stage of binned index s of the column (x - ox, y).
__device__ __forceinline__ int stage_index(const int* start, const int* at, int s, int ox, bool wrap_row) {
  const int r = 2 * ox + (wrap_row ? 1 : 0);
  return s - start[r] + at[r];
}

// ---------------------------------------------------------------------------
// Forward pass 1 (along z, real-to-complex) fused with the CIC scatter-add:
//   G_c(x_j) = sum_i g_i rhat_ic W_i(x_j)  (adjoint of the gather)
// Every output sums its contributions in a fixed order, so the result is
// deterministic.  The tile's points (at most four contiguous ranges of the
// binned arrays) are staged in LDS when they fit.
//  * Sparse grids (no column holds more than 8 points): a pencil has only a
//    few nonzero nodes, so each output coefficient is summed directly over
//    the points of the pencil's four stencil columns (corner by corner, in
//    binned order) instead of building the pencil and transforming it.
//  * Crowded grids: each real pencil is built in LDS and transformed, a few
//    pencil pairs a round (a small buffer keeps more tiles resident on a
//    compute unit for the sparse case).  The points of a column are sorted
//    by z cell, so the
//    points that reach node j are two runs per stencil column (z cell j - 1
//    with weight tz, then z cell j with weight 1 - tz); G lanes share each
//    (pencil, component) row, lane l owning the nodes of one z segment, and
//    node j sums in the order (corner, run, binned index) whatever G is.  The
//    tile's points are staged in LDS when they fit.
// G follows the most crowded column of the grid (found by the binning scan).
// Outputs Gx, Gy and n_z Gz on kz in [0, N/2).  Grid (N / P, N).
// ---------------------------------------------------------------------------
template <typename T, int N, int NT>
__device__ __forceinline__ void
fwd_z_scatter_body(const T* __restrict__ gsort, Binned<T> bins, const cplx_t<T>* __restrict__ tw,
                   cplx_t<T>* __restrict__ gx, cplx_t<T>* __restrict__ gy, cplx_t<T>* __restrict__ gz, int x0) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Pen;
  constexpr int P = S::P, H = S::H, PC = S::PC, FC = 3 * PC / 2;
  static_assert(P % PC == 0 && PC % 2 == 0, "rounds of whole pencil pairs");
  constexpr int GMAX_T = NT / (3 * PC) >= 16 ? 16 : (NT / (3 * PC) >= 8 ? 8 : (NT / (3 * PC) >= 4 ? 4 : 1));
  constexpr int GMAX = GMAX_T < N ? GMAX_T : N;
  // stage capacity (points); the FP64 path keeps its LDS small for occupancy
  constexpr int CAP = sizeof(T) == 4 ? 256 : 32;
  __shared__ C buf[LAY::size(FC)];
  __shared__ C twl[N];
  __shared__ int col[4 * P][2];     // binned range of the 4 stencil columns of each pencil
  __shared__ ZStage<T, CAP> stg;
  __shared__ unsigned tile_touch;   // bit p: pencil p in reach of a point (see PencilProbe)
  const int x = x0 + blockIdx.y, y0 = blockIdx.x * P;
  static_assert(4 * P + 4 <= 64, "tile set-up runs in the first wave");
  // Tile set-up, issued first so that its loads overlap the twiddle load:
  // lanes 0 .. 4P-1 load the stencil columns, lanes 4P .. 4P+3 the four
  // ranges of the binned arrays that hold them.
  if (threadIdx.x < 64) {
    const int t = threadIdx.x;
    int a = 0, b = 0;
    if (t < 4 * P) {
      const int p = t >> 2, corner = t & 3;
      const int ox = corner >> 1, oy = corner & 1;
      const int key = ((x - ox + N) & (N - 1)) * N + ((y0 + p - oy + N) & (N - 1));
      a = bins.off[key];
      b = bins.off[key + 1];
      col[t][0] = a;
      col[t][1] = b;
    } else if (t < 4 * P + 4) {
      const int r = t - 4 * P, ox = r >> 1, wrap = r & 1;
      const int kx = ((x - ox + N) & (N - 1)) * N;
      if (!wrap) {
        a = bins.off[kx + (y0 > 0 ? y0 - 1 : 0)];
        b = bins.off[kx + y0 + P];
      } else if (y0 == 0) {
        a = bins.off[kx + N - 1];
        b = bins.off[kx + N];
      }
      stg.start[r] = a;
    }
    const unsigned long long occ = __ballot(t < 4 * P && b > a);
    const int len = (t >= 4 * P && t < 4 * P + 4) ? b - a : 0;
    const int l0 = __shfl(len, 4 * P, 64), l1 = __shfl(len, 4 * P + 1, 64);
    const int l2 = __shfl(len, 4 * P + 2, 64), l3 = __shfl(len, 4 * P + 3, 64);
    if (t == 0) {
      stg.at[0] = 0;
      stg.at[1] = l0;
      stg.at[2] = l0 + l1;
      stg.at[3] = l0 + l1 + l2;
      stg.count = l0 + l1 + l2 + l3;
      unsigned tp = 0;
      for (int q = 0; q < P; ++q) tp |= ((occ >> (4 * q)) & 0xFull) ? 1u << q : 0u;
      tile_touch = tp;
    }
  }
  load_twiddles<T, N, NT>(twl, tw);
  const int most = bins.most[0];
  int G = 1;
  while (G < GMAX && 8 * G < most) G <<= 1;
  __syncthreads();
  // Only pencils in reach of a point are stored: the forward y pass reads
  // the others as zero.
  const unsigned tp = tile_touch;
  if (tp == 0) return;   // block-uniform
  auto touched = [&](int q) { return ((tp >> q) & 1u) != 0; };
  const bool staged = stg.count <= CAP;   // block-uniform
  if (staged) {
    for (int i = threadIdx.x; i < stg.count; i += NT) {
      int r = 0;
      while (r < 3 && i >= stg.at[r + 1]) ++r;
      const int s = stg.start[r] + (i - stg.at[r]);
      stg.g[i] = gsort[s];
      stg.tx[i] = bins.tx[s];
      stg.ty[i] = bins.ty[s];
      stg.tz[i] = bins.tz[s];
      stg.r[0][i] = bins.rx[s];
      stg.r[1][i] = bins.ry[s];
      stg.r[2][i] = bins.rz[s];
      stg.iz[i] = (int16_t)bins.iz[s];
    }
  }
  if (G == 1 && staged) {
    // Sparse tile: a pencil holds a few nonzero nodes, so each output is the
    // direct sum  X_c(k) = sum_points v_c [(1 - tz) w^(z0 k) + tz w^((z0+1) k)],
    // w = exp(-2 pi i / N), over the pencil's stencil columns (corner by
    // corner, binned order); the bracket is shared by the three components.
    __syncthreads();
    // two consecutive kz per thread (16-byte stores in FP32)
    constexpr int KT = sizeof(C) == 8 ? 2 : 1;
    constexpr int HK = H / KT;
    struct alignas(16) CK { C v[KT]; };
    for (int idx = threadIdx.x; idx < P * HK; idx += NT) {
      const int k0 = KT * (idx % HK), p = idx / HK;
      if (!touched(p)) continue;
      C wk[KT];
      T ax[KT], ay[KT], bx[KT], by[KT], cx[KT], cy[KT];
#pragma unroll
      for (int j = 0; j < KT; ++j) {
        wk[j] = twl[k0 + j];
        ax[j] = ay[j] = bx[j] = by[j] = cx[j] = cy[j] = (T)0;
      }
      for (int corner = 0; corner < 4; ++corner) {
        const int s0 = col[4 * p + corner][0], s1 = col[4 * p + corner][1];
        const int ox = corner >> 1, oy = corner & 1;
        const bool wrap_row = y0 == 0 && p - oy < 0;
        const int lo = stage_index(stg.start, stg.at, s0, ox, wrap_row);
        for (int i = lo; i < lo + (s1 - s0); ++i) {
          const T tx = stg.tx[i], ty = stg.ty[i], tz = stg.tz[i];
          const T v = stg.g[i] * ((ox ? tx : (T)1 - tx) * (oy ? ty : (T)1 - ty));
          const T vx = v * stg.r[0][i], vy = v * stg.r[1][i], vz = v * stg.r[2][i];
          const int iz = stg.iz[i];
#pragma unroll
          for (int j = 0; j < KT; ++j) {
            const C w0 = twl[(iz * (k0 + j)) & (N - 1)];
            const T ux = ((T)1 - tz) + tz * wk[j].x, uy = tz * wk[j].y;
            const T wx = w0.x * ux - w0.y * uy, wy = w0.x * uy + w0.y * ux;
            ax[j] += vx * wx;
            ay[j] += vx * wy;
            bx[j] += vy * wx;
            by[j] += vy * wy;
            cx[j] += vz * wx;
            cy[j] += vz * wy;
          }
        }
      }
      const size_t g = gofs<N>(x, y0 + p, k0);
      CK ox_, oy_, oz_;
#pragma unroll
      for (int j = 0; j < KT; ++j) {
        ox_.v[j] = cmake<C>(ax[j], ay[j]);
        oy_.v[j] = cmake<C>(bx[j], by[j]);
        oz_.v[j] = cmake<C>((T)(k0 + j) * cx[j], (T)(k0 + j) * cy[j]);
      }
      *reinterpret_cast<CK*>(&gx[g]) = ox_;
      *reinterpret_cast<CK*>(&gy[g]) = oy_;
      *reinterpret_cast<CK*>(&gz[g]) = oz_;
    }
    return;
  }
  // Dense tiles: pencils built in LDS and transformed, PC pencils (FC
  // transforms) a round; rounds with no pencil in reach are skipped.
  T* row = reinterpret_cast<T*>(buf);
  for (int p0 = 0; p0 < P; p0 += PC) {
    if (((tp >> p0) & ((1u << PC) - 1u)) == 0u) continue;   // block-uniform
    const int f0 = 3 * p0 / 2;
    for (int i = threadIdx.x; i < LAY::size(FC); i += NT) buf[i] = cmake<C>((T)0, (T)0);
    __syncthreads();
    if (threadIdx.x < 3 * PC * G) {
      const int lane = threadIdx.x % G, pc = threadIdx.x / G;
      const int p = p0 + pc / 3, c = pc % 3;
      const int seg = N / G, za = lane * seg, zb = za + seg;
      const int zl = (za - 1) & (N - 1);
      const int f = zslot_f(p, c) - f0, part = zslot_part(p, c);
      const T* rcs = c == 0 ? bins.rx : (c == 1 ? bins.ry : bins.rz);
      for (int corner = 0; corner < 4; ++corner) {
        const int s0 = col[4 * p + corner][0], s1 = col[4 * p + corner][1];
        if (s0 == s1) continue;
        const int ox = corner >> 1, oy = corner & 1;
        // the run of z cell za - 1 puts its upper weight on node za; cells
        // za .. zb - 1 put their lower weight on node z and their upper
        // weight on node z + 1 inside the segment
        auto scatter = [&](auto g_, auto tx_, auto ty_, auto tz_, auto r_, auto iz_, int lo, int hi) {
          auto value = [&](int s) {
            const T tx = tx_[s], ty = ty_[s];
            const T wxy = (ox ? tx : (T)1 - tx) * (oy ? ty : (T)1 - ty);
            return g_[s] * wxy * r_[s];
          };
          for (int s = lower_bound_cell(iz_, lo, hi, zl); s < hi && (int)iz_[s] == zl; ++s)
            row[2 * LAY::idx(za, f) + part] += value(s) * tz_[s];
          for (int s = lower_bound_cell(iz_, lo, hi, za); s < hi && (int)iz_[s] < zb; ++s) {
            const int z = iz_[s];
            const T v = value(s), tz = tz_[s];
            row[2 * LAY::idx(z, f) + part] += v * ((T)1 - tz);
            if (z + 1 < zb) row[2 * LAY::idx(z + 1, f) + part] += v * tz;
          }
        };
        if (staged) {
          const bool wrap_row = y0 == 0 && p - oy < 0;
          const int lo = stage_index(stg.start, stg.at, s0, ox, wrap_row);
          scatter(stg.g, stg.tx, stg.ty, stg.tz, stg.r[c], stg.iz, lo, lo + (s1 - s0));
        } else {
          scatter(gsort, bins.tx, bins.ty, bins.tz, rcs, bins.iz, s0, s1);
        }
      }
    }
    __syncthreads();
    lds_fft<T, N, FC, LAY, NT, -1, true>(buf, twl);
    // Split each transform Z of a + i b into the half spectra
    //   A_k = (Z_k + conj Z_{N-k}) / 2,   B_k = (Z_k - conj Z_{N-k}) / (2 i).
    for (int idx = threadIdx.x; idx < FC * H; idx += NT) {
      const int k = idx % H, fl = idx / H;
      const int m = (f0 + fl) / 3, r = (f0 + fl) % 3;
      const C zk = buf[LAY::idx(k, fl)];
      const C zm = buf[LAY::idx((N - k) & (N - 1), fl)];
      const T half = (T)0.5;
      const C av = cmake<C>(half * (zk.x + zm.x), half * (zk.y - zm.y));
      const C bv = cmake<C>(half * (zk.y + zm.y), half * (zm.x - zk.x));
      if (r == 1) {
        const size_t g0 = gofs<N>(x, y0 + 2 * m, k);
        if (touched(2 * m)) gz[g0] = cscale(av, (T)k);
        if (touched(2 * m + 1)) gz[g0 + H] = cscale(bv, (T)k);
      } else if (touched(2 * m + (r == 2 ? 1 : 0))) {
        const size_t g = gofs<N>(x, y0 + 2 * m + (r == 2 ? 1 : 0), k);
        gx[g] = av;
        gy[g] = bv;
      }
    }
    __syncthreads();   // the next round reuses the buffer
  }
}

// ---------------------------------------------------------------------------
// Forward pass 2 (along y): S1 = n_y FFT_y(Gy) + FFT_y(n_z Gz), S2 = FFT_y(Gx).
// Tile: fixed x, kz chunk, all ky.
// ---------------------------------------------------------------------------
template <typename T, int N, int NT>
__device__ __forceinline__ void
fwd_y_body(const cplx_t<T>* __restrict__ gx, const cplx_t<T>* __restrict__ gy, const cplx_t<T>* __restrict__ gz,
        const cplx_t<T>* __restrict__ tw, const int* __restrict__ off, cplx_t<T>* __restrict__ s1,
        cplx_t<T>* __restrict__ s2, int x0) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Row;
  using CV = ColVec<T>;
  __shared__ C tile[LAY::size(N)];
  __shared__ C twl[N];
  __shared__ bool touched[N];   // rows the scatter stored; the others are zero
  const int2 tl = strided_tile<T, N>();
  const int x = x0 + tl.y, z0 = tl.x * S::W;
  plane_flags<N, NT>(off, x, touched);
  load_twiddles<T, N, NT>(twl, tw);
  __syncthreads();
  const unsigned rows = row_bits<T, N, NT>(touched);
  // flagged rows into LDS, zeros for the others; every load is issued
  // before the first wait
  typename CV::V ld[vecs_per_thread<T, N, NT>()];
  auto load = [&](const C* g) {
    tile_vecs<T, N, NT>([&](int e, int, int) {
#pragma unroll
      for (int j = 0; j < CV::K; ++j) ld[e].v[j] = cmake<C>((T)0, (T)0);
    });
    tile_vecs<T, N, NT>([&](int e, int y, int w) {
      if ((rows >> e) & 1u) ld[e] = vec_load<T>(&g[gofs<N>(x, y, z0 + w)]);
    });
    tile_vecs<T, N, NT>([&](int e, int y, int w) { vec_to_lds<T, LAY>(tile, y, w, ld[e]); });
  };
  typename CV::V acc[vecs_per_thread<T, N, NT>()];
  load(gy);
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, -1>(tile, twl);
  tile_vecs<T, N, NT>([&](int e, int y, int w) {
    const T ny = (T)signed_freq(y, N);
#pragma unroll
    for (int j = 0; j < CV::K; ++j) acc[e].v[j] = cscale(tile[LAY::idx(y, w + j)], ny);
  });
  __syncthreads();
  load(gz);
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, -1>(tile, twl);
  tile_vecs<T, N, NT>([&](int e, int y, int w) {
    typename CV::V o;
#pragma unroll
    for (int j = 0; j < CV::K; ++j) o.v[j] = cadd(acc[e].v[j], tile[LAY::idx(y, w + j)]);
    vec_store<T>(&s1[gofs<N>(x, y, z0 + w)], o);
  });
  __syncthreads();
  load(gx);
  __syncthreads();
  lds_fft<T, N, S::W, LAY, NT, -1>(tile, twl);
  tile_vecs<T, N, NT>([&](int, int y, int w) { vec_store<T>(&s2[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY>(tile, y, w)); });
}

// What a pass that starts or ends a trajectory needs besides the state: the
// chain's key and iteration (the first pass of a chain's trajectory draws
// the momenta), where the start point is kept (modes, cached gradient), and
// the kinetic-energy partial of each block (one per x-pass block, in block
// order).
struct ChainSave {
  double2* q0;
  double2* g0;
  double* kin_part;
  uint64_t seed;
  uint32_t iteration;
  double2* sv_q;   // first step outside a chain: keep the start point's modes here (or nullptr)
  double2* sv_p;   // and its momenta
};

// ---------------------------------------------------------------------------
// Pass along x at the end of a gradient evaluation, optionally fused with the
// leapfrog update of the modes and the first inverse pass of the next
// evaluation (the tile is the same: fixed ky, kz chunk, all kx).
//
// Gradient (complex convention, 0 on excluded modes):
//   G = 2 dhat / sigma^2 - 2 i kfac (FFT_x(S1) + n_x FFT_x(S2))
// Modes:
//   kXGrad  : write G (times plane_scale on the kz = 0 plane).
//   kXFirst : G read from `gcache` (gradient at the current point); kick
//             p -= (eps/2) G, drift q += eps (sigma^2/2) p, then inverse pass 1
//             of the new q (A, B, prior energy).
//   kXMid   : G from S1, S2; kick p -= eps G (two half kicks merged), drift,
//             inverse pass 1 of the new q.
//   kXLast  : G from S1, S2; kick p -= (eps/2) G; write G to `gcache`.
// (eq:hamilton integrated by kick-drift-kick leapfrog, mass matrix eq:M_ab.)
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE, int NT, bool CHAIN, typename Q>
__device__ __forceinline__ void
x_pass_body(const cplx_t<T>* s1, const cplx_t<T>* s2, Q* __restrict__ modes, Q* __restrict__ mom,
            Q* __restrict__ gcache, ModeTables tab, const cplx_t<T>* __restrict__ tw,
            const double* __restrict__ eps_ptr, cplx_t<T>* outA, cplx_t<T>* outB, double* __restrict__ prior_part,
            double plane_scale, ChainSave save) {
  using C = cplx_t<T>;
  using S = PassShape<T, N>;
  using LAY = typename S::Row;
  constexpr bool kFromSpectra = MODE != kXFirst;
  constexpr bool kDrift = MODE == kXFirst || MODE == kXMid;
  // kinetic energy of the momenta: before the first kick of a chain's
  // trajectory (K0), after the last kick (K1)
  constexpr bool kStartOfChain = CHAIN && MODE == kXFirst;
  constexpr bool kKinetic = kStartOfChain || MODE == kXLast;
  // Paired tiles: where two tiles fit the LDS of two blocks per compute
  // unit, S2 and S1 sit side by side (columns [0, W) and [W, 2W)) and are
  // transformed as one batch of 2W columns, and so are the next A and B: two
  // transforms instead of four, with every thread busy in each stage (a
  // W-wide batch of 256-point transforms has half as many butterflies per
  // stage as 512 threads), and no tile held in registers across a transform.
  // Otherwise one tile at a time (also at 512^3 in FP32, whose two tiles just
  // fill 72 KB: paired there, the x pass was 7 % slower).
  constexpr bool kPair = 2 * LAY::size(N) * (int)sizeof(C) < 72 * 1024;
  using LAY2 = RowLayout<C, 2 * S::W>;
  constexpr int kTileSize = kPair ? LAY2::size(N) : LAY::size(N);
  __shared__ C tile[kTileSize];
  __shared__ C twl[N];
  __shared__ double red[2 * (NT / 64)];
  // twiddles into LDS once the first tile loads are issued
  TwiddleStage<T, N, NT> tws;
  tws.load(tw);
  const int2 tl = strided_tile<T, N>();
  const int y = tl.y, z0 = tl.x * S::W;
  const int sy = signed_freq(y, N);
  C acc[kPair ? 1 : elems_per_thread<T, N, NT>()];
  // complex64 momenta of a leapfrog step are loaded before the second
  // forward transform of unpaired tiles, whose time hides their latency
  // (complex128 ones, more than eight per thread, or across a paired
  // transform, they would spill)
  constexpr bool kPrefetchP =
      kFromSpectra && !kPair && MODE != kXGrad && sizeof(Q) == 8 && elems_per_thread<T, N, NT>() <= 8;
  Q ppf[elems_per_thread<T, N, NT>()];
  if constexpr (kFromSpectra && kPair) {
    tile_vecs<T, N, NT>([&](int, int x, int w) { vec_to_lds<T, LAY2>(tile, x, w, vec_load<T>(&s2[gofs<N>(x, y, z0 + w)])); });
    tile_vecs<T, N, NT>(
        [&](int, int x, int w) { vec_to_lds<T, LAY2>(tile, x, S::W + w, vec_load<T>(&s1[gofs<N>(x, y, z0 + w)])); });
    if constexpr (kPrefetchP)
      tile_elems<T, N, NT>([&](int e, int x, int w) { ppf[e] = ld_stream(&mom[gofs<N>(x, y, z0 + w)]); });
    tws.store(twl);
    __syncthreads();
    lds_fft<T, N, 2 * S::W, LAY2, NT, -1>(tile, twl);
  } else if constexpr (kFromSpectra) {
    tile_vecs<T, N, NT>([&](int, int x, int w) { vec_to_lds<T, LAY>(tile, x, w, vec_load<T>(&s2[gofs<N>(x, y, z0 + w)])); });
    tws.store(twl);
    __syncthreads();
    lds_fft<T, N, S::W, LAY, NT, -1>(tile, twl);
    tile_elems<T, N, NT>([&](int e, int x, int w) { acc[e] = cscale(tile[LAY::idx(x, w)], (T)signed_freq(x, N)); });
    __syncthreads();
    tile_vecs<T, N, NT>([&](int, int x, int w) { vec_to_lds<T, LAY>(tile, x, w, vec_load<T>(&s1[gofs<N>(x, y, z0 + w)])); });
    if constexpr (kPrefetchP)
      tile_elems<T, N, NT>([&](int e, int x, int w) { ppf[e] = ld_stream(&mom[gofs<N>(x, y, z0 + w)]); });
    __syncthreads();
    lds_fft<T, N, S::W, LAY, NT, -1>(tile, twl);
  } else {
    (void)s1;
    (void)s2;
    tws.store(twl);
  }
  const double eps = MODE == kXGrad ? 0.0 : eps_ptr[0];
  const double hk = MODE == kXMid ? eps : 0.5 * eps;
  CSum prior, kin;
  // B-input of the next inverse pass (n_x times the A-input), kept in
  // registers, or in the tile's second half when paired
  C bin[kPair ? 1 : elems_per_thread<T, N, NT>()];
  // Complex64 chain state in paired tiles: two consecutive kz per lane, so
  // that the modes, momenta, cached gradient and sigma^2 move as 16-byte
  // accesses like the spectra (half the memory instructions of one mode per
  // lane: the middle step 158 -> 138 us at 256^3; at 512^3 the two elements'
  // state spilled and the pass was 5 % slower).  Otherwise one element per
  // lane (16-byte complex128 state, larger grids, or tiles held in
  // registers), in the form those passes were tuned with.
  constexpr bool kPairedState = kPair && sizeof(Q) == 8 && ColVec<T>::K == 2 && N <= 256;
  struct PairIo {
    Q qs, ps, gs, q0s, g0s;
    __device__ Q q() const { return qs; }
    __device__ Q p() const { return ps; }
    __device__ Q g_() const { return gs; }
    __device__ void set_q(Q v) { qs = v; }
    __device__ void set_p(Q v) { ps = v; }
    __device__ void set_gc(Q v) { gs = v; }
    __device__ void set_q0(Q v) { q0s = v; }
    __device__ void set_g0(Q v) { g0s = v; }
  };
  if constexpr (kPairedState) {
    Q* const q0a = reinterpret_cast<Q*>(save.q0);
    Q* const g0a = reinterpret_cast<Q*>(save.g0);
    // The update of element (x, w) of the tile (the same as the one-element
    // form below).  Its state in the storage type goes through io: q() the
    // mode, p() the momentum, g_() the cached gradient, and set_q/p/gc/q0/g0
    // what it writes (the mode where it drifts, the momentum, the cached
    // gradient of the plain gradient and the last step, the kept start
    // point), held in registers for the caller to move two elements at a time.
    auto step = [&](int e, int x, int w, double var_ld, auto& io) {
      const int kz = z0 + w, sx = signed_freq(x, N);
      const bool keep = retained(sx, sy, kz, N);
      const int n2 = sx * sx + sy * sy + kz * kz;
      const double var = keep ? var_ld : 0.0;
      // the mode, read once (gradient and drift)
      double2 q = make_double2(0.0, 0.0);
      if (kStartOfChain || (keep && (kFromSpectra || kDrift))) q = widen(io.q());
      double2 G = make_double2(0.0, 0.0);
      if constexpr (kFromSpectra) {
        if (keep) {
          C tv;
          if constexpr (kPair)
            tv = cadd(cscale(tile[LAY2::idx(x, w)], (T)sx), tile[LAY2::idx(x, S::W + w)]);
          else
            tv = cadd(acc[e], tile[LAY::idx(x, w)]);
          const double iv2 = 2.0 * inv_or_zero(var) * tab.inv_a, kf2 = 2.0 * mode_kfac(tab.kfac_adj, n2);
          // -2 i kfac t = (2 kfac t.y, -2 kfac t.x)
          G = make_double2(iv2 * q.x + kf2 * (double)tv.y, iv2 * q.y - kf2 * (double)tv.x);
        }
      } else {
        G = widen(io.g_());
      }
      if constexpr (MODE == kXGrad) {
        // plane_scale 0.5: gradient per stored entry (each Hermitian partner of
        // the kz = 0 plane taken as its own variable carries half)
        io.set_gc(narrow<Q>(kz == 0 ? make_double2(plane_scale * G.x, plane_scale * G.y) : G));
      }
      if constexpr (MODE == kXLast) io.set_gc(narrow<Q>(G));
      if constexpr (kStartOfChain) {
        // the start of the trajectory, kept for a rejection (both already in
        // the storage type)
        io.set_q0(narrow<Q>(q));
        io.set_g0(narrow<Q>(G));
      }
      if constexpr (MODE != kXGrad) {
        double2 p = make_double2(0.0, 0.0);
        if constexpr (kStartOfChain) {
          // momentum refresh p ~ N(0, M): Re and Im of a retained mode each
          // with variance 2 / sigma_k^2; an entry of the kz = 0 plane whose
          // Hermitian partner (-kx, -ky, 0) is canonical (ny > 0, or ny = 0 and
          // nx > 0) takes the conjugate of the partner's draw
          if (keep) {
            const bool mirror = kz == 0 && (sy < 0 || (sy == 0 && sx < 0));
            const size_t src = mirror ? gofs<N>((N - x) & (N - 1), (N - y) & (N - 1), 0) : gofs<N>(x, y, kz);
            const double2 z = normal_pair(draw_words(save.seed, save.iteration, kPurposeModes, src));
            const double sc = sqrt(2.0 * inv_or_zero(var));
            // drawn in FP64; K0 and the kick take the value as stored
            p = rounded<Q>(make_double2(sc * z.x, mirror ? -sc * z.y : sc * z.y));
          }
        } else {
          p = widen(io.p());
        }
        if constexpr (MODE == kXFirst && !CHAIN) {
          // the state this step starts from, kept where the caller asks (the
          // callers outside chains hold complex128 states)
          static_assert(sizeof(Q) == 16, "complex128 state outside chains");
          const size_t g = gofs<N>(x, y, kz);
          if (save.sv_q) st_stream(&save.sv_q[g], narrow<double2>(q));
          if (save.sv_p) st_stream(&save.sv_p[g], narrow<double2>(p));
        }
        // per stored mode (w / 8) sigma^2 |p|^2, w = 1 on kz = 0 (both
        // Hermitian partners stored), else 2
        const double wk = kz == 0 ? 0.125 : 0.25;
        if (kStartOfChain && keep) kin.add(wk * var * (p.x * p.x + p.y * p.y));
        p.x -= hk * G.x;
        p.y -= hk * G.y;
        p = rounded<Q>(p);
        if (MODE == kXLast && keep) kin.add(wk * var * (p.x * p.x + p.y * p.y));
        io.set_p(narrow<Q>(p));
        if constexpr (kDrift) {
          double2 a = make_double2(0.0, 0.0);
          if (keep) {
            const double c = eps * (0.5 * var);
            q.x += c * p.x;
            q.y += c * p.y;
            q = rounded<Q>(q);   // the prior energy and the next gradient are those of the stored modes
            io.set_q(narrow<Q>(q));
            prior.add((kz == 0 ? 0.5 : 1.0) * (q.x * q.x + q.y * q.y) * inv_or_zero(var));
            const double kf = mode_kfac(tab.kfac0, n2);
            a = make_double2(-kf * q.y, kf * q.x);      // i kfac q
          }
          const C ain = cconvert<C>(a), bn = cconvert<C>(make_double2((double)sx * a.x, (double)sx * a.y));
          if constexpr (kPair) {
            // over this element's own spectra, which only this thread reads
            tile[LAY2::idx(x, w)] = ain;
            tile[LAY2::idx(x, S::W + w)] = bn;
          } else {
            acc[e] = ain;                                // A-input (acc is free now)
            bin[e] = bn;
          }
        }
      }
    };
    struct alignas(16) QPair { Q v[2]; };
    tile_vecs<T, N, NT>([&](int, int x, int w) {   // w even: elements w and w + 1
      const size_t g = gofs<N>(x, y, z0 + w);
      const double2 var2 = ld_stream(reinterpret_cast<const double2*>(&tab.var[var_ofs(N, S::W, x, y, z0 + w)]));
      const QPair qv = ld_stream(reinterpret_cast<const QPair*>(&modes[g]));
      QPair pv{}, gv{};
      if constexpr (!kFromSpectra) gv = ld_stream(reinterpret_cast<const QPair*>(&gcache[g]));
      if constexpr (MODE != kXGrad && !kStartOfChain) pv = ld_stream(reinterpret_cast<const QPair*>(&mom[g]));
      PairIo io[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        io[j].qs = qv.v[j];   // (an excluded mode is written back as it was read)
        io[j].ps = pv.v[j];
        io[j].gs = gv.v[j];
      }
      step(0, x, w, var2.x, io[0]);
      step(0, x, w + 1, var2.y, io[1]);
      if constexpr (MODE == kXGrad || MODE == kXLast)
        st_stream(reinterpret_cast<QPair*>(&gcache[g]), QPair{{io[0].gs, io[1].gs}});
      if constexpr (kStartOfChain) {
        st_stream(reinterpret_cast<QPair*>(&q0a[g]), QPair{{io[0].q0s, io[1].q0s}});
        st_stream(reinterpret_cast<QPair*>(&g0a[g]), QPair{{io[0].g0s, io[1].g0s}});
      }
      if constexpr (MODE != kXGrad) st_stream(reinterpret_cast<QPair*>(&mom[g]), QPair{{io[0].ps, io[1].ps}});
      if constexpr (kDrift) st_stream(reinterpret_cast<QPair*>(&modes[g]), QPair{{io[0].qs, io[1].qs}});
    });
  } else {
    // one element per lane, reading and writing the arrays where the update
    // needs them (the update of step above, in the form whose register use
    // the unpaired and complex128 passes were tuned with)
    tile_elems<T, N, NT>([&](int e, int x, int w) {
      const int kz = z0 + w, sx = signed_freq(x, N);
      const size_t g = gofs<N>(x, y, kz);
      const bool keep = retained(sx, sy, kz, N);
      const int n2 = sx * sx + sy * sy + kz * kz;
      const double var = keep ? ld_stream(&tab.var[var_ofs(N, S::W, x, y, kz)]) : 0.0;
      // the mode, read once (gradient and drift)
      double2 q = make_double2(0.0, 0.0);
      if (kStartOfChain || (keep && (kFromSpectra || kDrift))) q = widen(ld_stream(&modes[g]));
      double2 G = make_double2(0.0, 0.0);
      if constexpr (kFromSpectra) {
        if (keep) {
          C tv;
          if constexpr (kPair)
            tv = cadd(cscale(tile[LAY2::idx(x, w)], (T)sx), tile[LAY2::idx(x, S::W + w)]);
          else
            tv = cadd(acc[e], tile[LAY::idx(x, w)]);
          const double iv2 = 2.0 * inv_or_zero(var) * tab.inv_a, kf2 = 2.0 * mode_kfac(tab.kfac_adj, n2);
          // -2 i kfac t = (2 kfac t.y, -2 kfac t.x)
          G = make_double2(iv2 * q.x + kf2 * (double)tv.y, iv2 * q.y - kf2 * (double)tv.x);
        }
      } else {
        G = widen(ld_stream(&gcache[g]));
      }
      if constexpr (MODE == kXGrad) {
        // plane_scale 0.5: gradient per stored entry (each Hermitian partner of
        // the kz = 0 plane taken as its own variable carries half)
        st_stream(&gcache[g], narrow<Q>(kz == 0 ? make_double2(plane_scale * G.x, plane_scale * G.y) : G));
      }
      if constexpr (MODE == kXLast) st_stream(&gcache[g], narrow<Q>(G));
      if constexpr (kStartOfChain) {
        // the start of the trajectory, kept for a rejection (both already in
        // the storage type)
        st_stream(&reinterpret_cast<Q*>(save.q0)[g], narrow<Q>(q));
        st_stream(&reinterpret_cast<Q*>(save.g0)[g], narrow<Q>(G));
      }
      if constexpr (MODE != kXGrad) {
        double2 p = make_double2(0.0, 0.0);
        if constexpr (kStartOfChain) {
          // momentum refresh p ~ N(0, M): Re and Im of a retained mode each
          // with variance 2 / sigma_k^2; an entry of the kz = 0 plane whose
          // Hermitian partner (-kx, -ky, 0) is canonical (ny > 0, or ny = 0 and
          // nx > 0) takes the conjugate of the partner's draw
          if (keep) {
            const bool mirror = kz == 0 && (sy < 0 || (sy == 0 && sx < 0));
            const size_t src = mirror ? gofs<N>((N - x) & (N - 1), (N - y) & (N - 1), 0) : g;
            const double2 z = normal_pair(draw_words(save.seed, save.iteration, kPurposeModes, src));
            const double sc = sqrt(2.0 * inv_or_zero(var));
            // drawn in FP64; K0 and the kick take the value as stored
            p = rounded<Q>(make_double2(sc * z.x, mirror ? -sc * z.y : sc * z.y));
          }
        } else if constexpr (kPrefetchP) {
          p = widen(ppf[e]);
        } else {
          p = widen(ld_stream(&mom[g]));
        }
        if constexpr (MODE == kXFirst && !CHAIN) {
          // the state this step starts from, kept where the caller asks (the
          // callers outside chains hold complex128 states)
          static_assert(sizeof(Q) == 16, "complex128 state outside chains");
          if (save.sv_q) st_stream(&save.sv_q[g], narrow<double2>(q));
          if (save.sv_p) st_stream(&save.sv_p[g], narrow<double2>(p));
        }
        // per stored mode (w / 8) sigma^2 |p|^2, w = 1 on kz = 0 (both
        // Hermitian partners stored), else 2
        const double wk = kz == 0 ? 0.125 : 0.25;
        if (kStartOfChain && keep) kin.add(wk * var * (p.x * p.x + p.y * p.y));
        p.x -= hk * G.x;
        p.y -= hk * G.y;
        p = rounded<Q>(p);
        if (MODE == kXLast && keep) kin.add(wk * var * (p.x * p.x + p.y * p.y));
        st_stream(&mom[g], narrow<Q>(p));
        if constexpr (kDrift) {
          double2 a = make_double2(0.0, 0.0);
          if (keep) {
            const double c = eps * (0.5 * var);
            q.x += c * p.x;
            q.y += c * p.y;
            q = rounded<Q>(q);   // the prior energy and the next gradient are those of the stored modes
            st_stream(&modes[g], narrow<Q>(q));
            prior.add((kz == 0 ? 0.5 : 1.0) * (q.x * q.x + q.y * q.y) * inv_or_zero(var));
            const double kf = mode_kfac(tab.kfac0, n2);
            a = make_double2(-kf * q.y, kf * q.x);      // i kfac q
          }
          const C ain = cconvert<C>(a), bn = cconvert<C>(make_double2((double)sx * a.x, (double)sx * a.y));
          if constexpr (kPair) {
            // over this element's own spectra, which only this thread reads
            tile[LAY2::idx(x, w)] = ain;
            tile[LAY2::idx(x, S::W + w)] = bn;
          } else {
            acc[e] = ain;                                // A-input (acc is free now)
            bin[e] = bn;
          }
        }
      }
    });
  }
  if constexpr (kKinetic) {
    const double ks = block_csum(kin, red);
    if (threadIdx.x == 0) save.kin_part[blockIdx.y * gridDim.x + blockIdx.x] = ks;
  } else {
    (void)kin;
  }
  if constexpr (kDrift && kPair) {
    const double ps = block_csum(prior, red);
    if (threadIdx.x == 0) prior_part[blockIdx.y * gridDim.x + blockIdx.x] = ps;
    __syncthreads();
    lds_fft<T, N, 2 * S::W, LAY2, NT, +1>(tile, twl);
    tile_vecs<T, N, NT>([&](int, int x, int w) { vec_store<T>(&outA[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY2>(tile, x, w)); });
    tile_vecs<T, N, NT>(
        [&](int, int x, int w) { vec_store<T>(&outB[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY2>(tile, x, S::W + w)); });
    (void)bin;
  } else if constexpr (kDrift) {
    const double ps = block_csum(prior, red);
    if (threadIdx.x == 0) prior_part[blockIdx.y * gridDim.x + blockIdx.x] = ps;
    __syncthreads();
    tile_elems<T, N, NT>([&](int e, int x, int w) { tile[LAY::idx(x, w)] = acc[e]; });
    __syncthreads();
    lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
    tile_vecs<T, N, NT>([&](int, int x, int w) { vec_store<T>(&outA[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY>(tile, x, w)); });
    __syncthreads();
    tile_elems<T, N, NT>([&](int e, int x, int w) { tile[LAY::idx(x, w)] = bin[e]; });
    __syncthreads();
    lds_fft<T, N, S::W, LAY, NT, +1>(tile, twl);
    tile_vecs<T, N, NT>([&](int, int x, int w) { vec_store<T>(&outB[gofs<N>(x, y, z0 + w)], vec_from_lds<T, LAY>(tile, x, w)); });
  } else {
    (void)outA;
    (void)outB;
    (void)prior_part;
    (void)bin;
  }
}

// ---------------------------------------------------------------------------
// Shared launches: blockIdx.z selects the plan.  The x pass reads S1, S2
// from a, b and, in the leapfrog modes, writes the next A, B over them
// (every tile reads its own entries before it writes them).
// ---------------------------------------------------------------------------
// Tables of the fiducial cosmology (f, sigma_8 as given).
template <typename T, int N> __device__ __forceinline__ ModeTables tables(const Ws<T, N>& w) {
  return ModeTables{w.mvar(), w.pc().kfac0, w.pc().kfac0, 1.0};
}

// Tables of an evaluation: with u8 and phi sampled, the multiplier of the
// state now (phi has drifted on by the time the x pass of a leapfrog step
// runs) and, for the adjoint and the prior gradient, u8 and phi where the
// final sums took the gradient.
template <typename T, int N> __device__ __forceinline__ ModeTables tables(const Ws<T, N>& w, const StateDev& st) {
  const PlanConst& pc = w.pc();
  ModeTables t{w.mvar(), pc.kfac0, pc.kfac0, 1.0};
  if (pc.sample_c && st.qs) {   // (the field of a state alone, without them, takes the fiducial ones)
    const double* ce = w.cosmo_eval();
    t.kfac0 = pc.kfac0 * st.qs[2];
    t.kfac_adj = pc.kfac0 * ce[1];
    t.inv_a = 1.0 / (ce[0] * ce[0]);
  }
  return t;
}

template <typename T, int N> __device__ __forceinline__ Binned<T> binned(const Ws<T, N>& w) {
  Binned<T> b;
  b.off = w.off();
  b.rx = w.rx(); b.ry = w.ry(); b.rz = w.rz();
  b.tx = w.tx(); b.ty = w.ty(); b.tz = w.tz();
  b.iz = w.iz();
  b.most = w.most();
  return b;
}

// S32: the plans' modes are a chain state in complex64 (st.q points to it).
template <typename T, int N, int NT, bool S32 = false>
__global__ void __launch_bounds__(NT) k_inv_x(Launch L) {
  using Q = typename StateElt<S32>::type;
  const Pick<T, N> k(L);
  if (k.mode != kXGrad) return;
  inv_x_body<T, N, NT, false, Q>(reinterpret_cast<const Q*>(k.st.q), tables(k.w, k.st), k.w.tw(), k.w.a(), k.w.b(),
                                 k.w.prior_part());
}

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT) k_inv_y(Launch L, int x0) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  inv_y_body<T, N, NT>(k.w.a(), k.w.b(), k.w.tw(), k.w.v0(), k.w.v1(), k.w.v2(), k.w.off(), x0);
}

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT) k_inv_y_all(Launch L, int x0) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  inv_y_body<T, N, NT, true>(k.w.a(), k.w.b(), k.w.tw(), k.w.v0(), k.w.v1(), k.w.v2(), nullptr, x0);
}

template <typename T, int N, int NT, bool DENSITY = false>
__global__ void __launch_bounds__(NT) k_inv_z_field(Launch L, int x0, T* out) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  inv_z_field_body<T, N, NT, DENSITY>(k.w.v0(), k.w.v1(), k.w.v2(), k.w.tw(), out, x0);
}

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT) k_inv_x_density(Launch L) {
  const Pick<T, N> k(L);
  if (k.mode != kXGrad) return;
  inv_x_body<T, N, NT, true>(k.st.q, tables(k.w), k.w.tw(), k.w.a(), k.w.b(), k.w.prior_part());
}

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT) k_inv_z_gather(Launch L, int x0) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  inv_z_gather_body<T, N, NT>(k.w.v0(), k.w.v1(), k.w.v2(), k.w.tw(), binned(k.w), k.w.part(), x0);
}

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT) k_fwd_z_scatter(Launch L, int x0) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  fwd_z_scatter_body<T, N, NT>(k.w.gsort(), binned(k.w), k.w.tw(), k.w.v0(), k.w.v1(), k.w.v2(), x0);
}

template <typename T, int N, int NT>
__global__ void __launch_bounds__(NT) k_fwd_y(Launch L, int x0) {
  const Pick<T, N> k(L);
  if (k.mode == kXSkip) return;
  fwd_y_body<T, N, NT>(k.w.v0(), k.w.v1(), k.w.v2(), k.w.tw(), k.w.off(), k.w.a(), k.w.b(), x0);
}

// One launch per mode present in a batch; plans in another mode return.
// CHAIN: the first step of a chain's trajectory, which also draws the
// momenta, keeps the start point and sums K0.  S32: the chain state (modes,
// momenta, cached gradient, start point) is stored in complex64.  Four
// waves per SIMD (two blocks per compute unit): the FP64 middle step spills
// a few registers for it and still gains 5 %, the first step 10 % in both
// precisions.
template <typename T, int N, int MODE, int NT, bool CHAIN = false, bool S32 = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_x_pass(Launch L,
                                                                                    double plane_scale) {
  using Q = typename StateElt<S32>::type;
  const Pick<T, N> k(L);
  if (k.mode != MODE) return;
  ChainSave save{k.w.q0(), k.w.g0(), k.w.kin_part(), 0, 0, k.st.sv_q, k.st.sv_p};
  if constexpr (CHAIN) {
    const ChainScalars* cs = k.w.chain();
    save.seed = cs->seed;
    save.iteration = (uint32_t)cs->iter;
  }
  x_pass_body<T, N, MODE, NT, CHAIN, Q>(k.w.a(), k.w.b(), reinterpret_cast<Q*>(k.st.q), reinterpret_cast<Q*>(k.st.p),
                                        reinterpret_cast<Q*>(k.st.g), tables(k.w, k.st), k.w.tw(), k.st.eps,
                                        k.w.a(), k.w.b(), k.w.prior_part(), plane_scale, save);
}

}  // namespace hamlet
