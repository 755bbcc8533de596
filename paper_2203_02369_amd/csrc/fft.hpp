// LDS-staged Stockham FFT building blocks for gfx950 (wave64).
//
// The velocity field of eq:vel-field is three inverse 3-D transforms of the
// modes, and the gradient needs three forward transforms of the scattered
// galaxy weights (the hand-built inverse-transform gradient of Section 4).
// Each 3-D transform is done as three batched 1-D passes; this header holds
// the 1-D part: a batch of B transforms of length N held in LDS is
// transformed in place by self-sorting (Stockham) radix-R stages, each
// butterfly's R points kept in registers.
//
// Stage with sub-transform length L (product of the earlier radices): for
// butterfly j in [0, N/R), k = j mod L,
//     x_r = in[j + r N/R] * w^(r k),  w = exp(sign 2 pi i / (L R)),
//     y   = DFT_R(x),
//     out[(j / L) L R + k + s L] = y_s.
// Twiddles come from a table tw[m] = exp(-2 pi i m / N) staged in LDS.
#pragma once

#include "common.hpp"
#include "schedule.hpp"

namespace hamlet {

// exp(SIGN 2 pi i j / 16) for j in [0, 8): cos and sin of multiples of pi/8.
template <typename T> __device__ __forceinline__ T cos16(int j) {
  // j in [0, 8)
  constexpr double c[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                           0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
  return static_cast<T>(c[j]);
}
template <typename T> __device__ __forceinline__ T sin16(int j) {
  constexpr double s[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                           1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
  return static_cast<T>(s[j]);
}

// b * exp(SIGN 2 pi i j / 16), j in [0, 8) known after unrolling.
template <typename T, int SIGN>
__device__ __forceinline__ cplx_t<T> rot16(cplx_t<T> b, int j) {
  using C = cplx_t<T>;
  if (j == 0) return b;
  if (j == 4) return SIGN > 0 ? cmake<C>(-b.y, b.x) : cmake<C>(b.y, -b.x);
  const T c = cos16<T>(j);
  const T s = SIGN > 0 ? sin16<T>(j) : -sin16<T>(j);
  return cmake<C>(b.x * c - b.y * s, b.x * s + b.y * c);
}

__host__ __device__ constexpr int bitrev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}
__host__ __device__ constexpr int log2_c(int n) { return n <= 1 ? 0 : 1 + log2_c(n / 2); }

// In-register DFT of R = 2, 4, 8 or 16 points, natural order in and out:
// bit-reversal permutation, then radix-2 butterflies.
template <typename T, int R, int SIGN>
__device__ __forceinline__ void dft_reg(cplx_t<T> (&v)[R]) {
  using C = cplx_t<T>;
  constexpr int BITS = log2_c(R);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev_c(i, BITS);
    if (j > i) { C t = v[i]; v[i] = v[j]; v[j] = t; }
  }
#pragma unroll
  for (int half = 1; half < R; half *= 2) {
#pragma unroll
    for (int g = 0; g < R; g += 2 * half) {
#pragma unroll
      for (int k = 0; k < half; ++k) {
        const C a = v[g + k];
        const C b = rot16<T, SIGN>(v[g + k + half], k * (16 / (2 * half)));
        v[g + k] = cadd(a, b);
        v[g + k + half] = csub(a, b);
      }
    }
  }
}

// LDS layouts of a batch of transforms.  idx(n, b) is the slot of element n
// of transform b.  Both pad so that the store phase of a radix-16 stage
// (writes R*L apart) spreads over the 64 banks as evenly as 64-bit or
// 128-bit accesses allow.
//
// RowLayout: W transforms side by side (element n of all transforms is one
// row of W); used for passes along a strided axis, transforms on consecutive
// threads.  8-byte elements get one pad slot per row, 16-byte elements two
// pad slots every 16 rows.
template <typename C, int W> struct RowLayout {
  static constexpr int P1 = sizeof(C) == 8 ? 1 : 0;
  static constexpr int P16 = sizeof(C) == 8 ? 0 : 2;
  static constexpr bool kNFast = false;
  __device__ __forceinline__ static int idx(int n, int b) { return n * (W + P1) + (n >> 4) * P16 + b; }
  static constexpr int size(int n) { return n * (W + P1) + (n >> 4) * P16; }
};

// PencilLayout: each transform contiguous with one pad slot per 16 elements;
// used for passes along the contiguous axis, butterflies on consecutive threads.
template <int N> struct PencilLayout {
  static constexpr int SB = N + N / 16;
  static constexpr bool kNFast = true;
  __device__ __forceinline__ static int idx(int n, int b) { return b * SB + n + (n >> 4); }
  static constexpr int size(int f) { return f * SB; }
};

// One Stockham stage on a batch of B transforms held in LDS (layout L).
// Thread mapping follows the layout: butterflies of a transform on
// consecutive threads (pencils) or transforms on consecutive threads (rows).
// TWP: form a radix-16 stage's twiddles from two table reads (below).
template <typename T, int N, int R, int LEN, int B, typename LAY, int NT, int SIGN, bool TWP = false>
__device__ __forceinline__ void lds_stage(cplx_t<T>* buf, const cplx_t<T>* tw) {
  using C = cplx_t<T>;
  constexpr int NB = N / R;
  constexpr int TOT = NB * B;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int TSTEP = N / (LEN * R);
  constexpr bool NFAST = LAY::kNFast;
  C v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int idx = tid + p * NT;
    if (TOT % NT == 0 || idx < TOT) {
      const int b = NFAST ? idx / NB : idx % B;
      const int j = NFAST ? idx % NB : idx / B;
      const int k = j % LEN;
      if constexpr (TWP && R == 16 && LEN > 1) {
        // Read w^k and w^4k and form the other powers w^rk with at most
        // three products (a few ulp): 2 LDS reads instead of 15 and fewer
        // live registers, which is what the scatter's dense path gains by.
        C w1 = tw[k * TSTEP], w4 = tw[4 * k * TSTEP];
        if (SIGN > 0) {
          w1.y = -w1.y;
          w4.y = -w4.y;
        }
        C w[R];
        w[1] = w1;
        w[2] = cmul(w1, w1);
        w[3] = cmul(w[2], w1);
        w[4] = w4;
        w[5] = cmul(w4, w1);
        w[6] = cmul(w4, w[2]);
        w[7] = cmul(w4, w[3]);
        w[8] = cmul(w4, w4);
#pragma unroll
        for (int r = 9; r < R; ++r) w[r] = cmul(w[8], w[r - 8]);
        v[p][0] = buf[LAY::idx(j, b)];
#pragma unroll
        for (int r = 1; r < R; ++r) v[p][r] = cmul(buf[LAY::idx(j + r * NB, b)], w[r]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          C x = buf[LAY::idx(j + r * NB, b)];
          if (LEN > 1 && r > 0) {
            C w = tw[r * k * TSTEP];
            if (SIGN > 0) w.y = -w.y;
            x = cmul(x, w);
          }
          v[p][r] = x;
        }
      }
      dft_reg<T, R, SIGN>(v[p]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int idx = tid + p * NT;
    if (TOT % NT == 0 || idx < TOT) {
      const int b = NFAST ? idx / NB : idx % B;
      const int j = NFAST ? idx % NB : idx / B;
      const int k = j % LEN;
      const int base = (j / LEN) * LEN * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[LAY::idx(base + r * LEN, b)] = v[p][r];
    }
  }
  __syncthreads();
}

// The whole transform of a batch in LDS, in the Stockham stages of the
// schedule's radix plan (schedule.hpp); a stage's span is the product of
// the radices before it.
// Callers must have synchronised the LDS contents before the call; on
// return the result is in place and synchronised.
template <typename T, int N, int B, typename LAY, int NT, int SIGN, bool TWP = false>
__device__ __forceinline__ void lds_fft(cplx_t<T>* buf, const cplx_t<T>* tw) {
  static_assert(N >= 8 && N <= 1024 && (N & (N - 1)) == 0, "FFT length must be 8..1024, power of two");
  constexpr RadixPlan RP = radix_plan(N, Sched<T, N>::RADIX);
  static_assert(RP.r[0] * (RP.r[1] ? RP.r[1] : 1) * (RP.r[2] ? RP.r[2] : 1) == N, "radices multiply to N");
  lds_stage<T, N, RP.r[0], 1, B, LAY, NT, SIGN, TWP>(buf, tw);
  if constexpr (RP.r[1] > 0) lds_stage<T, N, RP.r[1], RP.r[0], B, LAY, NT, SIGN, TWP>(buf, tw);
  if constexpr (RP.r[2] > 0) lds_stage<T, N, RP.r[2], RP.r[0] * RP.r[1], B, LAY, NT, SIGN, TWP>(buf, tw);
}

// Stage the N-entry twiddle table into LDS (caller synchronises).
template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(cplx_t<T>* tw_lds, const cplx_t<T>* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += NT) tw_lds[i] = tw[i];
}

// The same in two steps: load() into registers, store() into LDS, so that a
// pass can issue its tile loads in between and wait once for both.
template <typename T, int N, int NT> struct TwiddleStage {
  static constexpr int R = (N + NT - 1) / NT;
  cplx_t<T> v[R];
  __device__ __forceinline__ void load(const cplx_t<T>* __restrict__ tw) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = threadIdx.x + r * NT;
      if (i < N) v[r] = tw[i];
    }
  }
  __device__ __forceinline__ void store(cplx_t<T>* tw_lds) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = threadIdx.x + r * NT;
      if (i < N) tw_lds[i] = v[r];
    }
  }
};

}  // namespace hamlet
