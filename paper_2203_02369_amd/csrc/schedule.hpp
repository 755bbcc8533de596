// The kernel schedule of a grid size and real type: threads per block of
// each pass kind, the tile shapes of the strided and z passes, and the radix
// plan of the LDS transforms (fft.hpp).
//
// The defaults below were picked by hand; the autotuner
// (paper_2203_02369_amd/autotune.py) times alternatives on the GPU, keeps the
// fastest per pass kind in tuned_schedules.json and writes tuned.hpp, whose
// specialisations of Tuned<T, N> replace the defaults.  A tuning build
// (-DHAMLET_SCHED_DEFAULTS) ignores tuned.hpp and moves one parameter of
// every grid's schedule with -DHAMLET_SCHED_{XY,X,ZG,ZS,RADIX}=value or
// -DHAMLET_SCHED_{W,PZ,PG}_SHIFT=s (the default times 2^s, clamped to the
// valid range).
#pragma once

namespace hamlet {

// kz columns per strided tile of the x and y passes: 16 (FP32) or 8 (FP64),
// halved at N = 512 and again at 1024 so that a tile of N rows keeps the
// LDS and registers it has at 256, and at most N/2.  The per-mode sigma^2
// array is laid out in these tiles, so the passes, the layout and the host
// all take the width from the schedule.
__host__ __device__ constexpr int default_tile_width(int real_bytes, int n) {
  const int w = (real_bytes == 4 ? 16 : 8) / (n >= 1024 ? 4 : (n >= 512 ? 2 : 1));
  return w < n / 2 ? w : n / 2;
}

__host__ __device__ constexpr int clamp_pow2(int v, int s, int lo, int hi) {
  const int x = s >= 0 ? v << s : v >> -s;
  return x < lo ? lo : (x > hi ? hi : x);
}

template <typename T, int N> struct DefaultSched {
  static constexpr int XY = N >= 512 ? 512 : 256;   // y passes (and the inverse x pass of a plain gradient)
  static constexpr int X = 512;                      // x pass
  static constexpr int ZG = 256;                     // inverse z pass with the gather
  static constexpr int ZS = 256;                     // forward z pass with the scatter
  static constexpr int RADIX = 0;                    // radix plan (fft.hpp)
  static constexpr int W = default_tile_width(sizeof(T), N);   // kz columns per strided tile
  // pencils per z tile of the scatter, and of the gather (half as many at
  // 512^3, where its LDS transform buffer would otherwise keep two tiles per
  // compute unit)
  static constexpr int PZ = (sizeof(T) == 4 ? 8 : 4) < N ? (sizeof(T) == 4 ? 8 : 4) : N;
  static constexpr int PG = N >= 512 ? PZ / 2 : PZ;
};

template <typename T, int N> struct Tuned : DefaultSched<T, N> {};

}  // namespace hamlet

#ifndef HAMLET_SCHED_DEFAULTS
#include "tuned.hpp"
#endif

namespace hamlet {

template <typename T, int N> struct Sched {
#ifdef HAMLET_SCHED_XY
  static constexpr int XY = HAMLET_SCHED_XY;
#else
  static constexpr int XY = Tuned<T, N>::XY;
#endif
#ifdef HAMLET_SCHED_X
  static constexpr int X = HAMLET_SCHED_X;
#else
  static constexpr int X = Tuned<T, N>::X;
#endif
#ifdef HAMLET_SCHED_ZG
  static constexpr int ZG = HAMLET_SCHED_ZG;
#else
  static constexpr int ZG = Tuned<T, N>::ZG;
#endif
#ifdef HAMLET_SCHED_ZS
  static constexpr int ZS = HAMLET_SCHED_ZS;
#else
  static constexpr int ZS = Tuned<T, N>::ZS;
#endif
#ifdef HAMLET_SCHED_RADIX
  static constexpr int RADIX = HAMLET_SCHED_RADIX;
#else
  static constexpr int RADIX = Tuned<T, N>::RADIX;
#endif
#ifndef HAMLET_SCHED_W_SHIFT
#define HAMLET_SCHED_W_SHIFT 0
#endif
#ifndef HAMLET_SCHED_PZ_SHIFT
#define HAMLET_SCHED_PZ_SHIFT 0
#endif
#ifndef HAMLET_SCHED_PG_SHIFT
#define HAMLET_SCHED_PG_SHIFT 0
#endif
  // FP32 loads and stores the strided tiles two columns at a time, so W >= 2
  static constexpr int W = clamp_pow2(Tuned<T, N>::W, HAMLET_SCHED_W_SHIFT, sizeof(T) == 4 ? 2 : 1, N / 2);
  // whole pencil pairs; the scatter's tile set-up (4 PZ + 4 lanes) runs in one wave
  static constexpr int PZ = clamp_pow2(Tuned<T, N>::PZ, HAMLET_SCHED_PZ_SHIFT, 2, N < 8 ? N : 8);
  // whole pencil pairs; a wave holds every (pencil, corner) of the gather's tile
  static constexpr int PG = clamp_pow2(Tuned<T, N>::PG, HAMLET_SCHED_PG_SHIFT, 2, N < 16 ? N : 16);
};

// Radix plans per transform length: the radices of the Stockham stages in
// order (0 past the last stage); plan 0 is the hand-picked one, the others
// are the alternatives the autotuner times.  An index beyond a length's
// plans falls back to its plan 0.
struct RadixPlan {
  int r[3];
};
__host__ __device__ constexpr int radix_plans(int n) {
  return n == 16 ? 2 : (n == 32 ? 3 : (n == 64 ? 3 : (n == 128 ? 3 : (n == 256 ? 4 : (n == 512 ? 3 : 1)))));
}
__host__ __device__ constexpr RadixPlan radix_plan(int n, int pl) {
  pl = pl >= 0 && pl < radix_plans(n) ? pl : 0;
  switch (n) {
    case 8: return {{8, 0, 0}};
    case 16: return pl == 1 ? RadixPlan{{16, 0, 0}} : RadixPlan{{4, 4, 0}};
    case 32: return pl == 1 ? RadixPlan{{4, 8, 0}} : (pl == 2 ? RadixPlan{{2, 16, 0}} : RadixPlan{{8, 4, 0}});
    case 64: return pl == 1 ? RadixPlan{{4, 16, 0}} : (pl == 2 ? RadixPlan{{16, 4, 0}} : RadixPlan{{8, 8, 0}});
    case 128: return pl == 1 ? RadixPlan{{8, 16, 0}} : (pl == 2 ? RadixPlan{{8, 4, 4}} : RadixPlan{{16, 8, 0}});
    case 256:
      return pl == 1 ? RadixPlan{{4, 4, 16}}
                     : (pl == 2 ? RadixPlan{{16, 4, 4}} : (pl == 3 ? RadixPlan{{8, 8, 4}} : RadixPlan{{16, 16, 0}}));
    case 512: return pl == 1 ? RadixPlan{{16, 8, 4}} : (pl == 2 ? RadixPlan{{4, 8, 16}} : RadixPlan{{8, 8, 8}});
    default: return {{16, 8, 8}};   // 1024
  }
}

// Grid sizes built into this library (a tuning build holds one).
#ifdef HAMLET_ONLY_N
constexpr bool has_grid(int n) { return n == HAMLET_ONLY_N; }
#else
constexpr bool has_grid(int) { return true; }
#endif

}  // namespace hamlet
