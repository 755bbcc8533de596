// Kernel schedules chosen by the autotuner (paper_2203_02369_amd/autotune.py)
// from tuned_schedules.json; grids and types not listed keep DefaultSched.
// Generated: do not edit by hand.
#pragma once

namespace hamlet {

template <> struct Tuned<float, 64> : DefaultSched<float, 64> {
  static constexpr int PG = 4;
  static constexpr int PZ = 2;
  static constexpr int W = 8;
};

template <> struct Tuned<float, 128> : DefaultSched<float, 128> {
  static constexpr int PZ = 4;
  static constexpr int ZS = 128;
};

template <> struct Tuned<float, 512> : DefaultSched<float, 512> {
  static constexpr int PG = 2;
};

template <> struct Tuned<float, 1024> : DefaultSched<float, 1024> {
  static constexpr int PG = 2;
  static constexpr int ZG = 512;
  static constexpr int ZS = 512;
  static constexpr int X = 1024;
  static constexpr int XY = 1024;
  static constexpr int W = 16;
};

template <> struct Tuned<double, 128> : DefaultSched<double, 128> {
  static constexpr int RADIX = 2;
  static constexpr int ZS = 128;
  static constexpr int X = 256;
};

template <> struct Tuned<double, 256> : DefaultSched<double, 256> {
  static constexpr int RADIX = 3;
};

template <> struct Tuned<double, 512> : DefaultSched<double, 512> {
  static constexpr int PZ = 8;
  static constexpr int ZS = 512;
  static constexpr int X = 1024;
  static constexpr int W = 8;
};

template <> struct Tuned<double, 1024> : DefaultSched<double, 1024> {
  static constexpr int PZ = 8;
  static constexpr int ZG = 512;
  static constexpr int ZS = 512;
  static constexpr int W = 8;
};

}  // namespace hamlet
