// Shared device/host helpers of the HAMLET gfx950 library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hamlet {

// Physical constants (units: Mpc/h, km/s; H0 = 100 km/s per Mpc/h).
constexpr double kC = 299792.458;
constexpr double kH0 = 100.0;
constexpr double kSigmaNlUnit = 100.0;   // s = sigma_NL / 100 km/s

// Complex type of a real type.
template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };
template <typename T> using cplx_t = typename Cplx<T>::type;

template <typename C> __device__ __forceinline__ C cmake(decltype(C{}.x) re, decltype(C{}.x) im) {
  C r; r.x = re; r.y = im; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C{}.x) s) { return cmake<C>(a.x * s, a.y * s); }
// i * a
template <typename C> __device__ __forceinline__ C cmuli(C a) { return cmake<C>(-a.y, a.x); }

template <typename To, typename From> __device__ __forceinline__ To cconvert(From a) {
  To r; r.x = static_cast<decltype(r.x)>(a.x); r.y = static_cast<decltype(r.y)>(a.y); return r;
}

// Signed frequency index of array index j on an axis of length n.
__device__ __host__ __forceinline__ int signed_freq(int j, int n) { return j < n / 2 ? j : j - n; }

// Retained mode: not k = 0 and no component on a Nyquist index.  Only
// kz in [0, N/2) is stored, so the kz = N/2 plane never appears.
__device__ __host__ __forceinline__ bool retained(int sx, int sy, int kz, int n) {
  const int h = n / 2;
  if (sx == -h || sy == -h) return false;
  return (sx | sy | kz) != 0;
}

}  // namespace hamlet
