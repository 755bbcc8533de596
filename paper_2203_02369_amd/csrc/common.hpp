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

// Storage type of a chain's mode state (modes, momenta, cached gradient,
// saved start point): complex128, or complex64 for the chains of the FP32
// path.  Updates are computed in FP64 and rounded to the storage type
// before any use, so that the energies and gradients are those of the state
// as stored.
template <bool S32> struct StateElt { using type = double2; };
template <> struct StateElt<true> { using type = float2; };
template <typename Q> __device__ __forceinline__ double2 widen(Q v) { return make_double2((double)v.x, (double)v.y); }
template <typename Q> __device__ __forceinline__ Q narrow(double2 v) { return cconvert<Q>(v); }
template <typename Q> __device__ __forceinline__ double2 rounded(double2 v) { return widen(narrow<Q>(v)); }

// Streaming (non-temporal) loads and stores, for the arrays a pass reads or
// writes once: on the MI355X they stream about 15 % faster than plain
// accesses (a 1 GiB copy: 5.2 vs 4.6 TB/s) and leave the caches to data that
// is reused.  The passes load every spectral and mode array this way, but
// store plainly what the very next pass reads (it then partly comes from the
// memory-side cache), and stream out only the modes, momenta and cached
// gradient, read again one evaluation later.  Elements of 8 or 16 bytes.
template <typename X> __device__ __forceinline__ X ld_stream(const X* p) {
  static_assert(sizeof(X) == 8 || sizeof(X) == 16, "8- or 16-byte elements");
  if constexpr (sizeof(X) == 8) {
    return __builtin_bit_cast(X, __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p)));
  } else {
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(X, __builtin_nontemporal_load(reinterpret_cast<const u64x2*>(p)));
  }
}
template <typename X> __device__ __forceinline__ void st_stream(X* p, X v) {
  static_assert(sizeof(X) == 8 || sizeof(X) == 16, "8- or 16-byte elements");
  if constexpr (sizeof(X) == 8) {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), reinterpret_cast<unsigned long long*>(p));
  } else {
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(__builtin_bit_cast(u64x2, v), reinterpret_cast<u64x2*>(p));
  }
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
