// The paper's flat parameter vector (Section 3.1): Re of the independent
// modes, Im of them, the distances, s (and u8, phi when sampled).
//
// Independent modes are the retained stored entries with kz > 0 and, on the
// kz = 0 plane, the canonical member of each Hermitian pair (ny > 0, or
// ny = 0 and nx > 0), in row-major (kx, ky, kz) order.  Their rank in that
// order has a closed form, so each thread maps its own entry without tables:
// with h = N/2, the rows (kx, ky) with no Nyquist index are retained, each
// holds h - 1 entries with kz > 0 and one more on kz = 0 when canonical.
#pragma once

#include "common.hpp"

namespace hamlet {

// Independent modes: m = ((N-1)^3 - 1) / 2.
__host__ __device__ inline int64_t flat_modes(int n) {
  const int64_t r = n - 1;
  return (r * r * r - 1) / 2;
}

// Canonical kz = 0 entry (ny > 0, or ny = 0 and nx > 0), in a retained row.
__device__ __forceinline__ bool canonical_row(int sx, int sy) { return sy > 0 || (sy == 0 && sx > 0); }

// Rank of the independent entry (x, y, kz) (array indices, row retained,
// and kz > 0 or the row canonical) among all independent entries.
__device__ __forceinline__ int64_t flat_rank(int n, int x, int y, int kz) {
  const int h = n / 2;
  const int rx = x - (x > h ? 1 : 0);   // retained rows before row x
  const int ry = y - (y > h ? 1 : 0);
  const int64_t rows = (int64_t)rx * (n - 1) + ry;   // retained rows before (x, y)
  // canonical kz = 0 entries before (x, y): per retained row x' < x, h - 1
  // with ny > 0 plus the ny = 0 one when 0 < nx' < h; in row x, the y' < y
  // with 0 < y' < h, plus y' = 0 when y > 0 and 0 < nx < h
  const int64_t canon_before = (int64_t)rx * (h - 1) + min(max(x - 1, 0), h - 1) + min(max(y - 1, 0), h - 1) +
                               ((y > 0 && x >= 1 && x <= h - 1) ? 1 : 0);
  const bool canon = canonical_row(signed_freq(x, n), signed_freq(y, n));
  const int64_t within = kz == 0 ? 0 : (canon ? 1 : 0) + (kz - 1);
  return rows * (h - 1) + canon_before + within;
}

// flat <- (modes, dist, the ns small coordinates).  Grid over max(stored
// entries, n + ns).
__global__ void __launch_bounds__(256)
k_pack_flat(const double2* __restrict__ modes, const double* __restrict__ dist, const double* __restrict__ snl,
            double* __restrict__ flat, int n, int n_gal, int ns) {
  const int h = n / 2;
  const size_t total = (size_t)n * n * h;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = flat_modes(n);
  if (g < total) {
    const int kz = (int)(g % h), y = (int)((g / h) % n), x = (int)(g / ((size_t)h * n));
    const int sx = signed_freq(x, n), sy = signed_freq(y, n);
    if (retained(sx, sy, kz, n) && (kz > 0 || canonical_row(sx, sy))) {
      const int64_t r = flat_rank(n, x, y, kz);
      const double2 v = modes[g];
      flat[r] = v.x;
      flat[m + r] = v.y;
    }
  }
  if (g < (size_t)n_gal) flat[2 * m + g] = dist[g];
  if (g < (size_t)ns) flat[2 * m + n_gal + g] = snl[g];
}

// (modes, dist, the ns small coordinates) <- flat.  Grid over max(stored
// entries, n + ns).
__global__ void __launch_bounds__(256)
k_unpack_flat(const double* __restrict__ flat, double2* __restrict__ modes, double* __restrict__ dist,
              double* __restrict__ snl, int n, int n_gal, int ns) {
  const int h = n / 2;
  const size_t total = (size_t)n * n * h;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = flat_modes(n);
  if (g < total) {
    const int kz = (int)(g % h), y = (int)((g / h) % n), x = (int)(g / ((size_t)h * n));
    const int sx = signed_freq(x, n), sy = signed_freq(y, n);
    double2 v = make_double2(0.0, 0.0);
    if (retained(sx, sy, kz, n)) {
      if (kz > 0 || canonical_row(sx, sy)) {
        const int64_t r = flat_rank(n, x, y, kz);
        v = make_double2(flat[r], flat[m + r]);
      } else {
        // mirror entry of the kz = 0 plane: conjugate of (-kx, -ky, 0)
        const int64_t r = flat_rank(n, (n - x) & (n - 1), (n - y) & (n - 1), 0);
        v = make_double2(flat[r], -flat[m + r]);
      }
    }
    modes[g] = v;
  }
  if (g < (size_t)n_gal) dist[g] = flat[2 * m + g];
  if (g < (size_t)ns) snl[g] = flat[2 * m + n_gal + g];
}

}  // namespace hamlet
