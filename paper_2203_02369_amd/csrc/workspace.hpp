// A plan's device workspace and the argument table of shared launches.
//
// Each plan owns one allocation whose layout is a fixed function of the grid
// size N, the real type and the catalogue size: a block of per-plan
// constants, the arrays whose size depends on N only (at offsets that are
// compile-time constants), then the per-galaxy arrays (each a whole number of
// "galaxy units" of 8 bytes per galaxy), then the distance-prior histogram.
// A kernel therefore needs only the workspace base and the catalogue size of
// each plan.  A shared launch takes a Launch table by value with those and
// the per-call state pointers of up to kMaxBatch plans, indexed by
// blockIdx.z: one scalar load from the argument segment per field, no
// pointer chasing before the first data load.
#pragma once

#include "common.hpp"
#include "schedule.hpp"

namespace hamlet {

constexpr int kMaxBatch = 16;

// What a plan does in one launch.  In an evaluation: a plain gradient
// (kXGrad), a step inside a leapfrog trajectory with the merged kicks and a
// drift (kXMid), or the last step of a trajectory (kXLast); the first kick
// and drift of a trajectory is kXFirst.  kXSkip: the plan sits the launch
// out (its blocks return at once).  Bookkeeping launches only test for
// kXSkip.
enum XMode { kXSkip = -1, kXGrad = 0, kXFirst = 1, kXMid = 2, kXLast = 3 };

// The small coordinates of a state: s = sigma_NL / 100 km/s, and when the
// plan samples the cosmological parameters u8 = sigma_8 / sigma_8,fid,
// phi = f / f_fid and eta = h / h_fid (kSmallMax values: q_snl, p_snl, g_snl
// hold 1 or 4).
constexpr int kSmallMax = 4;

// Per-plan constants, at the start of the workspace.
struct PlanConst {
  int n_gal, n_hist, sample_d, sample_s;
  int n_prior_part, n_like_part, n_kin_part, sample_c;   // sample_c: u8, phi and eta sampled
  double om, h;            // Omega_0, little h (for mu)
  double box, spacing;     // L, L / N
  double dmax;             // c / (3 Omega_0 H0): domain of zbar(d)
  double hist_w;           // bin width of the distance prior, Mpc/h
  double minv_d;           // inverse mass of a distance, (sigma_v / H0)^2
  double psd;              // sqrt of the mass of a distance, H0 / sigma_v
  double kfac0;            // H0 f / (N^3 k_f), k_f = 2 pi / L (fiducial f)
  double minv_u8, minv_phi, minv_eta;   // inverse masses of u8, phi and eta
  double d_modes;          // real mode coordinates, (N-1)^3 - 1
};

// What one call works on: the coordinates, their momenta, where the
// gradient and Psi go, the step, and the chain outputs.
struct StateDev {
  double2* q;              // modes
  double2* p;              // mode momenta
  double2* g;              // mode gradient target, or the cached gradient
  double* qd;              // distances
  double* pd;
  double* gd;
  double* qs;              // s = sigma_NL / 100 km/s
  double* ps;
  double* gs;
  double* psi;
  const double* eps;
  double* dh;              // Delta H per chain iteration (or nullptr)
  int32_t* acc;            // accept flag per chain iteration (or nullptr)
  double2* msum;           // running sum of post-warm-up mode samples (or nullptr)
  double* psi_out;         // Psi of a leapfrog end point
  // Where the first step of a leapfrog call keeps the state it starts from
  // (coordinates and momenta, before its kick and drift), or nullptr: the
  // No-U-Turn sampler keeps the leaves its tree still needs this way.
  double2* sv_q;
  double2* sv_p;
  double* sv_qd;
  double* sv_pd;
  double* sv_qs;
  double* sv_ps;
};

struct Launch {
  char* base[kMaxBatch];
  int n_gal[kMaxBatch];
  int mode[kMaxBatch];
  StateDev st[kMaxBatch];
};

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Offsets of the arrays whose size depends on N and the real size R only.
// Sphere moments of the velocity field (analysis.hpp): radii per call, radii
// per pass over the modes, blocks of a pass (one partial sum per block and
// value), values per pass.
constexpr int kMomentsMaxRadii = 16;
constexpr int kMomentsRadiiPerPass = 8;
constexpr int kMomentsBlocks = 1024;
constexpr int kMomentsPassValues = 4 * kMomentsRadiiPerPass;
constexpr size_t kMomentsPartBytes =
    8 * size_t(kMomentsBlocks) * kMomentsPassValues * (kMomentsMaxRadii / kMomentsRadiiPerPass);

// The x pass's tile width of a grid size and real width (bytes): sigma^2
// per mode is laid out in these tiles (schedule.hpp).
template <int N, int R> constexpr int layout_tile_width() {
  return R == 4 ? Sched<float, N>::W : Sched<double, N>::W;
}

template <int N, int R> struct FixedLayout {
  static constexpr size_t NM = size_t(N) * N * (N / 2);          // stored modes
  static constexpr size_t NPK = 3 * size_t(N / 2) * (N / 2) + 1; // |n|^2 table
  static constexpr int W = layout_tile_width<N, R>();
  static constexpr int N_PRIOR = N * ((N / 2) / W);              // x-pass blocks
  static constexpr int N_KIN_SMALL = 64;                         // blocks of the distance and s terms
  static constexpr int N_KIN = N_PRIOR + N_KIN_SMALL;            // kinetic-energy partials
  static constexpr size_t consts = 0;
  static constexpr size_t chain = align256(consts + sizeof(PlanConst));
  static constexpr size_t chain_bytes = 256;                     // ChainScalars
  static constexpr size_t var_n2 = align256(chain + chain_bytes);
  static constexpr size_t tw = align256(var_n2 + 8 * NPK);
  static constexpr size_t count = align256(tw + 2 * R * size_t(N));
  static constexpr size_t off = align256(count + 4 * size_t(N) * N);
  static constexpr size_t cursor = align256(off + 4 * (size_t(N) * N + 1));
  static constexpr size_t prior_part = align256(cursor + 4 * size_t(N) * N);
  static constexpr size_t kin_part = align256(prior_part + 8 * size_t(N_PRIOR));
  static constexpr size_t small = align256(kin_part + 8 * size_t(N_KIN));   // qs0, ps, eps_slot, most, ticket, cosmo_eval
  static constexpr size_t mom_part = align256(small + 256);       // sphere-moment partial sums
  static constexpr size_t wtab = align256(mom_part + kMomentsPartBytes);   // sphere window by |n|^2, one pass
  static constexpr size_t mvar = align256(wtab + 8 * size_t(kMomentsRadiiPerPass) * NPK);
  static constexpr size_t a = align256(mvar + 8 * NM);
  static constexpr size_t b = a + 2 * R * NM;
  static constexpr size_t v0 = b + 2 * R * NM;
  static constexpr size_t v1 = v0 + 2 * R * NM;
  static constexpr size_t v2 = v1 + 2 * R * NM;
  static constexpr size_t gcache = v2 + 2 * R * NM;
  static constexpr size_t q0 = gcache + 16 * NM;
  static constexpr size_t g0 = q0 + 16 * NM;
  static constexpr size_t pm = g0 + 16 * NM;
  static constexpr size_t qc = pm + 16 * NM;                     // a chain's complex64 modes (FP32 path)
  static constexpr size_t end = qc + (R == 4 ? 8 * NM : 0);      // start of the galaxy region
};

// Per-galaxy arrays, in galaxy units (8 bytes per galaxy, rounded up to 256
// bytes): index of the first unit of each array.
template <int R> struct GalaxyUnits {
  static constexpr size_t rhat = 0;        // 3 doubles per galaxy
  static constexpr size_t mu = 3, smu = 4, cz = 5, scz = 6;
  static constexpr size_t frac = 7;        // 3 doubles
  static constexpr size_t gd = 10, gd0 = 11, qd0 = 12, pd = 13;
  static constexpr size_t like_part = 14;  // kLikeVals doubles per likelihood block
  static constexpr size_t key = 15, cellz = 16, slot = 17, iz = 18;   // ints
  static constexpr size_t rx = 19, ry = 20, rz = 21, tx = 22, ty = 23, tz = 24, gsort = 25;   // reals
  static constexpr size_t bpos = 26;       // binned index of each galaxy
  static constexpr size_t dz = 27;         // redshift distance of each galaxy
  static constexpr size_t part = 28;       // 4 complex reals per galaxy
  static constexpr size_t count = part + (R == 4 ? 4 : 8);
};

__host__ __device__ inline size_t gal_unit(int n_gal) { return align256(8 * size_t(n_gal > 0 ? n_gal : 1)); }

template <int N, int R> __host__ __device__ inline size_t hist_offset(int n_gal) {
  return FixedLayout<N, R>::end + GalaxyUnits<R>::count * gal_unit(n_gal);
}

template <int N, int R> __host__ __device__ inline size_t workspace_bytes(int n_gal, int n_hist) {
  return align256(hist_offset<N, R>(n_gal) + 8 * size_t(n_hist > 0 ? n_hist : 1));
}

// ---------------------------------------------------------------------------
// Chain scalars kept on the device so a whole run is enqueued without a
// host round trip.  Each chain has its own seed and iteration counter, so a
// chain draws the same numbers whichever other chains share its launches.
// ---------------------------------------------------------------------------
struct ChainScalars {
  double eps;          // step size of the chain (adapted during warm-up)
  double eps_it;       // step of the current iteration (jittered)
  double da_mu, da_hbar, da_log_eps_bar, da_m;
  double psi;                  // Psi at the current state
  double gs[kSmallMax];        // dPsi/d(s, u8, phi, eta) there
  double psi_saved;            // at the start of the trajectory
  double gs_saved[kSmallMax];
  double kin0, kin1;
  double target;
  uint64_t seed;
  int iter;            // iterations done by this chain
  int warmup;          // adaptation iterations
  int jitter;          // jitter the step by U(0.9, 1.1)
  int accept;          // last iteration accepted
  int post;            // last iteration was past warm-up
};
static_assert(sizeof(ChainScalars) <= FixedLayout<16, 8>::chain_bytes, "chain scalars block");
static_assert(sizeof(PlanConst) <= 256, "plan constants block");
static_assert(16 * kSmallMax + 32 <= 256, "small-coordinate block (qs0, ps, eps, most, ticket, cosmo_eval)");

// Typed view of a plan's workspace.
template <typename T, int N> struct Ws {
  using C = cplx_t<T>;
  using F = FixedLayout<N, sizeof(T)>;
  using G = GalaxyUnits<sizeof(T)>;
  char* base;
  size_t unit;
  __host__ __device__ Ws(char* b, int n_gal) : base(b), unit(gal_unit(n_gal)) {}
  template <typename X> __host__ __device__ X* at(size_t o) const { return reinterpret_cast<X*>(base + o); }
  template <typename X> __host__ __device__ X* gal(size_t u) const { return at<X>(F::end + u * unit); }
  __host__ __device__ const PlanConst& pc() const { return *at<const PlanConst>(F::consts); }
  __host__ __device__ ChainScalars* chain() const { return at<ChainScalars>(F::chain); }
  __host__ __device__ double* var_n2() const { return at<double>(F::var_n2); }
  __host__ __device__ C* tw() const { return at<C>(F::tw); }
  __host__ __device__ int* count() const { return at<int>(F::count); }
  __host__ __device__ int* off() const { return at<int>(F::off); }
  __host__ __device__ int* cursor() const { return at<int>(F::cursor); }
  __host__ __device__ double* prior_part() const { return at<double>(F::prior_part); }
  __host__ __device__ double* kin_part() const { return at<double>(F::kin_part); }
  __host__ __device__ double* qs0() const { return at<double>(F::small); }                    // kSmallMax
  __host__ __device__ double* ps() const { return at<double>(F::small + 8 * kSmallMax); }     // kSmallMax
  __host__ __device__ double* eps_slot() const { return at<double>(F::small + 16 * kSmallMax); }
  __host__ __device__ int* most() const { return at<int>(F::small + 16 * kSmallMax + 8); }   // most points in one column
  __host__ __device__ int* ticket() const { return at<int>(F::small + 16 * kSmallMax + 12); } // likelihood blocks done
  // u8 and phi where the evaluation's gradient is taken (the adjoint pass
  // reads them after the small coordinates have drifted on)
  __host__ __device__ double* cosmo_eval() const { return at<double>(F::small + 16 * kSmallMax + 16); }
  __host__ __device__ double* mvar() const { return at<double>(F::mvar); }
  __host__ __device__ C* a() const { return at<C>(F::a); }
  __host__ __device__ C* b() const { return at<C>(F::b); }
  __host__ __device__ C* v0() const { return at<C>(F::v0); }
  __host__ __device__ C* v1() const { return at<C>(F::v1); }
  __host__ __device__ C* v2() const { return at<C>(F::v2); }
  __host__ __device__ double2* gcache() const { return at<double2>(F::gcache); }
  __host__ __device__ double2* q0() const { return at<double2>(F::q0); }
  __host__ __device__ double2* g0() const { return at<double2>(F::g0); }
  __host__ __device__ double2* pm() const { return at<double2>(F::pm); }
  __host__ __device__ float2* qc() const { return at<float2>(F::qc); }
  __host__ __device__ double* rhat() const { return gal<double>(G::rhat); }
  __host__ __device__ double* mu() const { return gal<double>(G::mu); }
  __host__ __device__ double* smu() const { return gal<double>(G::smu); }
  __host__ __device__ double* cz() const { return gal<double>(G::cz); }
  __host__ __device__ double* scz() const { return gal<double>(G::scz); }
  __host__ __device__ double* frac() const { return gal<double>(G::frac); }
  __host__ __device__ double* gd() const { return gal<double>(G::gd); }
  __host__ __device__ double* gd0() const { return gal<double>(G::gd0); }
  __host__ __device__ double* qd0() const { return gal<double>(G::qd0); }
  __host__ __device__ double* pd() const { return gal<double>(G::pd); }
  __host__ __device__ double* like_part() const { return gal<double>(G::like_part); }
  __host__ __device__ int* key() const { return gal<int>(G::key); }
  __host__ __device__ int* cellz() const { return gal<int>(G::cellz); }
  __host__ __device__ int* slot() const { return gal<int>(G::slot); }
  __host__ __device__ int* bpos() const { return gal<int>(G::bpos); }
  __host__ __device__ double* dz() const { return gal<double>(G::dz); }
  __host__ __device__ int* iz() const { return gal<int>(G::iz); }
  __host__ __device__ T* rx() const { return gal<T>(G::rx); }
  __host__ __device__ T* ry() const { return gal<T>(G::ry); }
  __host__ __device__ T* rz() const { return gal<T>(G::rz); }
  __host__ __device__ T* tx() const { return gal<T>(G::tx); }
  __host__ __device__ T* ty() const { return gal<T>(G::ty); }
  __host__ __device__ T* tz() const { return gal<T>(G::tz); }
  __host__ __device__ T* gsort() const { return gal<T>(G::gsort); }
  __host__ __device__ C* part() const { return gal<C>(G::part); }
  __host__ __device__ double* hist(int n_gal) const { return at<double>(hist_offset<N, sizeof(T)>(n_gal)); }
};

// The plan of this block of a shared launch, or nullptr when it sits the
// launch out.  `mode` receives the plan's mode.
template <typename T, int N> struct Pick {
  Ws<T, N> w;
  const StateDev& st;
  int mode;
  int n_gal;
  __device__ Pick(const Launch& L)
      : w(L.base[blockIdx.z], L.n_gal[blockIdx.z]), st(L.st[blockIdx.z]), mode(L.mode[blockIdx.z]),
        n_gal(L.n_gal[blockIdx.z]) {}
};

}  // namespace hamlet
