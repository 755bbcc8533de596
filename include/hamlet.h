/*
 * hamlet.h - C ABI of the HAMLET log-posterior / gradient / HMC library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the posterior of the peculiar-velocity
 * reconstruction of Valade, Hoffman, Libeskind & Graziani, "Hamiltonian
 * Monte Carlo reconstruction from peculiar velocities" (HAMLET), and runs
 * its Hamiltonian Monte Carlo sampler, on one GPU.
 *
 * Parameters q (eq:q): the Fourier modes of the linear density contrast on
 * a periodic N^3 grid, the true distances d_i of the n catalogue points and
 * s = sigma_NL / (100 km/s).  Psi(q) = -ln Pi(q) (eq:Psi) is the sum of
 *   - the Gaussian prior of the modes (eq:prior-k),
 *   - per point: (mu_i - mu(d_i))^2 / 2 sigma_mu,i^2 (eqn:lmu, Section 2.2),
 *     r_i^2 / 2 kappa_i^2 + ln kappa_i with r_i = v_obs,i(d_i) - rhat_i . v(d_i rhat_i)
 *     (eq:vrobs, eqn:lvr, eq:kappa), and -ln N_dz(d_i) (eq:D),
 * without pure constants.  The velocity field v is the linear-theory field of
 * the modes (eq:vel-field), interpolated cloud-in-cell (trilinear, periodic)
 * at d_i rhat_i with the observer at the box centre (Section 5.1).
 *
 * Units: distances Mpc/h, velocities km/s, H0 = 100 km/s per Mpc/h.
 *
 * Mode layout ("half spectrum"): double complex, interleaved (re, im),
 * index [kx][ky][kz] row-major with kx, ky in [0, N) and kz in [0, N/2)
 * (kz fastest): N * N * N/2 entries.  Fourier convention
 *   delta(x) = N^-3 sum_k dhat_k exp(+i k.x),  k = 2 pi n / L.
 * Retained modes exclude k = 0 and every mode with a Nyquist component
 * (|n_c| = N/2); those entries must be zero and stay zero.  On the kz = 0
 * plane both members of a Hermitian pair are stored and must be conjugate
 * (dhat(-kx, -ky, 0) = conj dhat(kx, ky, 0)); every routine preserves this.
 * Mode gradients use the convention G = dPsi/dRe + i dPsi/dIm with respect
 * to the independent coordinates of each mode; momenta use the same layout.
 *
 * Streams: every call is asynchronous on the plan's HIP stream (the stream
 * given at creation); only hamlet_plan_create and hamlet_plan_destroy
 * synchronise.  Calls on plans that share a stream run in call order.
 * Plans of one call with the same N and precision are batched: their
 * kernels run as shared launches on the stream of the first of them, ordered
 * after and before the other plans' streams with events.  When several such
 * groups of one call would use the same stream, every group after the first
 * runs on a side stream of it (owned by the library, created on first use
 * and kept until the process ends), ordered the same way, so independent
 * groups may run concurrently.  A plan may appear once per call.
 *
 * Errors: every entry point returns a hamlet_status; the message of the last
 * non-OK status of the calling thread is hamlet_last_error().  A parameter
 * state outside the domain of the posterior (a distance <= 0, beyond
 * c / (3 Omega0 H0), or outside the distance histogram) is not an error:
 * Psi is +inf there and the sampler rejects such a trajectory.
 */
#ifndef HAMLET_H
#define HAMLET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HAMLET_OK = 0,
  HAMLET_EINVAL = -1,       /* invalid argument (message says which) */
  HAMLET_ENOMEM = -2,       /* device allocation failed */
  HAMLET_EDEVICE = -3,      /* a HIP call failed */
  HAMLET_EUNSUPPORTED = -4  /* grid size or option not built */
} hamlet_status;

typedef enum {
  HAMLET_FP64 = 0,          /* every transform, gather and scatter in FP64 */
  HAMLET_FP32_FP64E = 1     /* transforms, gather, scatter in FP32; Hamiltonian,
                               likelihood, dH, Metropolis test, momentum draws in
                               FP64; a chain's mode state stored in complex64 */
} hamlet_precision;

/* Problem statement (Section 2; the grid and box of Section 5.1).  All
 * pointers are host memory, read during hamlet_plan_create only. */
typedef struct {
  int32_t n_grid;           /* N: 16, 32, 64, 128, 256, 512 or 1024 */
  int32_t precision;        /* hamlet_precision */
  double box;               /* L, Mpc/h */
  double omega_m;           /* Omega0 of zbar(d) (Section 2.2) */
  double h;                 /* little h in mu(d) = 5 log10(d (1 + zbar) / h) + 25 */
  double f_growth;          /* f(Omega0) of eq:vel-field */
  double sigma_v;           /* km/s; mass of a distance is sigma_v^2 / H0^2 (eq:M_ab) */
  const double* pk_n2;      /* P(|k|) in (Mpc/h)^3 at |k| = (2 pi / L) sqrt(j),
                               j = 0 .. 3 (N/2)^2; mode variance is N^6 P / L^3 */
  int32_t n_pk;             /* must be 3 (N/2)^2 + 1 */
  double hist_width;        /* bin width of the distance prior (eq:D), Mpc/h; <= 0: 5 */
  int32_t sample_distances; /* 0: distances frozen (no momentum) */
  int32_t sample_sigma_nl;  /* 0: s frozen */
  int32_t sample_cosmology; /* 1: h, sigma_8 and f sampled with the field (Section 6, item 3), see below */
} hamlet_plan_desc;

/* Cosmological parameters in q.  With sample_cosmology = 1 the state has
 * three more coordinates after s: u8 = sigma_8 / sigma_8,fid, which scales
 * P(k) (pk_n2) by u8^2, phi = f / f_fid, which scales f_growth, and
 * eta = h / h_fid, which scales h.  All three have flat priors on (0, inf)
 * (Psi = +inf elsewhere); the prior of the modes is the normalised Gaussian
 * of variance u8^2 sigma_k^2, so Psi gains E (1/u8^2 - 1) + D ln u8 (E the
 * prior energy at u8 = 1, D = (N-1)^3 - 1 real mode coordinates), and
 * dPsi/dphi = sum_i (dPsi/du_i) u_i / phi.  With distances in Mpc/h, h
 * enters only the distance modulus, mu(d) = 5 log10(d_L / (eta h)) + 25, so
 * dPsi/deta = sum_i (dmu_i / sigma_mu,i^2) 5 / (eta ln 10).  Inverse masses:
 * 1 / (2 D) for u8, 1 / max(n, 1) for phi, 1 / sum_i (5 / ln 10)^2 /
 * sigma_mu,i^2 for eta (1 without points).  Every "snl" buffer of such a plan
 * (q_snl, g_snl, p_snl, the s of hamlet_hmc_run and hamlet_nuts_run) then
 * holds 4 doubles (s, u8, phi, eta) and the flat vector 2m + n + 4 entries;
 * the field, density and statistics entry points use the fiducial f.  A
 * served job with sampled cosmology starts at u8 = phi = eta = 1
 * (hamlet_server_take returns s only). */

/* Catalogue (Section 2, Section 5.1): n points, host arrays of length n.
 * rhat is 3 n doubles (x, y, z per point), the unit vector
 * (cos SGB cos SGL, cos SGB sin SGL, sin SGB).  cz = c z (km/s). */
typedef struct {
  int64_t n;
  const double* rhat;
  const double* mu;
  const double* sigma_mu;
  const double* cz;
  const double* sigma_cz;
} hamlet_catalog;

typedef struct hamlet_plan hamlet_plan;

/* Creates a plan on the current HIP device: uploads tables and catalogue and
 * allocates the workspace (hamlet_plan_footprint_bytes).  The distance prior
 * (eq:D) is built here from the catalogue: redshift distances by the
 * integral of eq:e:dz (composite Simpson, 2000 intervals), a histogram of
 * bin width hist_width over [0, max d_z + 15 Mpc/h) with one pseudo-count per
 * bin, normalised to a density.  `stream` is a hipStream_t (NULL: default
 * stream).  On error *out is NULL. */
hamlet_status hamlet_plan_create(const hamlet_plan_desc* desc, const hamlet_catalog* cat, void* stream,
                                 hamlet_plan** out);
hamlet_status hamlet_plan_destroy(hamlet_plan* plan);

/* Device bytes a plan of this description with n_gal points would own. */
hamlet_status hamlet_plan_footprint_bytes(const hamlet_plan_desc* desc, int64_t n_gal, size_t* bytes);

/* Psi(q) and its gradient for n_plans plans (batch of independent chains).
 * All array arguments are device pointers owned by the caller, one per plan:
 *   q_modes[j], g_modes[j]: N*N*N/2 double complex (layout above)
 *   q_dist[j],  g_dist[j]:  n doubles
 *   q_snl[j], g_snl[j]:     1 double each (s and dPsi/ds)
 *   psi[j]:                 1 double (Psi, +inf outside the domain)
 * Inputs and outputs must not overlap. */
hamlet_status hamlet_logpost_grad(hamlet_plan* const* plans, int32_t n_plans,
                                  const void* const* q_modes, const double* const* q_dist,
                                  const double* const* q_snl,
                                  void* const* g_modes, double* const* g_dist, double* const* g_snl,
                                  double* const* psi);

/* As hamlet_logpost_grad, but the mode gradient is taken with respect to the
 * stored entries one by one (the convention of automatic differentiation,
 * where both members of a Hermitian pair on the kz = 0 plane are separate
 * variables): equal to the hamlet_logpost_grad gradient except on the kz = 0
 * plane, where it is half of it.  Ψ and the other outputs are the same. */
hamlet_status hamlet_logpost_grad_entries(hamlet_plan* const* plans, int32_t n_plans,
                                          const void* const* q_modes, const double* const* q_dist,
                                          const double* const* q_snl,
                                          void* const* g_modes, double* const* g_dist, double* const* g_snl,
                                          double* const* psi);

/* n_steps[j] kick-drift-kick leapfrog steps of size eps[j] (host arrays) of
 * Hamilton's equations (eq:hamilton) with the mass matrix of eq:M_ab, from
 * (q, p) in place (device pointers as above; p_* have the layout of q_*).
 * psi[j] receives Psi at the end point.  Frozen coordinates do not move. */
hamlet_status hamlet_leapfrog(hamlet_plan* const* plans, int32_t n_plans, const double* eps,
                              const int32_t* n_steps,
                              void* const* q_modes, double* const* q_dist, double* const* q_snl,
                              void* const* p_modes, double* const* p_dist, double* const* p_snl,
                              double* const* psi);

typedef struct {
  int32_t n_iter;           /* HMC iterations (trajectories) */
  int32_t n_leapfrog;       /* leapfrog steps per trajectory */
  int32_t warmup;           /* the chain's first `warmup` iterations adapt eps by dual averaging
                               (the adapted step is fixed after iteration warmup - 1) */
  int32_t jitter_eps;       /* 1: step of iteration t is eps (0.9 + 0.2 u_t) */
  double eps0;              /* initial step */
  double target_accept;     /* dual-averaging target (Section 3.3: 0.65) */
  uint64_t seed;            /* Philox4x32-10 key of plan j's chain: seed + j (or seeds[j]) */
  int32_t resume;           /* 1: continue each plan's chain (step, adaptation, iteration count,
                               cached gradient) from its last hamlet_hmc_run; q_* must still
                               hold that chain's state.  A chain with no such run (or after
                               hamlet_leapfrog on its plan) starts fresh. */
  const uint64_t* seeds;    /* host, n_plans keys, or NULL */
} hamlet_hmc_opts;

/* Runs the chain of Section 3.2 for each plan: fresh momenta p ~ N(0, M)
 * per trajectory (Philox4x32-10, counter (index, 0, iteration, purpose),
 * iteration = the chain's own count), n_leapfrog steps, Metropolis-Hastings
 * test ln u < -dH (a rejected trajectory repeats the state), dual averaging
 * of eps during the chain's first `warmup` iterations.
 * q_* (device, in/out): start state in, last state out.  A plan of
 *   precision HAMLET_FP32_FP64E runs its chain on a complex64 copy of the
 *   modes in its workspace (its momenta, cached gradient and kept start
 *   point in complex64 too; every update computed in FP64 and rounded before
 *   use, so H and dH are those of the stored state): q_modes[j] is rounded to
 *   complex64 on entry, and on return its retained modes hold the chain's
 *   last state (widened exactly); its other entries are left as they were.
 * mode_sum[j] (device, may be NULL): sum over post-warm-up iterations of the
 *   chain's mode state (eq:int_mc numerator); accumulated onto its contents
 *   in FP64.
 * dh[j], accepted[j] (device, may be NULL): indexed by the chain's iteration
 *   count, so n_iter entries for a fresh chain (more when resumed).
 * eps_out (host, may be NULL): n_plans, the step after warm-up (synchronises).
 * Batches: the plans of one call with the same N and precision share every
 * kernel launch (up to 16 plans per launch); each chain's numbers do not
 * depend on which other chains share its launches. */
hamlet_status hamlet_hmc_run(hamlet_plan* const* plans, int32_t n_plans, const hamlet_hmc_opts* opts,
                             void* const* q_modes, double* const* q_dist, double* const* q_snl,
                             void* const* mode_sum, double* const* dh, int32_t* const* accepted,
                             double* eps_out);

/* ---- The No-U-Turn sampler ----
 *
 * Section 3.3 samples with the No-U-Turn sampler of Hoffman & Gelman (JMLR
 * 15, 2014), whose step is tuned by their dual averaging.  Each iteration
 * draws momenta r0 ~ N(0, M) (eq:M_ab; the stream and index of
 * hamlet_hmc_run's momenta), a slice variable ln u = ln U - H0 (U in (0, 1],
 * purpose of the Metropolis uniform), then doubles the trajectory in random
 * directions, 2^j leapfrog steps at doubling j, until a subtree or the whole
 * trajectory turns back ((theta+ - theta-) . r < 0 at either end, over the
 * independent real coordinates), a leaf leaves the slice by more than
 * Delta_max = 1000, or max_depth doublings are done.  Within a doubling
 * the two halves of every subtree merge with probability n''/(n' + n'') for
 * the second half's sample (n = leaves in the slice); after a doubling the
 * chain moves to its sample with probability min(1, n'/n).  Each decision
 * takes one uniform of the chain's Philox4x32-10 stream: direction of
 * doubling j (purpose 5, index j), merge of the node of height h and
 * position k in doubling j (purpose 6, index ((16 j + h) << 32) | k), move
 * after doubling j (purpose 7, index j); "with probability a/b" is U b <= a,
 * direction -1 iff U <= 1/2.  During the first `warmup` iterations the step
 * adapts to the mean acceptance statistic alpha / n_alpha of the leaves; its
 * averaged value is kept after them. */
typedef struct {
  int32_t n_iter;           /* NUTS iterations */
  int32_t warmup;           /* iterations of dual averaging (the step is fixed after them) */
  int32_t max_depth;        /* most doublings per iteration, 1 .. 12 (Hoffman & Gelman use 10) */
  int32_t reserved;         /* 0 */
  double eps0;              /* initial step */
  double target_accept;     /* dual-averaging target of alpha / n_alpha (Section 3.3: 0.65) */
  uint64_t seed;            /* Philox4x32-10 key of plan j's chain: seed + j (or seeds[j]) */
  const uint64_t* seeds;    /* host, n_plans keys, or NULL */
} hamlet_nuts_opts;

/* Runs n_iter NUTS iterations of each plan's chain from its state q_*
 * (device, in: start, out: last state), on the plans' streams.  mode_sum[j]
 * (device, may be NULL) accumulates the post-warm-up states (eq:int_mc
 * numerator).  Host outputs per iteration (each may be NULL, n_iter entries):
 * depth[j] doublings done, n_leapfrog[j] leapfrog steps (gradient
 * evaluations), leaf[j] 2 ints per iteration, (doubling, position in it) of
 * the leaf the chain moved to, (-1, 0) if it stayed, accept_stat[j] the
 * iteration's alpha / n_alpha.  eps_out (host, may be NULL): the step after
 * warm-up.  Plans of one grid size and precision advance their trees
 * together, one leapfrog step per chain in shared launches; each chain's
 * numbers do not depend on which others share them.  The host builds the
 * trees and reads two scalars per chain and step back, so the call returns
 * when the chains are done.  Device memory: the first call on a plan
 * allocates, and keeps until hamlet_plan_destroy, 3 max_depth + 12 state-
 * sized buffers (modes, distances, s: 134 MB each at 256^3; a call with a
 * larger max_depth reallocates them).  Errors: HAMLET_EINVAL for bad
 * arguments, HAMLET_ENOMEM when the buffers do not fit. */
hamlet_status hamlet_nuts_run(hamlet_plan* const* plans, int32_t n_plans, const hamlet_nuts_opts* opts,
                              void* const* q_modes, double* const* q_dist, double* const* q_snl,
                              void* const* mode_sum, int32_t* const* depth, int32_t* const* n_leapfrog,
                              int32_t* const* leaf, double* const* accept_stat, double* eps_out);

/* ---- The paper's flat parameter vector ----
 *
 * Section 3.1 orders the parameters of the posterior as one real vector:
 * the real parts of the independent Fourier modes, then their imaginary
 * parts, the n distances and sigma_NL (here s = sigma_NL / 100 km/s, the
 * sampled coordinate).  The independent modes are the retained entries of
 * the stored layout (no k = 0, no Nyquist component) with kz > 0, and on
 * the kz = 0 plane the canonical member of each Hermitian pair (ny > 0, or
 * ny = 0 and nx > 0), taken in row-major (kx, ky, kz) order: m = ((N-1)^3 - 1)
 * / 2 of them, so the vector has 2m + n + 1 entries.  Applied to a gradient
 * (G = dPsi/dRe + i dPsi/dIm per independent coordinate, dPsi/dd, dPsi/ds)
 * packing gives dPsi/dq in the same order. */

/* Length 2m + n + 1 (+3 with sampled cosmology) of the plan's flat vector
 * (host only). */
hamlet_status hamlet_flat_size(const hamlet_plan* plan, int64_t* n_flat);

/* flat (device, n_flat doubles) <- modes (device, N x N x N/2 complex128),
 * dist (device, n doubles; may be NULL when n = 0), snl (device, 1 double).
 * Reads only the independent entries.  Asynchronous on the plan's stream. */
hamlet_status hamlet_pack_flat(hamlet_plan* plan, const void* modes, const double* dist, const double* snl,
                               double* flat);

/* modes, dist, snl (device) <- flat (device).  Writes every stored entry:
 * the independent ones from flat, each mirror entry of the kz = 0 plane as
 * the conjugate of its partner, excluded entries 0.  Asynchronous on the
 * plan's stream. */
hamlet_status hamlet_unpack_flat(hamlet_plan* plan, const double* flat, void* modes, double* dist, double* snl);

/* ---- The velocity field of a state ----
 *
 * eq:vel-field: v_c(x_j) = N^-3 sum_k m_c(k) dhat_k exp(i k.x_j), c = x, y, z,
 * on every node x_j = j L / N of the grid (km/s), from the modes of a state
 * (e.g. a sample, or the chain's mean state) for maps and statistics of the
 * reconstructed field (Section 5).
 *
 * modes (device): N x N x N/2 complex128.
 * out (device): 3 N^3 reals of the plan's precision (float for
 *   HAMLET_FP32_FP64E, double for HAMLET_FP64), out[((c N + x) N + y) N + z].
 * Uses the plan's workspace (the inverse passes of an evaluation); calls on
 * one plan are ordered by its stream.  Errors: HAMLET_EINVAL for NULL
 * buffers.  Asynchronous on the plan's stream. */
hamlet_status hamlet_velocity_field(hamlet_plan* plan, const void* modes, void* out);

/* The density contrast delta(x_j) = N^-3 sum_k dhat_k exp(i k.x_j) of a state
 * on every node (the modes' Fourier convention, eq:prior-k), e.g. for the
 * maps of the mean and the scatter of delta (Section 5).  modes as above;
 * out (device): N^3 reals of the plan's precision, out[(x N + y) N + z].
 * Uses the plan's workspace; errors and ordering as above. */
hamlet_status hamlet_density_field(hamlet_plan* plan, const void* modes, void* out);

/* Adds one state's density contrast delta and radial velocity v_r (km/s) on
 * every node, and their squares, to running sums, for the maps of the chain's
 * mean field and of its scatter Sigma(r) along the chain (Section 5): with
 * n states summed, mean = S1 / n and variance = S2 / n - mean^2.  v_r is the
 * velocity field's component along r = x - o from the observer o =
 * (L/2)(1, 1, 1), which is node N/2 of each axis; v_r = 0 on that node.
 * modes as above; acc (device, caller-owned): 4 N^3 doubles, the grids
 * [sum delta, sum delta^2, sum v_r, sum v_r^2], each [(x N + y) N + z];
 * zero it before the first state.  The values are added in the plan's
 * precision and summed in double.  Uses the plan's workspace; errors and
 * ordering as above. */
hamlet_status hamlet_field_stats_accumulate(hamlet_plan* plan, const void* modes, double* acc);

/* Statistics of fields in spherical shells about the observer (Section 5,
 * correlation coefficients: the mean and scatter of delta or v_r in shells,
 * and the correlation of the reconstruction with the target voxel by voxel).
 * Shell s holds the nodes j with |r_j| in [s width, (s + 1) width), r_j =
 * (j - N/2) L / N per axis (the observer is node N/2 of each axis).
 * a, b (device): N^3 doubles each, [(x N + y) N + z]; b may be NULL (then
 * b counts as zero).  out (device): n_shells x 6 doubles per shell: node
 * count, mean of a, scatter of a (population standard deviation), mean of
 * b, scatter of b, Pearson correlation coefficient of a and b over the
 * shell's nodes; NaN where undefined (an empty shell, a constant field).
 * The sums run in double in a fixed order: reruns are bit-identical.
 * Allocates its partial sums on the plan's stream (stream-ordered).
 * Errors: HAMLET_EINVAL for NULL buffers, n_shells outside [0, 4096] or a
 * width that is not positive and finite; HAMLET_ENOMEM.  Asynchronous on
 * the plan's stream. */
hamlet_status hamlet_shell_stats(hamlet_plan* plan, const double* a, const double* b, double width,
                                 int32_t n_shells, double* out);

/* As hamlet_shell_stats, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the partial sums live in a static device array of 4 MiB
 * that each device the library runs on holds until the process ends; the
 * call allocates and frees nothing.  Its partials need n_shells x N x 24
 * bytes (one per shell and x plane: 276 KB at 256^3 with 45 shells); a call
 * that would need more than 4 MiB (more than 682 shells at 256^3, 170 at
 * 1024^3) fails with HAMLET_EINVAL before anything is enqueued.  Every call on a device shares
 * that device's array: calls that overlap on one device (two streams, or
 * two host threads) race and must be ordered by the caller.  Results equal
 * hamlet_shell_stats bit for bit.  The first call on a device looks up the
 * array's address there (no allocation).  Asynchronous on the plan's stream. */
hamlet_status hamlet_shell_stats_static(hamlet_plan* plan, const double* a, const double* b, double width,
                                        int32_t n_shells, double* out);

/* ---- Sphere moments of the velocity field ----
 *
 * Section 5 (monopole and dipole) follows the reconstruction by the moments
 * of the linear velocity field in spheres of radius R about the observer
 * o = (L/2)(1, 1, 1): the monopole M(R), the mean of -div v / H0 over the
 * ball (f times the mean density contrast within R), and the dipole D(R),
 * the mean of v over the ball (the bulk velocity of the sphere, km/s).  The
 * field between grid nodes is the band-limited field of the modes (on the
 * nodes it is the velocity field of the evaluation); each mode contributes
 * through the top-hat window W(|k| R) = 3 (sin y - y cos y) / y^3, y = |k| R.
 *
 * modes (device): N x N x N/2 complex128, a state of the chain (e.g. a
 *   sample, or the mode sum of hamlet_hmc_run divided by its count).
 * radii (host): n_radii radii in Mpc/h, each positive and finite;
 *   0 <= n_radii <= 16.
 * out (device): 4 n_radii doubles (may be NULL when n_radii = 0);
 *   out[4 j] = M(R_j), out[4 j + 1 + c] the component c (x, y, z) of D(R_j).
 * Computed in FP64 for both precisions; the sums run in a fixed order, so a
 * rerun gives the same bits.  Uses the plan's scratch for its partial sums:
 * calls on one plan are ordered by its stream like every other call.
 * Errors: HAMLET_EINVAL for NULL buffers, a count outside [0, 16] or a radius
 * that is not positive and finite (nothing is enqueued).  Asynchronous on the
 * plan's stream. */
hamlet_status hamlet_sphere_moments(hamlet_plan* plan, const void* modes, const double* radii, int32_t n_radii,
                                    double* out);

/* ---- Serving: continuous batching of independent reconstruction jobs ----
 *
 * A server runs many chains (jobs) on one device.  Jobs are queued with
 * their problem; on each tick the server admits queued jobs in arrival
 * order while the next one's device footprint (plan workspace and chain
 * state) fits its budget, and advances every running job by one leapfrog
 * step: jobs of one grid size and precision share every kernel launch, a
 * newly admitted job joins at its first tick, each job runs its own
 * Metropolis-Hastings test at the end of each of its trajectories (Section
 * 3.2), and a job leaves after its last iteration.  Each job's numbers do not
 * depend on which other jobs run beside it.  Ticks are enqueued on the
 * server's stream at most `ticks_ahead` ahead of the device. */
typedef struct hamlet_server hamlet_server;

typedef struct {
  size_t hbm_budget;        /* device bytes the running jobs may hold */
  int32_t max_running;      /* at most this many running jobs (<= 0: no limit) */
  int32_t ticks_ahead;      /* <= 0: 2 */
} hamlet_server_desc;

typedef struct {
  int32_t queued, running, finished;   /* finished: done on the device, not yet taken */
  int64_t ticks;
  size_t bytes_in_use;
} hamlet_server_stats;

/* `stream`: a hipStream_t for all of the server's work (NULL: default stream). */
hamlet_status hamlet_server_create(const hamlet_server_desc* desc, void* stream, hamlet_server** out);
/* Waits for the device and releases every job, taken or not. */
hamlet_status hamlet_server_destroy(hamlet_server* server);

/* Queues a job.  desc, cat: as for hamlet_plan_create (copied).  opts: the
 * chain (n_iter iterations of n_leapfrog steps, warmup, step; opts->seed is
 * the job's Philox key; resume and seeds are ignored).  Start state (host,
 * copied): q_modes N*N*N/2 double complex or NULL (all modes zero), q_dist n
 * doubles or NULL (the redshift distances d_z of eq:e:dz), q_snl.  A job that
 * could never fit the budget is rejected (HAMLET_ENOMEM). */
hamlet_status hamlet_server_submit(hamlet_server* server, const hamlet_plan_desc* desc, const hamlet_catalog* cat,
                                   const hamlet_hmc_opts* opts, const double* q_modes, const double* q_dist,
                                   double q_snl, int64_t* job_id);

/* One tick (see above).  stats may be NULL. */
hamlet_status hamlet_server_tick(hamlet_server* server, hamlet_server_stats* stats);

/* state: 0 queued, 1 running, 2 finished (all its work done on the device),
 * -1 failed at admission (the tick that tried reported why). */
hamlet_status hamlet_server_job_state(hamlet_server* server, int64_t job_id, int32_t* state);

/* Copies a finished job's results to host memory and releases it; each
 * pointer may be NULL.  mode_sum: N*N*N/2 double complex, the sum of the
 * post-warm-up states (eq:int_mc numerator); q_modes, q_dist, q_snl: the last
 * state (an HAMLET_FP32_FP64E job's chain runs on complex64 modes, as in
 * hamlet_hmc_run: its retained modes come back widened from them, the other
 * entries as submitted); dh, accepted: n_iter; eps: the step after warm-up. */
hamlet_status hamlet_server_take(hamlet_server* server, int64_t job_id, double* mode_sum, double* q_modes,
                                 double* q_dist, double* q_snl, double* dh, int32_t* accepted, double* eps);

/* Measurement aid.  Kernel kinds that can be timed with HIP events: */
typedef enum {
  HAMLET_K_BIN = 0,         /* binning of the points into CIC columns (its kernels timed as one) */
  HAMLET_K_INV_X = 1,       /* inverse pass 1: multiplier, prior energy, FFT along x */
  HAMLET_K_INV_Y = 2,       /* inverse pass 2: FFT along y */
  HAMLET_K_INV_Z = 3,       /* inverse pass 3: complex-to-real FFT along z + CIC gather */
  HAMLET_K_LIKE = 4,        /* per-point likelihood and its gradient, and the final sums */
  HAMLET_K_FWD_Z = 5,       /* forward pass 1: CIC scatter + real-to-complex FFT along z */
  HAMLET_K_FWD_Y = 6,       /* forward pass 2: FFT along y */
  HAMLET_K_FWD_X = 7,       /* forward pass 3: FFT along x, adjoint multiply, prior gradient; inside a
                               leapfrog trajectory also the mode kick and drift and inverse pass 1 of
                               the next evaluation (then HAMLET_K_INV_X is not launched); the first
                               pass of a chain's trajectory also draws the mode momenta, sums their
                               kinetic energy and keeps the start point, the last sums the kinetic
                               energy after its half kick */
  HAMLET_K_COUNT = 8
} hamlet_kernel;

/* While armed, every launch of that kernel kind on the plan's stream is
 * bracketed by a pair of HIP events (host objects created on demand).
 * hamlet_profile_stop synchronises the plan's stream, returns the summed
 * event-measured duration (ms) and the number of launches since
 * hamlet_profile_start, and disarms. */
hamlet_status hamlet_profile_start(hamlet_plan* plan, int32_t kernel);
hamlet_status hamlet_profile_stop(hamlet_plan* plan, double* total_ms, int64_t* launches);

/* The kernel schedule this library was built with for a grid size and
 * precision: what the autotuner chose where it timed alternatives on the
 * MI355X (tuned_schedules.json beside the library), else the hand-picked
 * defaults.  Not part of the method; it describes how the passes of the
 * evaluation are launched, so that a measurement can name it. */
typedef struct {
  int32_t threads_xy;        /* threads per block: the y passes (and a plain gradient's inverse x pass) */
  int32_t threads_x;         /* the fused x pass */
  int32_t threads_gather;    /* the inverse z pass with the CIC gather */
  int32_t threads_scatter;   /* the forward z pass with the CIC scatter */
  int32_t tile_width;        /* kz columns per tile of the x and y passes */
  int32_t pencils_scatter;   /* z pencils per tile of the scatter */
  int32_t pencils_gather;    /* z pencils per tile of the gather */
  int32_t radix_plan;        /* index of the radix plan of the length-n transforms */
  int32_t radix[3];          /* its radices, stage by stage (0 past the last) */
} hamlet_schedule;

/* Fills *out for grid size n_grid and precision (hamlet_precision).
 * HAMLET_EINVAL: NULL out or unknown precision; HAMLET_EUNSUPPORTED: a
 * grid size this library does not hold.  Needs no GPU. */
hamlet_status hamlet_schedule_get(int32_t precision, int32_t n_grid, hamlet_schedule* out);

/* Message of the last non-OK status on this thread ("" if none). */
const char* hamlet_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HAMLET_H */
