/*
 * ksc.h -- C ABI of the MI355X library that evaluates the cost J^2 of a
 * discretized Kuramoto-Sivashinsky connecting curve, its adjoint gradient, and
 * takes adjoint-descent steps that deform the curve toward a connecting orbit
 * (O. Ashtari & T. M. Schneider, "Jacobian-Free Variational Method for
 * Constructing Connecting Orbits in Nonlinear Dynamical Systems",
 * arXiv:2301.11704).
 *
 * Discrete problem (one curve; every call works on a batch of curves):
 *   state        u_hat[j][k], j = 0..n_s-1 rows along the curve, k = 0..K the
 *                kept Fourier modes of the periodic field u(x) on [0, L),
 *                K = (n_x - 1) / 3 (2/3-rule dealiasing).  Row 0 is the endpoint
 *                at s = -inf, row n_s-1 the endpoint at s = +inf (the curve's
 *                asymptotic conditions, Sec. II, eq. connecting_orbit_def).
 *                Mode 0 is real; its imaginary part is ignored on input and
 *                written as 0.
 *   layout       curve-major, row-major, interleaved (re, im) scalars of the
 *                problem's dtype: curve c starts at ksc_state_offset(p, c)
 *                scalars, row j of it 2*(K+1)*j scalars later.
 *   s-grid       sigma_j = j / (n_s - 1); rational map s = s0 + S cot(theta),
 *                theta = pi (1 - sigma) (Sec. IV, eq. Rational_domain), or the
 *                finite map s = T sigma.  d/ds = g_j (.)_{j+1} - (.)_{j-1} over
 *                2 dsigma with g = d sigma / d s.
 *   residual     r = -u_s - u u_x - u_xx - u_xxxx (Sec. V.A, eq. KSE_residual)
 *                on interior rows, r = 0 on the two end rows (Sec. V.C.1).
 *   cost         J2 = int int r^2 dx ds (Sec. II, eq. cost_function_general):
 *                trapezoid in sigma with weights dsigma / g_j, Parseval in x.
 *   adjoint      L^dagger(u; r) = r_s + u r_x - r_xx - r_xxxx (Sec. V.A and
 *                Appendix A); this is the exact adjoint of the discrete
 *                directional derivative, so the Euclidean gradient of J2 is
 *                dJ2/d(Re,Im) u_hat[j][k] = 2 w_j L c_k L^dagger[j][k]
 *                (w_j = dsigma / g_j, c_0 = 1, c_k = 2 otherwise), zero on the
 *                end rows and for Im of mode 0.
 *   step         semi-implicit forward Euler of du/dtau = -L^dagger(u; r)
 *                (eq. KSE_G, Sec. V.C.3): the stiff Fourier-diagonal part is
 *                implicit, u_hat <- u_hat - dtau L^dagger / (1 + dtau A_k^2),
 *                A_k = q_k^2 - q_k^4, q_k = 2 pi k / L.
 *   J_arc        int |r| |u_s| ds / int |u_s| ds (eq. J_arc).
 *
 * Spectral d/ds (KSC_DS_SPECTRAL, ksc_create_opts; rational map only): d/ds is
 * the paper's rational Chebyshev differentiation matrix D_t (Sec. IV, eq.
 * rational_diff_matrix) on the n_s points of eq. t_grid, applied along s as a
 * dense matrix product, instead of the central difference.  The gradient is
 * the exact gradient of the discrete J2: the s-part of L^dagger r is
 * -(1/w_j) sum_i D_t[i][j] w_i r_i, the adjoint of -D_t in the weighted inner
 * product (it agrees with the paper's r_s = D_t r up to quadrature error), and
 * J_arc weights |D_t u|_j by w_j.
 *
 * Inversion-symmetric subspace (state space KSC_SPACE_ODD, ksc_create2): the
 * fields with u(-x) = -u(x), invariant under the descent because the inversion
 * operator commutes with the residual (symmetry-preservation subsection, eq.
 * reflection).  There u_hat_k = i b_k with real b_k, k = 1..K, and a state row
 * is the K reals b_1..b_K (layout: curve-major, row-major, K scalars per row).
 * Every call computes the same quantities as in the full space for the state
 * u_hat_0 = 0, u_hat_k = i b_k: J2 and J_arc are equal, the gradient is
 * dJ2/db_k (the imaginary part of the full gradient), and a step maps b to the
 * imaginary parts of the full step.
 *
 * Conventions for every call:
 *   - All data pointers are DEVICE pointers owned by the caller, except
 *     ksc_query_flags' output and the descriptor array of ksc_create, which
 *     are host pointers.  The library owns only the workspace it allocates in
 *     ksc_create and frees in ksc_destroy.
 *   - Work is enqueued asynchronously on the problem's HIP stream; nothing
 *     blocks the host except ksc_create, ksc_destroy, ksc_tune and
 *     ksc_query_flags.
 *   - Every call returns a ksc_status; on failure nothing was enqueued and
 *     ksc_last_error() returns a message (thread-local).  Argument, shape and
 *     support errors are detected on the host before any launch.
 *   - Supported: n_x in {8, 16, 32, 64, 128, 256}, n_s >= 3, L > 0,
 *     scale > 0; in KSC_SPACE_ODD with KSC_F64, n_x <= 128.  dtype KSC_F32
 *     computes in FP32 and accumulates J2 in FP64; KSC_F64 computes in FP64.
 *   - Kernels are deterministic: the same inputs give bitwise-equal outputs.
 */
#ifndef KSC_H
#define KSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KSC_OK = 0,
  KSC_ERR_ARG = -1,         /* null pointer, bad enum or out-of-range value */
  KSC_ERR_SHAPE = -2,       /* n_s < 3, curve index out of range, ... */
  KSC_ERR_UNSUPPORTED = -3, /* n_x not a supported power of two */
  KSC_ERR_HIP = -4,         /* a HIP runtime call failed */
  KSC_ERR_NONFINITE = -5,   /* reported through ksc_query_flags */
  KSC_ERR_DIVERGED = -6,    /* reported through ksc_query_flags */
  KSC_ERR_STATE = -7        /* call not valid in the problem's current state */
} ksc_status;

typedef enum { KSC_F32 = 0, KSC_F64 = 1 } ksc_dtype;

typedef enum {
  KSC_SPACE_FULL = 0, /* rows of K+1 complex coefficients u_hat_0..u_hat_K */
  KSC_SPACE_ODD = 1   /* inversion-symmetric subspace: rows of K reals b_1..b_K */
} ksc_space;

typedef enum {
  KSC_DS_STENCIL = 0, /* g_j (q_{j+1} - q_{j-1}) / (2 dsigma) */
  KSC_DS_SPECTRAL = 1 /* the paper's dense D_t along s (rational map) */
} ksc_ds;

/* Creation options (ksc_create_opts). */
typedef struct {
  int32_t dtype;    /* ksc_dtype */
  int32_t space;    /* ksc_space */
  int32_t ds;       /* ksc_ds */
  int32_t reserved; /* must be 0 */
} ksc_options;

typedef enum {
  KSC_MAP_RATIONAL = 0, /* s = s0 + scale * cot(pi (1 - sigma)); scale is the paper's S */
  KSC_MAP_FINITE = 1    /* s = scale * sigma; scale is the length T */
} ksc_map;

/* Descent scheme of ksc_step and ksc_descend (ksc_set_scheme). */
typedef enum {
  KSC_SCHEME_PAPER = 0,     /* the paper's semi-implicit step (Sec. V.C.3) */
  KSC_SCHEME_IMPLICIT_S = 1 /* the whole linear part implicit, including d/ds */
} ksc_scheme;

/* Per-curve flag bits reported by ksc_query_flags. */
#define KSC_FLAG_NONFINITE 1u  /* the last J2 of the curve was NaN or Inf */
#define KSC_FLAG_INCREASED 2u  /* J2 rose between two consecutive descent steps */

/* Launch policy (ksc_set_launch). */
#define KSC_LAUNCH_AUTO 0       /* one launch per call; tuned or default tile shape */
#define KSC_LAUNCH_PLAIN 1      /* one launch per curve per call (reference policy) */
#define KSC_LAUNCH_PERSISTENT 2 /* one persistent launch walking a static tile list */

typedef struct {
  int32_t n_s;   /* rows along the curve, including the two endpoint rows */
  int32_t n_x;   /* grid points in x (power of two, 8..256) */
  double L;      /* domain length (Sec. V.A, eq. KSE) */
  int32_t map;   /* ksc_map */
  double scale;  /* S (rational map) or T (finite map) */
  double s0;     /* centre of the rational map; ignored for the finite map */
} ksc_curve_desc;

typedef struct ksc_problem ksc_problem; /* opaque */

/* Create a problem for n_curves curves (descs: host array of n_curves).
 * hip_stream: the hipStream_t every call is enqueued on (may be NULL for the
 * default stream).  Allocates the workspace: metric and symbol tables, tile
 * list, per-tile partials, per-curve flags.  Out: *out, freed by ksc_destroy. */
ksc_status ksc_create(const ksc_curve_desc* descs, int32_t n_curves, int32_t dtype,
                      void* hip_stream, ksc_problem** out);
/* The same with an explicit state space (ksc_space); ksc_create is
 * ksc_create2 with KSC_SPACE_FULL.  KSC_ERR_ARG for an unknown space,
 * KSC_ERR_UNSUPPORTED for KSC_SPACE_ODD with KSC_F64 and n_x = 256. */
ksc_status ksc_create2(const ksc_curve_desc* descs, int32_t n_curves, int32_t dtype,
                       int32_t space, void* hip_stream, ksc_problem** out);
/* The same with every option (opts: host pointer).  KSC_DS_SPECTRAL (either
 * space) needs the rational map on every curve, one row per lane: n_x <= 128
 * in FP32, n_x <= 64 in FP64, and n_s <= 16384 (KSC_ERR_UNSUPPORTED or
 * KSC_ERR_ARG otherwise, before any device work).  It allocates D_t and its
 * transpose for every distinct n_s (2 n_s^2 FP64 scalars), three state-sized
 * work arrays and, for small batches, FP64 partial products of up to 8 state
 * sizes. */
ksc_status ksc_create_opts(const ksc_curve_desc* descs, int32_t n_curves, const ksc_options* opts,
                           void* hip_stream, ksc_problem** out);
ksc_status ksc_destroy(ksc_problem* p);

/* Change the stream later calls are enqueued on. */
ksc_status ksc_set_stream(ksc_problem* p, void* hip_stream);

/* Number of scalars (dtype elements) of a whole state / a whole physical-grid
 * array, and the offset (in scalars) of curve c inside each. -1 on error. */
int64_t ksc_state_numel(const ksc_problem* p);
int64_t ksc_state_offset(const ksc_problem* p, int32_t curve);
int64_t ksc_phys_numel(const ksc_problem* p);
int64_t ksc_phys_offset(const ksc_problem* p, int32_t curve);
/* Kept modes K+1 for n_x; -1 if n_x is unsupported. */
int32_t ksc_n_modes(int32_t n_x);

/* Write the two pinned endpoint rows of curve `curve` (the asymptotic states
 * u_- and u_+ of eq. connecting_orbit_def): a_hat -> row 0, b_hat -> row
 * n_s-1; each is one state row (K+1 interleaved complex values, or K reals in
 * KSC_SPACE_ODD; device pointers). */
ksc_status ksc_set_endpoints(ksc_problem* p, void* state, int32_t curve, const void* a_hat,
                             const void* b_hat);

/* Boundary conversions between the spectral state and physical samples on the
 * grid x_n = n L / n_x (Sec. V.C.1).  phys: curve-major [n_s][n_x] scalars.
 * phys_to_spec keeps modes k <= K (u_hat_k = (1/n_x) sum_n u_n e^{-2 pi i k n / n_x});
 * spec_to_phys evaluates the band-limited field.  In KSC_SPACE_ODD,
 * phys_to_spec stores b_k = Im u_hat_k (the odd part of the samples; the even
 * part is dropped) and spec_to_phys evaluates u_n = -2 sum_k b_k sin(q_k x_n). */
ksc_status ksc_phys_to_spec(ksc_problem* p, const void* phys, void* state);
ksc_status ksc_spec_to_phys(ksc_problem* p, const void* state, void* phys);

/* J2[c] (and J_arc[c] if Jarc != NULL) of every curve; FP64 device arrays of
 * n_curves entries. */
ksc_status ksc_eval_J(ksc_problem* p, const void* state, double* J2, double* Jarc);

/* Euclidean gradient of J2 in the state layout, times scale[c] if scale is not
 * NULL (FP64 device array, e.g. an autograd upstream gradient).  grad must not
 * alias state.  J2 (nullable) receives the cost of the same evaluation. */
ksc_status ksc_eval_grad(ksc_problem* p, const void* state, void* grad, double* J2,
                         const double* scale);

/* One descent step state_in -> state_out (distinct buffers; the endpoint rows
 * are copied).  J2 (nullable) receives the cost of state_in. */
ksc_status ksc_step(ksc_problem* p, const void* state_in, void* state_out, double dtau,
                    double* J2);

/* n_steps descent steps in place on `state`, ping-ponging through `scratch`
 * (same size as the state).  Each group of `every` steps is one captured HIP
 * graph; after each group the J2 of the group's last input state is copied to
 * J2_trace[g * n_curves + c] (nullable; n_steps / every rows).  active
 * (nullable, device uint8 [n_curves]): curves with 0 are left unchanged.
 * every must be >= 1; n_steps >= 0. */
ksc_status ksc_descend(ksc_problem* p, void* state, void* scratch, int64_t n_steps, double dtau,
                       double* J2_trace, int32_t every, const uint8_t* active);

/* Select the descent scheme of later ksc_step / ksc_descend calls.
 * KSC_SCHEME_PAPER (the default) is the step described at the top of this
 * file.  KSC_SCHEME_IMPLICIT_S (an extension, not in the paper) makes the
 * whole part of L^dagger(u; r(u)) that is linear in u implicit: on the
 * interior rows of every mode k it solves
 *     (I + dtau B_k) delta = -dtau L^dagger_k,  B_k = A_k^2 - D m D,
 * and writes u_hat + delta, where D is the central difference along s and m
 * zeroes the end rows of the residual (r = f(u) - u_s and
 * L^dagger r = r_s + u r_x - r_xx - r_xxxx of Sec. V.A; the cross terms
 * cancel).  B_k is self-adjoint and positive semi-definite in the weighted
 * inner product, so the step is a descent direction at any dtau > 0, its
 * fixed points are those of the paper's flow, and dtau is no longer bounded
 * by the s-resolution.  D m D couples rows two apart: two tridiagonal systems
 * per curve and mode, solved on the device in the problem's dtype.  Endpoint
 * rows, Im of mode 0 and the `active` mask behave as for the paper's step.
 * Needs KSC_DS_STENCIL (KSC_ERR_UNSUPPORTED for spectral d/ds) and
 * n_s <= 8194 (KSC_ERR_UNSUPPORTED).  Allocates one state-sized gradient
 * buffer and a solve table on first use; blocks the host. */
ksc_status ksc_set_scheme(ksc_problem* p, int32_t scheme);
ksc_status ksc_get_scheme(const ksc_problem* p, int32_t* scheme);

/* Heavy-ball momentum (Polyak) of later ksc_descend calls under
 * KSC_SCHEME_IMPLICIT_S (an extension, not in the paper): every step writes
 *     u_{n+1} = u_n + delta_n + beta (u_n - u_{n-1})
 * on the interior rows (delta_n the implicit-in-s increment of u_n), which
 * shortens the slow final approach along the smallest eigenvalues of the
 * descent flow.  A curve whose cost J2(u_n) rose against J2(u_{n-1}) takes
 * that step without the momentum term (an adaptive restart), so the cost can
 * rise only by single steps.
 * Every ksc_descend call starts from rest (u_{-1} = u_0); `every` must be
 * even while beta > 0 (KSC_ERR_ARG), and ksc_descend under the paper's scheme
 * with beta > 0 returns KSC_ERR_UNSUPPORTED.  ksc_step ignores it.
 * beta in [0, 1) (KSC_ERR_ARG otherwise); 0 (the default) turns it off. */
ksc_status ksc_set_momentum(ksc_problem* p, double beta);
ksc_status ksc_get_momentum(const ksc_problem* p, double* beta);

/* The implicit-in-s increment for a given Euclidean gradient (an extension,
 * not in the paper): on the interior rows of every mode k,
 *     (I + dtau B_k) out_k = -dtau grad_k / (2 w_j L c_k),
 * B_k = A_k^2 - D m D the linear part of the adjoint flow (the solve of the
 * implicit-in-s step, which this is for grad = the gradient of the state);
 * zero on the end rows and for Im of mode 0.  As a map of the stored real
 * and imaginary parts, out = -H0 grad with H0 symmetric positive definite
 * in the plain Euclidean inner product: the initial inverse Hessian of a
 * quasi-Newton descent over the state (paper_2301_11704_amd/lbfgs.py).
 * grad, out: device arrays in the state layout and dtype, distinct
 * (KSC_ERR_ARG otherwise); dtau > 0.  Needs the implicit-in-s scheme set
 * (ksc_set_scheme), else KSC_ERR_UNSUPPORTED.  Enqueued on the problem's
 * stream; allocates nothing. */
ksc_status ksc_precondition(ksc_problem* p, const void* grad, void* out, double dtau);

/* Choose the launch shape (waves per tile, persistent or not) by timing the
 * candidates on scratch buffers; the choice is cached in the JSON file at
 * cache_path (nullable: no file) keyed by device, ROCm version and problem
 * shape.  Blocks the host. */
ksc_status ksc_tune(ksc_problem* p, const char* cache_path);

/* Override the launch policy (KSC_LAUNCH_*) and waves per tile (1, 2 or 4;
 * 0 keeps the current value). */
ksc_status ksc_set_launch(ksc_problem* p, int32_t policy, int32_t waves);
/* Current waves per tile and policy. */
ksc_status ksc_get_launch(const ksc_problem* p, int32_t* policy, int32_t* waves);

/* Copy the per-curve flag words (KSC_FLAG_*) to flags_host[n_curves] and clear
 * them.  Synchronizes the problem's stream. */
ksc_status ksc_query_flags(ksc_problem* p, uint32_t* flags_host);

/* Kernel timing for measurement.  enable != 0 starts a new timing window:
 * every later ksc_eval_J / ksc_eval_grad / ksc_step call on the problem's own
 * stream has its kernel dispatches stamp HIP events (hipExtLaunchKernelGGL
 * start/stop events): the start and end of the fused tile kernel(s) and of
 * the post kernel.
 * Calls made under stream capture and ksc_descend's graphs are not timed;
 * under KSC_SCHEME_IMPLICIT_S a ksc_step's record covers its gradient
 * evaluation, not the banded solve that follows it.
 * enable == 0 stops recording (the window keeps what it holds).  At most
 * 65536 evaluations per window; later ones are not timed and
 * ksc_read_timing reports KSC_ERR_STATE. */
ksc_status ksc_set_timing(ksc_problem* p, int32_t enable);
/* Totals over the current window: milliseconds in the fused tile kernel(s),
 * milliseconds in the post kernel, and the number of timed evaluations.
 * Waits for the recorded events (blocks the host). */
ksc_status ksc_read_timing(ksc_problem* p, double* fused_ms, double* post_ms, int64_t* n_evals);

/* J2[c] of n_curves curves that share one descriptor, laid out as one
 * state of such a problem (curve-major, n_s rows of K+1 complex values each;
 * full space, central-difference d/ds), without a problem object and without
 * allocating device memory: for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * tables, tile list and per-wave partial sums live in one fixed array of
 * KSC_NOALLOC_SCRATCH_BYTES per GPU inside the library (held until the
 * process ends); a batch needing more returns KSC_ERR_SHAPE before any launch
 * (8 MiB holds, e.g., 64 curves of 1024 rows).  Every call on a GPU reuses
 * that GPU's array, so calls that overlap on one GPU (different streams or
 * threads) race.  state: device input; J2: device output of n_curves doubles;
 * hip_stream as for ksc_create.  Enqueued asynchronously; same kernels and
 * tolerance as ksc_eval_J. */
#define KSC_NOALLOC_SCRATCH_BYTES (8u << 20)
ksc_status ksc_eval_J_noalloc(const ksc_curve_desc* desc, int32_t n_curves, int32_t dtype,
                              const void* state, double* J2, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* ksc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KSC_H */
