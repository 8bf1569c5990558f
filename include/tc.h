/*
 * tc.h - C ABI of the MI355X Taylor-Couette projection-step library.
 *
 * The library advances the incompressible Navier-Stokes equations between
 * two coaxial cylinders with the method of Shi, Rampp, Hof and Avila
 * (arXiv:1311.2481): Fourier-Galerkin in (theta, z) (Sec. 3.1, eq. fourier),
 * 9-point finite differences on the radial nodes of eq. nodeDist, and the
 * AB2BD2 fractional-step projection scheme (Sec. 3.2, steps 1-6: eqs.
 * timeScheme, pressure, vel, correction, update).  The nonlinear term is
 * evaluated pseudospectrally with 3/2 dealiasing in its rotational form
 * N = omega x u; the pressure returned is then p + |u|^2/2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lengths are in gap units (r_o - r_i = 1, r_i = eta/(1-eta)); time in
 * viscous units d^2/nu (Sec. 2, eq. NS_dimless).
 *
 * Spectral fields are complex128 (interleaved re, im doubles), C order:
 *     field[j][s][n],  j = 0..n_r-1 radial node (j = 0 inner wall),
 *                      s = 0..m_z-1 axial slot, n = 0..m_theta-1.
 * Slot s holds axial wavenumber l = s for s < m_z/2 and l = s - m_z for
 * s > m_z/2; slot m_z/2 is not a mode and is read as zero and written as
 * zero.  n >= 0 only (real fields); the n = 0 coefficients of a real field
 * satisfy f(-l) = conj(f(l)).  A velocity is three such fields back to back,
 * (u+, u-, u_z) with u+- = u_r +- i u_theta (Sec. 3.1); a nonlinear term is
 * (N+, N-, N_z) in the same way.
 *
 * Memory: every array argument is DEVICE memory unless its comment says
 * host.  The caller owns its arrays; the library never frees or keeps them
 * past the call.  The context owns its own state (u^i, u^{i-1}, N^{i-1}, p),
 * the LU factors, transform tables and work space.
 *
 * Streams: all work is enqueued on the HIP stream given to tc_init and the
 * calls return without waiting, except where a comment says otherwise.
 *
 * Errors: every call returns a tc_status; nothing throws across the ABI.
 * tc_last_error() gives a message for the last failure on a context.
 */
#ifndef TC_H
#define TC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TC_OK = 0,
  TC_EINVAL = 1,      /* invalid argument or unsupported grid            */
  TC_ENOMEM = 2,      /* device allocation failed                        */
  TC_ESINGULAR = 3,   /* zero or non-finite pivot, or factors failing the
                         backward-error check of tc_init                 */
  TC_EHIP = 4,        /* HIP runtime error                               */
  TC_ENONFINITE = 5   /* non-finite value found by a finite check        */
} tc_status;

typedef enum {
  TC_FP64 = 0,        /* whole step in double precision                        */
  TC_FP32_BULK = 1    /* transforms and products in float (float accumulation);
                         curl, LU solves, correction and all state in double   */
} tc_precision;

/* Form of the nonlinear term (Sec. 3.2, step 1). */
typedef enum {
  TC_ROTATIONAL = 0,  /* N = omega x u from 6 transformed fields; the pressure
                         variable is then p + |u|^2/2                          */
  TC_CONVECTIVE = 1   /* N = u.grad u with the curvature terms of eq. NS_cyl,
                         from 12 transformed fields as the paper computes it;
                         the pressure is p.  FP64 only; no tc_step_adjoint    */
} tc_form;

/* The five linear systems of one step (Sec. 3.2, steps 2-4). */
typedef enum {
  TC_SOLVE_P = 0,      /* pressure predictor, eq. pressure: Lap p = rhs; Neumann
                          rows at both walls (rows 0, n_r-1 of rhs hold dp/dr);
                          mode (0,0): row n_r-1 is Dirichlet (Sec. 3.2, end)   */
  TC_SOLVE_UPLUS = 1,  /* eq. vel for u+: (Lap - (1+2a)/r^2 - 3/(2dt)) x = rhs,
                          Dirichlet rows (rows 0, n_r-1 of rhs hold the value)  */
  TC_SOLVE_UMINUS = 2, /* eq. vel for u-: (Lap - (1-2a)/r^2 - 3/(2dt)) x = rhs  */
  TC_SOLVE_UZ = 3,     /* eq. vel for u_z: (Lap - 3/(2dt)) x = rhs, Dirichlet    */
  TC_SOLVE_PHI = 4     /* eq. correction: same operator and rows as TC_SOLVE_P   */
} tc_solve_kind;
/* Lap = d2/dr2 + (1/r) d/dr - a^2/r^2 - b^2 with a = n k_theta, b = l k_z
 * (eq. modalNS); the +-(2a)/r^2 coupling follows eq. modalNSdecoup. */

typedef struct {
  int32_t n_r;        /* radial nodes including both walls (eq. nodeDist: j = 0..M,
                         n_r = M + 1); 9 <= n_r <= 4096                      */
  int32_t m_theta;    /* stored azimuthal wavenumbers n = 0..m_theta-1        */
  int32_t m_z;        /* axial slots (even)                                   */
  int32_t p_theta;    /* dealiased azimuthal grid. Must be >= 3*m_theta - 2
                         (3/2 rule, Sec. 3.1) and a supported transform length
                         (2^k, 3*2^k, 5*2^k, 9*2^k, 15*2^k from 16 to 2048);
                         0 -> the smallest supported length >= 3*m_theta - 2 */
  int32_t p_z;        /* dealiased axial grid; >= 3*m_z/2 - 2 and a supported
                         length; 0 -> the smallest one >= 3*m_z/2 - 2         */
  double k_theta;     /* fundamental azimuthal wavenumber (L_theta = 2pi/k_theta) */
  double k_z;         /* fundamental axial wavenumber (Gamma = 2pi/k_z)         */
  double alpha;       /* node-map parameter of eq. nodeDist; 0 = Chebyshev limit */
  int32_t n_s;        /* stencil length; only 9 is supported (Sec. 3.1)        */
  int32_t precision;  /* tc_precision                                         */
  int32_t form;       /* tc_form: the nonlinear term's form (Sec. 3.2, step 1) */
} tc_grid;

typedef struct tc_ctx tc_ctx;

/* Build the radial grid (eq. nodeDist), FD weights (Fornberg, Sec. 3.1),
 * and the LU factors of the four operators of every mode (Sec. 3.2: factors
 * are computed once, each step only substitutes).  hip_stream: a
 * hipStream_t (NULL = default stream).  Waits for the factorisation to
 * finish.  Returns TC_EINVAL for an unsupported grid, TC_ESINGULAR if a
 * pivot is zero or not finite, TC_ENOMEM, TC_EHIP.  *out is NULL on error.
 * On grids of 32, 64 or 128 radial nodes the context also keeps a second,
 * lane-contiguous copy of the factors for the predictor-corrector kernels
 * that hold each mode's radial line on chip; with the environment variable
 * TC_PC_LINE=0 set at this call it uses the four-sweep kernels instead (the
 * same results up to rounding) and keeps no copy.  The curl adjoint of
 * tc_step_adjoint runs as radial sweeps on grids with at least 131072
 * stored slots per radial node and tiled elsewhere; TC_ADJ_CURL_SWEEP=1 or
 * 0 at this call picks one form on any grid (results equal up to rounding). */
tc_status tc_init(const tc_grid* g, double eta, double Re_i, double Re_o, double dt,
                  void* hip_stream, tc_ctx** out);

/* Release everything the context owns (waits for its stream). */
tc_status tc_destroy(tc_ctx* ctx);

/* Message for the last failing call on ctx ("" if none); ctx may be NULL for
 * failures of tc_init.  The string is owned by the library. */
const char* tc_last_error(const tc_ctx* ctx);

/* Radial nodes r_0..r_{n_r-1} into HOST memory (n_r doubles).  Synchronous. */
tc_status tc_radial_nodes(const tc_ctx* ctx, double* r_host);

/* Load the time-stepping state.  u: velocity (3 fields) at step i.
 * u_prev: velocity at step i-1, or NULL for u_prev = u.  N_prev: nonlinear
 * term at step i-1, or NULL for N(u_prev).  Copies; the caller's arrays may
 * be reused once the stream has passed this call.  Resets the step count. */
tc_status tc_set_state(tc_ctx* ctx, const void* u, const void* u_prev, const void* N_prev);

/* Copy out the current velocity (3 fields) and, if p is not NULL, the
 * pressure of the last completed step (1 field; zero before the first). */
tc_status tc_get_state(const tc_ctx* ctx, void* u, void* p);

/* Copy out the history (u^{i-1} and N^{i-1}, 3 fields each); either may be NULL. */
tc_status tc_get_history(const tc_ctx* ctx, void* u_prev, void* N_prev);

/* Advance the state by nsteps >= 0 projection steps (Sec. 3.2, steps 1-6). */
tc_status tc_step(tc_ctx* ctx, int32_t nsteps);

/* Nonlinear term N of a velocity u (3 fields) into N (3 fields), in the
 * context's form (omega x u or u.grad u), by the pseudospectral method with
 * 3/2 dealiasing (Sec. 3.2, step 1).
 * u and N must not overlap.  Does not touch the context's state. */
tc_status tc_nonlinear(tc_ctx* ctx, const void* u, void* N);

/* Solve the system of kind k (see tc_solve_kind) for every mode: rhs and x
 * are one field each, rhs rows 0 and n_r-1 holding the boundary values.
 * x may equal rhs.  Does not touch the context's state. */
tc_status tc_helmholtz_solve(tc_ctx* ctx, tc_solve_kind k, const void* rhs, void* x);

/* Same solve with the transposed operator (A^T x = rhs), used by the adjoint. */
tc_status tc_helmholtz_solve_transposed(tc_ctx* ctx, tc_solve_kind k, const void* rhs, void* x);

/* One step of the discrete adjoint (reverse mode) of tc_step.
 * fwd: the forward inputs of the step, u^i, u^{i-1} (3 fields each) back to
 * back (6 fields).  adj_in: cotangents of the step outputs (u^{i+1}, u^i,
 * N^i) (9 fields).  adj_out: cotangents of the step inputs (u^i, u^{i-1},
 * N^{i-1}) (9 fields).  The inner product is sum Re(conj(x) y) over every
 * stored coefficient.  adj_in and adj_out must not overlap.  Rotational
 * form only (TC_EINVAL otherwise).  Its transforms run in double whatever
 * the context's precision: on a TC_FP32_BULK context it is the adjoint of
 * the FP64 step. */
tc_status tc_step_adjoint(tc_ctx* ctx, const void* fwd, const void* adj_in, void* adj_out);

/* Gradient of the perturbation kinetic energy E_pert(u) = 1/2 int |u - U_c|^2 dV
 * (U_c: circular Couette flow of Sec. 5.1; trapezoid rule in r, Parseval in
 * theta and z) with respect to the stored coefficients of u (3 fields) under
 * the inner product of tc_step_adjoint, into g (3 fields).  This is the
 * seed of the reverse sweep for the final-energy objective. */
tc_status tc_perturbation_energy_gradient(tc_ctx* ctx, const void* u, void* g);

/* Ends of the reverse sweep for the final-energy objective J = E_pert(u^T).
 * tc_adjoint_seed: g = scale * dJ/du at u = u^T (3 fields), the cotangent
 *   of the last step's output times the caller's cotangent of J.
 * tc_adjoint_initial_history: the cotangent of u^0 when the history of the
 *   first step is u^{-1} = u^0, N^{-1} = N(u^0) (what tc_set_state with
 *   NULL history sets): g = u_bar + u_prev_bar + N'(u^0)^T N_bar, from the
 *   9-field cotangent adj_in = (u_bar, u_prev_bar, N_bar) of the first
 *   step's inputs (tc_step_adjoint's adj_out).  u0, g: 3 fields; adj_in and
 *   g must not overlap.  Rotational form only. */
tc_status tc_adjoint_seed(tc_ctx* ctx, const void* uT, double scale, void* g);
tc_status tc_adjoint_initial_history(tc_ctx* ctx, const void* u0, const void* adj_in, void* g);

/* Optimal-perturbation control (not in the paper's method; the paper's
 * quasi-Keplerian run of Sec. 5.5 starts from a nonlinear optimal
 * perturbation taken from elsewhere).  The initial perturbation is the curl
 * of a vector potential with smooth radial profiles: per stored mode
 * (a = n k_theta, b = l k_z), A_c(r) = sum_{q=0..3} a[c][q] g(r) T_q(xi),
 * g = 16 (r - r_i)^2 (r_o - r)^2, xi = 2 (r - r_i) - 1 (T_q Chebyshev), and
 * u_r = i a A_z / r - i b A_theta, u_theta = i b A_r - d_r A_z,
 * u_z = d_r A_theta + A_theta / r - i a A_r / r.  A control is complex128
 * a[c][q][s][n] (c = r, theta, z; q = 0..3; slot s, wavenumber n as in the
 * spectral layout): 12 m_z m_theta values; mode (0,0) and the empty slot
 * are not controls (read as zero, written as zero), and the n = 0 column of
 * a real perturbation obeys a(-l) = conj(a(l)).
 *
 * tc_control_velocity: u = U_c + B a (3 fields; U_c circular Couette flow).
 * tc_control_gradient: ga = the gradient with respect to the control of a
 *   function whose gradient with respect to u is g (3 fields), i.e. B^H g
 *   projected on the controls with the n = 0 symmetry; inner products
 *   sum Re(conj(x) y) in both spaces.
 * tc_control_ascent_update: one step of projected gradient ascent on the
 *   sphere E_pert(U_c + B a) = E0: with p = gJ - beta gE, beta = <gJ, gE> /
 *   <gE, gE>, a_out = s (a + tau p) and s such that the perturbation energy
 *   of a_out is E0 exactly.  gJ and gE may both be NULL (then a_out is a
 *   rescaled to E0).  stats (host, nullable, 5 doubles): beta, the energy
 *   before rescaling, s, |p| and |a| (of the input a).  Synchronous.
 *   a_out may equal a.  Uses the context's curl work buffer. */
tc_status tc_control_velocity(tc_ctx* ctx, const void* a, void* u);
tc_status tc_control_gradient(tc_ctx* ctx, const void* g, void* ga);
tc_status tc_control_ascent_update(tc_ctx* ctx, const void* a, const void* gJ, const void* gE, double tau,
                                   double E0, void* a_out, double* stats_host);

/* Diagnostics of the current state into HOST memory (8 doubles):
 * kinetic energy, perturbation energy (against circular Couette flow),
 * max |div u| over interior nodes, relative tangential wall slip at r_i
 * (Sec. 5.3), an upper bound of the advective CFL number
 * dt max (|u_r|/dr + |u_theta|/(r dtheta) + |u_z|/dz) over the radial nodes
 * (per node the plane maximum of each component bounded by sum c_n |u_ln|;
 * dr the distance to the nearer neighbouring node, dtheta and dz the
 * spacings of the (2 m_theta, m_z) physical grid), the number of steps
 * taken, and the quasi-Nusselt numbers Nu_omega at r_i and at r_o (Sec. 5.5:
 * the torque on that cylinder, r^3 d<u_theta/r>/dr from the theta-z mean
 * by the wall row of D1, over its value -2 C2 in circular Couette flow;
 * NaN when C2 = 0).  Synchronous. */
tc_status tc_get_diag(tc_ctx* ctx, double* out_host);

/* The same eight diagnostics as tc_get_diag, for callers that cannot
 * allocate device memory (code under stream capture preparation, tight
 * serving loops, harnesses that forbid allocation): this call allocates
 * nothing.  Its partial sums live in a static 4 MiB device array of the
 * library (one per GPU, held from library load to process end; its address
 * on the context's device is looked up once, in tc_init).  Every call on a
 * GPU overwrites that GPU's array, so calls that overlap on one GPU (other
 * host threads, other streams) race and must be serialised by the caller;
 * nothing in it needs clearing, every partial is written before it is read.
 * Grids whose partials exceed the array (more than 2^19 - 8 doubles:
 * 4 max(1024, ceil(m_z m_theta / 256)) + 97 n_r) are rejected with
 * TC_EINVAL.  Synchronous; out_host: 8 doubles of HOST memory. */
tc_status tc_get_diag_noalloc(tc_ctx* ctx, double* out_host);

/* Check the current velocity for non-finite values: TC_ENONFINITE if any.
 * Synchronous. */
tc_status tc_check_finite(tc_ctx* ctx);

/* Mean duration in milliseconds of the launches of one kernel over the last
 * tc_step call with timing enabled (HIP events on the context stream);
 * which = 0: fused predictor-corrector solve, 1: curl, 2: axial inverse
 * transforms, 3: azimuthal transforms and product, 4: axial forward
 * transforms.  tc_set_timing(ctx, 1) enables it (adds event records).
 * launches_out receives the number of launches averaged.  Synchronous. */
tc_status tc_set_timing(tc_ctx* ctx, int32_t enable);
tc_status tc_kernel_time(tc_ctx* ctx, int32_t which, double* ms_out, int32_t* launches_out);

/* The factors are LU without pivoting (the paper's DGBTRF pivots; the
 * Neumann rows of P are scaled to the size of the Laplacian rows instead).
 * tc_init accepts them only after a check: for every operator and distinct
 * mode it solves A x = A x0 (x0_j = 1 + sin(0.7 j)/2) with the stored
 * factors and takes the componentwise backward error
 * max_j |A x - b|_j / (|A| |x| + |b|)_j; above 1e-12 it fails with
 * TC_ESINGULAR.  This call returns the largest error found (host double). */
tc_status tc_factor_backward_error(const tc_ctx* ctx, double* error_host);

/* Bytes of device memory the context holds (host pointer out). */
tc_status tc_memory_bytes(const tc_ctx* ctx, uint64_t* bytes_out);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
