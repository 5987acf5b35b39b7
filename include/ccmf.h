/*
 * ccmf.h -- C ABI of the MI355X solver for the effective crack energy on a
 * combinatorially consistent grid (Ernesti & Schneider, arXiv 2103.05968).
 *
 * The library computes, for a periodic voxel field gamma >= 0 of crack
 * resistances and a prescribed mean crack normal xibar, the CCMF
 * discretization of the effective crack energy
 *
 *     geff(xibar) = min { (1/N) sum_x gamma[x] |xi[x]| : xi in K_xibar }
 *                 = max { <xibar, v> : div^- v = 0, |A v| <= gamma }
 *
 * (Sec. 3.1, eq:CCMF_FFT_problem_primal_final and eq:CCMF_FFT_problemA) with the
 * damped ADMM of Sec. 3.2 (eq:CCMF_FFT_ADMM, second form): each iteration solves
 * the periodic discrete Laplacian div^- grad^+ in a separable spectral basis for
 * the node potential, projects each voxel's six incident edge quantities onto
 * the ball of radius gamma, updates the multiplier and reduces (in FP64) the
 * residual, energy and penalty statistics that drive the adaptive penalty.
 * All steps run in HIP kernels on the device; the host only launches them and
 * polls a convergence flag.
 *
 * Conventions for every entry point:
 *  - Fields are C-order [N1][N2][N3] (k = third index fastest), one contiguous
 *    block per field; vector fields are component-major [c][N1][N2][N3].
 *  - "device" pointers are HIP device allocations on the device that was
 *    current at ccmf_setup; "host" pointers are ordinary host memory.
 *  - Element type of device fields is the plan's dtype (double for CCMF_F64,
 *    float for CCMF_F32).  Scalars crossing the ABI are always double.
 *  - Every call is ordered on the stream given to ccmf_setup; calls returning
 *    host results synchronize that stream before returning.
 *  - The caller owns every pointer it passes; the plan copies what it keeps
 *    (kappa) and never retains a caller pointer past the call.
 *  - Return value 0 = success; negative = error (nothing written to outputs,
 *    message in ccmf_last_error()); CCMF_NOT_CONVERGED (= 1) is a warning:
 *    all outputs are written from the last iterate.
 *  - A plan is not thread safe; distinct plans are independent.
 *
 * Diagnostic environment variables (read by the library, never needed):
 *  - CCMF_TUNE_LOG: when set, the transform-tile autotuner prints every
 *    candidate's time to stderr.
 *  - CCMF_FFT_VARIANT = 0, 1 or 2: forces one register-blocked FFT plan variant
 *    in every power-of-two transform pass instead of the autotuner's choice
 *    (results agree to rounding; used to test each variant).
 *  - CCMF_TILE_WALK = 1 .. 64: forces the number of tiles each block of a
 *    power-of-two transform pass walks instead of the autotuner's choice (results
 *    are bit-identical; used to test the walk).
 */
#ifndef CCMF_H_
#define CCMF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ccmf_plan_s* ccmf_plan;

enum {
  CCMF_OK = 0,
  CCMF_NOT_CONVERGED = 1, /* max_iter reached; outputs hold the last iterate  */
  CCMF_EINVAL = -1,       /* invalid argument (message says which)             */
  CCMF_ENOMEM = -2,       /* device or pinned-host allocation failed           */
  CCMF_EDEVICE = -3,      /* a HIP call failed (HIP error text in the message) */
  CCMF_ESTATE = -4        /* call out of order (e.g. outputs before a solve)   */
};

enum { CCMF_F64 = 0, CCMF_F32 = 1 };

/* Penalty rules of Sec. 3.2: Barzilai-Borwein, constant rho0, Lorenz-Tran-Dinh. */
enum { CCMF_RHO_BB = 0, CCMF_RHO_CONST = 1, CCMF_RHO_LTD = 2 };

typedef struct {
  double delta;        /* damping of eq:CCMF_FFT_ADMM, in (0,1); 0 selects 0.25 (Sec. 4.1)  */
  double rho0;         /* initial penalty; 0 selects the smallest positive kappa of the field */
  int32_t rule;        /* CCMF_RHO_*                                                          */
  int32_t max_iter;    /* maximum number of xi-steps; 0 selects 20000                         */
  int32_t check_every; /* host polls the device convergence flags every this many
                          iterations (the kernels stop by themselves); 0 selects 32          */
  int32_t time_kernels;/* nonzero: time every launch of the fused update kernel with HIP
                          events on the plan's stream (read with ccmf_kernel_times); with
                          graph replay the events are part of the graph and are read after
                          each replay                                                      */
  double bb_min_corr;  /* Barzilai-Borwein estimate used only if <dv,de>/(|dv||de|) >= this,
                          else the Lorenz-Tran-Dinh value; 0 selects 0.2                    */
  double eta0;         /* safeguard: |log(rho_{k+1}/rho_k)| <= log(1 + eta0/(1+k/k0)^2), a
                          summable variation; 0 selects 1.0                                  */
  double k0;           /* see eta0; 0 selects 100                                             */
  int32_t eager;       /* nonzero: launch every kernel from the host; 0: capture one chunk of
                          check_every iterations into a HIP graph once and replay it         */
  int32_t no_autotune; /* nonzero: skip the tile-width autotuner of the spectral passes (run
                          once per plan and batch size, cached per process) and use defaults */
  int32_t warm_start;  /* nonzero: resume from the plan's state -- the stopping state of the
                          previous solve (same n_loads) or the one loaded by ccmf_set_state --
                          instead of the initial state; rho^k, rho^{k-1} and the iteration
                          index carry over (rho0 still sets the penalty limits), while tol,
                          delta, rule, max_iter and the loads are taken from this call.  The
                          stopping iterate is stepped again, so a solve stopped by max_iter
                          and resumed follows the uninterrupted sequence bit for bit. */
  int32_t record_history; /* nonzero: record, for each of the first max_iter iterations of
                          every problem, (|e^k - xi^{k+1/2}|_{L2}, rho^k, energy of
                          xi^{k+1/2}, |<v^k>|); read with ccmf_history.  Needs
                          B * max_iter * 32 bytes of device memory.                   */
} ccmf_options;

/* Create a plan for n_fields crack-resistance fields of size dims[0] x dims[1] x
 * dims[2] (each >= 1, N = product < 2^31, each dim <= 2048 in F64 / 4096 in F32).
 * kappa_dev: device, [n_fields][N1][N2][N3] of the plan's dtype, finite and >= 0
 * (zeros are pores).  Copied into the plan.  stream: hipStream_t; NULL makes the plan
 * create its own blocking stream (ordered with the null stream), since the null
 * stream cannot be captured into a HIP graph.
 * Errors: CCMF_EINVAL for bad sizes/dtype or a negative / non-finite kappa entry. */
int ccmf_setup(ccmf_plan* out, const int64_t dims[3], int64_t n_fields, int32_t dtype,
               const void* kappa_dev, void* stream);

/* Solve the damped ADMM of Sec. 3.2 for every (field f, load l) pair, problem
 * index b = f * n_loads + l, all in one batched launch sequence; every problem
 * stops by itself when |e^k - xi^{k+1/2}|_{L2} <= tol |<v^k>| (eq:convergence_criterion).
 * xi:        host, [n_loads][3] load directions (normalised to unit length).
 * tol:       > 0.   opt: host, may be NULL (all defaults).
 * geff:      host out, [B]: primal energy (1/N) sum gamma |xi^{k+1/2}| at the stopping iterate.
 * iters:     host out, [B]: number of xi-steps taken.  residual: host out, [B] (nullable).
 * dual_est:  host out, [B]: <A xibar, v^k> (nullable).
 * phi_dev:   device out, [B][N] double: node potential of the stopping iterate, zero mean
 *            (nullable).  Always FP64: phi has magnitude O(N) while only its
 *            differences enter the scheme, so it is computed and kept in FP64.
 * flux_dev:  device out, [B][3][N] face fluxes A* v^k, v_c[x] on face x + e_c/2 (nullable).
 * The solution state stays in the plan for ccmf_grad_kappa until the next solve. */
int ccmf_solve(ccmf_plan p, const double* xi, int64_t n_loads, double tol, const ccmf_options* opt,
               double* geff, int32_t* iters, double* residual, double* dual_est,
               void* phi_dev, void* flux_dev);

/* Envelope-theorem gradient of the last solve (not in the paper; Danskin's theorem
 * applied to the min-cut form eq:CCMF_FFT_problem_primal_final, linear in gamma):
 *   dkappa[f][x] = sum_l dL_dgeff[f*n_loads + l] * |xi^{k+1/2}_{f,l}[x]| / N.
 * dL_dgeff: host, [B].  dkappa_dev: device out, [n_fields][N] of the plan's dtype. */
int ccmf_grad_kappa(ccmf_plan p, const double* dL_dgeff, void* dkappa_dev);

/* Certified lower bound of geff for every problem of the last solve (strong duality
 * of Sec. 2.1 for the max-flow form eq:CCMF_FFT_problemA): with the face flux y = A* v^k
 * of the stopping iterate, its divergence-free part y_df = y - grad^+ L^dagger div^- y
 * (same spectral solve) and sigma = max over gamma > 0 of |A y_df| / gamma, the flux
 * y_df / max(1, sigma) is feasible, so cert = <xibar, y> / max(1, sigma) <= geff.
 * cert: host out [B]; -inf when a voxel with gamma = 0 carries flux.  sigma: host out
 * [B] (nullable).  Allocates scratch (N doubles per problem) for the duration of the call. */
int ccmf_certificate(ccmf_plan p, double* cert, double* sigma);

/* Mean face flux <A* v^k> (eq:CCMF_FFT_AOperator_adjoint) of every problem of the last
 * solve at its stopping iterate.  geff is the support function of the set of mean
 * fluxes of the admissible flows of the max-flow form eq:CCMF_FFT_problemA, so at the
 * optimum this is the gradient of the 1-homogeneous extension of geff with respect to
 * the load xibar (not stated in the paper; it follows from that max-flow form), and
 * <xibar, mflux> -> geff.  mflux: host out, [B][3].  Errors: CCMF_ESTATE before a solve. */
int ccmf_mean_flux(ccmf_plan p, double* mflux);

/* Convergence history of the last solve (options.record_history set): out, host
 * [B][max_len][4] with rows (residual, rho^k, energy, |<v^k>|) per iteration of the
 * solve (the quantities of eq:convergence_criterion and the penalty of Sec. 3.2);
 * rows at or beyond a problem's iteration count are NaN.  max_len >= 1; only the
 * first min(max_len, max_iter) rows are recorded.
 * Errors: CCMF_ESTATE when the last solve recorded no history. */
int ccmf_history(ccmf_plan p, int32_t max_len, double* out);

/* Checkpoint of the ADMM state of eq:CCMF_FFT_ADMM for every problem: the multiplier
 * v^k and e^k of the state the last solve stopped at (or the one set by ccmf_set_state),
 * the penalty rho^k and the global iteration index k.
 * v_dev, e_dev: device out, [B][6][N] of the plan's dtype (nullable); components 0..2
 * are the first half (xi1 of the operator A, eq:CCMF_FFT_AOperator), 3..5 the second.
 * rho: host out [B] (nullable).  k: host out [B] (nullable).
 * Errors: CCMF_ESTATE when the plan holds no state. */
int ccmf_get_state(ccmf_plan p, void* v_dev, void* e_dev, double* rho, int32_t* k);

/* Load a state (v^k, e^k, rho^k, k) for n_loads loads per field, b = f * n_loads + l,
 * for a following ccmf_solve with options.warm_start set and the same n_loads.
 * v_dev, e_dev: device, [B][6][N] of the plan's dtype, read during the call only.
 * At every voxel v and e must be non-negative multiples of one 6-vector (every ADMM
 * iterate is: v = P_C(z) and e = (z - v)/rho are both multiples of z); the plan stores
 * z = v + rho e and |v|/|z|.  rho: host [B], > 0.  k: host [B], >= 0 (enters the
 * penalty safeguard).  Errors: CCMF_EINVAL for bad sizes, rho or k, and for a pair
 * that is not of that form at some voxel (the plan then holds no state). */
int ccmf_set_state(ccmf_plan p, int64_t n_loads, const void* v_dev, const void* e_dev, const double* rho,
                   const int32_t* k);

/* Average device duration (ms) of the fused update kernel over the launches timed
 * since the last call (options.time_kernels), the number of launches, and the
 * kernel's algorithmic HBM bytes per launch per problem.  Resets the counters. */
int ccmf_kernel_times(ccmf_plan p, double* avg_ms, int64_t* count, double* bytes_per_launch);

/* Apply the spectral solve phi = (div^- grad^+)^dagger r (the pseudo-inverse in
 * eq:CCMF_FFT_Gamma_2) to `count` fields with the plan's transform kernels.
 * r_dev: device, [count][N] of the plan's dtype; phi_dev: device, [count][N] double
 * (may alias r_dev in FP64 mode). */
int ccmf_laplace_pinv(ccmf_plan p, const void* r_dev, void* phi_dev, int64_t count);

/* One separable Hartley transform pass along `axis` (0, 1, 2) of `count` fields,
 * in place: H[q] = sum_t x[t] (cos + sin)(2 pi q t / n), unnormalised.
 * data_dev: device, [count][N] of the plan's dtype.  A diagnostic of the spectral solve. */
int ccmf_hartley_axis(ccmf_plan p, void* data_dev, int64_t count, int32_t axis);

/* Plain device copy of nbytes (a multiple of 16) with a streaming kernel on
 * `stream`: the bandwidth reference used to calibrate traffic counters. */
int ccmf_stream_copy(void* dst_dev, const void* src_dev, int64_t nbytes, void* stream);

void ccmf_destroy(ccmf_plan p);

/* Message for the last non-zero status returned on the calling thread. */
const char* ccmf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CCMF_H_ */
