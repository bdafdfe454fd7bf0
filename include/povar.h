/*
 * povar.h — C ABI of the PoVar (Power Variable Projection) bundle-adjustment
 * hot path for AMD Instinct MI355X (gfx950).
 *
 * A problem is a set of observations (camera i, point j, 2-D measurement m_ij)
 * of n_cams projective 3x4 cameras and n_pts points (Sec. 3.2 of the paper).
 * The library minimises the pOSE objective, Eq. (6),
 *
 *   F(P, X) = sum_ij || ( sqrt(1-eta) (P_i^{1:2} x~_j - (P_i^3 x~_j) m_ij) ;
 *                         sqrt(eta)   (P_i^{1:2} x~_j - m_ij) ) ||^2 ,
 *   x~_j = (X_j, 1),
 *
 * by Variable Projection (Sec. 4.1): every landmark is eliminated in closed
 * form, Eq. (8); each outer iteration linearises the reduced problem (9) with
 * the RW2 normal equations (10)-(13), approximates the inverse of the Schur
 * complement (14)-(15) by the truncated power series (17), takes the camera
 * update in the tangent space of each camera's unit sphere in R^12 (Sec. 4.3,
 * (18)-(29)), retracts by normalisation, re-solves the landmarks and accepts
 * or rejects the step with a Levenberg-Marquardt damping schedule (Sec. 5.2).
 *
 * The stratified pipeline of Sec. 3 continues with two more calls: the
 * projective refinement of objective (7) with the Riemannian power-series
 * solver on both blocks (povar_refine_create, then the same solve/step
 * calls), and the metric upgrade with known intrinsics (povar_metric_upgrade,
 * the supplement's App. D).
 *
 * Conventions shared by every call:
 *  - Every call returns povar_status; 0 (POVAR_OK) is success.  No C++
 *    exception crosses this boundary.  On failure, povar_last_error(ctx)
 *    returns a message for the last failing call made on that context.
 *  - Cameras are row-major 3x4 matrices stored as 12 doubles (p_i), points are
 *    3 doubles, measurements are 2 doubles, all contiguous and unpadded.
 *  - Unless a name ends in _device, pointer arguments are HOST pointers.  The
 *    library copies inputs; the caller keeps ownership of every buffer it
 *    passes and may free it when the call returns.  Outputs are written into
 *    caller buffers of the documented size.
 *  - All device work of a context runs on the HIP stream given to
 *    povar_ctx_create (NULL = a stream the library creates).  Calls that
 *    return results to host memory synchronise that stream.
 *  - A context and the problems created from it are used from one host
 *    thread at a time.  The server (povar_server_*) is thread-safe.
 */
#ifndef POVAR_H
#define POVAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  POVAR_OK = 0,
  POVAR_EINVAL = 1,   /* invalid argument (sizes, indices, non-finite values, options) */
  POVAR_ENOMEM = 2,   /* device allocation failed, or request exceeds a server budget */
  POVAR_EDEVICE = 3,  /* a HIP runtime error */
  POVAR_EAGAIN = 4,   /* result not ready yet (server poll) */
  POVAR_ENUMERIC = 5, /* non-finite initial cost; from povar_debug_step: a damped camera
                         block that could not be factored (inside the LM loop such a
                         step is simply rejected) */
  POVAR_ESTATE = 6    /* call not valid in the object's current state */
} povar_status;

typedef enum {
  /* every step of the path in FP64 */
  POVAR_PREC_FP64 = 0,
  /* Jacobian evaluation and power-series matvecs in FP32 with FP32
     accumulation (the per-observation products and their per-landmark and
     per-camera sums); the V_j pseudo-inverse, the U_i factorisation (and
     their application to those sums inside the series) and the cost in FP64.
     U_i is formed in FP64 from FP64 landmarks and measurements (its FP64
     factorisation needs an FP64 input at small damping); b_p is FP32
     products accumulated in FP64. */
  POVAR_PREC_FP32_BULK = 1
} povar_precision;

typedef enum {
  /* camera update in the tangent space of the unit sphere of R^12, then
     retraction by normalisation (Sec. 4.3) */
  POVAR_MANIFOLD_SPHERE = 0,
  /* paper-literal Euclidean camera update of Sec. 4.1-4.2 (no projection) */
  POVAR_MANIFOLD_EUCLIDEAN = 1
} povar_manifold;

typedef struct {
  uint32_t struct_size;  /* = sizeof(povar_options); checked */
  double eta;            /* pOSE weight in [0,1], Eq. (6); default 0.01 */
  int32_t series_order;  /* m of Eq. (17): terms i = 0..m; >= 0; default 20 */
  int32_t max_iters;     /* LM iterations for povar_solve; default 50 */
  double ftol;           /* stop when an accepted step decreases the cost by
                            less than ftol relative; 0 disables; default 1e-6 */
  double lambda0;        /* initial damping (Sec. 5.2); default 1e-4 */
  double lambda_min;     /* damping bounds; defaults 1e-12, 1e12 */
  double lambda_max;
  int32_t precision;     /* povar_precision; default POVAR_PREC_FP64 */
  int32_t manifold;      /* povar_manifold; default POVAR_MANIFOLD_SPHERE */
  int32_t use_graph;     /* 1: replay each iteration as a captured HIP graph
                            (default) for problems of up to 2,000,000
                            observations, whose kernels are short enough for
                            launch costs to matter; larger problems and 0:
                            launch kernels one by one */
  int32_t reserved;
  double series_rtol;    /* optional early stop of the series, in [0, 1).
                            Sec. 5.2 gives the expansion methods a "threshold"
                            of 0.01 without defining it; read here as: after
                            term t >= 1, stop once ||x_t|| <= series_rtol *
                            ||x_0 + ... + x_t|| (2-norms over all cameras,
                            FP64 sums of the stored terms).  0 (default) runs
                            all series_order terms. */
  uint64_t init_seed;    /* seed of the initial cameras when cams0 is NULL
                            (Sec. 5.2 "Dataset": cameras drawn from an
                            isotropic Gaussian).  Camera c (caller's index)
                            takes 12 standard normals from three blocks of the
                            counter-based generator Philox4x64-10 (Salmon et
                            al., SC 2011) with key (init_seed, 0) and counters
                            (c, b, 0, 0), b = 0, 1, 2; each 64-bit output w
                            gives u = ((w >> 11) + 0.5) 2^-53 in (0, 1), and
                            the outputs (w0, w1), (w2, w3) of a block give two
                            normals each by the Box-Muller transform
                            (sqrt(-2 ln u0) cos(2 pi u1), then sin), in that
                            order; the 12-vector is then scaled to unit norm.
                            Default 0. */
} povar_options;

typedef struct {
  double cost_initial;   /* f* at the initial cameras */
  double cost_final;     /* f* at the current cameras */
  double lambda_final;   /* damping for the next step */
  double grad_norm_final;/* 2-norm over all cameras of the Riemannian gradient
                            of f* at the current cameras: 2 Pi_i b_p,i with
                            b_p,i = sum_k J_p,k^T r_k at X*(P) (the gradient of
                            the reduced cost (9) by the envelope theorem, Eq.
                            (10)), Pi_i the tangent projector of the unit sphere
                            at p_i (identity in Euclidean mode); computed by
                            povar_solve, povar_step and povar_get_report (one
                            linearisation pass when the current one is stale),
                            NaN in server reports */
  double seconds_total;  /* wall time of the call (0 for povar_get_report) */
  double seconds_series; /* device time of the power series (Eq. (17)) summed
                            over every iteration of the problem so far: from
                            the start of a step's camera-block factorisation
                            (x_0, the first term) to the end of its last
                            series pass, read from the GPU's constant-rate
                            clock */
  int32_t iters;         /* LM iterations taken so far (rejected ones count) */
  int32_t accepted;      /* accepted iterations so far */
  int32_t stop_reason;   /* 0 running / max_iters, 1 ftol reached */
  int32_t reserved;
} povar_report;

typedef struct povar_ctx_s* povar_ctx;
typedef struct povar_problem_s* povar_problem;
typedef struct povar_server_s* povar_server;

/* Fill *opts with the defaults listed above. */
povar_status povar_options_default(povar_options* opts);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
   (e.g. torch.cuda.current_stream().cuda_stream) or NULL for a private one. */
povar_status povar_ctx_create(int device, void* hip_stream, povar_ctx* out);
/* POVAR_ESTATE while problems created on ctx are still alive. */
povar_status povar_ctx_destroy(povar_ctx ctx);
/* Message of the last failing call on ctx (never NULL; "" if none).  With
   ctx == NULL: the last failure of a call that had no context. */
const char* povar_last_error(povar_ctx ctx);

/* Device bytes a problem of this size needs (all precisions' buffers that
   the chosen precision uses, plus the layout).  Used for server admission. */
povar_status povar_problem_footprint(int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                     int32_t precision, uint64_t* bytes);

/* Create a problem from observations (Sec. 3.2): cam_idx[k] in [0,n_cams),
   pt_idx[k] in [0,n_pts), meas[2k..2k+1] finite.  Every camera and every
   point needs at least one observation.  Sizes up to 67,108,863 cameras and
   1,073,741,822 observations.  cams0 (n_cams x 12) is the initial camera
   set, or NULL: cameras drawn from opts->init_seed as
   described there; on the sphere manifold each camera is normalised to
   unit norm.  The landmarks are then solved in closed form (8) and the
   initial cost is evaluated (POVAR_ENUMERIC if it is not finite).
   Errors: POVAR_EINVAL for any violated precondition, POVAR_ENOMEM,
   POVAR_EDEVICE. */
povar_status povar_problem_create(povar_ctx ctx, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                  const int32_t* cam_idx, const int32_t* pt_idx,
                                  const double* meas, const double* cams0,
                                  const povar_options* opts, povar_problem* out);
/* Same, with cam_idx, pt_idx, meas and cams0 in device memory of ctx's
   device (e.g. torch tensors); cams0 may be NULL as above. */
povar_status povar_problem_create_device(povar_ctx ctx, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                         const int32_t* cam_idx, const int32_t* pt_idx,
                                         const double* meas, const double* cams0,
                                         const povar_options* opts, povar_problem* out);
povar_status povar_problem_destroy(povar_problem pb);

/* Run LM iterations until opts.max_iters iterations in total or ftol. */
povar_status povar_solve(povar_problem pb, povar_report* report);
/* Run up to n_iters more iterations (fewer if ftol stops the solve). */
povar_status povar_step(povar_problem pb, int32_t n_iters, povar_report* report);
/* Enqueue n_iters iterations on the context stream without waiting and
   without reading anything back (for timing loops); povar_step/povar_report
   read the state afterwards. */
povar_status povar_enqueue(povar_problem pb, int32_t n_iters);
/* Current report (synchronises). */
povar_status povar_get_report(povar_problem pb, povar_report* report);

/* Current cameras (n_cams x 12) and points (n_pts x 3, caller's point order). */
povar_status povar_get_cameras(povar_problem pb, double* cams_out);
povar_status povar_get_points(povar_problem pb, double* pts_out);
/* Per-iteration trace: trial cost, damping used, accepted flag, for the
   first min(n, iters, 4096) iterations (the trace keeps the first 4096; the
   rest of each output is left untouched).  Any output pointer may be NULL. */
povar_status povar_get_trace(povar_problem pb, int32_t n, double* trial_cost,
                             double* lambda_used, int32_t* accepted);
/* Per-iteration diagnostics of the first stage, for the first
   min(n, iters, 4096) iterations (either pointer may be NULL): bl_norm, the 2-norm over all
   landmarks of b_l = sum_k J_l,k^T r_k at the trial cameras and their
   re-solved landmarks (zero up to rounding, since X* solves (8): the
   eliminated landmarks have zero gradient); series_seconds, the device time
   of that iteration's power series as in povar_report.seconds_series.
   Second-stage problems: POVAR_ESTATE. */
povar_status povar_get_trace_diag(povar_problem pb, int32_t n, double* bl_norm, double* series_seconds);

/* Checkpoint / resume: the state is (cameras, lambda, iteration count); the
   landmarks follow from the cameras by (8).  set_state re-solves them,
   re-evaluates the cost and forces a fresh linearisation.  On the sphere it
   normalises cameras whose squared norm differs from 1 by more than 1e-14
   and takes the others bit-exactly, so a state read by povar_get_state
   resumes bit-exactly. */
povar_status povar_get_state(povar_problem pb, double* cams_out, double* lambda_out,
                             int32_t* iter_out, double* cost_out);
povar_status povar_set_state(povar_problem pb, const double* cams, double lambda, int32_t iter);

/* ---- per-step hooks for parity tests ------------------------------------ */
/* Linearisation at the current cameras (Eq. (10)-(13)): U (n_cams x 144,
   row-major 12x12), b_p (n_cams x 12), g = b_p - W V^+ b_l (n_cams x 12),
   V^+ (n_pts x 9), X (n_pts x 3), z0 = V^+ b_l (n_pts x 3), and the cost.
   Points in the caller's order.  Any output pointer may be NULL. */
povar_status povar_debug_linearize(povar_problem pb, double* U, double* bp, double* g,
                                   double* Vpinv, double* X, double* z0, double* cost);
/* One camera step at the current linearisation with damping `lambda` and
   series order `order`, without changing the solver state: dp (n_cams x 12)
   is the ambient update (tangent on the sphere), p_trial the retracted
   cameras, cost_trial the cost after re-solving the landmarks there. */
povar_status povar_debug_step(povar_problem pb, double lambda, int32_t order, double* dp,
                              double* p_trial, double* cost_trial);
/* The damped camera block inverses at the current linearisation and damping
   `lambda`, without changing the solver state: K (n_cams x 144, host, caller's
   order, each block 12 x 12 row-major) receives K_i = B_i (B_i^T U_i,lambda
   B_i)^-1 B_i^T with B_i an orthonormal basis of the tangent space of camera
   i's unit sphere, i.e. the inverse of the camera block of Eq. (22) mapped
   back to the ambient space (Sec. 4.3); U_i,lambda = U_i + lambda diag(U_i)
   (Sec. 5.2), its diagonal floored at 1e-12 of its largest entry.  K_i =
   U_i,lambda^-1 in Euclidean mode.  Formed in FP64 in both precisions.
   POVAR_ESTATE on a finished or second-stage problem, POVAR_ENUMERIC (K of
   that camera zero) if a damped block could not be factored. */
povar_status povar_debug_camera_blocks(povar_problem pb, double lambda, double* K);
/* The truncated power series of Eq. (17) from a caller-supplied start, at
   the current linearisation and damping (the problem's lambda for its next
   step): x_out = sum_{t=0..order} M^t x0 with M = K W V^+ W^T, K the damped
   camera block inverse in the tangent space of each camera (Sec. 4.3; K =
   U_lambda^-1 in Euclidean mode).  x0 and x_out: n_cams x 12 ambient camera
   vectors (host, caller's order); x0 is used as given (the terms t >= 1 are
   tangent on the sphere).  The series precision is the problem's (an
   FP32-bulk problem rounds x0 to FP32 for its first term; x_out sums the
   terms in FP64); no early stop.  The solver state is kept.  POVAR_ESTATE on
   a finished or second-stage problem, POVAR_ENUMERIC if a damped camera
   block could not be factored. */
povar_status povar_debug_series(povar_problem pb, const double* x0, int32_t order, double* x_out);
/* Host only, no device needed: builds the device layout of a problem (same
   arguments as povar_problem_create) and checks it — every observation in
   exactly one packet entry, one camera-major position and, when the camera
   pass is landmark-blocked, one camera-slot entry; packet, chunk and slot
   headers consistent with their entries; run keys contiguous in each slot
   and run ids inside their camera's range; while every XCD has camera slots
   left, each slot's landmark block assigned to the XCD its workgroup runs
   on; the footprint from sizes alone at least the built layout's.  out[0..7] (if non-NULL): blocked, packet slots, chunks, camera
   slots, runs, landmarks per block, exact device bytes, footprint bound.
   POVAR_EINVAL with the reason in povar_last_error(NULL) on the first
   violated property or invalid input. */
povar_status povar_debug_layout_check(int32_t n_cams, int32_t n_pts, int64_t n_obs, const int32_t* cam_idx,
                                      const int32_t* pt_idx, const double* meas, int32_t precision,
                                      int64_t* out);

/* ---- second stage: projective refinement (RiPoBA) ----------------------- */
/* Objective (7) of Sec. 3 with the method of Sec. 4.3: the cameras (unit
   sphere of R^12) and the homogeneous landmarks (unit sphere of R^4) refined
   jointly by LM; each step solves the damped Riemannian normal equations
   (20)-(26) with the power series (29) of the inverse Riemannian Schur
   complement (27) for the cameras and back-substitution for the landmarks,
   then retracts both by normalisation.  Damping: Marquardt on the diagonal of
   each ambient camera / landmark block, then projected.
   cams0: n_cams x 12 (row-major 3x4), pts0: n_pts x 4 homogeneous, both in
   the caller's order (each row is normalised; host memory).  opts: precision
   POVAR_PREC_FP64, manifold POVAR_MANIFOLD_SPHERE; series_rtol as for the
   first stage (the early stop ends the camera series; the landmark update
   follows from the terms taken); the other fields as for
   povar_problem_create.  The handle works with povar_solve,
   povar_step, povar_enqueue, povar_get_report, povar_get_cameras,
   povar_get_trace, povar_get_state, povar_problem_info / _layout and
   povar_problem_destroy (povar_kernel_times counts no launches for it: the
   timing hooks bracket the first stage's series kernels); povar_get_points
   returns X / w per landmark, povar_get_points_h the unit 4-vectors.  The
   server does not take second-stage problems.  Errors: POVAR_EINVAL for
   invalid sizes, indices, options or non-finite / zero inputs, POVAR_ENOMEM,
   POVAR_EDEVICE, POVAR_ENUMERIC for a non-finite initial cost. */
povar_status povar_refine_create(povar_ctx ctx, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                 const int32_t* cam_idx, const int32_t* pt_idx, const double* meas,
                                 const double* cams0, const double* pts0, const povar_options* opts,
                                 povar_problem* out);
/* Homogeneous landmarks at the current point, n_pts x 4 in the caller's
   order: the unit 4-vectors of a second-stage problem, (X, 1) for a first-
   stage one. */
povar_status povar_get_points_h(povar_problem pb, double* out);
/* Test hooks of the second stage (each may be NULL; host arrays, caller's
   order).  povar_refine_debug_blocks: at the current point, U (n_cams x 144,
   undamped J_p^T J_p), b_p (n_cams x 12, J_p^T r), G (n_pts x 16, the ambient
   form B (B^T V_l B)^-1 B^T of the damped landmark block V_l at damping
   `lambda`, B a basis of the landmark's tangent space), b_l (n_pts x 4) and
   the cost (7).  povar_refine_debug_step: one step at `lambda` with series
   order `order` (the problem's state is kept): dp the ambient camera update
   (n_cams x 12), p_trial and x_trial (n_pts x 4) the retracted trial cameras
   and landmarks, cost_trial the cost there.  POVAR_ESTATE on a first-stage or
   finished problem; POVAR_ENUMERIC if a damped block could not be factored. */
povar_status povar_refine_debug_blocks(povar_problem pb, double lambda, double* U, double* bp, double* G,
                                       double* bl, double* cost);
povar_status povar_refine_debug_step(povar_problem pb, double lambda, int32_t order, double* dp, double* p_trial,
                                     double* x_trial, double* cost_trial);

/* ---- metric upgrade (autocalibration, supplement App. D) ----------------- */
/* From a projective reconstruction (for instance the refined cameras) and the
   cameras' known intrinsics, find H = [[A, 0], [c^T, 1]] such that every
   P_i H is a scaled K_i [R_i | t_i].  With Q_i = K_i^-1 P_i and H~ the three
   left columns of H, the plane at infinity c and the scales alpha_i minimise
   sum_i || alpha_i Q_i H~ H~^T Q_i^T - I ||_F^2: each alpha_i in closed form
   (variable projection), c by Levenberg-Marquardt on the reduced residual,
   in FP64 on the device.  The frame is first moved so that camera 0 is
   [I | 0], and A = K_0: camera 0 becomes K_0 [I | 0] and the metric frame is
   camera 0's, up to a global scale.  LM: Marquardt damping on diag(J^T J)
   (floored at 1e-12 of its largest entry), lambda0 = 1e-4, accept iff the
   cost decreases, lambda / 10 (>= 1e-12) on accept and x 10 on reject; stop
   when an accepted step lowers the cost by at most ftol (relative), when
   lambda reaches 1e12, or after max_iters iterations (attempted steps).

   cams: n_cams x 12 (row-major 3 x 4, any scale and sign per camera); K:
   n_cams x 9 (row-major, upper triangular, nonzero diagonal).  Outputs (each
   may be NULL): H (16, row-major 4 x 4; a projective point X maps to the
   metric frame as H^-1 X), c (3), alpha (n_cams), R (n_cams x 9, rotations:
   the orthogonal polar factor of K_i^-1 P_i H~ / s_i), t (n_cams x 3), with
   P_i H = s_i K_i [R_i | t_i], s_i = +-1/sqrt(alpha_i) of the sign that makes
   det R_i positive; trace_cost and trace_accept (max_iters each; the first
   report.iters entries are written) the trial cost and decision of every
   iteration.  Errors: POVAR_EINVAL (n_cams < 2, non-finite entries, a K that
   is not upper triangular with a nonzero diagonal, camera 0 with a singular
   left 3 x 3 block, max_iters outside [0, 2^20], ftol outside [0, 1)),
   POVAR_ENOMEM, POVAR_EDEVICE.  Device memory is allocated per call. */
typedef struct {
  double cost_initial; /* at c = 0 */
  double cost_final;
  double lambda;
  int32_t iters;
  int32_t stop;        /* 1: ftol, 2: lambda at its cap, 3: max_iters, 0: max_iters = 0 */
} povar_metric_report;

povar_status povar_metric_upgrade(povar_ctx ctx, int32_t n_cams, const double* cams, const double* K,
                                  int32_t max_iters, double ftol, double* H, double* c, double* alpha,
                                  double* R, double* t, double* trace_cost, int32_t* trace_accept,
                                  povar_metric_report* report);
/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   call as povar_metric_upgrade, with the same arguments, results and errors,
   but every device buffer of the call is carved from a static scratch array
   of 8 MiB per GPU instead of being allocated; it calls no hipMalloc or
   hipFree (nor any other allocating routine).  The call needs about
   n_cams x 368 + max_iters x 12 bytes (plus 80 bytes of partial sums per
   256 cameras and 256-byte alignment of each buffer), at most 8 MiB: up to
   22,700 cameras at 1,000 iterations; larger calls return POVAR_EINVAL with
   the bytes needed.
   The array of a GPU is shared by every call on it and keeps the last call's
   contents (each call initialises what it reads): calls that overlap on one
   GPU (two threads, or two contexts on one device) race and must not be
   issued.  POVAR_ESTATE if ctx was not made by povar_ctx_create. */
povar_status povar_metric_upgrade_noalloc(povar_ctx ctx, int32_t n_cams, const double* cams, const double* K,
                                          int32_t max_iters, double ftol, double* H, double* c, double* alpha,
                                          double* R, double* t, double* trace_cost, int32_t* trace_accept,
                                          povar_metric_report* report);
/* Test hook: the reduced problem at a given c (3 values): alpha (n_cams),
   J^T J (9, row-major 3 x 3), J^T r (3) and the cost. */
povar_status povar_metric_debug_reduced(povar_ctx ctx, int32_t n_cams, const double* cams, const double* K,
                                        const double* c, double* alpha, double* JtJ, double* Jtr, double* cost);

/* ---- kernel timing for roofline reports --------------------------------- */
/* enable != 0: subsequent povar_step / povar_enqueue launches bracket the
   two passes of every series order with HIP events recorded by the kernels'
   own dispatches on the context stream (graph replay is bypassed while
   enabled): the landmark pass, and the camera pass from the start of its
   chunk or slot kernel to the end of its last kernel (the combine kernel,
   where cameras have several partial sums).  povar_kernel_times returns the
   summed durations (ms) and counts of the two passes since timing was
   enabled and resets them. */
povar_status povar_kernel_timing(povar_problem pb, int32_t enable);
povar_status povar_kernel_times(povar_problem pb, double* ms_landmark_pass, int64_t* n_landmark_pass,
                                double* ms_camera_pass, int64_t* n_camera_pass);
/* Problem shape after layout: landmark-major packets (runs of whole
   landmarks of at most 64 observations), camera-major chunks (at most 2048
   observations of one camera), device bytes.  In a problem with a camera of
   more than 8 chunks, each accepted step adds every camera's chunk partials
   of the linearisation with one wave per camera (one more kernel) instead of
   one lane per camera, in the same order: the same sums, bit for bit. */
povar_status povar_problem_info(povar_problem pb, int64_t* n_obs, int64_t* n_packets,
                                int32_t* n_chunks, uint64_t* device_bytes);
/* Series camera pass of the problem.  *blocked = 0: one workgroup per camera
   chunk, landmark records gathered from anywhere (the records fit in L2).
   *blocked = 1 (records of the series precision above 4 MiB): landmarks in
   blocks of *lm_block internal ids (2 MiB of records), *n_slots 64-lane
   slots of 8 (FP32-bulk) or 4 (FP64) observations per lane, each block's
   slots run on one XCD, and *n_runs per-(camera, block
   part) partial sums added per camera afterwards.  *coop_gather = 1 when the
   landmark pass gathers the cameras' series records cooperatively, whole
   waves reading consecutive pieces of a few records: every FP64 problem, and
   FP32-bulk problems whose records are a full 128-byte line apart (more
   than 341 cameras).
   NULL outputs are skipped. */
povar_status povar_problem_layout(povar_problem pb, int32_t* blocked, int32_t* lm_block, int64_t* n_slots,
                                  int64_t* n_runs, int32_t* coop_gather);

/* ---- serving: continuous batching of many problems on one GPU ----------- */
/* A server owns a worker thread, an admission thread and the device state of
   up to max_slots problems whose summed footprint stays within
   hbm_budget_bytes. Requests wait in a FIFO queue until a slot and enough
   budget are free. Admitted problems form groups by precision and by size
   (up to 250,000 observations, or more); each group advances one LM
   iteration per batched launch sequence on a stream of its own, so small
   problems are not held to the pace of large ones. An admission thread
   initialises admitted requests (device allocation, upload, initial landmark
   solve) on a stream of its own while the groups' iterations run; an
   initialised problem joins its group before the group's next launch. A
   finished problem's result is copied out at once; its device memory (still
   counted against the budget) is freed when no group has work in flight, or,
   when a queued request needs that memory, after the groups in flight finish
   their current iterations. Each result is independent of which other
   problems shared the launches. */
povar_status povar_server_create(povar_ctx ctx, uint64_t hbm_budget_bytes, int32_t max_slots,
                                 povar_server* out);
/* Copies the request; *ticket identifies it.  cams0 may be NULL (seeded
   cameras from opts->init_seed, as for povar_problem_create).  POVAR_ENOMEM
   if the request alone exceeds the budget; POVAR_EINVAL as for
   povar_problem_create. */
povar_status povar_server_submit(povar_server sv, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                                 const int32_t* cam_idx, const int32_t* pt_idx, const double* meas,
                                 const double* cams0, const povar_options* opts, uint64_t* ticket);
/* POVAR_EAGAIN until the request has finished; then fills the report, the
   cameras (n_cams x 12) and points (n_pts x 3) if non-NULL, and releases the
   ticket.  Timestamps (seconds since server creation) of the submit call's
   entry (before its layout build), admission and completion go to
   times[0..2] if times is non-NULL. */
povar_status povar_server_poll(povar_server sv, uint64_t ticket, povar_report* report,
                               double* cams_out, double* pts_out, double* times);
/* Statistics: requests queued, active, finished; batched iterations run
   (summed over the groups). */
povar_status povar_server_stats(povar_server sv, int32_t* queued, int32_t* active,
                                int64_t* finished, int64_t* batch_iters);
/* Where the server's time went (seconds since creation, each may be NULL):
   seconds[0] the admission thread initialising requests (device allocation,
   layout upload, initial landmark solve), [1] the worker enqueueing batched
   launches, [2] waiting for the GPU while no group's read-back had arrived,
   [3] retiring finished problems and freeing their memory; counts[0] batched
   iterations summed over the groups, [1] control-block read-backs (a group
   enqueues up to four iterations per read-back while none of its problems
   can reach its iteration limit and no admitted request waits to join it),
   [2] requests whose admission the HBM budget deferred. */
povar_status povar_server_profile(povar_server sv, double* seconds, int64_t* counts);
/* Waits for the worker to drain nothing: pending requests are dropped. */
povar_status povar_server_destroy(povar_server sv);

#ifdef __cplusplus
}
#endif
#endif /* POVAR_H */
