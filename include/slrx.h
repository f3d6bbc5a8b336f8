/*
 * slrx -- structured low-rank recovery of damped-exponential image series on
 * AMD MI355X (gfx950).  C ABI.
 *
 * Method: Balachandrasekaran, Magnotta, Jacob, "Recovery of damped exponentials
 * using structured low rank matrix completion" (arXiv 1704.04511).  The
 * library runs the IRLS loop of Algorithm 1 on one GPU:
 *   step 1 (Sec. III.B): Gram matrix R of the multi-fold Toeplitz lifting of
 *     the k-space samples, formed by Fourier autocorrelation of the images
 *     (eq. "eq:block-expression for R", eq. "eq:P_ij modified"); its FP64
 *     eigen-decomposition; weights alpha_i = (lambda_i + eps)^(p/2-1); the
 *     summed filter power spectra as per-pixel penalty masks (Sec. III.A);
 *   step 2 (Sec. III.A, eq. "eq:grad_ls"): a fixed number of conjugate-gradient
 *     iterations on (S + lam F G F^H) x = S b;
 *   then eps <- eps / gamma (Sec. III.C).
 *
 * Conventions
 *   - k-space and images are complex64 (interleaved re, im float) arrays
 *     [T][P][Q], frame-major, row-major frames, DC at index [0][0].  F is the
 *     unitary 2-D DFT; images = F^-1 x per frame.
 *   - Masks are uint8 [T][P][Q] with values 0 or 1 (nonzero counts as 1).
 *   - lam is the penalty weight per least-squares step:
 *     min ||S x - b||^2 + lam J(x);  lam = 2/(mu p) for the paper's mu.
 *   - Filter support N1 x N2 x M (spatial x spatial x taps); s = N1 N2 M.
 *   - Supported frame sizes P, Q in {8,16,32,64,96,128,160,192,256};
 *     1 <= M <= min(T, 8); T <= 32; 1 <= N1 <= P; 1 <= N2 <= Q;
 *     s = N1 N2 M <= 3000 (the size the eigensolver chain handles).
 *
 * Ownership and errors
 *   - The library owns every device buffer it allocates.  Host inputs are
 *     copied before the call returns.  Device inputs (SLRX_MEM_DEVICE) are
 *     read on the plan's stream in stream order; they must stay valid until
 *     the next slrx_sync on that plan.
 *   - Every call returns an slrx_status; no C++ exception crosses the ABI.
 *     Argument validation happens before any device work and is testable
 *     without a GPU.  slrx_last_error(plan) returns the message of the plan's
 *     last failed call, slrx_last_error(NULL) that of the calling thread's.
 *   - One plan is used by one thread at a time; different plans may run
 *     concurrently on different streams.
 */
#ifndef SLRX_H
#define SLRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLRX_OK = 0,
  SLRX_EINVAL = -1,      /* invalid argument or unsupported size */
  SLRX_ENOMEM = -2,      /* device allocation failed or budget exceeded */
  SLRX_EDEVICE = -3,     /* HIP / rocSOLVER error */
  SLRX_ESTATE = -4,      /* call not allowed in the plan's current state */
  SLRX_ENUMERIC = -5,    /* eigen-decomposition failed or non-finite values */
  SLRX_EBUSY = -6,       /* plan is running */
  SLRX_ENOTREADY = -7,   /* no completed run / request not finished */
  SLRX_ECANCELED = -8,   /* server request canceled before admission */
  SLRX_ETIMEDOUT = -9    /* server request waited longer than the queue timeout */
} slrx_status;

typedef enum { SLRX_MEM_HOST = 0, SLRX_MEM_DEVICE = 1 } slrx_mem;

/* Problem dimensions: T frames of P x Q; filter support N1 x N2 x M. */
typedef struct {
  int32_t P, Q, T;
  int32_t N1, N2, M;
} slrx_dims;

/* Algorithm parameters.  lambda >= 0; p in [0, 1] (Schatten exponent,
 * Sec. II.D); gamma > 1 (eps decrease, Sec. III.C); eps0_frac > 0
 * (eps^(0) = eps0_frac * lambda_max of the first Gram matrix); n_irls >= 1
 * outer iterations; n_cg >= 0 CG iterations per outer iteration. */
typedef struct {
  double lambda, p, gamma, eps0_frac;
  int32_t n_irls, n_cg;
  uint32_t flags; /* SLRX_FLAG_* */
} slrx_params;

#define SLRX_FLAG_TIMING 1u /* record per-phase device times (hipEvents) */
#define SLRX_FLAG_KTIME 2u  /* record every launch of each kernel class (hipEvents) */
#define SLRX_FLAG_LIBEIGH 4u /* test reference only: the eigen-decomposition by rocSOLVER
                                zheevd instead of the library's own chain (Householder
                                tridiagonalisation, divide and conquer, back-transformation),
                                to check the latter against an independent solver; its
                                handle and workspace are allocated at the first such run,
                                outside slrx_footprint; servers reject it */
#define SLRX_FLAG_GIRAF 8u  /* the GIRAF approximation the paper compares with (Sec. IV,
                               Fig. 3): the lifting circular along the parameter axis
                               as well as in space (all T shifts, frame indices mod T)
                               in the Gram matrix and the penalty; default: the hybrid
                               lifting, linear along the parameter axis (Sec. III.A) */
#define SLRX_FLAG_NO_GRAPH 32u /* launch the CG kernels one by one; default for a plan run
                                 alone (slrx_run, slrx_step_cg): the CG of every
                                 least-squares step (initial residual and n_cg iterations)
                                 is captured once per plan as a HIP graph and replayed (same
                                 kernels, same results), except when a CG kernel class is
                                 timed under SLRX_FLAG_KTIME; lock-step batches and servers
                                 launch one by one (graph launches on their many
                                 concurrent streams measured slower) */
#define SLRX_FLAG_HLR_VOXEL 64u /* the pixel-wise Hankel low-rank prior the paper compares with
                                  (HLR-Voxel; Sec. II.E, eq. "eq: MORASA-objective", solved by
                                  IRLS, Sec. IV): every pixel's series gets its own
                                  (T-M+1) x M Toeplitz matrix T_r and its own weight
                                  H_r = (T_r^H T_r + eps I)^(p/2-1) (eigenvalues clamped at 0),
                                  the penalty is sum_r ||T_r H_r^(1/2)||_F^2, and eps^(0) is
                                  eps0_frac times the largest eigenvalue over all pixels.
                                  Requires N1 = N2 = 1 (a filter of M taps per pixel); not
                                  combinable with SLRX_FLAG_GIRAF or SLRX_FLAG_LIBEIGH.  There
                                  is no global Gram matrix: slrx_step_gram and the lam / H
                                  outputs of slrx_step_weights are rejected */
#define SLRX_FLAG_DIRECT 128u /* IRLS-direct, the method without the FFT-based approximations
                                 that the paper compares with (Sec. IV, Fig. 2): the lifting
                                 linear in all three dimensions (k-space in centred order,
                                 DC at (P/2, Q/2); rows n = M-1..T-1 and the
                                 (P-N1+1)(Q-N2+1) shifts whose N1 x N2 support lies inside
                                 the grid), R = T^H T from the explicit lifted matrix
                                 (complex128) and the least-squares operator
                                 S + lam T^*(T(.) H) on the explicit lifted matrix of the
                                 CG direction (complex64), the same eps schedule.  Memory:
                                 16 + 2 x 8 bytes per lifted-matrix entry
                                 ((T-M+1)(P-N1+1)(Q-N2+1) x s entries) plus 8 s^2, allocated
                                 at the first run outside slrx_footprint, and a rocBLAS
                                 handle.  Single-channel only; not combinable with
                                 SLRX_FLAG_GIRAF, SLRX_FLAG_HLR_VOXEL or SLRX_FLAG_LIBEIGH;
                                 servers reject it; the single-step entry points other than
                                 slrx_step_tdeig reject direct plans */
/* With SLRX_FLAG_KTIME: time only the classes whose bits are set here (none set:
 * every class).  Each timed region adds two events to the stream. */
#define SLRX_FLAG_KTIME_CLASS(c) (1u << (16 + (c)))

/* Kernel classes timed under SLRX_FLAG_KTIME. */
enum {
  SLRX_K_ROWS = 0,    /* inverse row pass of the CG operator (fused p update) */
  SLRX_K_COLS = 1,    /* column pass: inverse column DFT, penalty G (plus the coil
                         combination with coil maps), forward column DFT */
  SLRX_K_FIN = 2,     /* forward row pass + data term S o v + dot */
  SLRX_K_UPDATE = 3,  /* CG vector update + residual norm */
  SLRX_K_GRAM = 4,    /* Gram matrix (lagged products, pruned DFT, window) */
  SLRX_K_TRI = 5,     /* Householder tridiagonalisation (one launch per column) */
  SLRX_K_TDEIG = 6,   /* eigenpairs of the real tridiagonal (divide and conquer), or the
                         whole library eigen-decomposition with SLRX_FLAG_LIBEIGH */
  SLRX_K_BACKTR = 7,  /* blocked back-transformation U = Q Z */
  SLRX_K_FILTER = 8,  /* weights + filter product H = U diag(alpha) U^H */
  SLRX_K_MASKS = 9,   /* diagonal sums + mask synthesis */
  SLRX_K_COIL = 10,   /* multichannel data term (with coil maps only): coil images
                         and their forward DFT, sampling mask, inverse DFT and
                         coil combination */
  SLRX_K_VOXEL = 11,  /* SLRX_FLAG_HLR_VOXEL: per-pixel Gram matrices, eigen-decompositions
                         and masks, and the eps schedule on their eigenvalues */
  SLRX_K_DIRECT = 12, /* SLRX_FLAG_DIRECT: the CG of each least-squares step on the explicit
                         lifting (lifting, GEMM with H, adjoint, vector updates) */
  SLRX_K_NCLASS = 13
};

/* Per-run statistics, filled by slrx_get_stats after a completed run. */
#define SLRX_MAX_IRLS 256
typedef struct {
  int32_t n_irls_done;
  double eps[SLRX_MAX_IRLS];        /* eps used by each outer iteration */
  double lambda_max[SLRX_MAX_IRLS]; /* largest Gram eigenvalue per iteration */
  double cg_rr_final[SLRX_MAX_IRLS];/* squared CG residual norm after each LS step */
  double ms_total;                  /* device time of the whole run (ms) */
  double ms_gram, ms_eigh, ms_weights, ms_cg; /* per phase, SLRX_FLAG_TIMING */
  double kt_ms[16];      /* summed durations per class (index SLRX_K_*), SLRX_FLAG_KTIME */
  int32_t kt_count[16];  /* timed regions per class (a region may hold several launches) */
} slrx_stats;

typedef struct slrx_plan slrx_plan;
typedef struct slrx_server slrx_server;

/* Default parameters: p = 0.6, gamma = 1.4, eps0_frac = 0.01, lambda = 1e-3,
 * n_irls = 15, n_cg = 10, flags = 0. */
void slrx_default_params(slrx_params* out);

/* Validate dims/params without touching the device.  SLRX_OK or SLRX_EINVAL. */
slrx_status slrx_validate(const slrx_dims* dims, const slrx_params* params);

/* Device bytes a plan of these dims allocates (its buffer arena; a server adds
 * the request's share of the engine's eigen-decomposition buffers). */
size_t slrx_footprint(const slrx_dims* dims);

/* Create a plan on the current HIP device.  hip_stream: a hipStream_t to run
 * on, or NULL for a stream owned by the plan.  Allocates all device state. */
slrx_status slrx_plan_create(const slrx_dims* dims, const slrx_params* params,
                             void* hip_stream, slrx_plan** out);
void slrx_plan_destroy(slrx_plan* plan);

/* Inputs.  b: complex64 [T][P][Q] sampled k-space (entries off the mask are
 * ignored);  S: uint8 [T][P][Q];  x0: optional complex64 k-space initial
 * guess (default x0 = S o b, the zero-filled data; Algorithm 1 init). */
slrx_status slrx_set_kspace(slrx_plan* plan, const void* b, slrx_mem mem);
slrx_status slrx_set_mask(slrx_plan* plan, const uint8_t* S, slrx_mem mem);
slrx_status slrx_set_init(slrx_plan* plan, const void* x0, slrx_mem mem);
slrx_status slrx_clear_init(slrx_plan* plan);
/* Multichannel measurements (the model of Sec. II.A, eq. "measurement_ij"):
 * frame i of coil j is sampled as b_ij = S_i F C_j F^* rho_hat_i + noise, with
 * C_j a pointwise image-domain sensitivity shared by all frames and S_i the
 * frame's mask (slrx_set_mask) shared by all coils.  The reconstruction then
 * solves (A^H A + lam F G F^*) rho_hat = A^H b in every least-squares step and
 * starts from A^H b = sum_j F C_j^* F^* (S o b_j) (or x0).
 *   ncoils: 1..SLRX_MAX_COILS, or 0 to return to the single-channel model
 *           (b of slrx_set_kspace; C and b are then ignored);
 *   C: complex64 [ncoils][P][Q] sensitivities, row-major frames;
 *   b: complex64 [ncoils][T][P][Q] coil k-space, DC at [0][0] (entries off
 *      the mask are ignored).
 * Copies both (host or device memory per mem).  Allocates 8 (ncoils P Q +
 * (2 ncoils + 1) T P Q) + 16 (ncoils + min(ncoils, 4)) T P Q bytes of device
 * memory beyond slrx_footprint (the adjoint half of the coil data term runs in
 * complex128), released by
 * slrx_plan_destroy or a later call.  SLRX_EINVAL for ncoils out of range,
 * NULL pointers or a bad mem; SLRX_EBUSY while the plan runs.  Plans with coils
 * can be run alone or in slrx_run_batch; servers take single-channel requests. */
#define SLRX_MAX_COILS 32
slrx_status slrx_set_coils(slrx_plan* plan, int32_t ncoils, const void* C, const void* b, slrx_mem mem);
/* Change the filter support; N1 N2 M must not exceed the sizes the plan was
 * created with (buffers are sized at creation).  Algorithm parameters: */
slrx_status slrx_set_filter(slrx_plan* plan, int32_t N1, int32_t N2, int32_t M);
slrx_status slrx_set_params(slrx_plan* plan, const slrx_params* params);

/* Enqueue the whole reconstruction on the plan's stream.  The FP64
 * eigen-decomposition may synchronise the stream internally. */
slrx_status slrx_run(slrx_plan* plan);
/* Wait for the plan's work; reports numerical failures of the run. */
slrx_status slrx_sync(slrx_plan* plan);

/* Outputs (after slrx_sync): images F^-1 x and k-space x, complex64 [T][P][Q]. */
slrx_status slrx_get_images(slrx_plan* plan, void* out, slrx_mem mem);
slrx_status slrx_get_kspace(slrx_plan* plan, void* out, slrx_mem mem);
slrx_status slrx_get_stats(slrx_plan* plan, slrx_stats* out);

/* Mono-exponential fit per pixel (Sec. IV: T2 maps are obtained by fitting a
 * mono-exponential model to every pixel of the reconstructed series): the
 * least-squares line through log|rho_t| (|rho| floored at 1e-30) against the
 * echo times, in FP64.
 *   img: complex64 [T][P][Q] series, or NULL for the plan's reconstruction
 *        (after slrx_sync of a completed run);
 *   te_ms: T echo times, host memory (T2 comes out in the same unit);
 *   t2_out: float64 [P][Q]: -1/slope where the slope is negative, +inf otherwise;
 *   amp_out: float64 [P][Q] amplitude exp(intercept at TE = 0), or NULL.
 * img and the outputs are host or device memory per mem.  Overwrites the
 * plan's image and CG scratch buffers (the reconstruction itself, x, is kept).
 * SLRX_EINVAL for T < 2, equal or non-finite echo times or NULL pointers;
 * SLRX_ENOTREADY without img before a completed run; SLRX_EBUSY while running. */
slrx_status slrx_fit_t2(slrx_plan* plan, const void* img, const double* te_ms, double* t2_out, double* amp_out,
                        slrx_mem mem);

/* Run several independent plans.  hip_stream NULL: in lock step, one outer
 * iteration of every plan per step; plans with equal Gram size s share one
 * launch sequence of the eigen-decomposition (every kernel covers all of them,
 * each with the arithmetic of a single plan), every other kernel runs on the
 * plan's own stream.  A plan's result is bit-identical to slrx_run on that
 * plan (plans using the library eigensolver take their own path).  With
 * hip_stream: the plans run back to back on it, each as slrx_run would.
 * Returns once the work is enqueued; call slrx_sync on each plan. */
slrx_status slrx_run_batch(slrx_plan* const* plans, int32_t n, void* hip_stream);

/* --- single steps of the loop, for testing each step against a reference --- */
/* Images F^-1 x of the plan's current iterate (complex64 [T][P][Q]). */
/* Gram matrix of the current iterate: complex128 s x s, column-major. */
slrx_status slrx_step_gram(slrx_plan* plan, void* R_out, slrx_mem mem);
/* Weight update from the current iterate with a given eps: eigenvalues
 * (ascending, s doubles), filter product H = U diag(alpha) U^H (complex128
 * s x s, row-major) and penalty masks E (complex64 [W][P][Q], W = M(M+1)/2,
 * pairs m <= m' in row-major upper-triangle order).  Any output may be NULL. */
slrx_status slrx_step_weights(slrx_plan* plan, double eps, double* lam_out,
                              void* H_out, void* E_out, slrx_mem mem);
/* Eigenpairs of the real symmetric tridiagonal matrix with diagonal D (s
 * doubles) and off-diagonal E (s - 1 doubles), s = N1 N2 M of the plan, by the
 * divide-and-conquer stage of the weight update: lam_out gets the s
 * eigenvalues ascending, Z_out the eigenvectors as complex128, column-major
 * s x s, imaginary parts 0.  SLRX_EINVAL if s > 3000. */
slrx_status slrx_step_tdeig(slrx_plan* plan, const double* D, const double* E, double* lam_out,
                            void* Z_out, slrx_mem mem);
/* Apply the normal operator to k-space v with masks E (complex64 [W][P][Q]):
 * out = S o v + lam F G F^H v, complex64 k-space. */
slrx_status slrx_step_apply(slrx_plan* plan, const void* E, const void* v,
                            void* out, slrx_mem mem);
/* Run n_cg CG iterations from the current iterate with given masks E. */
slrx_status slrx_step_cg(slrx_plan* plan, const void* E, int32_t n_cg);

/* --- continuous-batching server ------------------------------------------
 * Requests queue in arrival order and are admitted (first fit) between
 * engine steps, when fewer than max_slots requests are active and their
 * device footprint (slrx_footprint) fits the remaining budget_bytes.  One
 * scheduler thread advances every active request by one outer iteration per
 * step, exactly as slrx_run_batch does; a request arriving while others run
 * joins at the next step.  A request's result is bit-identical to slrx_run on
 * the same data.  A request is charged its plan's footprint plus its share of
 * the engine's shared eigen-decomposition buffers (about 72 s^2 bytes for Gram
 * size s); the budget bounds every device byte the server holds: running
 * requests, idle plans kept for reuse, and engine buffers left from earlier
 * steps (freed when an admission needs the room).  Every request runs on a
 * stream of its own and the engine's on another, so hip_stream is ignored.
 * Thread-safe: any thread may submit, poll, wait, cancel or fetch. */
typedef struct {
  double t_submit, t_admit, t_done; /* steady-clock seconds */
  int32_t state;                    /* 0 queued, 1 running, 2 done */
  int32_t status;                   /* slrx_status of a finished request */
  size_t bytes;                     /* footprint charged against the budget */
} slrx_request_info;

slrx_status slrx_server_create(size_t budget_bytes, int32_t max_slots,
                               void* hip_stream, slrx_server** out);
/* Cancels queued requests (SLRX_ECANCELED), waits for running ones and for
 * threads inside slrx_wait to return, frees server-owned state. */
void slrx_server_destroy(slrx_server* srv);
/* Submit an existing plan (k-space and mask set); it is run in place and its
 * footprint is charged while it runs.  The plan must not be used until done;
 * SLRX_EBUSY if it is already queued or running on this server, SLRX_EINVAL
 * for a plan with SLRX_FLAG_LIBEIGH. */
slrx_status slrx_submit(slrx_server* srv, slrx_plan* plan, uint64_t* ticket);
/* Submit host data; at admission the server takes an idle plan of the same
 * shape or creates one (allocating its device state), keeps it resident while
 * the request runs, and on completion copies the images to host memory
 * (slrx_fetch_images) and releases the request's budget share; the plan stays
 * idle for reuse until the budget is needed.  Fails with SLRX_ENOMEM if the
 * footprint alone exceeds the budget. */
slrx_status slrx_submit_data(slrx_server* srv, const slrx_dims* dims, const slrx_params* params,
                             const void* b_host, const uint8_t* S_host, uint64_t* ticket);
slrx_status slrx_poll(slrx_server* srv, uint64_t ticket, int32_t* done);
/* Block until the request is done; returns its status. */
slrx_status slrx_wait(slrx_server* srv, uint64_t ticket);
/* As slrx_wait, but returns SLRX_ENOTREADY if the request is not done within
 * timeout_s seconds (>= 0; 0 polls). */
slrx_status slrx_wait_for(slrx_server* srv, uint64_t ticket, double timeout_s);
/* Cancel a queued request: it completes with SLRX_ECANCELED.  SLRX_EBUSY if it
 * is already running (it then runs to completion), SLRX_ESTATE if done. */
slrx_status slrx_cancel(slrx_server* srv, uint64_t ticket);
/* Requests not admitted within `seconds` of their submission complete with
 * SLRX_ETIMEDOUT (0, the default: no limit).  Checked by the scheduler at
 * least every seconds / 4. */
slrx_status slrx_server_set_queue_timeout(slrx_server* srv, double seconds);
slrx_status slrx_get_request_info(slrx_server* srv, uint64_t ticket, slrx_request_info* out);
/* Device bytes the server holds (running requests, idle plans kept for reuse
 * by later requests of the same shape, engine buffers beyond the running
 * requests' shares; idle plans are evicted and engine buffers trimmed when a
 * request needs the room) and number of queued requests. */
slrx_status slrx_server_usage(slrx_server* srv, size_t* used, int32_t* queued);
/* Copy a done server-owned request's images (complex64 [T][P][Q]) to host memory. */
slrx_status slrx_fetch_images(slrx_server* srv, uint64_t ticket, void* out_host);
/* Forget a done request, freeing whatever it still holds. */
slrx_status slrx_release(slrx_server* srv, uint64_t ticket);

/* --- launch configuration tuning -----------------------------------------
 * The library times the candidate launch configurations of its kernels on the
 * first calls for each shape and keeps the fastest (only configurations that
 * leave results bit for bit unchanged are tuned; the calls made while tuning
 * are ordinary calls).  With the environment variable SLRX_TUNE_CACHE naming a
 * file, choices are appended to it and read back by later processes.
 * slrx_tri_workgroup_budget: the workgroups per column launch chosen for the
 * tridiagonalisation of nbatch problems of Gram size n (decompositions run
 * together in a batch), or 0 while that shape is still being tuned. */
int32_t slrx_tri_workgroup_budget(int32_t n, int32_t nbatch);

/* --- the normal operator without allocation ------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * out = S o v + lambda F G F^-1 v, the operator of slrx_step_apply, without a
 * plan: dims gives P, Q, T and M (N1, N2 are not used); S uint8 [T][P][Q], E
 * the masks complex64 [W][P][Q] (W = M(M+1)/2, pairs m <= m' in row-major
 * upper-triangle order), v and out complex64 [T][P][Q] k-space; every pointer
 * is device memory, read and written on hip_stream (NULL: the default stream)
 * in stream order; the call returns once the work is enqueued.  flags: 0 or
 * SLRX_FLAG_GIRAF.  Its scratch (the transposed volume and masks, twiddles,
 * partial sums) is one device array inside the library, held by each GPU it
 * runs on until the process ends: 8 (T P Q + W P Q) bytes (each rounded up to
 * 256) must not exceed slrx_apply_noalloc_limit() = 24 MiB, else SLRX_EINVAL.
 * The call makes no device allocation.  Calls on one GPU share that array, so
 * calls that overlap on one GPU (different streams, different threads) race;
 * nothing in it has to start at zero.  Same errors as slrx_validate for the
 * sizes, SLRX_EINVAL for NULL pointers or bad flags. */
size_t slrx_apply_noalloc_limit(void);
slrx_status slrx_apply_noalloc(const slrx_dims* dims, double lambda, uint32_t flags, const uint8_t* S,
                               const void* E, const void* v, void* out, void* hip_stream);

const char* slrx_status_str(slrx_status s);

/* Test hook (fault injection): the n-th device allocation of the library from now
 * on (0 = the next one) fails as if the device were out of memory, without
 * allocating; the call that made it returns SLRX_ENOMEM and leaves the object
 * it was allocating for unchanged or destroyed.  n < 0 switches it off.  The
 * environment variable SLRX_FAULT_ALLOC=n does the same from the first
 * allocation of the process.  Other environment variables: SLRX_LOG (print every
 * failure to stderr), SLRX_TUNE_CACHE (the tuner's cache file). */
void slrx_fault_alloc(int32_t n);

/* CG strategy of lock-step batches and servers (process-wide): -1 (default)
 * picks, per step shape, by timing both on the first steps (online tuner, after
 * the tridiagonalisation's launch shape is settled); 0 runs each problem's CG
 * on its own stream; 1 runs the CG of all single-channel problems of a step
 * that share the tap count M and the CG count in one launch per pass.  Results
 * are bit-identical either way. */
void slrx_set_cg_grouping(int32_t mode);
/* Message of the last failed call on `plan`, or of the calling thread's last
 * failed call when plan is NULL ("" if none).  Valid until the next call. */
const char* slrx_last_error(const slrx_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* SLRX_H */
