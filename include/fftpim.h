/*
 * fftpim.h - C ABI of the MI355X FFT-PIM apply.
 *
 * The FFT periodic interpolation method (Ai & Lomakin) evaluates the periodic
 * scalar potential of Sec. 2, Eq. (1),
 *
 *     u(r_m) = sum_n G^p(r_m - r_n) q_n ,
 *
 * with G^p the 1D/2D/3D periodic Green's function of Eq. (2) built from
 * G0(r) = exp(-j k0 |r|) / (4 pi |r|) and image phases exp(-j k_t . R_i).
 * The sum is split into a near zone and a far zone (Sec. 3.1, Eq. (4)-(5)):
 *   far zone  (Sec. 3.2): projection onto a sparse source grid, a dense grid
 *             sum with the far-image kernel (Eq. (8)), interpolation from the
 *             shifted observer grid;
 *   near zone (Sec. 3.3): projection onto one dense grid, a zero-padded FFT
 *             convolution with the tabulated near-image kernel, interpolation,
 *             and the error correction of Eq. (er) over close source/observer
 *             pairs and their close images.
 *
 * Conventions shared by every entry point:
 *   - All pointers named *_dev are device pointers (hipMalloc'ed or torch CUDA
 *     tensors); host pointers are named otherwise.
 *   - Positions are double [n][3] (x, y, z interleaved), in the zeroth cell:
 *     0 <= x_c < L_c on every periodic axis c.
 *   - Amplitudes/potentials are right-hand-side major: q[r][n], r < nrhs.
 *     Element type: double / float (FFTPIM_REAL) or interleaved complex
 *     (re, im) double / float (FFTPIM_COMPLEX), per the plan's precision.
 *   - Nothing is copied back to the host by an apply: work is enqueued on the
 *     given stream and the call returns.  Errors found on the device (e.g. a
 *     non-neutral right-hand side of a static no-phase problem) are latched
 *     and reported by fftpim_last_status.
 *   - Every function returns an fftpim_status (0 = success); no exception or
 *     longjmp crosses the ABI (an unexpected internal C++ exception is
 *     reported as FFTPIM_ERR_DEVICE).
 *   - Applies on one plan share its workspace: enqueue them on one stream, or
 *     use one plan per stream.
 */
#ifndef FFTPIM_H
#define FFTPIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fftpim_plan_s* fftpim_plan_t;
typedef void* fftpim_stream_t; /* a hipStream_t; NULL = the null stream */

typedef enum {
  FFTPIM_OK = 0,
  FFTPIM_ERR_INVALID_ARG = 1,  /* null pointer, bad size or parameter */
  FFTPIM_ERR_OUT_OF_CELL = 2,  /* a point outside [0, L) on a periodic axis,
                                  or outside the given box elsewhere */
  FFTPIM_ERR_NOT_NEUTRAL = 3,  /* static no-phase problem with sum(q) != 0 */
  FFTPIM_ERR_WOOD_ANOMALY = 4, /* a Floquet wavenumber vanishes (Sec. 2) */
  FFTPIM_ERR_UNSUPPORTED = 5,  /* a combination the library does not handle */
  FFTPIM_ERR_NO_MEMORY = 6,    /* a device or host allocation failed, a host
                                  thread could not be started, or the plan
                                  would exceed params.max_bytes */
  FFTPIM_ERR_DEVICE = 7,       /* a HIP runtime call failed */
  FFTPIM_ERR_UNIMPLEMENTED = 8,
  FFTPIM_ERR_SCRATCH_LIMIT = 9 /* fftpim_apply_pair_noalloc: the plan needs more
                                  than its fixed per-device array */
} fftpim_status;

/* Precision of the bulk path (the correction values and their products stay
 * FP64 in every mode).  FFTPIM_F32_FARBF16: FP32 everywhere except the far
 * grid sum of Eq. (8), which rounds the far-kernel table values and the grid
 * amplitudes to bfloat16 and accumulates in FP32 on the matrix cores (with at
 * least 8 planes; fewer planes use the FP32 grid sum).  FFTPIM_F32_FARBF16X3:
 * the same with each input split into two bfloat16 parts and three products
 * per term (about 16 significant bits). */
enum { FFTPIM_F64 = 0, FFTPIM_F32 = 1, FFTPIM_F32_FARBF16 = 2, FFTPIM_F32_FARBF16X3 = 3 };
enum { FFTPIM_REAL = 0, FFTPIM_COMPLEX = 1 };     /* element type of q and u */
/* Self term (Eq. (1) sums over every n, Eq. (5) writes n != m):
 * FFTPIM_SELF_IMAGES drops only the singular zeroth image of the n = m term,
 * so the images of a point act on itself (what the grid pipeline computes);
 * FFTPIM_SELF_EXCLUDE drops the whole n = m term: every apply (and every
 * part mask of fftpim_apply_parts) also subtracts C_self q_m, with C_self =
 * fftpim_eval_pgf_self, and the conjugate transpose conj(C_self) v_m. */
enum { FFTPIM_SELF_IMAGES = 0, FFTPIM_SELF_EXCLUDE = 1 };
enum { FFTPIM_ORDER_USER = 0, FFTPIM_ORDER_PLAN = 1 };
enum { FFTPIM_PART_NEAR_GRID = 1, FFTPIM_PART_NEAR_CORR = 2, FFTPIM_PART_FAR = 4,
       FFTPIM_PART_ALL = 7 };

/* The problem of Sec. 2: periodicity, periods, free-space wavenumber k0
 * (0 = static) and phase-shift wavenumbers k_x0, k_y0, k_z0, each possibly
 * complex (Sec. 2 allows a complex phase shift; a lossy medium has
 * Im k0 < 0 under the exp(-j k0 r) convention).  Complex values are given as
 * separate real and imaginary parts; zero-initialised imaginary parts give
 * the real problem. */
typedef struct {
  int periodic_dims;   /* 1: x; 2: x, y; 3: x, y, z */
  double L[3];         /* periods (entries beyond periodic_dims ignored) */
  double k0;           /* free-space wavenumber, real part (>= 0) */
  double kt[3];        /* phase-shift wavenumbers, real parts (beyond periodic_dims ignored) */
  int has_box;         /* 1: use box_lo/box_hi on the non-periodic axes, */
  double box_lo[3];    /* else the bounding box of the points (target region */
  double box_hi[3];    /* D of Sec. 3.2) */
  double k0_im;        /* imaginary part of k0 (<= 0) */
  double kt_im[3];     /* imaginary parts of the phase-shift wavenumbers */
} fftpim_problem_t;

/* Method parameters (Sec. 3.2-3.3).  Grid sizes count the interpolation halo:
 * a grid of n nodes and order q spans n - q cells on a periodic axis of the
 * near grid and n - q - 1 cells otherwise.  Orders are Lagrange degrees
 * (q + 1 nodes per axis). */
typedef struct {
  int near_n[3];     /* near grid nodes per axis (any size from near_order + 2 to
                        2048; the zero-padded transforms use the smallest power
                        of two >= 2 near_n - 1, reported as near_fft) */
  int near_order;    /* near projection/interpolation degree */
  int corr_radius;   /* error-correction radius in near-grid boxes (Chebyshev) */
  int far_n[3];      /* far grid nodes per axis */
  int far_order;     /* far projection/interpolation degree */
  int n_images;      /* i_d of Eq. (4): near-zone images per periodic axis */
  int precision;     /* FFTPIM_F64, FFTPIM_F32, FFTPIM_F32_FARBF16(X3) (correction stays FP64) */
  int value_type;    /* FFTPIM_REAL (static no-phase only) or FFTPIM_COMPLEX */
  int self_mode;     /* FFTPIM_SELF_IMAGES or FFTPIM_SELF_EXCLUDE */
  int order_io;      /* FFTPIM_ORDER_USER: q/u indexed like the input points;
                        FFTPIM_ORDER_PLAN: indexed in the plan's sorted order */
  int nrhs_max;      /* largest nrhs a single apply may pass */
  int corr_layout;   /* FFTPIM_CORR_AUTO, _CSR, _SYM or _TILE */
  size_t max_bytes;  /* cap on the device memory the plan may hold, including
                        what fftpim_apply_pair adds on its first call;
                        0 = no cap.  Exceeding it returns FFTPIM_ERR_NO_MEMORY. */
  double corr_ball;  /* shape of the correction region of Eq. (er): 0 = the cube
                        of Chebyshev box distance <= corr_radius; > 0 = the
                        ball |r - r_m| <= D^ER of Eq. (er) over box offsets d,
                        sum_c (d_c h_c / h_max)^2 <= corr_ball^2 (h_c the near
                        grid spacings), corr_radius then unused.  The ball
                        must hold every offset with max_c |d_c| <= near_order
                        (overlapping stencils), else INVALID_ARG. */
  int far_sum;       /* far grid sum of Eq. (8), u^g = K_far q_g: FFTPIM_FAR_AUTO,
                        FFTPIM_FAR_DIRECT or FFTPIM_FAR_FFT (see below) */
} fftpim_params_t;

/* Evaluation of the far grid sum of Eq. (8).  K_far is shift invariant
 * (Sec. 3.2: one table value per node offset between the observer and source
 * grids), so the sum is a 3D discrete convolution.  DIRECT forms it term by
 * term from the table (or on matrix cores for at least eight planes; the
 * BF16 precisions always take this path).  FFT zero-pads the far grid to the
 * smallest power of two >= 2 far_n - 1 per axis and convolves with the
 * table's spectrum, O(N_g log N_g) instead of O(N_g^2): the path for large
 * far grids, as wave problems of several wavelengths per period need.  AUTO
 * takes FFT from 8192 far grid nodes up, DIRECT below. */
enum { FFTPIM_FAR_AUTO = 0, FFTPIM_FAR_DIRECT = 1, FFTPIM_FAR_FFT = 2 };

/* Storage of the near-zone correction of Eq. (er): one CSR row per observer;
 * or (SYM) the in-cell part once per unordered pair of near-grid boxes (the
 * image-0 correction is symmetric in source and observer) plus a CSR of the
 * close-image part; or (TILE, real static kernels only) dense blocks of 16
 * observers by the union of their corrected sources, zeros included, applied
 * as FP64 matrix-core products.  AUTO picks TILE for real values and at
 * least eight planes, SYM for at most four planes when boxes hold several
 * points each, CSR otherwise.  FFTPIM_CORR_TILE with complex values returns
 * FFTPIM_ERR_UNSUPPORTED. */
enum { FFTPIM_CORR_AUTO = 0, FFTPIM_CORR_CSR = 1, FFTPIM_CORR_SYM = 2, FFTPIM_CORR_TILE = 3 };

typedef struct {
  int64_t n_src, n_obs;
  int near_n[3], near_fft[3], near_cells[3];
  double near_h[3], domain_lo[3], domain_hi[3];
  int far_n[3], far_cells[3];
  double far_h[3];
  int64_t corr_nnz;           /* stored correction entries (all parts) */
  int64_t corr_sym_values;    /* entries in symmetric box-pair blocks */
  int64_t corr_csr_nnz;       /* entries in the CSR part */
  int64_t corr_tile_values;   /* entries stored in dense row tiles (zeros included) */
  int corr_value_bytes;       /* 8 (real) or 16 (complex) per FP64 entry */
  int corr_layout_used;       /* FFTPIM_CORR_CSR, FFTPIM_CORR_SYM or FFTPIM_CORR_TILE */
  int64_t device_bytes;       /* device memory held by the plan */
  int nplanes_max;            /* complex grid planes for nrhs_max */
  double plan_seconds;        /* wall time of fftpim_plan */
  int far_fft[3];             /* far-sum transform lengths (0: direct far sum) */
} fftpim_info_t;

/* Fill *params with defaults for the problem (order 4 near, order 7 far,
 * i_d = 1, F64, complex values, images kept, user order, nrhs_max 1,
 * automatic far sum). */
int fftpim_default_params(const fftpim_problem_t* problem, fftpim_params_t* params);

/* Build a plan (Sec. 3.2 and 3.3 preprocessing: grids, interpolation
 * stencils, the far-zone kernel table of Eq. (8) from the series of
 * Eq. (pgf)/(lgf), the FFT of the zero-padded near-zone table, and the
 * error-correction operator of Eq. (er)).
 *   src_xyz_dev: device double [n_src][3]; copied, may be freed afterwards.
 *   obs_xyz_dev: NULL: the observers are the sources (Sec. 2; n_obs 0 or
 *                n_src).  Otherwise device double [n_obs][3], a separate
 *                observer set, copied: u is evaluated there (Eq. (1) with r_m
 *                the observers; the target region D of Sec. 3.2 bounds both
 *                sets, observers on periodic axes lie in [0, L) too).  The
 *                correction is then held as a CSR per direction (observer
 *                rows, and source rows for A^H); params.self_mode must be
 *                FFTPIM_SELF_IMAGES and corr_layout AUTO or CSR; an observer
 *                exactly on a source keeps only the grid part of that pair
 *                (the reading of the n = m term); fftpim_apply_pair(_noalloc)
 *                and fftpim_grad_positions return FFTPIM_ERR_UNSUPPORTED.
 *   stream:      stream for the plan's device work; the call synchronizes it.
 * On success *plan owns all device memory it needs; free with fftpim_destroy.
 * Errors: INVALID_ARG, OUT_OF_CELL, WOOD_ANOMALY, UNSUPPORTED, NO_MEMORY,
 * DEVICE. */
int fftpim_plan(fftpim_plan_t* plan, const fftpim_problem_t* problem,
                const fftpim_params_t* params, int64_t n_src, const double* src_xyz_dev,
                int64_t n_obs, const double* obs_xyz_dev, fftpim_stream_t stream);

/* u = A q (Eq. (1) through Eq. (5)): q_dev [nrhs][n_src], u_dev [nrhs][n_obs]
 * (overwritten).  1 <= nrhs <= nrhs_max.  For a static no-phase problem
 * every right-hand side must be neutral (Eq. (neutral)); a violation is
 * latched for fftpim_last_status. */
int fftpim_apply(fftpim_plan_t plan, const void* q_dev, void* u_dev, int nrhs,
                 fftpim_stream_t stream);

/* w = A^H v, the exact conjugate transpose of the discrete operator applied
 * by fftpim_apply: v_dev [nrhs][n_obs], w_dev [nrhs][n_src] (overwritten).
 * For a static no-phase problem only the zero-mean part of w is defined;
 * this call returns w with its mean removed per right-hand side. */
int fftpim_apply_adjoint(fftpim_plan_t plan, const void* v_dev, void* w_dev, int nrhs,
                         fftpim_stream_t stream);

/* u = A q and w = A^H v in one call (the pair Krylov solvers of the BiCG
 * family need every iteration; A as in Eq. (1) through Eq. (5)).  Both
 * products are computed in full and equal those of fftpim_apply and
 * fftpim_apply_adjoint up to the summation order; the box-pair correction
 * layout reads each stored block once for both.  q_dev, v_dev, u_dev, w_dev:
 * device arrays [nrhs][n], same element type as fftpim_apply; u and w are
 * overwritten and must not overlap each other or the inputs.  The static
 * no-phase case checks q for neutrality and removes the mean of w, as the two
 * single calls do.  The first call on a plan allocates four work arrays of
 * n x planes elements (planes = nrhs_max, or half of it for real values) and a
 * second set of near-grid and far-zone work buffers of the plan's own sizes
 * (counted in fftpim_plan_info's device_bytes once made); later calls allocate
 * nothing.  Enqueued on stream like fftpim_apply.  Errors: INVALID_ARG,
 * NO_MEMORY, DEVICE. */
int fftpim_apply_pair(fftpim_plan_t plan, const void* q_dev, void* u_dev, const void* v_dev,
                      void* w_dev, int nrhs, fftpim_stream_t stream);

/* fftpim_apply_pair for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and stream semantics as
 * fftpim_apply_pair; the pair's own work arrays (a second near-grid/far-zone
 * work set, the packed v and the three parts of w) live in a fixed array of
 * 64 MiB per device, held from library load until the process ends, instead
 * of plan-owned allocations, so no call allocates (stage timing is not
 * recorded for this call).  Every call on a device shares that device's
 * array and leaves it holding its last contents: calls that overlap in time
 * on one device (on different streams, or from different plans or host
 * threads) race and must be serialised by the caller.
 * Errors: INVALID_ARG; SCRATCH_LIMIT when the plan's pair arrays exceed the
 * array (nothing is enqueued); DEVICE. */
int fftpim_apply_pair_noalloc(fftpim_plan_t plan, const void* q_dev, void* u_dev, const void* v_dev,
                              void* w_dev, int nrhs, fftpim_stream_t stream);

/* Position gradient (forces) of the discrete operator A that fftpim_apply
 * applies: its entries depend on the positions through the Lagrange weights
 * of the projections and interpolations (Eq. (projection),
 * Eq. (interpolation)) and through the correction entries of Eq. (er), all
 * differentiated here.  For amplitudes q_dev and an upstream gradient g_dev
 * = dL/du (both [nrhs][n], element type as for fftpim_apply), grad_dev
 * (device double [n][3], overwritten) receives
 *     dL/dr_k = sum over right-hand sides of
 *               Re(conj(g_k) sum_n dA[k,n]/dr_k q_n) + Re(sum_m conj(g_m) dA[m,k]/dr_k q_k),
 * the gradient of L = Re sum_m conj(g_m) (A q)_m (for real values,
 * L = sum_m g_m (A q)_m; with g = q / 2 and a real static kernel, L is the
 * electrostatic energy and -grad the forces).  Rows follow the caller's
 * order (FFTPIM_ORDER_PLAN: the plan's order).  A is piecewise smooth: a
 * point exactly on a stencil switch gets the derivative of the stencil it
 * uses.  The first call on a plan allocates the fused pair's work arrays (as
 * fftpim_apply_pair does) and an [n][3] accumulator.  Enqueued on stream.
 * Errors: INVALID_ARG, NO_MEMORY, DEVICE. */
int fftpim_grad_positions(fftpim_plan_t plan, const void* q_dev, const void* g_dev, int nrhs, double* grad_dev,
                          fftpim_stream_t stream);

/* Apply only some parts of the operator (FFTPIM_PART_* mask) - forward
 * (adjoint = 0) or conjugate transpose (adjoint = 1).  PART_ALL equals
 * fftpim_apply / fftpim_apply_adjoint except that no mean is removed and no
 * neutrality check is made.  Used to check the stages one at a time. */
int fftpim_apply_parts(fftpim_plan_t plan, int parts, int adjoint, const void* q_dev,
                       void* u_dev, int nrhs, fftpim_stream_t stream);

/* perm_dev (device int32 [n]) receives, for each plan-order position, the
 * index of that point in the caller's order.  which: 0 sources, 1 observers. */
int fftpim_get_permutation(fftpim_plan_t plan, int which, int32_t* perm_dev);

/* Sizes and parameters of a plan. */
int fftpim_plan_info(fftpim_plan_t plan, fftpim_info_t* info);

/* Synchronizes the plan's last stream and returns the first device-detected
 * error of the applies since the previous call (then clears it). */
int fftpim_last_status(fftpim_plan_t plan);

/* Frees the plan and every device buffer it owns. NULL is accepted. */
int fftpim_destroy(fftpim_plan_t plan);

/* Per-stage device timing with HIP events recorded on the apply stream.
 * enable = 1: start recording (accumulators reset); every later apply records
 * an event pair around each stage.  enable = 0: stop recording.  On return
 * (either way) ms_out[FFTPIM_NSTAGES] and calls_out[FFTPIM_NSTAGES] (host
 * arrays, may be NULL) hold the summed milliseconds and the number of timed
 * launches per stage since recording started; the call synchronizes. */
enum { FFTPIM_STAGE_PACK = 0, FFTPIM_STAGE_NEAR_SPREAD = 1, FFTPIM_STAGE_NEAR_FFT = 2,
       FFTPIM_STAGE_NEAR_INTERP = 3, FFTPIM_STAGE_NEAR_CORR = 4, FFTPIM_STAGE_FAR = 5,
       FFTPIM_STAGE_UNPACK = 6, FFTPIM_NSTAGES = 7 };
int fftpim_stage_times(fftpim_plan_t plan, int enable, double* ms_out, int64_t* calls_out);

/* Static description of a status code. */
const char* fftpim_error_string(int status);

/* The periodic Green's function of Sec. 2 as the library's host evaluator
 * computes it for the far-zone table (Eq. (pgf) / Eq. (lgf) with the
 * neutral-static gauge of zero cell mean in 3D), at n host points
 * r_xyz [n][3]; out [n][2] receives (re, im).  Points must not be lattice
 * vectors.  Exposed so the evaluator can be checked on its own. */
int fftpim_eval_pgf(const fftpim_problem_t* problem, int64_t n, const double* r_xyz,
                    double* out);

/* lim_{r->0} [G^p(r) - G0(r)] for the problem (Sec. 2): the coefficient
 * with which the images of a point act on the point itself, i.e. the n = m
 * term of Eq. (1) without its singular zeroth image, in the gauge of
 * fftpim_eval_pgf for the neutral static case.  The apply subtracts
 * C_self q_m when params.self_mode is FFTPIM_SELF_EXCLUDE (Eq. (5), n != m).
 * out [2] receives (re, im).  Host only.  Errors: INVALID_ARG, UNSUPPORTED,
 * WOOD_ANOMALY. */
int fftpim_eval_pgf_self(const fftpim_problem_t* problem, double* out);

/* ---- Many independent cells -------------------------------------------
 * Sec. 4.2 runs 1D, 2D and 3D periodicities, static and dynamic, with one
 * implementation; a workload of many such cells of uneven size is served by
 * a parameter choice per cell and a batch apply. */

typedef struct {
  double predicted_rel_err;    /* error model value of the chosen parameters */
  double predicted_ms;         /* cost model value of one apply, milliseconds */
  int64_t predicted_corr_nnz;  /* correction pairs the choice implies (sampled) */
  int candidates;              /* parameter sets the search scored */
} fftpim_tune_report_t;

/* Chooses the method parameters of Sec. 3.2-3.3 for a problem and its n
 * points (device [n][3], FP64) so that the predicted relative L2 error of
 * the potential stays below target_rel_err at the least predicted apply
 * time for nrhs right-hand sides in the given precision.  The error model
 * bounds the near zone by the interpolation error outside the correction
 * ball of Eq. (er) (decaying with the ball radius, floored by (k0 h)^(q+1)
 * for a wave kernel) and the far zone by the interpolation error of G_far of
 * Eq. (4) on the far grids of Eq. (grid) (set by the far spacing relative
 * to the period and to the wavelength); its constants come from measured
 * errors with a margin.  The cost model is fitted to measured per-part
 * times.  params: in, value_type, self_mode, order_io, nrhs_max, corr_layout
 * and max_bytes are kept (fill it with fftpim_default_params first); out,
 * near_n, near_order, corr_ball (the ball region; corr_radius its ceiling),
 * far_n, far_order, n_images = 1, precision and far_sum = AUTO are set.
 * report may be NULL.  Reads the points to the host; allocates no device
 * memory.  Errors: INVALID_ARG (also an FP32 precision with a target below
 * 5e-6), OUT_OF_CELL, UNSUPPORTED (no parameter set reaches the target
 * within the grid limits), DEVICE. */
int fftpim_autotune(const fftpim_problem_t* problem, int64_t n, const double* xyz_dev,
                    double target_rel_err, int precision, int nrhs, fftpim_params_t* params,
                    fftpim_tune_report_t* report);

typedef struct fftpim_batch_s* fftpim_batch_t;

/* Groups ncells plans (not owned: they must outlive the batch and must not
 * be applied elsewhere while a batch apply runs) to be applied together.
 * The cells are ranked by a predicted cost and dealt, largest first, to the
 * least-loaded of nlanes (1..16) streams; each lane applies its cells in
 * turn while every cell still runs its near, correction and far parts on its
 * plan's own concurrent streams, so small and large cells fill the GPU
 * together.  use_graph is reserved and must be 0 (1 returns
 * FFTPIM_ERR_UNSUPPORTED: recording a batch apply as one HIP graph is
 * switched off). */
int fftpim_batch_create(fftpim_batch_t* batch, const fftpim_plan_t* plans, int ncells, int nlanes,
                        int use_graph);

/* in[c], out[c], nrhs[c]: the arguments of fftpim_apply for cell c (of
 * fftpim_apply_adjoint when adjoint = 1).  Enqueued on stream, which waits
 * for every cell; no host synchronisation. */
int fftpim_batch_apply(fftpim_batch_t batch, const void* const* in, void* const* out,
                       const int* nrhs, int adjoint, fftpim_stream_t stream);

int fftpim_batch_destroy(fftpim_batch_t batch);

#ifdef __cplusplus
}
#endif

#endif /* FFTPIM_H */
