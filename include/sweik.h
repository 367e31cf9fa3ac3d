/*
 * sweik.h -- C ABI of the MI355X (gfx950) linearised eikonal solver.
 *
 * The solver computes the viscosity-regularised distance S on a regular grid
 * from a positive forcing f and a point set {y_k} with S(y_k) = 0, by the
 * perturbation method of the paper (Section 5, algorithm in Table 1):
 *
 *   ftilde   reference forcing (Section 5.1): nu = sqrt((fmin^2+fmax^2)/2),
 *            sup f, or a caller value
 *   phi_0    = sum_k exp(-ftilde |x - y_k| / hbar)       (eq. phi_0Solution)
 *   phi_i    = h^D G (*) ((f^2 - ftilde^2) phi_{i-1}),  i = 1..T,  with the
 *            screened-Poisson Green's function G of eq. GreensFunction2D /
 *            GreensFunction3D; a linear (zero-padded) convolution over the
 *            grid, evaluated by FFT (eqs. phiRecRelation, phi_i_Solution and
 *            Section 5.2)
 *   phi      = sum_{i=0..T} (-1)^i phi_i                   (eq. phiSolution)
 *   S        = -hbar ln phi                                 (eq. SfromPhi)
 *
 * The value of G at the singular origin is its average over the ball of one
 * cell's volume.  Points where phi <= 0 get S = +inf and are counted.
 *
 * In 3D the real transform along the last axis samples the odd frequencies
 * (k + 1/2)/M; with zero padding to M >= 2n - 1 the nega-cyclic convolution
 * it implies equals the linear convolution (Section 5.2's discrete
 * convolution), like the cyclic one.
 *
 * Conventions
 *   - Arrays are C order (last index fastest).  Grid point index m has
 *     position h*m.  Sources are distinct grid indices, int32 [n_src][ndim].
 *   - Every pointer passed to a solve is DEVICE memory owned by the caller,
 *     except where marked host.  The library allocates no device memory and
 *     never synchronises the stream: all work is enqueued on `stream`
 *     (a hipStream_t; NULL = the default stream).  A solve can therefore be
 *     captured into a HIP graph.
 *   - Precision SWEIK_F32_SCALED: f and S are float32; FFTs run in float32
 *     on power-of-two-rescaled series terms; the series is accumulated and
 *     the logarithm taken in float64.  SWEIK_F64: everything float64.
 *   - Errors in arguments are reported synchronously through the return
 *     value before anything is enqueued.  Errors in the data (f <= 0, NaN or
 *     Inf in f, a source outside the grid) are reported asynchronously in
 *     the device-side sweik_info.flags.
 *   - Plans are immutable after creation and may be shared by concurrent
 *     solves that use distinct workspaces.
 */
#ifndef SWEIK_H
#define SWEIK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWEIK_ABI_VERSION 1
#define SWEIK_MAX_TERMS 64 /* largest T */
#define SWEIK_MAX_TILTS 64 /* most tilts of one sweik_solve_tilted */

typedef enum {
  SWEIK_OK = 0,
  SWEIK_EINVAL = 1,       /* invalid argument */
  SWEIK_EUNSUPPORTED = 2, /* valid but not supported: a grid beyond the sizes
                             below (2D n0 <= 4096 and n1 <= 8192; 3D every
                             axis <= 1024), a
                             2D-only call on a 3D plan, or a schedule the
                             plan cannot run */
  SWEIK_EWORKSPACE = 3,   /* workspace or checkpoint buffer too small */
  SWEIK_EDEVICE = 4,      /* a HIP call failed */
  SWEIK_ENOMEM = 5        /* host allocation failed */
} sweik_status;

typedef enum { SWEIK_F32_SCALED = 0, SWEIK_F64 = 1 } sweik_precision;

typedef enum {
  SWEIK_FT_NU = 0,    /* sqrt((fmin^2 + fmax^2)/2), Section 5.1 optimum */
  SWEIK_FT_FMAX = 1,  /* sup f: every term has one sign (Section 5.1) */
  SWEIK_FT_GIVEN = 2  /* the value in sweik_problem.ftilde */
} sweik_ftilde_mode;

/* Bits of sweik_info.flags */
#define SWEIK_FLAG_F_NONFINITE 1   /* f holds NaN or Inf */
#define SWEIK_FLAG_F_NONPOSITIVE 2 /* f holds a value <= 0 */
#define SWEIK_FLAG_C0_GE_1 4       /* sup|f^2-ftilde^2|/ftilde^2 >= 1 */
#define SWEIK_FLAG_BAD_SOURCE 8    /* a source lies outside the grid */

typedef struct {
  int32_t ndim;      /* 2 or 3 */
  int64_t dims[3];   /* grid points per axis, each >= 2 (dims[2] unused in 2D) */
  double h;          /* grid spacing > 0 */
  double hbar;       /* > 0 */
  int32_t T;         /* number of correction terms, 0..SWEIK_MAX_TERMS */
  int32_t n_src;     /* >= 1 */
  int32_t prec;      /* sweik_precision */
  int32_t ft_mode;   /* sweik_ftilde_mode */
  double ftilde;     /* used when ft_mode == SWEIK_FT_GIVEN; > 0 */
} sweik_problem;

/* Written on the device by every solve (when info is non-NULL); read it
 * after synchronising the stream. */
typedef struct {
  double f_min, f_max;
  double ftilde;
  double beta;      /* ftilde h / hbar: decay per cell */
  double c0_bound;  /* sup|f^2 - ftilde^2| / ftilde^2 (eq. OperatorNormUpperBound) */
  int64_t n_nonpositive_phi; /* points with phi <= 0 (S = +inf) */
  int32_t flags;    /* SWEIK_FLAG_* */
  int32_t T;
  int32_t scale_exp[SWEIK_MAX_TERMS + 1]; /* term i is stored as 2^scale_exp[i] * m_i */
} sweik_info;

typedef struct sweik_plan_s *sweik_plan;

/* Validate a problem and choose the kernel schedule.  Host only: makes no
 * HIP call.  Returns SWEIK_EINVAL for invalid fields, SWEIK_EUNSUPPORTED for
 * grids beyond the supported sizes.  Padded FFT lengths (the next power of
 * two >= 2n-1, at least 64): 2D axis 0 <= 8192 and axis 1 <= 16384; 3D
 * every axis <= 2048.  In grid points: 2D n0 <= 4096 and n1 <= 8192, 3D n0,
 * n1, n2 <= 1024, in both precisions.  The bound is the line
 * length one work-group transforms in its registers and LDS (a column of
 * 8192 points, a real row of 16384); the
 * method itself has none, and a larger grid would need a two-level
 * (four-step) transform along the long axis. */
sweik_status sweik_plan_create(const sweik_problem *problem, sweik_plan *out);
void sweik_plan_destroy(sweik_plan plan);

/* Bytes of device workspace a solve (and an adjoint) needs. */
size_t sweik_workspace_bytes(sweik_plan plan);
/* Bytes of the checkpoint buffer a solve writes for a later adjoint. */
size_t sweik_checkpoint_bytes(sweik_plan plan);
/* Padded FFT sizes per axis (out[0..2]); returns ndim. */
int32_t sweik_plan_padded_dims(sweik_plan plan, int64_t *out);

/* Host-side check of a host copy of the source list: SWEIK_EINVAL when a
 * source lies outside the grid or two sources coincide. */
sweik_status sweik_check_sources(sweik_plan plan, const int32_t *src_host);

/* Forward solve (Table 1).
 *   f      device, dims, float32 (F32_SCALED) or float64 (F64)
 *   src    device, int32 [n_src][ndim]
 *   S      device, dims, same type as f (output)
 *   ws     device workspace of ws_bytes >= sweik_workspace_bytes(plan)
 *   ckpt   device, nullable: when given, the series terms and phi are kept
 *          for sweik_solve_adjoint (sweik_checkpoint_bytes(plan) bytes; 2D
 *          and 3D)
 *   stream hipStream_t
 *   info   device, nullable: sweik_info written asynchronously */
sweik_status sweik_solve(sweik_plan plan, const void *f, const int32_t *src,
                         void *S, void *ws, size_t ws_bytes, void *ckpt,
                         void *stream, sweik_info *info);

/* Forward solve with prescribed values S(y_k) = s_k at the sources: each
 * source's exponential in phi_0 (eq. phi_0Solution) carries the weight
 * exp(-s_k / hbar), so that S is a smooth minimum of s_k + distance.
 *   src_s  device, n_src values of the type of f (nullable: all 0, which is
 *          sweik_solve).  Other arguments as sweik_solve.  An adjoint taken
 *          from this solve's checkpoint holds the seed values fixed. */
sweik_status sweik_solve_seeded(sweik_plan plan, const void *f,
                                const int32_t *src, const void *src_s, void *S,
                                void *ws, size_t ws_bytes, void *ckpt,
                                void *stream, sweik_info *info);

/* Far-field stabilised solve (2D).  FFT convolution rounds with an absolute
 * error of about eps max|phi_i| over the whole grid while phi decays like
 * exp(-S/hbar), so far from the sources the plain solve loses all relative
 * accuracy (Section 5.3; the paper turns to multiprecision there).  This
 * solve runs the same series once per tilt a = beta (tilts[2d],
 * tilts[2d+1]) (a per grid index along axes 0 and 1) on the tilted terms
 * phi_i(x) exp(a . x - A) with the kernel kappa(m) exp(a . m): in exact
 * arithmetic the same convolution (kappa (*) psi times exp(a . x) equals
 * (kappa exp(a . m)) (*) (psi exp(a . y))), so S is unchanged, but the terms
 * are flat in the direction of a and their rounding noise is small there.
 * A = max_k (a . y_k) keeps the tilted phi_0 at most n_src.  Per point the
 * result of the tilt with the best score ln(tilted phi) - ln B is kept,
 * B = sum_i max|tilted phi_i| / (1 - |tilt|^2) being the tilt's noise scale
 * (exp(-score) is about the relative error to expect).  A tilt gains little
 * near sources that lie behind the one furthest along it; with per_source
 * set the solve is split over the sources instead (at a fixed reference
 * forcing the series is linear in phi_0, so phi = sum_k phi^(k)): each
 * source is solved alone with all tilts, and S = -hbar ln sum_k
 * exp(-S_k / hbar) in float64, at n_src times the cost.
 *   tilts  HOST, n_tilt pairs (tilt0, tilt1) in units of beta, each with
 *          tilt0^2 + tilt1^2 < 1 (the tilted kernel must decay); (0, 0) is
 *          the plain solve.  E.g. (0, 0) and 8 directions at 0.9.
 *   n_tilt 1 .. SWEIK_MAX_TILTS
 *   per_source  0: one tilted solve over all sources; 1: one per source
 *   ws     device workspace of ws_bytes >= sweik_tilted_workspace_bytes(plan,
 *          n_tilt): the solve's, plus per tilt its own spectra, complex
 *          kernel spectrum ((H1 + 1) M0 complex values), T stored terms, S
 *          and a float score per point (about 9 N values of the plan's
 *          precision plus T N per tilt), plus the tilts' work lists
 *   src_s  device, nullable: values of S at the sources, as sweik_solve_seeded
 *   f, src, S, stream, info as sweik_solve (no checkpoint); info counts the
 *          points that no tilt resolved (S = +inf) and reports the first
 *          tilt's term scales.
 * The tilts run side by side: each pass is one launch over the work-groups
 * of every tilt, so the launches do not grow with n_tilt; the work grows
 * as about one solve per tilt (per source with per_source; the kernel
 * spectrum of a tilt is complex: about 1.6 x the column pass's bytes).
 * With T = 0 it is sweik_solve.  Enqueues kernels only (no copies, no
 * memset): it can be captured into a HIP graph.
 * SWEIK_EINVAL for a tilt outside the unit disc or n_tilt out of range,
 * SWEIK_EUNSUPPORTED in 3D (sweik_tilted_workspace_bytes returns 0 there
 * and for n_tilt out of range). */
size_t sweik_tilted_workspace_bytes(sweik_plan plan, int32_t n_tilt);
sweik_status sweik_solve_tilted(sweik_plan plan, const void *f, const int32_t *src,
                                const void *src_s, void *S, const double *tilts, int32_t n_tilt,
                                int32_t per_source, void *ws, size_t ws_bytes, void *stream,
                                sweik_info *info);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): sweik_solve
 * without a caller workspace.  The workspace is a static device array of
 * sweik_noalloc_scratch_bytes() bytes (64 MiB) inside the library; each GPU
 * the library runs on holds its own copy until the process ends.  The call
 * allocates nothing (no hipMalloc, no library allocation); its first call on
 * a device looks up that device's copy of the array.
 *   f, src, S, stream, info  as sweik_solve (no checkpoint)
 * Returns SWEIK_EWORKSPACE when sweik_workspace_bytes(plan) exceeds the
 * array (e.g. 1024^2 in FP32 with T = 16 needs about 109 MB), before
 * anything is enqueued.  Every call on one GPU uses the same array, which
 * keeps the last call's contents (a solve writes every workspace buffer
 * before reading it, so nothing needs clearing): calls that overlap in time
 * on one GPU (other streams, other threads) race and give wrong results. */
size_t sweik_noalloc_scratch_bytes(void);
sweik_status sweik_solve_noalloc(sweik_plan plan, const void *f, const int32_t *src, void *S,
                                 void *stream, sweik_info *info);

/* Adjoint (2D and 3D) of the solve with ftilde held fixed (reverse sweep of
 * the recurrence eq. phiRecRelation; the kernel is even, so the transposed
 * convolution is the convolution itself).
 *   dLdS   device, dims, same type as f: gradient of a loss w.r.t. S
 *   dLdf   device, dims, same type as f (output)
 *   ckpt   the checkpoint written by sweik_solve for the same f and src */
sweik_status sweik_solve_adjoint(sweik_plan plan, const void *f,
                                 const int32_t *src, const void *ckpt,
                                 const void *dLdS, void *dLdf, void *ws,
                                 size_t ws_bytes, void *stream);

/* Full gradient (2D and 3D) of a loss L(S) of a solve: not in the paper, the
 * derivative of all of its steps.  With beta = ftilde h / hbar,
 * gamma = f^2/ftilde^2 - 1 and w_k = exp(-s_k / hbar):
 *   dLdf   device, dims, type of f (output): dL/df including the dependence
 *          of ftilde on f (Section 5.1): the adjoint of sweik_solve_adjoint
 *          plus dL/dftilde times a subgradient of ftilde(f), which for nu
 *          puts fmin/(2 ftilde) on the first grid point (C order) where f is
 *          smallest and fmax/(2 ftilde) on the first where it is largest; for
 *          sup f, 1 on the first maximum; nothing for a given ftilde
 *   grads  device, 4 doubles, nullable (output): dL/dhbar (through beta, the
 *          weights and the logarithm), dL/dftilde, dL/dbeta, 0
 *   src_s  device, nullable: the source values of the forward solve
 *          (sweik_solve_seeded); ckpt its checkpoint
 *   ws     device workspace of ws_bytes >= sweik_adjoint_full_workspace_bytes
 * The beta-derivative of the kernel (2D: (beta/pi) K0(x) - (beta/2pi) x
 * K1(x), x = beta|m|; 3D: beta e^{-x} (2 - x) / (4 pi |m|); at the origin
 * that of the cell average) is convolved with every adjoint term, so the
 * sweep costs about 1.7 adjoints (3D: two y, z, y chains per term). */
size_t sweik_adjoint_full_workspace_bytes(sweik_plan plan);
sweik_status sweik_solve_adjoint_full(sweik_plan plan, const void *f, const int32_t *src,
                                      const void *src_s, const void *ckpt, const void *dLdS,
                                      void *dLdf, double *grads, void *ws, size_t ws_bytes,
                                      void *stream);

/* ---- finite-difference screened Poisson solve (Section 6) ----------------
 * The paper's second method: eq. phiEquation discretised with the standard
 * Laplacian (five-point in 2D, seven-point in 3D; phi = 0 outside the grid),
 * the sparse system of eq. sparse-system,
 *   (2D + (h f_m / hbar)^2) phi_m - sum_{grid neighbours n} phi_n = b_m,
 * b = 1 at the sources and 0 elsewhere (eq. deltakron), then
 * S = -hbar ln phi (eq. SfromPhi).  (The printed diagonal term f(X_i) is read
 * as (h f / hbar)^2; with the printed right-hand side, phi at a source is a
 * value of the discrete Green's function, so S there is O(hbar), not 0.)
 * Solved matrix-free by conjugate gradients preconditioned with the
 * diagonal, in float64 for either precision of f and S, until
 * ||r|| <= rtol ||b|| or max_iter iterations.
 *   plan      any plan (uses ndim, dims, h, hbar, n_src and the precision of
 *             f and S; T and the reference forcing are not used)
 *   f, src, S as sweik_solve (device)
 *   ws        device workspace of ws_bytes >= sweik_fd_workspace_bytes(plan)
 *             (about 72 bytes per grid point)
 *   max_iter  0 .. 2^24; rtol >= 0, finite
 *   info      HOST, nullable
 * Unlike the FFT solve this call synchronises the stream: it reads a
 * convergence flag from the device after every 64 iterations (so it cannot
 * be captured into a graph).  Sources are distinct grid points; a source
 * outside the grid sets SWEIK_FLAG_BAD_SOURCE and is ignored. */
typedef struct {
  int32_t iterations;   /* CG iterations taken */
  int32_t converged;    /* 1 when ||r|| <= rtol ||b|| was reached */
  double rel_residual;  /* ||r|| / ||b|| of the recursively updated residual */
  int64_t n_nonpositive_phi; /* points with phi <= 0 (S = +inf) */
  int32_t flags;        /* SWEIK_FLAG_* for f and the sources */
  int32_t n_sources;    /* distinct sources inside the grid */
} sweik_fd_info;

size_t sweik_fd_workspace_bytes(sweik_plan plan);
sweik_status sweik_fd_solve(sweik_plan plan, const void *f, const int32_t *src, void *S,
                            void *ws, size_t ws_bytes, int32_t max_iter, double rtol,
                            void *stream, sweik_fd_info *info);

/* ---- path backtracking (Section 6, path planning) -------------------------
 * From each start point, integrate dx/dt = -grad S / |grad S| (eq.
 * PathPlanning-backTrackOnS) on a computed S, in grid units (position x_d
 * is grid index x_d along axis d, C order):
 *   - the node gradient of S is its central difference along each axis
 *     (one-sided at the first and last node); the gradient at x is the
 *     multilinear interpolation of the node gradients of x's cell;
 *   - each step is a classical fourth-order Runge-Kutta step of length
 *     `step` on the unit field -g/|g|; stage positions and new points are
 *     clamped to the box [0, dims[d] - 1];
 *   - a path stops when it comes within `radius` of a source (status 0),
 *     after max_steps steps (1), or where the gradient vanishes or is not
 *     finite, e.g. where S = +inf (2).  A start outside the box or not
 *     finite records no point (status 3).
 * Arguments:
 *   ndim, dims  host: 2 or 3 axes, each 2 .. 2^20 points
 *   prec        type of S: float32 (SWEIK_F32_SCALED) or float64
 *   S           device, dims (as written by a solve)
 *   src         device, int32 [n_src][ndim] (n_src >= 0)
 *   start       device, float64 [n_paths][ndim]
 *   max_steps   0 .. 2^20; step > 0 and radius >= 0, finite
 *   path        device, float64 [n_paths][max_steps + 1][ndim] (output; the
 *               first n_points[p] points of path p are written)
 *   n_points    device, int32 [n_paths] (output)
 *   status      device, int32 [n_paths] (output)
 *   stream      hipStream_t
 * Argument errors return SWEIK_EINVAL before anything is enqueued; nothing
 * is allocated and the stream is not synchronised.  All arithmetic is
 * float64.  n_paths = 0 is a no-op. */
sweik_status sweik_backtrack(int32_t ndim, const int64_t *dims, sweik_precision prec,
                             const void *S, const int32_t *src, int32_t n_src,
                             const double *start, int32_t n_paths, int32_t max_steps,
                             double step, double radius, double *path, int32_t *n_points,
                             int32_t *status, void *stream);

/* ---- measurement ---------------------------------------------------------
 * Kernel classes of a solve, for sweik_solve_timed. */
enum {
  SWEIK_KC_PREP = 0,      /* reduction of f, twiddle table */
  SWEIK_KC_GHAT_ROW = 1,  /* kernel table lines + real FFT (last axis) */
  SWEIK_KC_GHAT_COL = 2,  /* kernel spectrum: 2D columns; 3D axis 1 */
  SWEIK_KC_PHI0_ROW = 3,  /* phi_0, first forcing term, real FFT */
  SWEIK_KC_CONV_COL = 4,  /* FFT * kernel spectrum * inverse FFT (2D columns, 3D axis 0) */
  SWEIK_KC_TERM_ROW = 5,  /* inverse real FFT, accumulate, next forcing, real FFT */
  SWEIK_KC_LAST_ROW = 6,  /* inverse real FFT, accumulate, S = -hbar ln phi */
  SWEIK_KC_Y_FWD = 7,     /* 3D: FFT along axis 1 */
  SWEIK_KC_Y_INV = 8,     /* 3D: inverse FFT along axis 1 */
  SWEIK_KC_GHAT_Z = 9,    /* 3D: kernel spectrum along axis 0 */
  SWEIK_KC_PHI0_FFT = 10, /* phi_0 by FFT: exp(-beta|m|) spectrum, source grid, product */
  SWEIK_KC_COUNT = 11
};

/* Same work as sweik_solve (no checkpoint, no info) with a HIP event
 * recorded on `stream` before the first kernel and after every kernel.
 * Synchronises the stream, then writes to the HOST arrays
 * ms[SWEIK_KC_COUNT] (per class, the summed intervals between the event
 * before and the event after each of its kernels: the kernel plus the
 * dispatch gap before it) and count[SWEIK_KC_COUNT] (launches per class).
 * For benchmarks: the events add a little time between launches. */
sweik_status sweik_solve_timed(sweik_plan plan, const void *f, const int32_t *src,
                               void *S, void *ws, size_t ws_bytes, void *stream,
                               float *ms, int32_t *count);

/* ---- uneven batches of independent 2D problems ------------------------ */
typedef struct sweik_batch_s *sweik_batch;

/* All problems must be 2D with the same precision and the same T.  Host
 * only: validates the problems and lays out the workspace (no HIP call). */
sweik_status sweik_batch_create(const sweik_problem *problems, int32_t count,
                                sweik_batch *out);
/* Creates, on the calling thread's current device, the HIP resources the
 * batch's solves use: one stream and one event per size class beyond the
 * first (class chains run side by side), a capture stream, and a ring of
 * pinned host staging buffers for the per-instance argument lists.  Call
 * once before the first solve; the batch then runs on that device only.
 * Returns SWEIK_EINVAL when called again from another device, SWEIK_EDEVICE
 * when a HIP call fails.  The batch owns these until sweik_batch_destroy. */
sweik_status sweik_batch_prepare(sweik_batch batch);
void sweik_batch_destroy(sweik_batch batch);
size_t sweik_batch_workspace_bytes(sweik_batch batch);

/* f, src, S: HOST arrays of `count` device pointers.  infos: device array of
 * `count` sweik_info (nullable).  Creates no HIP resource and allocates
 * nothing: SWEIK_EINVAL until sweik_batch_prepare has been called.  The
 * argument lists are copied from the pinned ring; a slot is reused only
 * after the copy issued from it four calls earlier has completed (the one
 * host wait of this call). */
sweik_status sweik_batch_solve(sweik_batch batch, const void *const *f,
                               const int32_t *const *src, void *const *S,
                               void *ws, size_t ws_bytes, void *stream,
                               sweik_info *infos);

/* Same work, captured once into a HIP graph owned by the batch and replayed
 * on later calls with the same pointers (a call with other pointers waits
 * for the stream and re-captures).  Capturing instantiates a graph: the
 * first call, and a call with new pointers, create one graph executable;
 * replays create nothing.  SWEIK_EINVAL until sweik_batch_prepare. */
sweik_status sweik_batch_solve_graph(sweik_batch batch, const void *const *f,
                                     const int32_t *const *src,
                                     void *const *S, void *ws,
                                     size_t ws_bytes, void *stream,
                                     sweik_info *infos);

/* ---- schedules and tuning ------------------------------------------------
 * A schedule fixes, per pass family, the FFT radix and the work-group shape:
 * E elements per team thread, i.e. radix-E Stockham stages and 4096/E
 * threads per work-group (the rows or columns per work-group do not change).
 *   row_e     2D row passes (all modes): 16, 8, or 4 (float32 only)
 *   col_e     2D column passes (all modes): 16, 8, or 4 (float32 only);
 *             16 only for n0 > 2048 (8192-point columns); likewise row_e
 *             for n1 > 4096
 *   phi0_fft  2D and 3D: 0 = phi_0 by the direct sum over the sources (eq.
 *             phi_0Solution), 1 = by FFT as in Table 1 steps 1-5 (the
 *             spectrum of exp(-beta |m|) times the transform of the source
 *             grid).  2D plans start with 1 when n_src > 64, 3D plans
 *             when n_src > 128 (float32) or n_src > 32 (float64).
 * 3D plans have row_e = col_e = 16 (phi0_fft as above).  New plans take row_e and
 * col_e from the process-wide table filled by sweik_autotune (default 16).
 * Batches always sum over the sources. */
typedef struct {
  int32_t row_e, col_e;
  int32_t phi0_fft;
  int32_t reserved[5];
} sweik_schedule;

sweik_status sweik_plan_get_schedule(sweik_plan plan, sweik_schedule *out);
/* SWEIK_EINVAL for a value other than 16, 8 or 4 (0 or 1 for phi0_fft);
 * SWEIK_EUNSUPPORTED for 4 in a float64 plan, col_e other than 16 with
 * n0 > 2048, row_e other than 16 with n1 > 4096, or a 3D plan with a radix
 * other than 16.  Host only.  Not to be called while a
 * solve with this plan is being enqueued on another thread. */
sweik_status sweik_plan_set_schedule(sweik_plan plan, const sweik_schedule *s);

/* Times every candidate schedule of the 2D per-term passes with HIP events
 * on `stream` (radix 16, 8 and, in float32, 4): each (col_e, row_e) pair
 * as 4 back-to-back [column
 * convolution; row pass] launches, 5 times (the pairs taking turns within
 * each repetition), keeping the median (with T < 2
 * only the column pass is timed).  Works on the workspace `ws`, whose
 * contents are overwritten: run it before a solve, not between a solve and
 * its adjoint.  Keeps the fastest in the plan and in the process-wide table
 * keyed by (pass, length, precision) that later plans start from.
 * Synchronises the stream.  Returns the number of schedules timed (9 in
 * float32, 4 in float64; 3 or 2 when T < 2; 0 for 3D plans; negative on a
 * HIP error or a too-small workspace). */
int32_t sweik_autotune(sweik_plan plan, void *ws, size_t ws_bytes,
                       void *stream);

const char *sweik_status_string(sweik_status s);
int32_t sweik_abi_version(void);
/* Description of the last kernel launch that failed on the calling thread
 * (the kernel family, mode, length, schedule and the HIP error name), or ""
 * when none has; the text behind a SWEIK_EDEVICE.  Owned by the library,
 * valid until the thread's next failing launch. */
const char *sweik_last_error(void);
/* Number of HIP resources (streams, events, pinned host buffers, graph
 * executables) the library has created in this process so far.  Solves,
 * adjoints, batch solves and graph replays create none; plan and batch
 * creation are host only; sweik_batch_prepare, the first capture of a batch
 * graph, sweik_solve_timed and sweik_autotune do create some.  For tests
 * and diagnostics. */
int64_t sweik_resource_count(void);

#ifdef __cplusplus
}
#endif
#endif /* SWEIK_H */
