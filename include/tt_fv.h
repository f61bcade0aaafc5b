/*
 * tt_fv.h -- C ABI of the MI355X (gfx950) tensor-train finite-volume library.
 *
 * Method: Danis et al., "High-order Tensor-Train Finite Volume Method for Shallow Water
 * Equations" (arXiv 2408.03483).  Every field is a 2-core tensor train
 *     X(i1, i2) = sum_a G1(i1, a) * G2(a, i2)          (Section 3.1, 2-D form of the TT)
 * stored as two column-major device arrays: g1 = G1 (n1 x rank) and g2 = G2^T (n2 x rank).
 * For a solution field i1 is the x cell and i2 the y cell.
 *
 * Conventions for every entry point
 *   - Pointers inside tt_matrix are DEVICE pointers owned by the caller.  Their column
 *     capacity `cap` must be at least the rank written into them; the library never
 *     frees or reallocates them.  Leading dimensions are n1 and n2 (no padding).
 *   - All work is enqueued on the stream of the tt_ctx (or solver) and the call returns
 *     after the stream has been synchronised: ranks chosen on the device are read back
 *     to set tt_matrix.rank.  Outputs may not alias inputs.
 *   - Temporary device memory comes from the context's arena, allocated once by
 *     tt_ctx_create / tt_fv_init (tt_ens_create for an ensemble's workers), which also
 *     make the split-K arrival counters, the pinned staging buffer of small read-backs and
 *     the events a context uses; rounding, cross, reciprocal and step calls allocate no
 *     device or pinned memory and create no event.  The exceptions are opt-in: kernel
 *     timing (tt_fv_time_kernel) and the GEMM tile autotuner (tt_gemm_autotune) create
 *     events as they measure.
 *   - A context, solver or ensemble is used by one host thread at a time (the library runs
 *     its own threads inside a call); different objects may be used from different threads.
 *   - Return value: 0 on success, a negative TT_E* code on error (outputs untouched
 *     or partially written), or a positive bitmask of TT_W* warnings.
 *     tt_last_error() gives a message for the last failure in the calling thread.
 */
#ifndef TT_FV_H
#define TT_FV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes (negative) */
#define TT_EINVAL  (-1)   /* bad argument: shape, rank, capacity, parameter out of range   */
#define TT_ENOMEM  (-2)   /* the context arena is too small for this call                  */
#define TT_EHIP    (-3)   /* a HIP runtime call failed (message in tt_last_error)          */
#define TT_ENONFINITE (-4)/* NaN or Inf met in a factorisation                             */
#define TT_EDOMAIN (-5)   /* the Taylor series of 1/x diverges: its term norms grew twice in a
                             row, i.e. |1 - x / mean(x)| >= 1 somewhere (Algorithm 1)       */
/* warning bits (positive) */
#define TT_WRANKCAP  1    /* a rounding hit r_max with a tail above eps                      */
#define TT_WNOCONV   2    /* the Taylor reciprocal stopped at max_terms with Err > eps       */
#define TT_WSKETCH   4    /* a randomized rounding of rank > 96 reached its subspace-iteration
                             limit before its leak bound (rank <= 96 is redone exactly)      */
#define TT_WJACOBI   8    /* a Jacobi SVD stopped at its sweep cap while still rotating      */

/* A 2-core TT.  Cores are always stored in FP64: the FP32 form (TT_PREC_F32) changes the
 * arithmetic of the contractions, not the storage, so the type carries no dtype. */
typedef struct {
  int n1, n2;      /* mode sizes (rows of g1, rows of g2)                                  */
  int rank;        /* current rank: number of valid columns                                */
  int cap;         /* column capacity of both buffers                                      */
  double *g1;      /* device, n1 x cap, column-major, first core G1                        */
  double *g2;      /* device, n2 x cap, column-major, second core transposed (G2^T)        */
} tt_matrix;

typedef struct tt_ctx tt_ctx;   /* stream + device arena + tuning knobs */
typedef struct tt_fv tt_fv;     /* solver: parameters, state, context   */

/* Create a context whose work runs on `hip_stream` (a hipStream_t, NULL = default stream)
 * with a device arena of `arena_bytes` (allocated here, once). */
int  tt_ctx_create(tt_ctx **out, size_t arena_bytes, void *hip_stream);
void tt_ctx_destroy(tt_ctx *ctx);
/* Rounding sketch width (0 = automatic: min(96, max(2 r_max, 16))) and the number of
 * subspace iterations always run (>= 0; more are added while the sketch has not converged). */
int  tt_ctx_set_sketch(tt_ctx *ctx, int width, int power_iters);
/* Arithmetic of the core contractions (rounding GEMMs and Householder QR panels):
 * TT_PREC_F64 (default) or TT_PREC_F32 (FP32 operands and accumulation on the matrix cores;
 * the small SVD, maxvol, the Taylor mean and error estimates and all stored cores stay FP64).
 * Results in FP32 mode are accurate to about 1e-6 relative, so tolerances below that
 * saturate the rank cap. */
/* Iteration limits: the sweep cap of the Jacobi SVDs (default 40; TT_WJACOBI when reached
 * while still rotating) and the number of subspace iterations after which a randomized
 * rounding stops (default 8; an unconverged rounding of rank <= 96 is then redone exactly,
 * otherwise TT_WSKETCH).  Ranges [1, 100] and [0, 16]. */
int  tt_ctx_set_limits(tt_ctx *ctx, int jacobi_max_sweeps, int sketch_max_iters);
#define TT_PREC_F64 0
#define TT_PREC_F32 1
int  tt_ctx_set_precision(tt_ctx *ctx, int precision);
/* QR of the tall-skinny factors inside roundings and cross orthogonalisations (Section 3.2's
 * orthogonalisation step).  TT_QR_CHOLESKY: repeated shifted Cholesky QR on the FP64 matrix
 * cores, at most max_passes passes (default 6, range [2, 8]); a call whose columns are not
 * orthonormal after them is redone with Householder QR (tt_fv_stats.qr_redos).
 * TT_QR_HOUSEHOLDER: Householder TSQR always.  TT_QR_AUTO (default): Cholesky QR for more
 * than 64 columns, Householder QR otherwise (the faster of the two at each width when eight
 * chains share the GPU).  All give the same factors up to round-off. */
#define TT_QR_AUTO        0
#define TT_QR_CHOLESKY    1
#define TT_QR_HOUSEHOLDER 2
int  tt_ctx_set_qr(tt_ctx *ctx, int method, int max_passes);
/* Column enrichment of this context's crosses (tt_cross): TT_ENRICH_KICKS (default) or
 * TT_ENRICH_RESIDUAL (see tt_fv_params.cross_enrich). */
int  tt_ctx_set_enrichment(tt_ctx *ctx, int mode);
/* Fixed shapes for this context's tt_round and tt_cross (on = 1; 0 restores the default):
 * the decisions those calls take on the host are taken on the device (see
 * tt_fv_params.graph).  tt_round: Householder QR, the range finder runs exactly
 * max(1, power iterations) subspace iterations, the output buffers hold the static rank
 * min(r_max, m) of which the columns after the device's rank are zero, and y->rank is the
 * device's rank; sigma_out is not written.  tt_cross: nJ0 <= r_max, the column set lives on
 * the device (r_max entries), the kicks use the key's high word as site and its low word as
 * step.  Each call still reads its rank back; the point of the mode is the solver's graph. */
int  tt_ctx_set_fixed(tt_ctx *ctx, int on);

/* Host-only (no GPU, no context): the decision rules the library takes on the host in its
 * dynamic path and in its fixed-shape kernels (one definition for both), exposed for checking.
 * tt_rule_trunc_rank: the kept rank of a rounding (Section 3.2) from its singular values s
 * (host, m values, descending): the fewest leading values whose discarded tail is within eps
 * of the total, never one at or below max(1e-17, floor_rel) ||s||, at most r_max (>= 1);
 * *capped (optional) = 1 when r_max, not eps or the floor, decided.  Returns the rank, or
 * TT_EINVAL for m < 1, m > 128, r_max < 1 or a null s.
 * tt_rule_kicks: the seeded fresh columns of a cross sweep (Section 3.3): up to `count` indices
 * in [0, n) outside have[0 .. nhave) (distinct), drawn as SplitMix64 outputs mod n from `key`
 * with at most 64 (count + 1) draws; written to out (host, room for count); returns how many,
 * or TT_EINVAL for bad arguments (nhave > 4096, count > 4096). */
int  tt_rule_trunc_rank(const double *s, int m, double eps, int r_max, double floor_rel,
                        int *capped);
int  tt_rule_kicks(const int *have, int nhave, int n, int count, uint64_t key, int *out);

/* TT rounding (Section 3.2): y = best approximation of x with relative Frobenius accuracy
 * eps and rank <= r_max.  x may have any rank <= x->cap; y->cap must be >= r_max.
 * Returns TT_WRANKCAP when the cap truncated more than eps.  The kept singular values
 * are written to sigma_out (host, length >= r_max) when not NULL. */
int tt_round(tt_ctx *ctx, const tt_matrix *x, double eps, int r_max, tt_matrix *y,
             double *sigma_out);

/* A d-core tensor train (Section 3.1, equation TT_def): core k (0-based) is an
 * r[k] x n[k] x r[k+1] array on the device with the left rank index fastest, element
 * G_k(a, i, b) at a + r[k] (i + n[k] b), so both of its unfoldings are column-major;
 * r[0] = r[d] = 1. */
typedef struct {
  int d;
  const int *n;          /* host, d mode sizes                                          */
  int *r;                /* host, d + 1 ranks                                           */
  double *const *cores;  /* host array of d device pointers                             */
} tt_tensor;
/* Rounding of a d-core TT (Section 3.2 extended to d cores: right-to-left orthogonalisation,
 * then left-to-right truncated SVDs at eps / sqrt(d - 1) of the norm each, ranks <= r_max):
 * ||x - y|| <= eps ||x|| when no cap binds.  x's ranks <= 96.  y: same d and modes; each
 * y->cores[k] holds r_max * n[k] * r_max doubles; y->r receives the ranks.  The kept singular
 * values of the d - 1 bonds are written one after another to sigma_out (host, length >=
 * (d - 1) r_max) when not NULL.  Returns TT_WRANKCAP when a cap truncated more than its share
 * of eps. */
int tt_round_nd(tt_ctx *ctx, const tt_tensor *x, double eps, int r_max, tt_tensor *y,
                double *sigma_out);

/* Compression of a full field into a TT (the TT-native replacement of an initial-condition
 * SVD on the host; Section 3.2's truncated SVD applied to a dense matrix): y = a rank-k
 * approximation of F with ||F - y||_F <= eps ||F||_F and k <= r_max as small as the SVD allows,
 * found by a randomized range finder with subspace iterations on the matrix cores (Halko,
 * Martinsson and Tropp 2011) that runs until the discarded directions can move the kept ones
 * by at most 1e-13 of the largest singular value.  F: device, n1 x n2, column-major with
 * leading dimension ld >= n1 (not modified).  y->cap >= r_max; y's first core has orthonormal
 * columns, the second carries the singular values, which are written to sigma_out (host,
 * length >= r_max) when not NULL.  Returns TT_WRANKCAP when r_max (or the 96-column sketch) is
 * what limited the rank, TT_WSKETCH when the iterations stopped unconverged. */
int tt_compress(tt_ctx *ctx, const double *F, int n1, int n2, int ld, double eps, int r_max,
                tt_matrix *y, double *sigma_out);

/* TT rounding that allocates nothing, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same result
 * and arguments as tt_round with a default context (FP64 contractions, automatic sketch), but
 * without a tt_ctx: work runs on hip_stream (a hipStream_t, NULL = default stream) and every
 * temporary lives in one fixed device array of TT_NOALLOC_SCRATCH_BYTES that the library holds
 * on each GPU it runs on until the process ends; the call allocates no device or pinned host
 * memory and creates no events.  The call returns after synchronising hip_stream.
 * Errors: TT_EINVAL for bad arguments (as tt_round); TT_ENOMEM, before any work is enqueued,
 * when an n1 x n2 input of this rank could need more scratch than the maximum (the message
 * gives both sizes; e.g. 1024 x 3072 at rank 1024 with r_max 32 fits, 20000 x 20000 at rank
 * 2000 does not).  All calls on one GPU share that GPU's array, which keeps the last call's
 * contents: calls that overlap in time on the same GPU (several threads, or several streams)
 * race and must be serialised by the caller. */
#define TT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tt_round_noalloc(const tt_matrix *x, double eps, int r_max, tt_matrix *y,
                     double *sigma_out, void *hip_stream);

/* Elementwise (Hadamard) product of two TTs on the same index space followed by rounding:
 * y = round(x o z, eps, r_max).  The product has rank x.rank * z.rank (Section 4.2). */
int tt_hadamard_round(tt_ctx *ctx, const tt_matrix *x, const tt_matrix *z, double eps,
                      int r_max, tt_matrix *y);

/* Taylor-series reciprocal, Algorithm 1 of the paper: y ~ 1/x.  max_terms counts the
 * constant term (at most max_terms - 1 products); the loop also stops when
 * Err = ||dy||_F / sqrt(n1 n2) <= eps.  err_out / terms_out (host) report the last Err and
 * the number of terms.  Returns TT_WNOCONV when it stopped at max_terms with Err > eps. */
int tt_reciprocal(tt_ctx *ctx, const tt_matrix *x, double eps, int max_terms, int r_max,
                  tt_matrix *y, double *err_out, int *terms_out);

/* Maximum-volume rows of a tall matrix (n x r, n >= r, r <= 96, device, column-major,
 * leading dimension ldq), as in the maxvol algorithm of Goreinov et al. cited in
 * Section 3.3: greedy start, then swaps until max |Q Q[I]^-1| <= tau or maxit swaps.
 * rows_out: host array of r indices. */
int tt_maxvol(tt_ctx *ctx, const double *q, int n, int r, int ldq, double tau, int maxit,
              int *rows_out);

/* Cross interpolation (Section 3.3): an alternating skeleton cross with maxvol pivots of
 * the n1 x n2 matrix whose entries are fn(inputs) (fn is a TT_FN_* id below), started from
 * the column set J0 (host, nJ0 >= 1 distinct indices < n2), `sweeps` sweeps, `kick` fresh
 * column indices per non-final sweep from SplitMix64 keyed by `key`, final rounding at
 * (eps, r_max).  J_out (host, capacity >= r_max + kick * sweeps) receives the column set
 * of the last sweep, *nJ_out its size.  fparams: see TT_FN_*. */
#define TT_FN_IDENTITY   0  /* inputs[0] = X; entry X(i,j)                                   */
#define TT_FN_LLF_LAMBDA 1  /* inputs = h-, m-, h+, m+ (face/quadrature TTs); fparams[0] = g;
                               entry max(|m-/h-| + sqrt(g h-), |m+/h+| + sqrt(g h+))         */
#define TT_FN_WENO_FACE_M 2 /* inputs[0] = cell TT v (n x n); entry (f, j): WENO5 value at face
                               f from the left (cell f-1); fparams = {periodic, sign, eps_w} */
#define TT_FN_WENO_FACE_P 3 /* as above from the right (cell f), mirrored stencils           */
#define TT_FN_WENO_QUAD  4  /* inputs[0] = face TT v (n_f x n); entry (f, j*3+m): WENO5 value
                               at Gauss point m of cell j; fparams = {periodic, sign, eps_w} */
#define TT_FN_RECIP      5  /* inputs[0] = X; entry 1 / X(i,j) (the cross alternative to
                               Algorithm 1 that Section 4.2 names)                          */
#define TT_FN_LLF_FLUX   6  /* LF-cross (the alternative Section 4.2 contrasts with its flux
                               products): inputs = h-, m-, t-, h+, m+, t+ (face/quadrature
                               TTs, n1 x n2/3, normal-first variables); fparams[0] = g;
                               entry (f, c n2/3 + j): component c of the LLF flux
                               (F(U-) + F(U+))/2 - lambda/2 (U+ - U-), F = (m, m^2/h + g h^2/2,
                               m t/h), lambda = max(|m-/h-| + sqrt(g h-), |m+/h+| + sqrt(g h+)) */
int tt_cross(tt_ctx *ctx, int fn, const tt_matrix *inputs, int n_inputs, const double *fparams,
             int n1, int n2, const int *J0, int nJ0, double eps, int r_max, int sweeps,
             int kick, uint64_t key, tt_matrix *y, int *J_out, int *nJ_out);

/* The final step of tt_cross for given pivots (Section 3.3, skeleton decomposition): with Qc
 * the nI leading orthonormal directions of the columns fn(:, J), y = round(Qc Qc[I]^-1
 * fn(I, :), eps, r_max).  J, I: host index arrays (1 <= nJ <= 96 columns < n2, nI <= nJ rows
 * < n1; nI = 0 gives the zero TT).  Inputs and fparams as tt_cross.  TT_EINVAL when the
 * columns have fewer than nI nonzero directions. */
int tt_cross_skeleton(tt_ctx *ctx, int fn, const tt_matrix *inputs, int n_inputs,
                      const double *fparams, int n1, int n2, const int *J, int nJ, const int *I,
                      int nI, double eps, int r_max, tt_matrix *y);

/* Linear reconstruction of one core (Section 4.3.1).  core: n x rank cell values (device).
 * scheme: 3 = Upwind3, 5 = Upwind5.  face_m / face_p (n_f x rank, n_f = n periodic or n + 1
 * with walls) get the face values from the left / right; quad (n*nq x rank, row j*nq + m)
 * gets the Gauss-point values.  Ghost cells: periodic wrap, or mirrored with `sign`. */
int tt_recon_core(tt_ctx *ctx, const double *core, int n, int rank, int scheme, int periodic,
                  double sign, double *face_m, double *face_p, double *quad);

/* ---------------------------------------------------------------------------------------
 * Solver: explicit SSP-RK3 of the TT finite-volume scheme (Sections 4.1-4.4).           */
typedef struct {
  int n;              /* cells per direction on [0, 1]^2 (dx = dy = 1/n)                  */
  int nonlinear;      /* 0: (eta, u, v), Section 2.1 linear SWE; 1: (h, hu, hv) nonlinear  */
  int scheme;         /* 3 Upwind3, 5 Upwind5, 55 WENO5                                    */
  int periodic;       /* 1 periodic in x and y; 0 reflective walls                         */
  double g, H0, f;    /* gravity, mean depth (linear), Coriolis parameter                  */
  double eps;         /* rounding tolerance (relative Frobenius)                           */
  int r_max;          /* rank cap of every rounding, <= 64                                 */
  int taylor_terms;   /* Algorithm 1 terms including the constant (nonlinear)              */
  int cross_sweeps;   /* maxvol cross sweeps                                               */
  int cross_kick;     /* fresh columns per non-final sweep                                 */
  int recip;          /* 1/h: 0 = Taylor series (Algorithm 1), 1 = cross of 1/x            */
  int workers;        /* own worker streams: 0 = default (8), k = k (1: every kernel of the
                         step on one stream), -1 = none (the solver then steps only inside
                         an ensemble, tt_ens_step)                                         */
  int precision;      /* TT_PREC_F64 or TT_PREC_F32 (contractions; see tt_ctx_set_precision) */
  int qr;             /* TT_QR_AUTO, TT_QR_CHOLESKY or TT_QR_HOUSEHOLDER (tt_ctx_set_qr)    */
  double cross_drop;  /* a cross drops fiber directions below this fraction of the largest
                         singular value; 0 = 1e-13, or 1e-6 with FP32 contractions          */
  int eps_rule;       /* TT_EPS_FIXED: `eps` for every rounding.  TT_EPS_PAPER: Section 4.4's
                         rule, set at the start of each step from the state's norms with
                         base = c_eps V^(1/2) dx^(p - 1/2) (V = 1, dx = 1/n, p = 3 for
                         Upwind3, 5 for Upwind5 and WENO5): eq. eps-tt-formula,
                         base / max_q ||q||, for the roundings inside L(Q), the Taylor
                         reciprocal and the crosses; eq. modified-eps-tt-formula,
                         min(1e-3, base / ||q||), for the forward-Euler and SSP-RK3
                         combination roundings of each variable q.  ||q|| is the L2 norm of
                         the cell averages on the unit square (dx times the Frobenius norm of
                         the n x n array); a zero state takes 1e-3.  `eps` is then unused.  */
  double c_eps;       /* C_eps of the paper's rule (> 0; Table 1 lists it per case/scheme)  */
  int bc_x, bc_y;     /* boundary of each axis: 0 = as `periodic` says, TT_BC_PERIODIC,
                         TT_BC_WALL, or TT_BC_EXACT (ghost cells from the TT_TERM_X_* /
                         TT_TERM_Y_* terms of tt_fv_set_terms, Section 5's exact-solution
                         boundaries; at most one axis)                                      */
  double t0;          /* time at the start of the first step (for the terms' time factors) */
  int flux;           /* nonlinear LLF flux: TT_FLUX_PRODUCTS (Section 4.2: 1/h, Hadamard
                         products and roundings, lambda by cross) or TT_FLUX_LF_CROSS (the
                         whole flux vector of a direction by one cross, TT_FN_LLF_FLUX)     */
  int cross_enrich;   /* columns a cross adds per non-final sweep (cross_kick of them):
                         TT_ENRICH_KICKS, seeded fresh indices; TT_ENRICH_RESIDUAL, the
                         4 x cross_kick seeded candidates with the largest residual of the
                         current skeleton (AMEn-style enrichment, Section 3.3)              */
  int graph;          /* 1: fixed shapes captured in a HIP graph.  Every decision the step
                         otherwise takes on the host is taken on the device: a rounding's
                         kept rank (the same rule; the TT keeps the static rank min(r_max, m)
                         of its buffer, zero columns after the device's rank), a cross's kept
                         directions, maxvol rows and seeded kicks (column sets stay on the
                         device per cross site), the Taylor reciprocal's stop (all
                         taylor_terms terms are formed; those after the first with
                         Err <= eps enter times zero).  Inputs of rank <= 96 are rounded
                         exactly, larger ones by the range finder with graph_iters subspace
                         iterations (TT_WSKETCH when its stopping test fails).  The first
                         tt_fv_step step runs eagerly and sets the static ranks and the cross
                         sites' starting columns (with the GEMM tile autotuner on, a second
                         eager step tunes the static shapes); the next step is captured on
                         the solver's own stream (again after a change of dt) and every later
                         step replays the graph, with no host round trip.  Needs Upwind3/5,
                         TT_EPS_FIXED, TT_FLUX_PRODUCTS, seeded kicks, no exact boundaries or
                         terms (tt_fv_set_terms refuses them), plain maxvol pivots
                         (tt_fv_set_pivots refuses the other modes), n > 2 r_max.
                         `workers` sets the branch streams the
                         independent tasks of a phase fork onto inside the graph (0: 4; -1, a
                         member for tt_ens_step: 1, one chain).  Results equal the dynamic
                         path's up to what the fixed iteration count leaves of the range
                         finder's leak.  0: off.                                            */
  int graph_iters;    /* graph mode: subspace iterations of every randomized rounding;
                         0 = 2 with FP64 contractions, 1 with FP32 (whose own rounding
                         error is above what the second iteration removes)                 */
} tt_fv_params;
#define TT_FLUX_PRODUCTS 0
#define TT_FLUX_LF_CROSS 1
#define TT_ENRICH_KICKS    0
#define TT_ENRICH_RESIDUAL 1
#define TT_BC_PERIODIC 1
#define TT_BC_WALL     2
#define TT_BC_EXACT    3

/* A separable term amp cos(omega t + phase) X (x) Y (y) of variable `var` (0..2), t the stage
 * time of SSP-RK3 (t, t + dt, t + dt/2 from the step's start).  `where`:
 *   TT_TERM_FORCING: added to L(Q) (a manufactured solution's forcing, Section 5.4); X has n
 *                    values along x, Y n values along y (cell averages);
 *   TT_TERM_X_LO / TT_TERM_X_HI: ghost cells -3, -2, -1 / n, n+1, n+2 along x on an exact x
 *                    boundary (X, 3 values, ascending) times Y (n cells along y);
 *   TT_TERM_Y_LO / TT_TERM_Y_HI: X (n cells along x) times the ghost cells along y (Y, 3).
 * Ghost cells sum the terms of their side; corners follow the other axis's rule. */
typedef struct {
  int var;
  int where;
  double amp, omega, phase;
  const double *X;    /* host */
  const double *Y;    /* host */
} tt_fv_term;
#define TT_TERM_FORCING 0
#define TT_TERM_X_LO    1
#define TT_TERM_X_HI    2
#define TT_TERM_Y_LO    3
#define TT_TERM_Y_HI    4
#define TT_EPS_FIXED 0
#define TT_EPS_PAPER 1

typedef struct {
  long long steps;            /* steps taken                                              */
  int ranks[3];               /* current state ranks                                      */
  long long roundings;        /* roundings performed                                      */
  long long crosses;          /* crosses performed                                        */
  int last_taylor_terms;      /* terms used by the last reciprocal (graph mode: the terms
                                 formed, taylor_terms)                                     */
  double last_taylor_err;     /* its final Err (graph mode: not read back, 0)              */
  int warnings;               /* OR of TT_W* bits since init                              */
  double flops;               /* algorithmic flop count since init                        */
  double bytes;               /* algorithmic HBM bytes since init                         */
  double timed_ms;            /* event-timed duration of the timed kernel family          */
  long long timed_launches;   /* its launches since tt_fv_time_kernel                     */
  double timed_flops;         /* its algorithmic flops                                    */
  double timed_bytes;         /* its algorithmic bytes                                    */
  long long cross_sweeps_run; /* maxvol sweeps actually run by all crosses                */
  long long learned_crosses;  /* crosses accepted from the learned pivot proposer          */
  long long learned_fallbacks;/* proposer results rejected (plain crosses run instead)     */
  double max_learned_err;     /* largest validation error of an accepted proposer cross    */
  long long sketch_fallbacks; /* randomized roundings redone exactly (limit reached)       */
  long long sketch_unconverged; /* randomized roundings kept unconverged (TT_WSKETCH)      */
  long long jacobi_capped;    /* Jacobi SVDs stopped at the sweep cap (TT_WJACOBI)         */
  long long qr_redos;         /* roundings or orthogonalisations redone with Householder QR
                                 because a Cholesky QR ended without orthonormal columns   */
  double eps_inner;           /* tolerance of the last step's roundings inside L(Q)        */
  double eps_var[3];          /* tolerances of its time-stepping roundings, per variable   */
  double time;                /* time reached (t0 + dt of every step taken)                */
  long long graph_launches;   /* steps replayed from the captured graph (graph mode)       */
} tt_fv_stats;

/* Copy the three initial TTs (caller's device buffers) into solver-owned state and build
 * the reconstruction tables.  Allocates its arena once here. */
int  tt_fv_init(tt_fv **out, const tt_fv_params *p, const tt_matrix q0[3], void *hip_stream,
                size_t arena_bytes);
/* Advance nsteps SSP-RK3 steps of size dt. */
int  tt_fv_step(tt_fv *s, double dt, int nsteps);
/* Largest wave speed per direction over the cells, speed[0] = max |hu/h| + sqrt(g h) and
 * speed[1] = max |hv/h| + sqrt(g h) (nonlinear; sqrt(g H0) for both in the linear case),
 * estimated on the TTs without forming the field: rook pivoting on the pointwise function
 * from every maxvol column of h's second core (a lower bound of the true maximum, which it
 * found on every smooth field tested). */
int  tt_fv_max_speed(tt_fv *s, double speed[2]);
/* The explicit step for a CFL number: *dt = cfl / (speed[0] / dx + speed[1] / dy). */
int  tt_fv_cfl_dt(tt_fv *s, double cfl, double *dt);
/* Replace the solver's separable forcing and boundary terms (copied; count 0 clears them).
 * Errors: TT_EINVAL for a bad var or where, a null factor, or ghost terms on a non-exact
 * axis. */
int  tt_fv_set_terms(tt_fv *s, const tt_fv_term *terms, int count);
/* Copy the state into caller buffers (cap >= rank). */
int  tt_fv_get_state(tt_fv *s, tt_matrix q[3]);
int  tt_fv_get_stats(tt_fv *s, tt_fv_stats *out);
/* Time one launch in `every` of a kernel family: the sampled launches carry a start and a stop
 * event on the stream they run on, which HIP sets to the kernel's own start and end.  The
 * family is every kernel whose timing name starts with `name`: "jacobi", "gemm", the
 * Householder factorisations "tsqr_qr_leaf" and "tsqr_qr_node" ("tsqr_qr" for both), their
 * Q formation "tsqr_wy_node" and "tsqr_wy_leaf" ("tsqr" for all four), "cholqr_slab" and
 * "cholqr_factor" ("cholqr" for both); NULL or "" switches timing off.  The timed_*
 * statistics are reset. */
int  tt_fv_time_kernel(tt_fv *s, const char *name, int every);
void tt_fv_destroy(tt_fv *s);

/* ---------------------------------------------------------------------------------------
 * Full-grid comparator: the same finite-volume scheme (Sections 2.2-2.4: reconstruction,
 * LLF flux, Gauss-Legendre face sums, Coriolis source; SSP-RK3 of Section 4.4 without
 * rounding) on n x n arrays of cell averages, the full-tensor form of Section 4.1 that the
 * paper's speed-ups are measured against.  One fused kernel per RK stage. */
typedef struct tt_grid tt_grid;
/* Uses n, nonlinear, scheme, periodic, bc_x, bc_y, t0, g, H0 and f of `p` (the other fields
 * are ignored).  Allocates two stage buffers of
 * 3 n^2 doubles once here; work runs on hip_stream. */
int  tt_grid_init(tt_grid **out, const tt_fv_params *p, void *hip_stream);
/* Replace the comparator's separable forcing and boundary terms (as tt_fv_set_terms). */
int  tt_grid_set_terms(tt_grid *s, const tt_fv_term *terms, int count);
/* Advance U nsteps SSP-RK3 steps of size dt in place.  U: device, 3 x n x n doubles, variable
 * major, then the x cell, then the y cell (y contiguous), the variables of tt_fv_params'
 * equation set.  Enqueues the stage kernels on the solver's stream and returns; the caller
 * synchronises that stream before reading U. */
int  tt_grid_step(tt_grid *s, double *U, double dt, int nsteps);
void tt_grid_destroy(tt_grid *s);

/* ---------------------------------------------------------------------------------------
 * Learned pivot proposer for the crosses (an addition to the paper, whose crosses choose
 * pivots by alternating maxvol sweeps, Section 3.3).  A perceptron 16 -> 256 -> 256 -> 1
 * (ReLU; BF16 weights and activations, FP32 accumulation) scores every column index of a
 * cross from 16 features of the cross's starting TT (second core B0) and the call site's
 * previous pivots; the previous pivots together with the top K = min(r_max, |J_prev| + kick)
 * indices (at most 96 columns) are the columns of one refinement sweep, accepted or replaced
 * by the plain maxvol cross by the rule of tt_fv_set_pivot_acceptance.  The model is trained
 * with Adam on (features, final maxvol pivots) pairs logged from plain crosses.  Weights:
 * flat FP32 vector of TT_PM_NPARAM entries, W1 (16 x 256, row-major) | b1 | W2 (256 x 256) |
 * b2 | w3 | b3. */
#define TT_PM_NPARAM 70401
#define TT_PIV_MAXVOL  0    /* plain alternating maxvol sweeps                              */
#define TT_PIV_LOG     1    /* plain sweeps; log (features, pivots) into the model          */
#define TT_PIV_LEARNED 2    /* proposer + one sweep, plain sweeps as the fallback           */
#define TT_PIV_REPLAY  3    /* each cross takes the (J, I) given by tt_fv_replay_pivots for
                               its (step, site) and forms only the skeleton (no model)       */
#define TT_PIV_KICKS   4    /* ablation of TT_PIV_LEARNED without a model: the one sweep starts
                               from the previous pivots and fresh SplitMix64 columns          */
typedef struct tt_pm tt_pm;
/* max_rows: capacity of the training log (rows of 16 features); seed: weight init. */
int  tt_pm_create(tt_pm **out, size_t max_rows, unsigned long long seed);
void tt_pm_destroy(tt_pm *pm);
int  tt_pm_set_weights(tt_pm *pm, const float *host, size_t n);
int  tt_pm_get_weights(tt_pm *pm, float *host, size_t n);
/* Scores s (N, device FP32) of features X (N x 16 row-major, device FP32, cast to BF16). */
int  tt_pm_forward(tt_pm *pm, const float *X_dev, int N, float *s_dev);
/* Loss and gradients (flat, host FP32, n = TT_PM_NPARAM) of the weighted logistic loss
 * sum_i w_i (log(1 + e^s_i) - y_i s_i) / N, w_i = pos_weight where y_i = 1, else 1. */
int  tt_pm_grad(tt_pm *pm, const float *X_dev, const float *y_dev, int N, double pos_weight,
                float *grad_host, size_t n, double *loss_out);
/* One Adam step (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8, FP32) of the weights
 * with the caller's gradient (host FP32, n = TT_PM_NPARAM), step count continuing from the
 * model's previous updates. */
int  tt_pm_adam(tt_pm *pm, const float *grad_host, size_t n, double lr);
/* Adam (lr) over the logged samples, positive weight = negatives / positives. */
int  tt_pm_train(tt_pm *pm, int epochs, int batch, double lr, double *loss_out);
int  tt_pm_dataset(tt_pm *pm, size_t *rows, size_t *positives);
/* The 16 features of every index of a cross (B0: n2 x r, ld ldb, device FP64; J_dev: the
 * nJ <= 128 previous pivots) into X_dev (n2 x 16 row-major FP32). */
int  tt_pm_features(tt_ctx *ctx, const double *B0, int n2, int r, int ldb, const int *J_dev,
                    int nJ, float *X_dev);
/* Indices of the k largest scores (ties: smaller index first), ascending, into idx_dev. */
int  tt_pm_topk(tt_ctx *ctx, const float *s_dev, int n, int k, int *idx_dev);
/* Pivot mode of a solver's crosses (TT_PIV_*); pm must outlive its use (NULL with modes 0,
 * 3 and 4). */
int  tt_fv_set_pivots(tt_fv *s, int mode, tt_pm *pm);
/* Acceptance of a one-sweep cross from proposed columns (TT_PIV_LEARNED, TT_PIV_KICKS): its
 * error on 16 seeded validation columns outside J, |f - Y|_F / |Y|_F, must be <= abs_tol;
 * with rel_slack >= 0 a cross is also accepted when that error is <= (1 + rel_slack) times
 * the same error of the site's last plain cross (equal accuracy), and proposals are tried
 * only at sites that have one.  Otherwise the plain maxvol cross runs.  Default: abs_tol
 * 1e-6, rel_slack -1 (the absolute rule alone). */
int  tt_fv_set_pivot_acceptance(tt_fv *s, double abs_tol, double rel_slack);

/* Pivot replay (Section 3.3: a skeleton is fixed by its column and row sets).  At the rank
 * cap several pivot sets of a cross are equally valid and maxvol's choice among them can flip
 * under round-off, so two implementations of the same step are compared by giving both the
 * same sets.  Store the column set J (host, 1 <= nJ <= 96 distinct indices < n2 of that
 * cross) and row set I (host, nI = the rank of the columns f(:, J) after dropping directions
 * below 1e-13 of the largest, 1e-6 with FP32 contractions; the skeleton uses exactly nI
 * leading directions) for the cross at `site` in step
 * `step` (0 = the first step after tt_fv_init).  Sites: base = ((direction * 3 + stage) << 6),
 * direction 0 = x, 1 = y, stage 0..2; lambda cross base + 0; cross 1/h base + 8 + side
 * (0 = minus, 1 = plus); WENO5 Algorithm 2 base + 16 + 4 variable + side and Algorithm 3 the
 * same + 2 (variables in normal-first order h, normal momentum, tangential momentum).  In
 * mode TT_PIV_REPLAY a step fails with TT_EINVAL when a cross finds no entry or its columns
 * have fewer than nI nonzero directions.  Entries are kept until the solver is destroyed. */
int  tt_fv_replay_pivots(tt_fv *s, long long step, int site, const int *J, int nJ, const int *I,
                         int nI);
/* The last sweep's column and row sets of the latest cross at `site` (host outputs of
 * capacity capJ / capI).  Returns 1 when the site has run, 0 (and nJ = nI = 0) when not. */
int  tt_fv_get_pivots(tt_fv *s, int site, int *J, int capJ, int *nJ, int *I, int capI, int *nI);

/* ---------------------------------------------------------------------------------------
 * Batched ensemble: independent solvers advanced together.  Their independent chains of TT
 * operations share one pool of `workers` worker streams; `concurrency` host threads take
 * the members in decreasing cost order (n r_max^4, longest first) and step each one.  A
 * member's result is the same as stepping it alone.  Members must not be stepped
 * elsewhere during the call. */
typedef struct tt_ens tt_ens;
int  tt_ens_create(tt_ens **out, int workers, size_t arena_bytes_per_worker);
int  tt_ens_step(tt_ens *e, tt_fv *const *members, int count, const double *dts, int nsteps,
                 int concurrency);
void tt_ens_destroy(tt_ens *e);

/* GEMM tile-shape autotuner (process-wide; off by default): while on, the first rounding GEMM
 * of each shape class (transposes, precision, M and K rounded up to powers of two, N) times
 * the candidate tile shapes (output tile width 64 or 128; split-K chunks of at least 256,
 * 512 or 1024, or no split) on its stream and keeps the fastest for later calls.  With it on,
 * choices and hence the last bits of results can differ from run to run.  classes_out (may be
 * NULL) receives the number of tuned shape classes. */
int  tt_gemm_autotune(int on, int *classes_out);

const char *tt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TT_FV_H */
