// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tt_fv.h"

namespace ttfv {

// ---------------------------------------------------------------------------------------
// errors: internal code throws, the C ABI layer converts to return codes

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &m);

#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      throw ::ttfv::Error(TT_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

#define TT_REQUIRE(cond, msg)                                                             \
  do {                                                                                    \
    if (!(cond)) throw ::ttfv::Error(TT_EINVAL, msg);                                     \
  } while (0)

// ---------------------------------------------------------------------------------------
// device arena: one hipMalloc at creation, stack-like sub-allocation afterwards

class Arena {
 public:
  Arena() = default;
  ~Arena();
  void init(size_t bytes);
  // use caller-owned device memory (not freed here); its first 256 bytes become the status
  // words, which the caller must have zeroed
  void adopt(void *base, size_t bytes);
  void *alloc(size_t bytes);                 // 256-byte aligned
  double *dalloc(size_t n) { return static_cast<double *>(alloc(n * sizeof(double))); }
  int *ialloc(size_t n) { return static_cast<int *>(alloc(n * sizeof(int))); }
  // status words at the arena's base (zeroed at init, never sub-allocated): [0] counts the
  // Jacobi SVDs on this arena's stream that stopped at their sweep cap
  int *status() const { return reinterpret_cast<int *>(base_); }
  // [FX_WARN]: TT_W* bits and [FX_ERRORS]: FX_ERR_* bits raised by fixed-shape kernels
  size_t mark() const { return top_; }
  void release(size_t m) { top_ = m; }
  size_t capacity() const { return cap_; }
  size_t high_water() const { return hw_; }

 private:
  char *base_ = nullptr;
  size_t cap_ = 0, top_ = 0, hw_ = 0;
  bool owned_ = false;
};

struct Scope {  // releases everything allocated after construction
  Arena &a;
  size_t m;
  explicit Scope(Arena &ar) : a(ar), m(ar.mark()) {}
  ~Scope() { a.release(m); }
};

// ---------------------------------------------------------------------------------------
// a device TT: X = A * B^T, A: n1 x r (ld n1), B: n2 x r (ld n2), column-major

struct DTT {
  int n1 = 0, n2 = 0, r = 0;
  double *A = nullptr, *B = nullptr;
};

struct Counters {
  long long roundings = 0, crosses = 0, extra_power_iters = 0;
  long long sketch_fallbacks = 0;    // range finders unconverged at the limit, redone exactly
  long long sketch_unconverged = 0;  // range finders unconverged at the limit, kept (warning)
  long long qr_redos = 0;            // roundings and orthogonalisations redone with Householder
                                     // QR after a Cholesky QR ended without orthonormal columns
  double flops = 0, bytes = 0;
  int warnings = 0;
};

// status words of fixed-shape execution (fixed.hip) at the arena's base, after the Jacobi count
constexpr int FX_WARN = 1, FX_ERRORS = 2;
constexpr int FX_ERR_NONFINITE = 1, FX_ERR_MEAN = 2, FX_ERR_DOMAIN = 4;

// Optional event timing of one kernel family: one launch in `every` of the kernels whose
// timing name starts with `name` is launched with a start and a stop event, which HIP sets to
// that kernel's own start and end on its stream; pairs are resolved at the next sync.
struct KernelTimer {
  std::string name;                         // empty: off
  int every = 32;                           // one launch in `every` of the family is timed
  long long seen = 0;
  struct Rec {
    hipEvent_t start, stop;
    double flops, bytes;
  };
  std::vector<Rec> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;
  double ms = 0, flops = 0, bytes = 0;
  long long launches = 0;
};

struct Ctx {
  hipStream_t stream = nullptr;
  Arena arena;
  int sketch_width = 0;     // 0: automatic
  int power_iters = 1;      // subspace iterations always run; more are added on demand
  bool fp32 = false;        // core contractions (GEMM, face-splitting products, TSQR) in FP32
  int qr = TT_QR_AUTO;      // QR method of tsqr() (TT_QR_*)
  double cross_drop = 0.0;  // relative singular value below which a cross drops a fiber
  int enrich = 0;           // cross enrichment: 0 seeded kicks, 1 largest residual
                            // direction (0: 1e-13, or 1e-6 with FP32 contractions)
  double drop() const { return cross_drop > 0.0 ? cross_drop : (fp32 ? 1e-6 : 1e-13); }
  int cqr_passes = 6;       // pass limit of the Cholesky QR
  bool householder = false; // force Householder TSQR (the redo after a failed Cholesky QR)
  int jacobi_max_sweeps = 40;     // sweep cap of the one-sided Jacobi SVD
  int sketch_max_iters = 8;       // subspace iterations after which a range finder stops
  // fixed shapes (fixed.hip): ranks and the other decisions stay on the device, every TT keeps
  // its buffer's static rank (zero columns beyond the device's), no host round trip; capturing:
  // the stream is being captured into a HIP graph (sync() does nothing, host reads are errors)
  bool fixed = false;
  bool capturing = false;
  Counters cnt;
  KernelTimer timer;
  int *tile_cnt = nullptr;  // zeroed per-tile arrival counters of split-K GEMMs (this stream)
  int *tile_counters();     // allocates them on first use
  // the context allocates nothing: arena and tile counters are preset on caller memory,
  // small reads go to pageable host memory, sync() waits on the stream, no GEMM autotuning
  bool no_alloc = false;
  double *pinned = nullptr; // pinned host staging for small device-to-host reads
  hipEvent_t sync_ev = nullptr;   // recorded and waited for by sync()
  // events of the sampled launch in progress (set by TimedLaunch, used by TT_LAUNCH)
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  static constexpr size_t kPinnedDoubles = 4096;
  double *pinned_staging(); // allocates it on first use (nullptr in a no_alloc context)
  // events of the Taylor partial sums handed to a helper context, one per term
  std::vector<hipEvent_t> term_ev;
  static constexpr int kTermEvents = 64;
  // allocates now what the context would otherwise allocate on first use (split-K counters,
  // pinned staging, the sync event, the term events), so that rounding, cross and step
  // calls allocate nothing
  void prepare(int term_events = kTermEvents);
  void sync();
  int jacobi_capped();      // syncs; Jacobi SVDs of this context stopped at the sweep cap
  int jacobi_seen = 0;      // the count at the last check (jacobi_warning)
  ~Ctx();
};

// RAII bracket around one launch (made with TT_LAUNCH): when the launch is a sampled one of
// the timed family, the context's launch events are set for it
struct TimedLaunch {
  Ctx &c;
  bool on;
  TimedLaunch(Ctx &ctx, const char *name, double flops, double bytes);
  ~TimedLaunch();
};

// kernel launch on the context's stream carrying the events of a sampled TimedLaunch (none
// otherwise): HIP records the kernel's own start and end in them
#define TT_LAUNCH(c, kernel, grid, block, shmem, ...)                                        \
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, (c).stream, (c).ev_start, (c).ev_stop, 0, \
                        __VA_ARGS__)

struct Solver;

// TT_WJACOBI when Jacobi SVDs of this context stopped at their sweep cap since the last check
int jacobi_warning(Ctx &c);

// ---------------------------------------------------------------------------------------
// launchers (kernels.hip)

void fill_gauss(Ctx &c, double *O, int rows, int cols, int ld, uint64_t seed);
void copy_scale(Ctx &c, double *dst, int ldd, const double *src, int lds, int rows, int cols,
                double alpha);
void axpby(Ctx &c, double *dst, int ldd, const double *x, int ldx, double a, const double *y,
           int ldy, double b, int rows, int cols);
void fill_value(Ctx &c, double *dst, int ld, int rows, int cols, double v);
void khatri_rao(Ctx &c, double *out, int n, const double *X, int rx, const double *Y, int ry);
void colsum(Ctx &c, const double *A, int n, int r, int ld, double *out);
// out[c] = sum of squares of column c
void colsumsq(Ctx &c, const double *A, int n, int r, int ld, double *out);
void gather_rows(Ctx &c, double *dst, int ldd, const double *src, int lds, const int *rows_dev,
                 int nrows, int cols);
// dst (cols x rows) = src^T (src: rows x cols)
void transpose(Ctx &c, double *dst, int ldd, const double *src, int lds, int rows, int cols);

struct StencilSet {          // weights of the combined linear stencils, offsets -k..k
  int k = 0, nq = 0;
  double face[5] = {0};      // value at the right face (x0 = +1/2)
  double quad[3][5] = {{0}}; // value at Gauss point m
  double gw[3] = {0};        // Gauss-Legendre weights (sum 1)
};
// ghost cells of a core column along its mode: periodic wrap; mirror times sign (walls);
// zero (an exact boundary, whose values come as separate columns); or an explicitly extended
// column of n + 6 rows (cells -3 .. n + 2), which the kernels read as is
enum class Ghost : int { Periodic = 0, Wall = 1, Zero = 2, Explicit = 3 };
void recon_face(Ctx &c, const double *A, int n, int r, Ghost rule, double sign,
                const StencilSet &st, double *Am, double *Ap, int nf);
void recon_quad(Ctx &c, const double *B, int n, int r, Ghost rule, double sign,
                const StencilSet &st, double *Bq);
void quad_sum(Ctx &c, const double *Bq, int n, int nq, int r, const StencilSet &st, double *Bo);
void face_diff(Ctx &c, const double *A, int nf, int n, int r, bool periodic, double scale,
               double *Ao, int ldo);
void ghost_extend(Ctx &c, const double *A, int n, int r, Ghost rule, double sign, double *E);

// gemm.hip: C = alpha * op(A) * B + beta * C, op = identity or transpose
void gemm(Ctx &c, bool transA, int M, int N, int K, double alpha, const double *A, int lda,
          const double *B, int ldb, double beta, double *C, int ldc);
void gemm2(Ctx &c, bool transA, bool transB, int M, int N, int K, double alpha, const double *A,
           int lda, const double *B, int ldb, double beta, double *C, int ldc);
// arena bytes of the split-K partial tiles one gemm/gemm2 call of these sizes draws (default
// tile rule; alignment included)
size_t gemm_arena_bytes(int M, int N, int K);
// tile-shape autotuner of the GEMMs (process-wide; off by default)
void gemm_autotune(bool on);
bool gemm_autotune_on();
int gemm_tuned_classes();

// tsqr.hip: Q (n x m, ldq) and R (m x m, ldr) of Y (n x m, n >= m, m <= 96); Q == nullptr
// forms R only
constexpr int QR_MAXM = 96;
int qr_max_cols();   // largest m the device's LDS allows (<= QR_MAXM)
void tsqr(Ctx &c, const double *Y, int n, int m, int ldy, double *Q, int ldq, double *R,
          int ldr);
// arena bytes one FP64 tsqr call of these sizes draws (upper bound, alignment included)
size_t tsqr_arena_bytes(int n, int m);
// cholqr.hip: the same outputs by repeated Cholesky QR on the matrix cores (FP64); tsqr()
// uses it unless the context asks for Householder.  When it ends without orthonormal
// columns, Q and R are NaN.
void cholqr(Ctx &c, const double *Y, int n, int m, int ldy, double *Q, int ldq, double *R,
            int ldr);
size_t cholqr_arena_bytes(int n, int m, bool with_q);

// jacobi.hip
// One-sided Jacobi on M (m x m, ld m, m <= 96): writes U*Sigma columns sorted by norm into
// US (m x m) and the norms into sig (device, m).
// trans: M holds the transpose of the matrix to decompose.  Columns with norm below
// floor_rel ||M||_F take no rotations (a rounding passes eps / 100).
void jacobi_svd(Ctx &c, const double *M, int m, double *US, double *sig, bool trans = false,
                double floor_rel = 0.0, bool accumulate = false);
// accumulate (m <= 96): with trans and M = R, return the product of the rotations scaled by
// the norms, i.e. the left singular vectors of R times Sigma.
// Same outputs for M (m x m, ld m, m <= 96) from a column-pivoted QR M P = Q2 R2 and one-sided
// Jacobi on R2^T (U = Q2 times the accumulated rotations): the pivoting grades R2 so that the
// sweeps drop from ~20 to ~7 on the graded cores of the crosses.
void svd_pivoted(Ctx &c, const double *M, int m, double *US, double *sig, double floor_rel);
// inverse of a small square matrix (m <= 96) with partial pivoting
void small_inverse(Ctx &c, const double *M, int m, int ldm, double *Minv);
// normalise the first k columns of US by sig into U
void normalise_cols(Ctx &c, const double *US, const double *sig, int m, int k, double *U);

// cross.hip.  k_dev (fixed shapes): Q's columns from *k_dev on are zero; the rows chosen for
// them are valid indices but carry no meaning
void maxvol_dev(Ctx &c, const double *Q, int n, int r, int ldq, double tau, int maxit,
                int *rows_dev, const int *k_dev = nullptr);

// fixed.hip: device-side decisions of fixed-shape execution.  trunc_mask: kept rank by the
// rounding rule (rule 0: eps, floor_rel, rmax; q >= 0 also checks a range finder's stop after q
// subspace iterations) or the orthogonalisation rule (rule 1: s_j > eps s_0), written to
// *k_out when not null, and U (m x kcap) = US / s for the kept columns, zero after them;
// *ss_out = sum of the kept s^2 when not null
void trunc_mask(Ctx &c, const double *sg, const double *US, int m, int kcap, int rule,
                double eps, double floor_rel, int rmax, int q, double *U, int *k_out,
                double *ss_out);
void qi_pad(Ctx &c, double *QI, int m, const int *k_dev);
void mask_cols(Ctx &c, double *X, int ld, int rows, int m, const int *k_dev);
// *nJ = *src, then the seeded fresh columns of sweep `sweep` (as kick_indices) while < rmax
void device_kicks(Ctx &c, int *J, int *nJ, const int *src, int n, int kick, int rmax,
                  uint64_t site, const long long *step_dev, int sweep);
// dst = (mul * s[0]) src (mode 0) or (mul / s[0]) src (mode 1), s on the device
void scale_dev(Ctx &c, double *dst, int ldd, const double *src, int lds, int rows, int cols,
               const double *s, double mul, int mode);
void mean_dev(Ctx &c, const double *cs, int r, double N, double *out);
void taylor_start(Ctx &c, double *hist);
void taylor_err(Ctx &c, const double *ss, double N, double eps, double *hist, int terms,
                bool last);
void inc_step(Ctx &c, long long *step);
void count_rank(Ctx &c, const double *B, int n, int r, int *out);
// reads and clears the fixed-shape status words: throws on an error bit, returns TT_W* bits
int fixed_status(Ctx &c);

struct WenoTables {          // candidate stencils and weights for WENO5 (k = 2)
  double face_C[3][3];       // Step 1 candidate r, cell j-r+l, at +1/2
  double face_d[3];          // ideal weights
  double quad_C[3][3][3];    // Step 2, Gauss point m
  double quad_g[3][3];       // linear weights (m = 0, 2); m = 1: unused
  double gp[3], gm[3];       // normalised split weights at m = 1
  double sp, sm;             // sigma+-
};
struct FiberInput {
  const double *A; const double *B; int lda, ldb, r;
};
struct FiberSpec {
  int fn = 0;
  int n_in = 0;
  FiberInput in[6];
  double g = 0, eps_w = 0;
  int nq = 3;
  int ncol = 0;                     // TT_FN_LLF_FLUX: columns per flux component
  const WenoTables *wt = nullptr;   // host table, copied into the kernel arguments
};
// entries fn(i, j) for i in [0,n1), j in J (|J| = nj) into out (n1 x nj, ld n1)
void fiber_cols(Ctx &c, const FiberSpec &fs, int n1, const int *J_dev, int nj, double *out);
// entries fn(i, j) for i in I, j in [0,n2) into outT (n2 x ni, ld n2): transposed rows
void fiber_rows(Ctx &c, const FiberSpec &fs, int n2, const int *I_dev, int ni, double *outT);

// tt_ops.hip (host algorithms)
int round_tt(Ctx &c, const DTT &x, double eps, int rmax, DTT &y, std::vector<double> *sig);
// Frobenius norm of x (sqrt of sum((A^T A) o (B^T B)), the Gram matrices on the matrix cores)
double norm_tt(Ctx &c, const DTT &x);
// tt_nd.hip: rounding of a d-core TT (cores left-rank-fastest; see tt_round_nd)
int round_nd(Ctx &c, int d, const int *n, const int *r, const double *const *in, double eps,
             int rmax, double *const *out, int *r_out, std::vector<double> *sig);
// 2-core TT of a dense n1 x n2 matrix F (device, column-major, leading dimension ld) at
// relative Frobenius accuracy eps, rank <= rmax (randomized range finder; y->cap >= rmax)
int compress_dense(Ctx &c, const double *F, int n1, int n2, int ld, double eps, int rmax, DTT &y,
                   std::vector<double> *sig);
// upper bound of the arena bytes round_tt draws for an n1 x n2 input of rank R with the
// context's default sketch settings (FP64), every branch included
size_t round_arena_bound(int n1, int n2, int R, int rmax);
// orthonormal basis of range(C) (n x m): QR, SVD of R, keep directions above drop * s_0, or
// exactly `want` leading directions when want >= 0
void orth(Ctx &c, const double *C, int n, int m, int ldc, double drop, double *Q, int *k_out,
          int want = -1);
// aux: optional second context (own stream and arena) on which a helper thread forms the
// partial sums while this thread forms the next term
int reciprocal_tt(Ctx &c, const DTT &x, double eps, int K, int rmax, DTT &y, double *err,
                  int *terms, Ctx *aux = nullptr);
std::vector<int> maxvol_host(Ctx &c, const double *Q, int n, int r, int ldq, double tau,
                             int maxit);
int cross_tt(Ctx &c, const FiberSpec &fs, int n1, int n2, std::vector<int> J, double eps,
             int rmax, int sweeps, int kick, uint64_t key, DTT &y, std::vector<int> *J_out,
             std::vector<int> *I_out = nullptr);
// the final step of a cross for given pivots: Qc = the |I| leading orthonormal directions of
// f(:, J), y = round(Qc Qc[I]^-1 f(I, :), eps, rmax)
int skeleton_tt(Ctx &c, const FiberSpec &fs, int n1, int n2, const std::vector<int> &J,
                const std::vector<int> &I, double eps, int rmax, DTT &y);
// fixed shapes: a rounding whose output keeps the static rank min(rmax, m) with zero columns
// after the rank chosen on the device (into *k_dev when not null; *ss_dev = sum of the kept
// s^2); the range finder runs exactly max(power_iters, 1) subspace iterations
int round_fixed(Ctx &c, const DTT &x, double eps, int rmax, DTT &y, int *k_dev = nullptr,
                double *ss_dev = nullptr);
// fixed shapes: orth with the kept count on the device (Q: n x m, zero after it)
void orth_fixed(Ctx &c, const double *C, int n, int m, int ldc, double drop, double *Q,
                int *k_dev);
// fixed shapes: the maxvol cross from the device column set Jd (capacity m, *nJ active, every
// entry a valid column), updated in place to the set of the last sweep; kicks keyed by site
// and *step_dev as cross_tt's
int cross_fixed(Ctx &c, const FiberSpec &fs, int n1, int n2, int *Jd, int *nJ, int m,
                double eps, int rmax, int sweeps, int kick, uint64_t site,
                const long long *step_dev, DTT &y, int *k_dev = nullptr);
// fixed shapes: Algorithm 1 with K terms, the stopping test as a device predicate (terms after
// the first with Err <= eps are added times zero)
int reciprocal_fixed(Ctx &c, const DTT &x, double eps, int K, int rmax, DTT &y);
uint64_t splitmix64_next(uint64_t &state);
std::vector<int> kick_indices(const std::vector<int> &have, int n, int count, uint64_t key);

// mlp.hip: learned pivot proposer (16 features -> 256 -> 256 -> 1, BF16 on the matrix cores)
typedef unsigned short bf16_t;
constexpr int PM_F = 16, PM_H = 256;
constexpr size_t PM_W1_N = (size_t)PM_F * PM_H, PM_W2_N = (size_t)PM_H * PM_H, PM_W3_N = PM_H;
// flat FP32 parameter vector: W1 (F x H, row-major) | b1 | W2 (H x H) | b2 | w3 | b3
constexpr size_t PM_W1 = 0, PM_B1 = PM_W1 + PM_W1_N, PM_W2 = PM_B1 + PM_H,
                 PM_B2 = PM_W2 + PM_W2_N, PM_W3 = PM_B2 + PM_H, PM_B3 = PM_W3 + PM_W3_N,
                 PM_NPARAM = PM_B3 + 1;

struct PivotModel {
  PivotModel(size_t max_rows, uint64_t seed);
  ~PivotModel();
  void set_weights(const float *host);
  void get_weights(float *host);
  void refresh_bf16();
  void forward(Ctx &w, const bf16_t *Xb, int N, float *s, bf16_t **H1, bf16_t **H2);
  double grad(Ctx &w, const bf16_t *Xb, const float *y, int N, double pos_weight);
  void adam(Ctx &w, double lr);
  void append(Ctx &w, const bf16_t *Xb, const int *J_dev, int nJ, int n2);
  double train(int epochs, int batch, double lr);

  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // FP32 params, grads, Adam
  bf16_t *wb = nullptr;                                              // BF16 W1 | W2 | w3
  bf16_t *Xd = nullptr;                                              // logged features
  float *Yd = nullptr;                                               // logged labels
  size_t cap = 0, rows = 0, positives = 0;
  int t = 0;
  Ctx c;
  std::mutex mu;
};
void pivot_features(Ctx &c, const double *B0, int n2, int r, int ldb, const int *J_dev, int nJ,
                    float *Xf, bf16_t *Xb);
void topk_indices(Ctx &c, const float *s, int n, int K, int *out);
void to_bf16(Ctx &c, const float *x, size_t n, bf16_t *y);

// stencil derivation (stencils.cpp part of fv.hip)
StencilSet derive_stencils(int scheme);
WenoTables derive_weno_tables();

}  // namespace ttfv
