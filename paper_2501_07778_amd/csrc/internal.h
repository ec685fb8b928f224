// internal.h — shared declarations of the QTT library (host and device).
//
// Internal tensor trains are "slotted": core k lives at a fixed element
// offset computed on the host from rank caps, and the actual ranks live in
// device memory.  Kernels read the ranks and exit early on work beyond them,
// so sequences of kernels (a rounding sweep, a CG iteration) run without
// host round trips.  Cores are column-major: element (a, i, j, b) of a
// matrix core with ranks (r0, r1) and modes (n, m) sits at
// a + r0 * (i + n * (j + m * b)); vectors have m = 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/qtt.h"

#define QTT_MAXD QTT_MAX_CORES

namespace qtt {

struct TTView {
  int32_t D;
  int32_t n[QTT_MAXD];      // row modes
  int32_t m[QTT_MAXD];      // column modes (1 for vectors)
  int64_t off[QTT_MAXD];    // element offset of slot k in `data`
  int32_t cap[QTT_MAXD + 1];  // rank caps the slots are sized for
  int32_t *rk;              // device ranks (D + 1 entries)
  double *data;
};

// ---------------------------------------------------------------- errors
// Entry points that launch kernels start by clearing HIP's per-thread last
// error: a failed runtime call made earlier by another library in the same
// thread would otherwise be reported by the first launch check.
inline void clear_stale_error() { (void)hipGetLastError(); }

void set_error(const std::string &msg);
qtt_status fail(qtt_status st, const std::string &msg);
// Validates a caller's train: core count and modes in range; with
// need_ranks also boundary ranks 1, interior ranks in range, capacity for
// the packed cores and non-NULL data.
qtt_status check_tt(const qtt_tt *t, const char *name, bool need_ranks);
hipError_t publish_ranks(const qtt_tt *t, hipStream_t s);
#define QTT_HIP(call)                                                     \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      return ::qtt::fail(QTT_E_HIP, std::string(#call) + ": " +           \
                                        hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------- timing
// Kernels that qtt_kernel_timing can time (ktimer.cpp): ktimer_begin
// records an event on `s` before the launch and returns a handle (-1 when
// timing is off), ktimer_end records the closing event after it.
enum KernelTimerId { KT_SVD_STEP = 0, KT_SKETCH_QR = 1, KT_QR_STEP = 2, KT_COUNT = 3 };
int ktimer_begin(int id, hipStream_t s);
void ktimer_end(int handle, hipStream_t s);

// ---------------------------------------------------------------- arena
// Bump allocator over the caller's workspace; `dry` mode only counts.
struct Arena {
  char *base = nullptr;
  size_t size = 0;
  size_t used = 0;
  bool dry = false;
  void *take(size_t bytes) {
    size_t a = (used + 255) & ~size_t(255);
    used = a + ((bytes + 255) & ~size_t(255));
    if (dry || used > size) return nullptr;
    return base + a;
  }
  bool ok() const { return dry || used <= size; }
};

// slotted TT bookkeeping on the host
struct TTDesc {
  TTView v;          // passed by value to kernels
  int64_t elems = 0; // total slot elements
  int rmax_cap() const {
    int r = 1;
    for (int k = 0; k <= v.D; ++k) r = r > v.cap[k] ? r : v.cap[k];
    return r;
  }
};

// Fill modes and caps, compute slot offsets; returns total elements.
int64_t layout(TTView &v, int D, const int32_t *n, const int32_t *m,
               const std::vector<int> &caps);
// caps for a TT of uniform cap r limited by the mode products from each end
std::vector<int> bounded_caps(int D, const int32_t *n, const int32_t *m,
                              int r);
// allocate a slotted TT (data + device ranks) from the arena
bool arena_tt(Arena &ar, TTDesc &t, int D, const int32_t *n,
              const int32_t *m, const std::vector<int> &caps);

// ---------------------------------------------------------------- kernels
// All launchers enqueue on `s` and return hipGetLastError().
hipError_t launch_matvec(const TTView &A, const TTView &x, const TTView &y,
                         qtt_dtype compute, hipStream_t s);
hipError_t launch_set_product_ranks(const TTView &A, const TTView &x,
                                    const TTView &y, hipStream_t s);

// packed <-> slotted copies; `ranks_dev` of the packed side are the
// slotted side's device ranks.
hipError_t launch_unpack(const double *packed, const TTView &dst,
                         hipStream_t s);
hipError_t launch_pack(const TTView &src, double *packed, hipStream_t s);
hipError_t launch_copy_tt(const TTView &src, const TTView &dst,
                          hipStream_t s);

// z = a*x + b*y by core concatenation.  a_dev/b_dev (may be NULL) multiply
// the host scalars.
hipError_t launch_axpby(double a, const double *a_dev, const TTView &x,
                        double b, const double *b_dev, const TTView &y,
                        const TTView &z, hipStream_t s);
// v <- c v (the first core is scaled); c_dev (may be NULL) multiplies c
hipError_t launch_scale(const TTView &v, double c, hipStream_t s, const double *c_dev = nullptr);
// <x, y> into *out (device), workspace of `ws_elems` doubles
hipError_t launch_dot(const TTView &x, const TTView &y, double *out,
                      double *ws, int64_t ws_elems, hipStream_t s);
int64_t dot_ws_elems(const TTView &x, const TTView &y);
// <x, A y> (A a TT matrix) without forming A y; ws of dot3_ws_elems doubles
hipError_t launch_dot3(const TTView &x, const TTView &A, const TTView &y, double *out,
                       double *ws, int64_t ws_elems, hipStream_t s);
int64_t dot3_ws_elems(const TTView &x, const TTView &A, const TTView &y);
// tiny scalar programs on device scalars
hipError_t launch_scalar(int op, double *s0, const double *s1,
                         const double *s2, double c, hipStream_t s);
enum ScalarOp {
  SC_DIV = 0,        // s0 = s1 / s2
  SC_NEG = 1,        // s0 = -s1
  SC_COPY = 2,       // s0 = s1
  SC_SQRT_DIV = 3,   // s0 = sqrt(max(s1,0)) / c
  SC_SET = 4,        // s0 = c
  SC_DIV_POS = 5,    // s0 = s2 > 0 ? s1 / s2 : 0
  SC_NORM2 = 6,      // s0 = s1[0]^2 - s1[1] (squared norm after truncation)
  SC_DIFF_DIV = 7    // s0 = s2[0] > 0 ? (s1[0] - s1[1]) / s2[0] : 0
};

// rounding (exact algorithm); ws sized by round_workspace_elems
struct RoundWs {
  double *carry, *rbuf, *work, *vbuf, *fold, *scal;  // scal: norm, err2
  double *rotlog = nullptr;                           // Jacobi rotations
  int *iwork;
  int64_t carry_elems, sq_elems;
};
int64_t round_ws_bytes(const TTView &x);
bool round_ws_take(Arena &ar, const TTView &x, RoundWs &w);
// rounds x in place: ranks stay on the device; norm -> w.scal[0],
// sum of discarded sigma^2 -> w.scal[1].  eps_dev (may be NULL) replaces
// eps by *eps_dev (device scalar).
// left_orth: cores 0..D-2 are already left-orthogonal (e.g. the output of
// sketch_tt), so the QR sweep is skipped.  rank_bound > 0: the device ranks
// are known to be <= rank_bound (it selects faster kernel variants).
hipError_t round_tt(const TTView &x, double eps, int rmax, const RoundWs &w,
                    hipStream_t s, bool left_orth = false, int rank_bound = 0);

// randomised rounding of y to ranks <= ell (Gaussian sketch, seed/call
// select the random numbers); ws holds sketch_ws_elems(y, ell) doubles
int64_t sketch_ws_elems(const TTView &y, int ell);
hipError_t sketch_tt(const TTView &y, int ell, uint64_t seed, uint64_t call, double *ws,
                     hipStream_t s);

// dense vector of a TT vector (first core least significant); host ranks
// `rk` must equal the device ranks.  ws: full_ws_elems doubles.
int64_t full_ws_elems(const TTView &v, const int32_t *rk);
hipError_t tt_full(const TTView &v, const int32_t *rk, double *out, double *ws,
                   hipStream_t s);
// out[0] = sum_i (a_i - b_i)^2 over n entries, out[1] = sum_i a_i^2
hipError_t launch_diff_norm2(const double *a, const double *b, int64_t n, double *out,
                             hipStream_t s);

// fills the device ranks from a host array
hipError_t upload_ranks(const TTView &v, const int32_t *ranks,
                        hipStream_t s);

// ---------------------------------------------------------------- ALS
// Kernels of the one-site ALS solve (k_als.hip); all dimensions are host
// values, cores column-major as above, environments P[a, al, a'] (vector
// rank, operator rank, vector rank) and Q[a, c] (vector rank, load rank).
hipError_t als_env3_left(const double *P, const double *X, const double *A, const double *Y,
                         double *Pn, double *W1, double *W2, int r0, int ra0, int n, int ra1,
                         int r1, hipStream_t s);
hipError_t als_env3_right(const double *Pn, const double *X, const double *A, const double *Y,
                          double *P, double *W1, double *W2, int r0, int ra0, int n, int ra1,
                          int r1, hipStream_t s);
hipError_t als_env2_left(const double *Q, const double *X, const double *F, double *Qn,
                         double *Tm, int r0, int rf0, int n, int r1, int rf1, hipStream_t s);
hipError_t als_env2_right(const double *Qn, const double *X, const double *F, double *Q,
                          double *Tm, int r0, int rf0, int n, int r1, int rf1, hipStream_t s);
// B (N x N, N = r0 n r1) and g (N) of the local system of one core; T holds
// r0^2 n^2 ra1 doubles
hipError_t als_local_system(const double *L, const double *K, const double *R, const double *Lf,
                            const double *F, const double *Rf, double *T, double *B, double *g,
                            int r0, int ra0, int n, int ra1, int r1, int rf0, int rf1,
                            hipStream_t s);
// B y = g for SPD B: B below its diagonal blocks is overwritten by the
// Cholesky factor L, the diagonal blocks of L go to Lst (als_chol_diag_elems
// doubles), z = L^-1 g to z (N doubles), y receives the solution, g is
// consumed; zz (may be NULL) receives <y, g> (computed as <z, z>); *flag
// becomes nonzero on a pivot <= 0
int64_t als_chol_diag_elems(int64_t N);
hipError_t als_cholesky_solve(double *B, int64_t N, double *g, double *y, double *Lst, double *z,
                              int *flag, double *zz, hipStream_t s);
// thin Householder QR of W (rows x cols, cols <= rows): Q -> W, R -> R
hipError_t als_qr(double *W, int rows, int cols, double *R, double *tau, hipStream_t s);
hipError_t als_gemm(const double *A, int lda, const double *B, int ldb, bool tb, double *C, int ldc,
                    int M, int N, int K, hipStream_t s);
hipError_t als_fill(double *x, int64_t n, uint64_t seed, double scale, hipStream_t s);
hipError_t als_fill_value(double *x, int64_t n, double v, hipStream_t s);
hipError_t als_vdot(const double *a, const double *b, int64_t n, double *out, hipStream_t s);
hipError_t als_transpose(const double *src, int rows, int cols, double *dst, hipStream_t s);
hipError_t als_pad_core(const double *src, int r0s, int n, int r1s, double *dst, int r0d, int r1d,
                        hipStream_t s);

// the ALS method of qtt_solve (als.cpp)
qtt_status check_als_opts(const qtt_solve_opts *o);
size_t als_workspace_bytes(const qtt_tt *K, const qtt_tt *f, const qtt_solve_opts *o);
qtt_status solve_als(const qtt_tt *K, const qtt_tt *f, const qtt_tt *x0,
                     const qtt_solve_opts *o, qtt_tt *u, qtt_solve_report *rep, void *ws,
                     size_t ws_bytes, hipStream_t s);

}  // namespace qtt
