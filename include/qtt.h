/* qtt.h — C ABI of the MI355X QTT finite element hot path.
 *
 * The operations follow the paper's statement of the problem (Alg. 1 and
 * Sec. 4 of "A Low-Rank QTT-based Finite Element Method for Elasticity
 * Problems"): assemble the global stiffness matrix K and load vector f in
 * Z-ordered QTT form, multiply a QTT matrix by a QTT vector core by core
 * (strong Kronecker product), round a tensor train to a relative accuracy
 * (left-to-right QR sweep, right-to-left truncated SVD sweep; the cited
 * TT-rounding algorithm), and solve K u = f to a stated accuracy.
 *
 * Conventions shared by every call
 * --------------------------------
 * - A tensor train (qtt_tt) is D cores.  Core k of a vector has shape
 *   (r_k, n_k, r_{k+1}); core k of a matrix (r_k, n_k, m_k, r_{k+1}).  Cores
 *   are packed back to back in `data` in the order k = 0..D-1, each stored
 *   column-major (the left rank index varies fastest, then n, then m, then
 *   the right rank).  r_0 = r_D = 1.
 * - The first core carries the least significant digit of the global index:
 *   i = i_0 + n_0 (i_1 + n_1 (i_2 + ...)).  For the elasticity problem the
 *   cores are [component | subdomain (q > 1 only) | i1 j1 i2 j2 ... id jd],
 *   so the global dof index is c + 2 (m + q Z(i, j)) with Z the Z-order of
 *   Sec. 3.2.
 * - All values are FP64 in device memory.  `ranks`, `nrow`, `ncol` are host
 *   arrays.  The caller owns every buffer; the library never allocates
 *   device memory: each call takes a caller-provided device workspace
 *   (`ws`, `ws_bytes`, 256-byte aligned) whose size the matching
 *   *_workspace call reports.  (The graph form of the batched step holds
 *   HIP graphs, streams and events of its own, which the runtime owns.)
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *   their kernels on it.  A call whose outputs include host-side ranks or
 *   scalars synchronises that stream before returning; this is stated per
 *   call.
 * - Errors: every call returns a qtt_status; a negative value is an error
 *   and qtt_last_error() returns a description (thread-local).  Nothing
 *   throws across the ABI.  On error the outputs are unspecified.
 */
#ifndef QTT_H
#define QTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QTT_MAX_CORES 40

typedef enum {
  QTT_OK = 0,
  QTT_E_INVAL = -1,       /* bad argument (NULL pointer, bad value)          */
  QTT_E_SHAPE = -2,       /* modes or ranks of the operands do not agree     */
  QTT_E_CAPACITY = -3,    /* an output buffer or the workspace is too small  */
  QTT_E_NOCONV = -4,      /* the solve did not reach its tolerance           */
  QTT_E_HIP = -5,         /* a HIP runtime call failed                       */
  QTT_E_UNSUPPORTED = -7  /* valid request that this library does not do     */
} qtt_status;

typedef enum { QTT_F64 = 0, QTT_F32 = 1, QTT_BF16 = 2 } qtt_dtype;

/* A tensor train in caller-owned memory (the TT/QTT format of Sec. 4:
 * core k holds r_k x n_k (x m_k) x r_{k+1} values, column-major with the
 * left rank fastest, cores packed one after another).  `ncol == NULL` marks
 * a vector. */
typedef struct {
  int32_t ncores;
  const int32_t *nrow;   /* host, ncores mode sizes (1..64)                 */
  const int32_t *ncol;   /* host, ncores column mode sizes (1..64), or NULL */
  int32_t *ranks;        /* host, ncores + 1 ranks; inputs read them,
                            producers write them                           */
  double *data;          /* device, packed cores                            */
  int64_t capacity;      /* number of values available at `data`            */
  int32_t *d_ranks;      /* optional device mirror of ranks (ncores + 1
                            int32 in device memory, or NULL): producers
                            also write the ranks there, on their stream    */
  qtt_dtype dtype;       /* storage type of `data`: QTT_F64 (the only one
                            this library stores; others are refused with
                            QTT_E_UNSUPPORTED).  Low-precision arithmetic is
                            chosen per call by its `compute` argument.     */
} qtt_tt;

/* ------------------------------------------------------------ problem
 * One subdomain carrying 2^level x 2^level nodes (Sec. 3.2): the square
 * [x0, x0+side] x [y0, y0+side], or, when edges = (ax, ay, bx, by) is not
 * all zero, the parallelogram {(x0, y0) + s (ax, ay) + t (bx, by)} with
 * its nodes at s, t = i / (2^level - 1) (an affine image of the square
 * mesh: every element has the same constant Jacobian, the case of the
 * Jacobian expansion of Sec. 3.4 where it is exact).  fixed[s][c] != 0
 * clamps component c (0 = x, 1 = y) on side s (0 = west s = 0, 1 = east
 * s = 1, 2 = south t = 0, 3 = north t = 1) (Sec. 3.8).                   */
typedef struct {
  double x0, y0, side;
  uint8_t fixed[4][2];
  double edges[4];
} qtt_square;

/* Traction t_comp(s) = constant + sum_{k=1..nmodes} amp[k-1] sin(k pi s)
 * on side `side` of subdomain `sub`, s in [0, 1] the normalised arclength. */
typedef struct {
  int32_t sub, side, comp, nmodes;
  const double *amp;
  double constant;
} qtt_traction;

typedef struct {
  int32_t level;            /* d: 2^d nodes per subdomain side              */
  int32_t q;                /* number of subdomains (1..32)                 */
  const qtt_square *sub;    /* q > 1: squares of equal side, edge-to-edge;
                               q = 1: a square or a parallelogram          */
  double E, nu;             /* Young's modulus and Poisson's ratio (Sec. 2) */
  int32_t plane_strain;     /* 1 plane strain, 0 plane stress              */
  double body[2];           /* constant body force                          */
  int32_t ntrac;
  const qtt_traction *trac;
  int32_t coupling;         /* q > 1: QTT_COUPLING_PAPER (0), the paper's
                               coupling rows (Sec. 3.6.1; not symmetric, for
                               assembly only), or QTT_COUPLING_SYMMETRIC
                               (1), the symmetric exact coupling (copy
                               averaging plus copy Laplacian) that the
                               solvers take                                */
  double gamma;             /* q > 1: the coupling penalty; <= 0 selects the
                               paper's choice, the mean diagonal of one
                               subdomain's stiffness (Sec. 3.6.1)          */
} qtt_problem;

enum { QTT_COUPLING_PAPER = 0, QTT_COUPLING_SYMMETRIC = 1 };

/* qtt_assemble_stiffness — Alg. 1: global stiffness K and load f in
 * Z-ordered QTT form after coupling and Dirichlet conditions.
 *   K_bc = P K P + gamma_D (I - P), f_bc = P f, P = diag(mask),
 *   gamma_D = trace(K)/N; q > 1 couples replicated interface nodes
 *   (coupling field above) with gamma = mean diagonal of one subdomain's
 *   stiffness.
 * The stiffness uses exact 2x2 Gauss quadrature of the Q1 element integrals
 * (Sec. 3.3-3.4), the loads are mass matrices times nodal intensities
 * (the load-vector equation of Sec. 3.5 and its edge analogue).  Both results are
 * rounded to relative accuracy `eps` (use 1e-14).
 * K: matrix with ncores = 1 + (q>1) + 2 level, nrow = ncol = modes; f: vector
 * with the same modes.  The caller provides nrow/ncol arrays and data
 * buffers; ranks are written.  Synchronises `stream`.                      */
qtt_status qtt_assemble_stiffness(const qtt_problem *prob, double eps,
                                  qtt_tt *K, qtt_tt *f, void *ws,
                                  size_t ws_bytes, void *stream);
qtt_status qtt_assemble_workspace(const qtt_problem *prob, size_t *bytes,
                                  int64_t *K_capacity, int64_t *f_capacity);

/* qtt_assemble_bpx — additive multilevel (BPX) preconditioner for the
 * stiffness of one square subdomain (q = 1), the tensor-structured
 * preconditioning the paper points to for very fine grids (Sec. 1):
 *   C = sum_{l=0}^{d} P_l P_l^T per displacement component,
 * P_l interpolating level-l coarse nodal values (fine indices 2^l j, linear
 * between coarse nodes, constant past the last one) onto the fine grid, the
 * coarse node on a clamped end dropped (a clamp at the far end mirrors the
 * construction), then C_bc = P C P + (1/gamma_D)(I - P) with the Dirichlet
 * mask P and gamma_D of qtt_assemble_stiffness.  Each 1-D level has QTT rank
 * <= 5 and C <= ~40 at any level.  C has K's modes; caller-provided data
 * (capacity as K's from qtt_assemble_workspace), ranks written; same
 * workspace as qtt_assemble_stiffness.  QTT_E_UNSUPPORTED for q > 1 or for
 * clamps on both ends of one direction.  Synchronises `stream`.           */
qtt_status qtt_assemble_bpx(const qtt_problem *prob, double eps, qtt_tt *C,
                            void *ws, size_t ws_bytes, void *stream);

/* qtt_matvec — y = A x core by core (strong Kronecker product, Sec. 4):
 *   y_k[(a,b), i, (c,d)] = sum_j A_k[a, i, j, c] x_k[b, j, d],
 * with the pair index (a,b) -> a r^x + b.  Output ranks are products of the
 * input ranks and are written to y->ranks (host, no synchronisation).
 * `compute`: QTT_F64, or QTT_F32 / QTT_BF16 to read the operands rounded to
 * that type and accumulate in FP32 (the result is stored in FP64).         */
qtt_status qtt_matvec(const qtt_tt *A, const qtt_tt *x, qtt_tt *y,
                      qtt_dtype compute, void *ws, size_t ws_bytes,
                      void *stream);

/* qtt_round — TT rounding in place (the cited rounding algorithm): a
 * left-to-right Householder QR sweep moves the norm into the last core,
 * then a right-to-left sweep of truncated SVDs keeps at each bond the
 * smallest rank r with sqrt(sum_{i>=r} sigma_i^2) <= eps ||x|| / sqrt(D-1),
 * capped at rmax (rmax <= 0: no cap).  Matrices are rounded with the long
 * index (i, j) as one mode.  Writes the new ranks to x->ranks, the norm
 * ||x||_F to *norm and sqrt(sum of all discarded sigma^2) to *err (either
 * pointer may be NULL).  Synchronises `stream`.                            */
qtt_status qtt_round(qtt_tt *x, double eps, int32_t rmax, double *norm,
                     double *err, void *ws, size_t ws_bytes, void *stream);
qtt_status qtt_round_workspace(const qtt_tt *x, int32_t rmax, size_t *bytes);

/* qtt_round_sketch — randomised rounding in place for trains whose ranks are
 * far above the result's (products such as K x): randomize-then-orthogonalize
 * (Al Daas et al., SIAM J. Sci. Comput. 2023) with a Gaussian train of rank
 * `ell` drawn from Philox4x32-10 keyed by `seed`, followed by qtt_round(eps,
 * rmax) of the rank-<=ell result.  The error is close to the best rank-ell
 * approximation's with high probability (not a deterministic bound).  *norm
 * and *err are those of the final exact rounding.  Vectors only.
 * Synchronises `stream`.                                                   */
qtt_status qtt_round_sketch(qtt_tt *x, int32_t ell, uint64_t seed, double eps, int32_t rmax,
                            double *norm, double *err, void *ws, size_t ws_bytes,
                            void *stream);
/* Workspace bytes of qtt_round_sketch for x's current ranks and `ell`.    */
qtt_status qtt_round_sketch_workspace(const qtt_tt *x, int32_t ell, size_t *bytes);

/* qtt_matvec_round — the hot step of every solver iteration in one call:
 * y = round(A x), the product formed in the workspace (never in y) and
 * rounded in place there: with ell > 0 by a Gaussian sketch of rank ell
 * (as qtt_round_sketch), then the exact rounding to (eps, rmax); with
 * ell = 0 by the exact rounding alone.  y receives the rounded train
 * (capacity for ranks min(rmax, ...) is enough) and its ranks; *norm and
 * *err as qtt_round.  compute as qtt_matvec.  Synchronises `stream`.      */
qtt_status qtt_matvec_round(const qtt_tt *A, const qtt_tt *x, qtt_tt *y, qtt_dtype compute,
                            int32_t ell, uint64_t seed, double eps, int32_t rmax, double *norm,
                            double *err, void *ws, size_t ws_bytes, void *stream);
qtt_status qtt_matvec_round_workspace(const qtt_tt *A, const qtt_tt *x, int32_t ell,
                                      size_t *bytes);

/* qtt_dot — <x, y> of two TT vectors of equal modes (left-to-right
 * environment sweep): the inner product of the TT format of Sec. 4, which
 * the iterative solves use for step lengths and norms.  Synchronises
 * `stream`.                                                                */
qtt_status qtt_dot(const qtt_tt *x, const qtt_tt *y, double *out, void *ws,
                   size_t ws_bytes, void *stream);

/* qtt_dot_noalloc — qtt_dot for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same kernels, with the
 * scratch (device ranks, result, environments) in a library-owned device
 * array of 16 MiB per GPU, held from the first call on that GPU until the
 * process ends.  It allocates nothing.  Returns QTT_E_CAPACITY (before any
 * device work) when the operands need more scratch than that: 2 (r_x r_y)
 * + r_x n r_y doubles at the widest core plus 64.  Every call on one GPU
 * shares the array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Synchronises
 * `stream`.                                                               */
qtt_status qtt_dot_noalloc(const qtt_tt *x, const qtt_tt *y, double *out, void *stream);

/* qtt_axpby — z = a x + b y in the TT format of Sec. 4, whose sum is a
 * core concatenation (ranks add): the first
 * cores sit side by side, middle cores block-diagonally, last cores stacked;
 * a and b scale the first core.  z must not alias x or y.  Writes z->ranks
 * (host, no synchronisation); the workspace needs 1 KiB.                   */
qtt_status qtt_axpby(double a, const qtt_tt *x, double b, const qtt_tt *y,
                     qtt_tt *z, void *ws, size_t ws_bytes, void *stream);

/* qtt_tt_combine — z = sum_i coeffs[i] x[i] for nterms TT vectors of equal
 * modes (at least two cores) by core concatenation (ranks add): first
 * cores side by side, each scaled by its coefficient, middle cores
 * block-diagonal, last cores stacked.  coeffs is a host array; z must not
 * alias a term and needs capacity for the summed ranks, which are written
 * to z->ranks (host, no synchronisation).  Used to form superposed
 * solutions of a linear problem (the training targets of the learned warm
 * start).                                                                 */
qtt_status qtt_tt_combine(int32_t nterms, const double *coeffs, const qtt_tt *const *x,
                          qtt_tt *z, void *stream);

/* ------------------------------------------------------------ solve   */
typedef enum {
  QTT_SOLVE_CG_IR = 0,     /* truncated CG with FP64 iterative refinement      */
  QTT_SOLVE_CHEBYSHEV = 1, /* preconditioned Chebyshev iteration, true residual
                              every step (needs `precond`)                      */
  QTT_SOLVE_FCG = 2,       /* flexible preconditioned CG (one stored direction),
                              true residual every step, exact step length
                              (needs `precond`)                                */
  QTT_SOLVE_ALS = 3,       /* one-site alternating least squares at fixed
                              ranks: the core update of the paper's AMEn
                              solver (Sec. 4) without residual enrichment   */
  QTT_SOLVE_AMEN = 4       /* one-site ALS sweeps with residual enrichment
                              between them: ranks adapt to the solution     */
} qtt_solve_method;

typedef struct {
  double tol;        /* CG_IR: stop when ||f - K u|| <= tol ||f|| (FP64).
                        CHEBYSHEV, FCG: stop when sqrt(<r, C r>) <= tol sqrt(<f, C f>)
                        with r = f - K u: the preconditioned residual, equal to
                        the relative energy-norm error within sqrt(lmax/lmin).
                        ALS: stop when the change of u over a sweep is
                        <= tol ||u||                                          */
  double eps;        /* rounding accuracy of the iterate u                    */
  int32_t rmax;      /* rank cap of u                                         */
  double eps_in;     /* rounding accuracy of the residual, the preconditioned
                        residual and the search direction (relative to each
                        vector's own norm)                                    */
  int32_t rmax_in;   /* rank cap of those vectors (<= rmax for CHEBYSHEV);
                        ALS: first rank of the rank ramp (>= rmax: none)     */
  double red_in;     /* CG_IR: residual reduction of each correction solve   */
  int32_t maxit_in;  /* CG_IR: CG iterations per correction solve;
                        CHEBYSHEV, FCG: iterations in total                   */
  int32_t maxit_out; /* CG_IR: refinement steps; ALS: sweeps in total        */
  int32_t check_every; /* iterations between host convergence checks        */
  qtt_dtype compute; /* products of the correction: QTT_F64, QTT_F32 or
                        QTT_BF16 with FP32 accumulation (CG_IR: K p; CHEBYSHEV
                        and FCG: C r and the power steps); the residual
                        f - K u, QR, SVD and inner products stay FP64        */
  int32_t sketch;    /* 0: exact rounding of every product; > 0: round
                        products by a randomised sketch of this oversampling
                        before the exact rounding                            */
  uint64_t seed;     /* seed of the sketch generator (Philox4x32-10)         */
  const qtt_tt *precond; /* NULL, or a QTT matrix C ~ K^-1 (symmetric positive
                        definite, e.g. from qtt_assemble_bpx)                */
  int32_t method;    /* qtt_solve_method                                     */
  double lmin;       /* CHEBYSHEV: lower bound of the spectrum of C K; <= 0
                        takes 0.09, the bound measured for qtt_assemble_bpx's
                        operator on the cantilever family (levels 2..6)      */
  double lmax;       /* CHEBYSHEV: upper bound of the spectrum of C K; <= 0
                        estimates it by 12 power steps on C K started from f,
                        times 1.12 (reported back in the report)            */
} qtt_solve_opts;

typedef struct {
  int32_t status;         /* QTT_OK or QTT_E_NOCONV                           */
  int32_t outer;          /* CG_IR: refinement steps taken                    */
  int32_t inner;          /* CG iterations (CG_IR) or Chebyshev iterations    */
  double residual;        /* final ||f - K u|| / ||f|| in FP64 (dense check)  */
  double residual_hist[64]; /* CG_IR: residual before each refinement step;
                             CHEBYSHEV: stop criterion at each check        */
  int32_t max_rank;       /* largest bond rank of u                           */
  double criterion;       /* value of the stop criterion at exit              */
  double lmax;            /* CHEBYSHEV: the upper spectral bound used         */
  int32_t warm_start;     /* 0: no x0; 1: the iteration started from
                             alpha x0 (see qtt_solve); -1 (ALS): x0 was
                             rejected (no component along the solution, or
                             not finite) and the cold start ran instead    */
  double warm_energy;     /* ALS with x0: J(alpha x0) = -<f, x0>^2 /
                             (2 <x0, K x0>), the energy of the scaled start
                             (the solution's is -<f, u>/2; their difference
                             is half the squared energy-norm error of the
                             start); 0 otherwise                           */
} qtt_solve_report;

/* qtt_solve — solve K u = f (K symmetric positive definite), the linear
 * system of the discretised elasticity problem (Sec. 3.7, with the
 * Dirichlet conditions of Sec. 3.8), on the QTT format with every iterate
 * rounded (the paper solves it in the TT format by AMEn, Sec. 4, Sec. 5).
 * CG_IR: the outer loop forms the residual f - K u exactly (product,
 * difference), checks its FP64 norm and rounds it; the inner loop runs
 * truncated (P)CG on K e = r with its vectors rounded to (eps_in, rmax_in);
 * u <- round(u + e, eps, rmax).
 * FCG: z = round(C r), p = round(z - beta p) with beta = <z, K p>/<p, K p>,
 * u = round(u + alpha p) with alpha = <f - K u, p>/<p, K p> evaluated from u
 * and p themselves (three-operand inner products, no product formed), so
 * the energy error decreases at every step whatever the truncation of z and
 * p (Notay's flexible CG with one stored direction); r = round(f - K u) is
 * recomputed from the iterate; stop as CHEBYSHEV.
 * ALS: one-site alternating least squares at fixed ranks (the bounded caps
 * of rmax): each core in turn minimises the energy <u, K u>/2 - <u, f>
 * with the other cores fixed and orthogonal (a dense SPD local system of
 * r_k n_k r_{k+1} unknowns solved by Cholesky), sweeping left-right and back;
 * stop when the change of u over a sweep, bounded by the sum of the local
 * changes ||y_k - x_k|| (exact per core: the frames are orthonormal),
 * relative to ||u||, is <= tol (criterion = that bound, one entry of
 * residual_hist per sweep), at most maxit_out sweeps; eps > 0 then rounds u
 * (exact rounding).  rmax_in < rmax ramps the rank: 3 sweeps at rmax_in,
 * 3 at 2 rmax_in, ... (each stage zero-pads the cores of the last), then
 * sweeps at rmax until tol; maxit_out counts the sweeps of all stages.
 * Local systems, QR and the final residual are FP64 (compute must be
 * QTT_F64); precond, eps_in, red_in, maxit_in, check_every and sketch are
 * unused; seed selects the random start cores when x0 is NULL (x0 is
 * zero-padded to the ranks of the first stage that holds it).  x0 enters
 * scaled by alpha = <f, x0> / <x0, K x0>, the minimiser of the energy
 * J(alpha x0) = alpha^2 <x0, K x0>/2 - alpha <f, x0>; an x0 with
 * <f, x0> = 0 (no better than no start at all) or non-finite values is
 * rejected and the cold start runs (report warm_start = -1), so a learned
 * start can only cost its check.  The
 * workspace holds one local matrix (8 (r n r)^2 bytes at the widest core)
 * and the trains of the final FP64 residual check (ranks R_k r_k).
 * rmax <= 512.
 * AMEN: the solver the paper uses (Sec. 4, Sec. 5), in the form of ALS
 * sweeps alternated with a global enrichment step (the ALS(t+z) scheme of
 * Dolgov and Savostyanov 2014 that AMEn localises): the sweeps start at the
 * ranks rmax_in (random cores, or x0); after every pair of sweeps the
 * residual z = f - K u is formed exactly and rounded by a rank-(rmax_in + 8)
 * sketch to (eps_in, rmax_in), then u <- round(u + alpha z, eps, rmax - rmax_in)
 * with the energy-optimal alpha = <f - K u, z> / <z, K z> (three-operand
 * inner products).  The enrichment adds the residual's directions to every
 * core's basis and the rounding keeps only what the accuracy eps needs,
 * so the ranks grow where the solution needs them instead of following
 * caps.  Stop when the sweep change is <= tol and the enrichment moved u
 * by at most tol ||u||; eps > 0 then rounds u.  rmax >= 2 rmax_in and
 * rmax_in >= 1 are required; otherwise as ALS (FP64 local systems, the
 * start check of x0, report fields; inner counts local solves).
 * CHEBYSHEV: u_{k+1} = u_k + d_k with d_k = c1 d_{k-1} + c2 round(C r_k),
 * r_k = round(f - K u_k) recomputed from u_k at every step (so rounding
 * errors do not accumulate in a recurrence), c1, c2 from the Chebyshev
 * polynomials on [lmin, lmax] (Golub-Varga two-term form).
 * x0 (NULL: zero) is the starting guess.  u must have capacity for rank
 * rmax.  Writes u->ranks and the report.  Synchronises `stream`.  Returns
 * QTT_E_NOCONV (with the last iterate in u) when the iteration limit is
 * reached.                                                                 */
qtt_status qtt_solve(const qtt_tt *K, const qtt_tt *f, const qtt_tt *x0,
                     const qtt_solve_opts *opts, qtt_tt *u,
                     qtt_solve_report *report, void *ws, size_t ws_bytes,
                     void *stream);
qtt_status qtt_solve_workspace(const qtt_tt *K, const qtt_tt *f,
                               const qtt_solve_opts *opts, size_t *bytes);

/* ------------------------------------------------------------ batched  */
/* One independent solve of a batch: the arguments of qtt_solve, with its
 * own workspace and stream (streams of default priority, all on one
 * device).                                                                 */
typedef struct {
  const qtt_tt *K, *f, *x0;
  const qtt_solve_opts *opts;
  qtt_tt *u;
  qtt_solve_report *report;
  void *ws;
  size_t ws_bytes;
  void *stream;
  int32_t status;         /* written: the case's qtt_status                 */
} qtt_solve_case;

/* qtt_solve_batched — many load cases (any levels, ranks and options) solved
 * concurrently: `concurrency` host workers each take the next unsolved case
 * and run qtt_solve on that case's stream, so up to `concurrency` solves
 * keep the GPU busy at once (each solve alone is a chain of small,
 * mostly one-workgroup kernels).  concurrency <= 0 uses the value the
 * autotuner stored for the batch's largest level, else 8.  Returns QTT_OK
 * when every case converged, otherwise the first failing case's status;
 * every case's own status is in cases[i].status.  Synchronises all the
 * cases' streams.  No multi-GPU split: the batch runs on the current
 * device.                                                                  */
qtt_status qtt_solve_batched(int32_t n, qtt_solve_case *cases, int32_t concurrency);

/* qtt_autotune_batched — times qtt_solve_batched on the given cases at
 * concurrency 1, 2, 4, 8, 16 and 32 (each run solves all n cases), stores
 * the fastest for the batch's largest level and returns it in *best (and
 * the converged solves/s of each candidate in rates[6] when rates is not
 * NULL).  A case that stops at its iteration limit (QTT_E_NOCONV) is a
 * finished run for the timing but not a solve; any other failure stops the
 * tuning and is returned.  The cases' results are those of the last run and
 * the return value is their aggregate status (QTT_E_NOCONV when some case
 * did not converge; *best is written either way).                          */
qtt_status qtt_autotune_batched(int32_t n, qtt_solve_case *cases, int32_t *best,
                                double *rates);

/* One y = round(A x) of a batch of hot steps (arguments of qtt_matvec_round
 * without the workspace and stream, which belong to the workers).          */
typedef struct {
  const qtt_tt *A, *x;
  qtt_tt *y;
  qtt_dtype compute;
  int32_t ell;
  uint64_t seed;
  double eps;
  int32_t rmax;
  double norm, err;       /* written */
  int32_t status;         /* written */
} qtt_matvec_round_case;

/* qtt_matvec_round_batched — n independent hot steps (any levels and ranks)
 * run by `nworkers` host workers, worker w using ws[w] (ws_bytes[w] bytes,
 * enough for the largest case: qtt_matvec_round_workspace) and streams[w].
 * Returns QTT_OK or the first failing case's status (each case's own in
 * cases[i].status).  Synchronises the workers' streams.                    */
qtt_status qtt_matvec_round_batched(int32_t n, qtt_matvec_round_case *cases, int32_t nworkers,
                                    void *const *ws, const size_t *ws_bytes,
                                    void *const *streams);

/* The batched hot step as one HIP graph.  The launches of n independent
 * steps y_i = round(A_i x_i) (each exactly the launch sequence of
 * qtt_matvec_round, Sec. 4's product and TT rounding) are captured once
 * into `nbranch` independent branches; each replay runs the whole batch
 * with no host synchronisation: as one graph whose branches are parallel
 * paths (per_branch = 0: one hipGraphLaunch), or as one graph per branch,
 * each replayed on a stream of the handle's own, forked from the caller's
 * stream and joined back into it by events (per_branch = 1).
 *
 * qtt_matvec_round_graph_aux_bytes — bytes of the device buffer `aux` that
 *   receives every case's ranks and (norm, squared error).
 * qtt_matvec_round_graph_create — validates every case as qtt_matvec_round
 *   does, and y_i's capacity against the largest ranks the rounding can
 *   leave (the product ranks capped by rmax); assigns the cases to branches
 *   (largest workspace first, least loaded branch), branch b running its
 *   cases in sequence in ws[b] (ws_bytes[b] bytes, enough for each of them:
 *   qtt_matvec_round_workspace); captures and instantiates the graph.  The
 *   graph keeps the addresses of A_i, x_i, y_i (data and d_ranks), the
 *   workspaces and aux, and the ranks of A_i and x_i and the scalars of
 *   each case as they are now: all must stay allocated, and a change of a
 *   rank or scalar needs a new graph.  Refused while qtt_kernel_timing is
 *   on.  Captures on streams of its own (kept by the handle for the
 *   per-branch replays); enqueues nothing.
 * qtt_matvec_round_graph_launch — enqueues one replay on `stream`: y_i's
 *   data and device ranks (d_ranks, when set) are written, host ranks are
 *   not.  Replays that overlap in time race on the workspaces.
 * qtt_matvec_round_graph_collect — synchronises `stream` (the one of the
 *   last replay) and writes y_i's host ranks and cases[i].norm, .err and
 *   .status (cases: the array of n given at creation, or a copy of it).
 * qtt_matvec_round_graph_destroy — frees the graph (NULL is a no-op).    */
typedef struct qtt_graph qtt_graph;
qtt_status qtt_matvec_round_graph_aux_bytes(int32_t n, size_t *bytes);
qtt_status qtt_matvec_round_graph_create(int32_t n, const qtt_matvec_round_case *cases,
                                         int32_t nbranch, void *const *ws,
                                         const size_t *ws_bytes, void *aux, size_t aux_bytes,
                                         int32_t per_branch, qtt_graph **out);
qtt_status qtt_matvec_round_graph_launch(qtt_graph *g, void *stream);
qtt_status qtt_matvec_round_graph_collect(qtt_graph *g, qtt_matvec_round_case *cases,
                                          void *stream);
qtt_status qtt_matvec_round_graph_destroy(qtt_graph *g);

/* ------------------------------------------------------------ warm start */
/* A multilayer perceptron from load parameters to the QTT cores of the
 * displacement (the learned warm start of the solve; not in the paper).
 * sizes[0] inputs, sizes[1..nlayers-1] hidden widths with ReLU,
 * sizes[nlayers] outputs = the packed size of the train's rank pattern.
 * params holds, layer after layer, W_l (sizes[l+1] x sizes[l], column-major)
 * then b_l; adam_m and adam_v have the same layout.  FP32, device memory,
 * caller-owned.  step counts the Adam steps taken.                         */
typedef struct {
  int32_t nlayers;
  const int32_t *sizes;   /* host, nlayers + 1 entries */
  float *params;
  float *adam_m, *adam_v; /* training only (may be NULL for inference) */
  int64_t step;
  int32_t gemm_dtype;     /* QTT_BF16: every layer GEMM (forward and backward)
                             rounds its operands to BF16 and accumulates in
                             FP32 on the matrix cores; QTT_F32 (or QTT_F64,
                             0): FP32 GEMMs.  Parameters, Adam moments,
                             activations and gradients stay FP32.          */
  int32_t loss;           /* QTT_LOSS_TT (0): the gauge-invariant distance of
                             the trains (see qtt_warmstart_train_step);
                             QTT_LOSS_CORES: ||o_j - u_j||^2 / ||u_j||^2 over
                             the packed cores themselves, for targets brought
                             to one gauge by qtt_tt_align (no metric);
                             QTT_LOSS_ANGLE: 1 - <x, u>^2 / (<x, x> <u, u>)
                             with x = TT(o_j), in the metric's norm if one is
                             given: the squared relative error of the best
                             multiple of x, which is the start qtt_solve
                             makes of x (scale-invariant, gauge-invariant). */
} qtt_mlp;

enum { QTT_LOSS_TT = 0, QTT_LOSS_CORES = 1, QTT_LOSS_ANGLE = 2 };

/* Number of floats in params for these layer sizes (-1 on bad input).      */
int64_t qtt_mlp_param_count(int32_t nlayers, const int32_t *sizes);

/* Workspace bytes for a batch (ncores = 0: inference only; otherwise the
 * train's modes nrow[ncores], rank pattern ranks[ncores + 1] and the
 * optional metric of qtt_warmstart_train_step).                            */
qtt_status qtt_warmstart_workspace(const qtt_mlp *net, int32_t batch, int32_t ncores,
                                   const int32_t *nrow, const int32_t *ranks,
                                   const qtt_tt *metric, size_t *bytes);

/* qtt_warmstart_infer — out (sizes[nlayers] x batch, column-major, device)
 * = MLP(a) for a (sizes[0] x batch); each column is the packed train.      */
qtt_status qtt_warmstart_infer(const qtt_mlp *net, const float *a, int32_t batch, float *out,
                               void *ws, size_t ws_bytes, void *stream);

/* qtt_warmstart_train_step — one Adam step (learning rate lr) on the mean
 * over the batch of the loss of net->loss; for QTT_LOSS_TT the
 * gauge-invariant ||TT(o_j) - u_j||^2/||u_j||^2,
 * where o_j = MLP(a_j) and u_j (column j of targets, packed with the same
 * rank pattern, zero-padded) is the target train: forward pass, loss and
 * gradient through the TT inner products (FP64 environments), backward
 * pass, Adam.  With metric (a symmetric positive definite QTT matrix with
 * the train's modes, FP64, e.g. the stiffness matrix) the norm is the
 * energy norm ||v||_A^2 = <v, A v> (three-operand environments); metric
 * NULL: the Frobenius norm.  *loss receives the batch's mean loss before
 * the step.  Synchronises `stream`.                                         */
qtt_status qtt_warmstart_train_step(qtt_mlp *net, const float *a, const float *targets,
                                    int32_t batch, int32_t ncores, const int32_t *nrow,
                                    const int32_t *ranks, const qtt_tt *metric, float lr,
                                    double *loss, void *ws, size_t ws_bytes, void *stream);

/* qtt_warmstart_fit — trains the network natively: `epochs` passes over the
 * n samples (a: sizes[0] x n, targets: sizes[nlayers] x n, column-major
 * device FP32), each pass in a new seeded order (Fisher-Yates with
 * splitmix64 from `seed`) split into n / batch full batches, one Adam step
 * of qtt_warmstart_train_step per batch, the learning rate decaying from
 * lr to lr_final along a half cosine over all steps.  loss_hist (host,
 * `epochs` entries, may be NULL) receives each pass's mean batch loss.
 * Synchronises `stream` once per pass.  Workspace: qtt_warmstart_fit_workspace. */
qtt_status qtt_warmstart_fit(qtt_mlp *net, const float *a, const float *targets, int32_t n,
                             int32_t batch, int32_t epochs, float lr, float lr_final,
                             uint64_t seed, int32_t ncores, const int32_t *nrow,
                             const int32_t *ranks, const qtt_tt *metric, double *loss_hist,
                             void *ws, size_t ws_bytes, void *stream);
qtt_status qtt_warmstart_fit_workspace(const qtt_mlp *net, int32_t n, int32_t batch,
                                       int32_t ncores, const int32_t *nrow, const int32_t *ranks,
                                       const qtt_tt *metric, size_t *bytes);

/* qtt_warmstart_infer_tt — the warm start of one load: x0 (an FP64 TT
 * vector with the given modes, capacity >= sizes[nlayers]) receives the
 * network's output for the parameters a (sizes[0] floats, device) as the
 * packed cores of the rank pattern `ranks`, which are written to
 * x0->ranks.  Pass x0 to qtt_solve; the solve checks it and falls back to
 * its cold start when x0 is no better than zero.  Workspace:
 * qtt_warmstart_workspace(net, 1, 0, ...).                                 */
qtt_status qtt_warmstart_infer_tt(const qtt_mlp *net, const float *a, int32_t ncores,
                                  const int32_t *nrow, const int32_t *ranks, qtt_tt *x0,
                                  void *ws, size_t ws_bytes, void *stream);

/* qtt_tt_contract_last — evaluates a parametric train at one parameter
 * vector: x (D >= 3 cores, FP64, device) whose last core carries a
 * parameter index of size n = x->nrow[D-1]; y (D - 1 cores with x's first
 * D - 1 modes) receives x's cores 0..D-3 unchanged and, as its last core,
 * core D-2 contracted with v = X_{D-1} w (w: n weights, device memory),
 * so that y = sum_i w_i x[..., i].  Writes y->ranks (x's first D - 1 ranks
 * and a final 1; host, no synchronisation).  The last bond rank of x must
 * be <= 1024.  Used for the learned warm start's targets: the solutions of
 * the 16 unit loads as one train with the load index as its last core,
 * rounded once, then evaluated at each load, so every target shares the
 * same cores but the last.                                                */
qtt_status qtt_tt_contract_last(const qtt_tt *x, const double *w, qtt_tt *y, void *stream);

/* qtt_tt_align — brings the TT vector x to the gauge of ref (same modes and
 * ranks, every inner rank <= 48, FP64, device) without changing the vector
 * x represents: for k = D-1 down to 1, with M = X_k R_k^T (the r_k x r_k
 * contraction of core k of x with that of ref over its mode and right
 * index), Q = U V^T from the SVD M = U S V^T is the orthogonal matrix that
 * brings Q^T X_k closest to R_k in the Frobenius norm; core k becomes
 * Q^T X_k and core k-1 absorbs Q.  For trains in a right-orthogonal gauge
 * this removes the sign and rotation freedom of the SVD, so that targets of
 * nearby loads have nearby cores (the training targets of QTT_LOSS_CORES).
 * A bond whose M has a singular value below 1e-13 of its largest keeps
 * Q = I.  Enqueued on `stream`.                                            */
qtt_status qtt_tt_align(qtt_tt *x, const qtt_tt *ref, void *stream);

/* ------------------------------------------------------------ timing   */
/* qtt_kernel_timing — enable (nonzero) or disable per-launch timing of the
 * rounding's one-workgroup kernels ("k_svd_step", "k_sketch_qr",
 * "k_qr_step"): while enabled, every launch of them is bracketed by two HIP
 * events recorded on the stream it is launched on.  Either call clears the
 * records.  qtt_kernel_timing_read sums the device time (ms) and counts the
 * launches of one kernel recorded since; it waits for the recorded events.
 * For benchmarking only: the events add a few microseconds per launch.    */
qtt_status qtt_kernel_timing(int32_t enable);
qtt_status qtt_kernel_timing_read(const char *kernel, double *ms, int64_t *launches);

/* Thread-local text of the last error of this thread.                      */
const char *qtt_last_error(void);

/* Library version string.                                                  */
const char *qtt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QTT_H */
