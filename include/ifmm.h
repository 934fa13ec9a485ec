/*
 * ifmm.h - C ABI of the MI355X inverse fast multipole method (IFMM) library.
 *
 * The library builds an H2 (black-box FMM, Chebyshev) representation of a
 * dense kernel matrix A_ij = K(|r_i - r_j|) + s*delta_ij on a point cloud,
 * turns it into the extended sparse system E and factorizes E level by level
 * up the tree with compression of well-separated fill-in to a tolerance
 * eps (Coulier, Pouransari & Darve, "The inverse fast multipole method",
 * Sec. 2 and Alg. 1-3). The factorization gives an approximate direct solve
 * x = A~^-1 b for any number of right-hand sides and serves as a
 * preconditioner for GMRES (Sec. 3.2).
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers (memory of the current HIP device),
 *     owned by the caller, unless the argument says "host".
 *   - Vectors and blocks of right-hand sides are column-major with a leading
 *     dimension ld >= n, in the caller's point order.
 *   - Points are row-major, n x dim, float64.
 *   - All work is ordered on the stream given in ifmm_options.stream (0 =
 *     the null stream). Calls on one handle must not overlap; different
 *     handles may be used concurrently from different host threads.
 *   - No exception crosses the ABI: every entry point returns an ifmm_status
 *     code; ifmm_strerror() gives a short message and ifmm_last_error()
 *     a longer, thread-local description of the last failure.
 *   - Handle life cycle: BUILT (after ifmm_build) -> FACTORIZED (after
 *     ifmm_factorize). ifmm_matvec is legal in both states; ifmm_solve and
 *     the preconditioner handle of ifmm_gmres(_left) need FACTORIZED; factorizing
 *     again is allowed.
 */
#ifndef IFMM_H
#define IFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IFMM_OK = 0,
  IFMM_ERR_ARG = 1,        /* invalid argument (null pointer, bad size, dim, order...) */
  IFMM_ERR_OOM = 2,        /* device allocation failed or the HBM budget was exceeded */
  IFMM_ERR_SINGULAR = 3,   /* a pivot block or the top system is exactly singular */
  IFMM_ERR_NUMERICAL = 4,  /* a non-finite value appeared */
  IFMM_ERR_STATE = 5,      /* call not legal in the handle's state */
  IFMM_ERR_HIP = 6,        /* a HIP runtime call failed */
  IFMM_ERR_INTERNAL = 7    /* an internal consistency check failed */
} ifmm_status;

/* Matrix-entry kernel K(r) (Sec. 2.1; Sec. 3.1 gives the paper's own kernel). */
typedef enum {
  IFMM_K_IMQ = 0,    /* 1/sqrt(r^2 + c^2),           param = c */
  IFMM_K_GAUSS = 1,  /* exp(-r^2/h^2),               param = h */
  IFMM_K_PAPER = 2,  /* 1 at r=0, r/d below d, d/r above (Sec. 3.1), param = d */
  IFMM_K_POLY2 = 3   /* 1 + r^2 (reproduced exactly by order >= 3; for tests) */
} ifmm_kernel_kind;

typedef struct {
  int kind;            /* ifmm_kernel_kind */
  double param;        /* c, h or d */
  double diag_shift;   /* s: added to the diagonal a_ii only */
} ifmm_kernel;

typedef struct {
  int precision;              /* 64 (default) or 32: arithmetic of the factors and
                                 of ifmm_solve; the matvec is always float64 */
  int leaf_max;               /* used when depth <= 0: the smallest uniform depth
                                 >= 2 whose leaves hold at most leaf_max points */
  int rank_max;               /* > 0: no basis keeps more than rank_max columns
                                 (0 = bounded only by the box size) */
  double sigma0_override;     /* > 0: use this value as sigma_0(E) instead of the
                                 power-iteration estimate */
  int64_t hbm_budget_bytes;   /* > 0: fail with IFMM_ERR_OOM rather than let the
                                 handle's device memory exceed this */
  void* stream;               /* hipStream_t; 0 = null stream */
  /* Optional device allocator of the handle (both set, or both NULL = the
   * library's own cache of hipMalloc blocks). Every device buffer of the
   * handle is then taken from dev_alloc(bytes, alloc_ctx), which returns a
   * device pointer of at least that many bytes aligned to 256 (NULL: the call
   * fails with IFMM_ERR_OOM), and returned through dev_free(ptr, bytes,
   * alloc_ctx) with the same byte count. A buffer handed to dev_free may still
   * be read or written by work already queued on the handle's stream: the
   * allocator may reuse it only for work ordered after that on the same
   * stream, or after the stream has been synchronised (stream-ordered reuse,
   * as PyTorch's caching allocator does when given the handle's stream). The
   * callbacks may be called from the calling thread and, in
   * ifmm_factorize_batch, from the library's worker threads, until
   * ifmm_destroy returns. */
  void* (*dev_alloc)(size_t bytes, void* alloc_ctx);
  void (*dev_free)(void* ptr, size_t bytes, void* alloc_ctx);
  void* alloc_ctx;
} ifmm_options;

/* Counters and phase times of a handle (host struct, filled by ifmm_query). */
typedef struct {
  int64_t n;
  int dim, depth, cheb_order, precision;
  double eps, sigma0, tau;
  int levels;                 /* number of eliminated levels (depth - 1) */
  int max_rank[32];           /* by level: largest final rank */
  double mean_rank[32];       /* by level: mean final rank */
  int64_t boxes[32];          /* by level: occupied boxes */
  double t_build_ms, t_sigma0_ms, t_factor_ms, t_last_solve_ms, t_last_matvec_ms;
  double factor_flops;        /* algorithmic flops of the last factorization
                                 (LU, triangular solves, Schur products,
                                 recompressions, edge updates, merge, top) */
  double schur_flops;         /* of which Schur-complement products */
  int64_t factor_bytes;       /* bytes of the stored factors (read once per solve) */
  int64_t device_bytes;       /* device memory held by the handle now */
  int64_t device_bytes_peak;  /* peak over the handle's life */
  int error_level, error_box; /* where IFMM_ERR_SINGULAR / NUMERICAL arose, else -1 */
  int gmres_iters;            /* of the last ifmm_gmres(_left) call (max over columns) */
  double gmres_relres;        /* monitored residual of that call (max over columns) */
  /* Device time by kernel family, measured with HIP events on the handle's
     stream when the environment variable IFMM_KTIMING=1 is set at build time
     (IFMM_KTIMING=m<hex>: only the families whose bits are set; otherwise
     zero); totals since the handle was built. Families:
     0 Schur-complement GEMM, 1 pivot LU (panels, swaps, trailing GEMM),
     2 triangular solves W = E_PP^-1 E_PF, 3 Householder QR of the
     recompression matrices, 4 Jacobi SVD, 5 basis changes of the edges and
     redirection, 6 forward/backward substitution, 7 H2 matvec, 8 other.
     Families 9-14 hold one kernel each, every launch timed on its own (the
     kernel is not counted in the families above): 9 block-Jacobi round,
     10 Householder QR panel, 11 truncated pivoted QR, 12 one-workgroup
     Jacobi SVD, 13 row basis change, 14 column basis change. Family 15
     holds the launches of the step-wise truncated pivoted QR (batches of
     few problems: one launch per Householder step). Family 16 holds one
     kernel, the streaming R-only QR of matrices at most 64 columns wide (one
     column per lane). Family 17 holds one kernel, the products
     R_i K_o R_j^T of the weighted system by interaction offset. Entries
     18-23 are zero. */
  double kfam_ms[24];
  double kfam_flops[24];      /* algorithmic flops attributed to the family */
  double kfam_bytes[24];      /* algorithmic bytes attributed to the family */
  int64_t kfam_launches[24];
  int gmres_restarts;         /* column restarts from the true residual in the
                                 last ifmm_gmres call (see ifmm_gmres) */
} ifmm_stats;

typedef struct ifmm_problem* ifmm_handle;

/* Fill *opt with the defaults (precision 64, leaf_max 64, no rank cap, no
   sigma_0 override, no budget, null stream). */
void ifmm_default_options(ifmm_options* opt);

/*
 * ifmm_build - tree, H2 operators and the initial extended system
 * (Alg. 1: octree and initial operators; Sec. 3 opening: Chebyshev
 * interpolation followed by an SVD; Sec. 2.4: sigma_0(E) and the rank rule).
 *   points      device, n x dim row-major float64; copied, not retained
 *   n           number of points (>= 1)
 *   dim         1, 2 or 3
 *   k           kernel and diagonal shift
 *   depth       leaf level L (>= 2); <= 0 selects it from opt->leaf_max
 *   cheb_order  Chebyshev nodes per dimension n (1..8)
 *   eps         relative tolerance of the compressions (>= 0)
 *   opt         host; may be NULL for defaults
 *   out         host; receives the handle (NULL on failure)
 * The handle owns all device memory it allocates; free it with ifmm_destroy.
 */
int ifmm_build(const double* points, int64_t n, int dim, ifmm_kernel k, int depth,
               int cheb_order, double eps, const ifmm_options* opt, ifmm_handle* out);

/*
 * ifmm_factorize - eliminate levels L..2 in colour (independent-set) order,
 * compress and redirect well-separated fill-in, merge each level into its
 * parent and factorize the dense top system (Alg. 1 and 2; Alg. 3; eqs.
 * P2P_kj to K_merge). Stores the factors for any number of later solves.
 * Errors: IFMM_ERR_SINGULAR (a zero pivot; stats error_level / error_box),
 * IFMM_ERR_NUMERICAL (a NaN or infinity in the stored factors; stats
 * error_level = the finest level holding one, 1 = top system).
 */
int ifmm_factorize(ifmm_handle h);

/*
 * ifmm_factorize_batch - ifmm_factorize of count independent handles at once
 * (each problem factorized as in Alg. 1 and 2). Host worker threads take the
 * problems largest first; each problem's launches go to its own handle's
 * stream, so problems on distinct streams overlap on the device. Results are
 * identical to factorizing each handle alone.
 *   hs        host array of count handles (distinct; non-NULL)
 *   count     >= 0
 *   nthreads  host worker threads (>= 1; capped at count)
 *   status    host array of count, may be NULL: per-problem status code
 * Returns IFMM_OK when every problem succeeded, else the first failing
 * problem's code (its message is in ifmm_last_error of the calling thread).
 */
int ifmm_factorize_batch(ifmm_handle* hs, int count, int nthreads, int* status);

/*
 * ifmm_solve - x = IFMM^-1 b for nrhs right-hand sides (Alg. 1, substitution).
 *   b, x   device, n x nrhs column-major float64, leading dimension ld;
 *          x may alias b
 * Returns when x is complete. IFMM_ERR_NUMERICAL if b holds a NaN or an
 * infinity, or if the result does (x is then not meaningful).
 */
int ifmm_solve(ifmm_handle h, const double* b, double* x, int nrhs, int64_t ld);

/*
 * ifmm_solve_noalloc - ifmm_solve that allocates no device memory, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation. Same arguments and result as
 * ifmm_solve (x = IFMM^-1 b; x may alias b), with these differences:
 *   - its work storage is one fixed device array of 64 MiB per GPU, set up at
 *     the first ifmm_build on that GPU and held until the process ends; a call
 *     whose work exceeds it (about (rows of the substitution) x nrhs plus
 *     partial sums, in the factor precision) fails with IFMM_ERR_ARG and
 *     names the bytes it would need;
 *   - every call on one GPU shares that array: calls that overlap on one GPU
 *     (two streams, two host threads, two handles) race and must be ordered
 *     by the caller;
 *   - the call only enqueues work on the handle's stream and returns without
 *     waiting; there is no non-finite check (it would need a host read).
 */
int ifmm_solve_noalloc(ifmm_handle h, const double* b, double* x, int nrhs, int64_t ld);

/*
 * ifmm_query_ranks - final rank of every box of one level, i.e. the size of
 * y_i when box i is eliminated (Alg. 2), after the recompressions of Sec. 2.2.
 *   level  in [2, depth]
 *   out    host array of count ints, boxes in the level's order (occupied
 *          boxes sorted by Morton code)
 *   count  must equal the occupied boxes of the level (ifmm_stats.boxes)
 * Needs a factorized handle (IFMM_ERR_STATE otherwise).
 */
int ifmm_query_ranks(ifmm_handle h, int level, int* out, int count);

/*
 * ifmm_matvec - y = A~ x with the H2 operators of the build (eq. A_decomp_l3
 * and A_decomp_l2; the FMM product used by GMRES in Sec. 3.2), float64.
 *   x, y   device, n x nrhs column-major, leading dimension ld; must not alias
 */
int ifmm_matvec(ifmm_handle h, const double* x, double* y, int nrhs, int64_t ld);

/*
 * ifmm_gmres - right-preconditioned, non-restarted GMRES (Sec. 3.2): the
 * products use op's H2 matvec in float64, the preconditioner is prec's
 * factorization (float32 or float64); orthogonalisation is float64.
 * op and prec must describe the same points (same n); they may be the same
 * handle, or live on different streams (the calls order the two streams with
 * events). prec = NULL runs GMRES without a preconditioner (the comparison
 * runs of Sec. 3.2); op then need not be factorized. Each column is an
 * independent GMRES run. Rounding can leave the true residual, recomputed at
 * exit, above tol when the monitored one has met it. Such a column is then
 * restarted from its true residual (x += d, A~ d = b - A~ x). There are at
 * most 3 restarts of at most 10 iterations each, within the iterations the
 * column has left. The restarts stop when one takes less than 1% off the
 * residual. The column is refined alone, so its result does not depend on the
 * other columns.
 *   b, x        device, n x nrhs, leading dimension ld; x is overwritten;
 *               x and b must not overlap (IFMM_ERR_ARG)
 *   tol         stop when ||b - A~ x|| <= tol ||b|| (per column)
 *   maxit       iteration limit per column, restarts included (<= 1000)
 *   iters_out   host, may be NULL: largest iteration count over the columns
 *   relres_out  host, may be NULL: largest true relative residual at exit
 * IFMM_ERR_NUMERICAL if b holds a NaN or an infinity.
 */
int ifmm_gmres(ifmm_handle op, ifmm_handle prec, const double* b, double* x, int nrhs,
               int64_t ld, double tol, int maxit, int* iters_out, double* relres_out);

/*
 * ifmm_gmres_left - left-preconditioned, non-restarted GMRES (App. B): GMRES
 * on P^-1 A~ x = P^-1 b, with P^-1 prec's factorization and A~ op's H2
 * matvec in float64; orthogonalisation is float64, x = V_k y_k. The
 * monitored residual is the preconditioned one, as the App. B tables report
 * it for the left variant. Arguments, states and errors as ifmm_gmres;
 * prec = NULL gives P = I (then the method equals ifmm_gmres without a
 * preconditioner).
 *   tol              stop when ||P^-1 (b - A~ x)|| <= tol ||P^-1 b|| (per column)
 *   relres_out       host, may be NULL: largest preconditioned relative
 *                    residual at exit (recomputed from x)
 *   true_relres_out  host, may be NULL: largest ||b - A~ x|| / ||b|| at exit
 */
int ifmm_gmres_left(ifmm_handle op, ifmm_handle prec, const double* b, double* x, int nrhs,
                    int64_t ld, double tol, int maxit, int* iters_out, double* relres_out,
                    double* true_relres_out);

/* ifmm_query - copy counters and phase times into *s (host). */
int ifmm_query(ifmm_handle h, ifmm_stats* s);

/* ifmm_destroy - release the handle and all its device memory; NULL is a no-op. */
int ifmm_destroy(ifmm_handle h);

/* Static message for a status code. */
const char* ifmm_strerror(int code);

/* Thread-local description of the last failure of this thread (never NULL). */
const char* ifmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IFMM_H */
