/*
 * kdcd.h -- C-ABI of the MI355X (gfx950) library for s-step dual coordinate
 * descent on kernel methods:
 *
 *   s-step DCD for kernel SVM (paper: "Scalable Dual Coordinate Descent for
 *   Kernel Methods", Sec. 3.1-3.2, Algorithms 1-2), and
 *   s-step block DCD for kernel ridge regression (Sec. 3.3-3.4,
 *   Algorithms 3-4, Eq. (3)).
 *
 * Every outer iteration k of both solvers runs on the device:
 *   1. the index block S_k: s*b entries of the caller's sequence idx;
 *   2. the kernel-block product P = A A_S^T (m x sb), dense (MFMA) or CSR;
 *   3. the kernel map of Table 1 (RBF from precomputed row norms, or
 *      polynomial), fused into the product's epilogue;
 *   4. the right-hand side r = U^T beta (U = K(A, A_S) is never stored);
 *   5. the sampled Gram W = K(A_S, A_S) (sb x sb, FP64);
 *   6. the s inner coordinate (K-SVM) or b x b block (K-RR) updates;
 *   7. the scatter alpha_{S_t} += theta_t (or Delta alpha_t), in t order.
 *
 * Conventions shared by every entry point
 *  - Pointers marked "device" are HIP device pointers owned by the caller;
 *    the library never frees them.  Pointers marked "host" are host memory.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    Solver entry points synchronise `stream` before returning so that they
 *    can report errors found on the device.
 *  - No exception crosses this boundary.  On any error the contents of
 *    output arrays (alpha, r, W, trace, snapshots) are unspecified.
 *  - All floating-point inputs and outputs are FP64.  Indices are int32,
 *    0-based.  Dense A is row-major with leading dimension ld >= n.
 *  - Calls are reentrant; they share no hidden state across calls.
 */
#ifndef KDCD_H
#define KDCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;
typedef struct ihipStream_t *kdcd_stream; /* identical to hipStream_t */

typedef enum {
    KDCD_OK = 0,
    KDCD_ERR_INVALID_ARG = -1,     /* a host-checkable argument is out of its domain       */
    KDCD_ERR_UNSUPPORTED = -2,     /* valid but not implemented (e.g. b > 32, sb > 1024)   */
    KDCD_ERR_INDEX_RANGE = -3,     /* some idx entry is outside [0, m)                      */
    KDCD_ERR_INDEX_DUPLICATE = -4, /* a K-RR block repeats a coordinate (Alg. 3/4 draw a   */
                                   /* block without replacement)                            */
    KDCD_ERR_NOT_SPD = -5,         /* a K-RR block matrix G = W_jj/lambda + m I failed its */
                                   /* factorisation (non-positive or non-finite pivot)      */
    KDCD_ERR_NONFINITE = -6,       /* NaN/Inf in y, alpha_0, or produced by an update       */
    KDCD_ERR_HIP = -7,             /* a HIP runtime call failed                             */
    KDCD_ERR_ALLOC = -8,           /* device workspace allocation failed                   */
    KDCD_ERR_WORKSPACE = -9        /* caller workspace smaller than kdcd_workspace_bytes    */
} kdcd_status;

/* Kernel functions of Table 1:
 *   LINEAR  K(x, z) = x . z
 *   POLY    K(x, z) = (c + x . z)^degree,  c >= 0, integer degree >= 1
 *   RBF     K(x, z) = exp(-sigma ||x - z||^2),  sigma > 0                     */
typedef enum { KDCD_KERNEL_LINEAR = 0, KDCD_KERNEL_POLY = 1, KDCD_KERNEL_RBF = 2 } kdcd_kernel_kind;

typedef struct {
    int32_t kind;   /* kdcd_kernel_kind */
    int32_t degree; /* POLY only */
    double sigma;   /* RBF only */
    double c;       /* POLY only */
} kdcd_kernel;

typedef enum { KDCD_DENSE = 0, KDCD_CSR = 1 } kdcd_format;

/* Precision of the kernel-block product P = A A_S^T only.  The Gram W, the
 * right-hand side r, the recurrence and alpha are always FP64.  F32/BF16/F16
 * use MFMA with FP32 accumulation; BF16X3 splits A = hi + lo in bf16 and sums
 * hi*hi + hi*lo + lo*hi.  Low-precision copies of A are library workspace.  */
typedef enum { KDCD_F64 = 0, KDCD_F32 = 1, KDCD_BF16 = 2, KDCD_F16 = 3, KDCD_BF16X3 = 4 } kdcd_compute;

typedef struct {
    int32_t format; /* kdcd_format */
    int32_t reserved;
    int64_t m, n;   /* rows (samples) and columns (features) */
    int64_t ld;     /* DENSE: leading dimension (>= n), in elements */
    int64_t nnz;    /* CSR: number of stored entries */
    const double *values;    /* device. DENSE: m x ld row-major. CSR: nnz values      */
    const int64_t *row_ptr;  /* device. CSR: m+1 offsets, row_ptr[0] = 0              */
    const int32_t *col_idx;  /* device. CSR: nnz columns, strictly increasing per row */
} kdcd_matrix;

/* Optional per-call stage timings, measured with HIP events recorded on the
 * call's stream around every launch of the named stage. */
typedef struct {
    double kblock_ms;        /* kernel-block product + map + r partials + Gram    */
                             /* (the product kernel alone where the Gram rows are */
                             /* gathered from it, s*b >= 256 dense FP64)          */
    int64_t kblock_launches;
    double finish_ms;        /* partial reduction of r, K-RR block inverses, and  */
                             /* the row-position / repeated-row kernels of the    */
                             /* gathered Gram                                     */
    int64_t finish_launches;
    double recur_ms;         /* s-step recurrence + scatter                         */
    int64_t recur_launches;
    double total_ms;         /* first to last event of the solve                   */
} kdcd_profile;

/*
 * KDCD_FLAG_GRAPH (kdcd_ksvm_solve, kdcd_krr_solve, kdcd_batch_solve): the
 * call's whole launch sequence (validation, norms, every outer iteration,
 * snapshot copies) is captured once into a hipGraph on a private stream of
 * the current device and kept in a process-wide cache of 8 entries keyed by
 * every argument (pointers included, stream excluded); an identical later
 * call launches the instantiated graph on `stream`, so it re-reads the
 * current contents of A, y, idx and alpha.  A cache entry keeps its own
 * workspace (allocated once with hipMalloc) unless opt->workspace is given,
 * which then must stay valid while the entry lives.  Graph-mode calls are
 * serialised by one lock.  With a profile, only total_ms is reported.
 * kdcd_ksvm_solve / kdcd_krr_solve without trace, snapshots, profile or a
 * caller workspace, with at least 18 whole blocks (floor(H/s) >= 18), are
 * replayed by windows instead: one graph holds 16 outer iterations -- a
 * kernel that copies the window's index blocks out of idx, the block index
 * taken from a counter in device memory that the same kernel moves on, then
 * the window's launches -- and is launched window after window; the set-up,
 * the first outer iteration and the iterations after the last whole window
 * run eagerly, in the graph's workspace.  That graph does not depend on H or
 * on the contents of idx (only on its address), so such calls share it.
 */
/*
 * KDCD_FLAG_TIME_PRODUCT (with a profile; dense kdcd_ksvm_solve /
 * kdcd_krr_solve, any compute): only the kernel-block product is timed (for
 * low-precision computes the product launch alone, not the FP64 Gram launch)
 * (kblock_ms, kblock_launches and total_ms from its first start to its last
 * end; the other stages report 0).  Stage kernels record their own
 * timestamps in their dispatch (hipExtLaunchKernelGGL), and each timed
 * dispatch costs a few microseconds of device time, so a timed measurement
 * of whole-solve throughput times the product only.
 * KDCD_FLAG_TIME_SAMPLE (with KDCD_FLAG_TIME_PRODUCT): only the product
 * launches of outer iterations k with k % 8 == 0 are timed (kblock_launches
 * counts them), which keeps the timing's device cost to one launch in eight.
 */
/*
 * Lookahead loop (kdcd_krr_solve and kdcd_krr_solve_noalloc; dense A, any
 * compute, b <= 8, 256 <= s*b <= 512, at least two outer iterations, no
 * snapshots; FP64 also needs n a multiple of 16 with 16-byte aligned rows;
 * the monitor only in FP64 and without a caller workspace, whose size does
 * not include the second stored kernel block the loop then keeps): the s-step
 * recurrence of index
 * block k (Algorithm 4's inner loop) runs in one workgroup of the launch that
 * computes the kernel block of index block k+1.  That product reduces r_{k+1}
 * against the iterate before block k's updates; the kernel rows of block k's
 * coordinates come from the same launch (FP64) or from the FP64 Gram launch
 * after it (low precision), and the finish pass of block k+1 adds those rows
 * times the updates to r_{k+1} and the updates to alpha, which is Algorithm
 * 4's r_{k+1} = U_{k+1}^T alpha up to rounding.  Used by default
 * when 2 m n s b >= 4e9 (the product then outlasts the recurrence it hides);
 * KDCD_FLAG_LOOKAHEAD asks for it at any size, KDCD_FLAG_SERIAL never.  Calls
 * that KDCD_FLAG_GRAPH replays by windows run the serial loop.
 */
/* Any other bit of flags is refused with KDCD_ERR_INVALID_ARG. */
enum {
    KDCD_FLAG_GRAPH = 1,
    KDCD_FLAG_TIME_PRODUCT = 4,
    KDCD_FLAG_TIME_SAMPLE = 8,
    KDCD_FLAG_LOOKAHEAD = 16,
    KDCD_FLAG_SERIAL = 32
};

typedef struct {
    int32_t compute;         /* kdcd_compute; default KDCD_F64                               */
    int32_t loss;            /* K-SVM: 1 = hinge (K-SVM-L1, default), 2 = squared hinge (L2) */
    int32_t snapshot_every;  /* > 0: copy alpha after every this many outer iterations       */
    int32_t flags;           /* KDCD_FLAG_*                                                  */
    double *snapshots;       /* device, (ceil(ceil(H/s)/snapshot_every)) x m, row-major       */
    double *trace;           /* device, H*b: theta (K-SVM) / Delta alpha (K-RR) per update    */
    void *workspace;         /* device; NULL = allocated on `stream` and freed before return  */
    size_t workspace_bytes;
    kdcd_profile *profile;   /* host; NULL = no timing                                      */
    int32_t monitor_every;   /* > 0: convergence monitor every this many outer iterations   */
    int32_t reserved;
    double tol;              /* monitor: stop once the certified relative error <= tol      */
    int64_t *outer_done;     /* host or NULL: outer iterations performed                    */
    double *rel_err;         /* host or NULL: last certified relative objective error       */
    double *monitor_log;     /* device or NULL: monitor_log_len records of 4 doubles        */
    int64_t monitor_log_len;
} kdcd_options;

/*
 * Convergence monitor (monitor_every > 0; kdcd_ksvm_solve / kdcd_krr_solve on
 * dense A in FP64, BF16, FP16 or BF16X3, on CSR A in FP64,
 * kdcd_ksvm_solve_sampled, and kdcd_batch_solve in FP64; not with
 * KDCD_FLAG_GRAPH, not in FP32).  A batch keeps every problem's dual vector
 * (one pass over each sigma group's stored block updates all of the group's
 * problems), evaluates every problem's bound and stops once the largest is
 * <= tol; rel_err and the log report that largest bound (objective: the sum
 * of the problems').  With a
 * low-precision compute the gradient is carried with the kernel values the
 * product computed, so the bound certifies the problem with those values (the
 * exact problem's objective differs by the kernel's rounding).
 * The solve keeps the full dual gradient current on the device (K-SVM:
 * g = Q alpha - 1 + omega alpha; K-RR: the residual y - M alpha, M =
 * K/lambda + m I) from the kernel block it already computes, and every
 * monitor_every outer iterations (and after the last) evaluates in O(m) a
 * certified bound on the relative objective error (f - f*) / |f*|:
 *   K-RR: ||y - M alpha||^2 / (2m) / (|f| - that), since lambda_min(M) >= m;
 *   K-SVM: the duality gap P(alpha) + f(alpha), divided by |f|.
 * Once the bound is <= tol every later launch of the solve returns at once,
 * and the host, which checks the outcome of the evaluation two periods back
 * before each period, stops enqueuing; alpha stops changing, every later
 * snapshot holds the final iterate, and trace (and idx_out) entries past that
 * point are unspecified.  The monitor adds about
 * 8 (m (s b + 2) + s b) bytes + 8 KiB to the workspace (not counted by
 * kdcd_workspace_bytes).
 * Costs per outer iteration: m*s*b*8 bytes written and read (the stored
 * kernel block) plus the O(m) evaluation.
 * monitor_log (optional): evaluation i writes record i (i < monitor_log_len)
 * = {outer iterations done, certified relative error, objective f, seconds
 * since the solve's first launch by the device's wall clock}; records past
 * the last evaluation are left as they were.
 */

/*
 * kdcd_ksvm_solve -- s-step DCD for K-SVM-L1/L2 (Algorithm 2; s = 1 is
 * Algorithm 1).  The dual Hessian is Q_pq = y_p y_q K(a_p, a_q) (Sec. 3.1).
 *   A       device matrix (dense or CSR), m x n
 *   y       device, m labels, each exactly +1 or -1
 *   kernel  host, kernel function
 *   C       > 0; hinge: box [0, C]; squared hinge: nu = inf, omega = 1/(2C)
 *   b       must be 1 (DCD updates one coordinate per inner step)
 *   s       >= 1 inner steps per outer iteration (s*b <= 1024)
 *   H       >= 1 inner steps in total; the last outer iteration holds
 *           H - s*floor(H/s) of them
 *   idx     device, H coordinates in [0, m); duplicates allowed anywhere
 *   alpha   device, m: alpha_0 on entry (0 <= alpha_0 <= nu), alpha_H on exit
 *   opt     host, may be NULL (defaults)
 * Errors: INVALID_ARG (host checks), UNSUPPORTED, INDEX_RANGE, NONFINITE
 * (y not +-1 or non-finite, alpha_0 outside the box, or a non-finite update),
 * HIP, ALLOC, WORKSPACE.
 */
kdcd_status kdcd_ksvm_solve(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                            double C, int32_t b, int32_t s, int64_t H, const int32_t *idx,
                            double *alpha, const kdcd_options *opt, kdcd_stream stream);

/*
 * kdcd_krr_solve -- s-step BDCD for K-RR (Algorithm 4 / Eq. (3); s = 1 is
 * Algorithm 3).  Minimises 1/2 a^T (K/lambda + m I) a - y^T a, so the fixed
 * point is alpha* = (K/lambda + m I)^{-1} y = lambda (K + m lambda I)^{-1} y.
 *   A, kernel as above; y device, m finite targets
 *   lambda  > 0 (the paper's lambda)
 *   b       1 <= b <= 32 coordinates per block, b <= m
 *   s       >= 1 blocks per outer iteration (s*b <= 1024)
 *   H       >= 1 block updates in total
 *   idx     device, H*b coordinates, block-major; every block holds b distinct
 *           coordinates, different blocks may overlap
 *   alpha   device, m: alpha_0 on entry, alpha_H on exit
 * Errors: INVALID_ARG, UNSUPPORTED, INDEX_RANGE, INDEX_DUPLICATE, NOT_SPD,
 * NONFINITE, HIP, ALLOC, WORKSPACE.
 */
kdcd_status kdcd_krr_solve(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                           double lambda, int32_t b, int32_t s, int64_t H, const int32_t *idx,
                           double *alpha, const kdcd_options *opt, kdcd_stream stream);

/*
 * kdcd_krr_solve_noalloc -- kdcd_krr_solve for callers that cannot allocate
 * device memory: code under stream capture, tight serving loops, harnesses
 * that forbid allocation.  The workspace is a fixed array of
 * KDCD_NOALLOC_SCRATCH_BYTES in the library's device memory (each device
 * holds its own copy from the first such call on it until the process ends);
 * the call allocates nothing.  Arguments and results are those of
 * kdcd_krr_solve on the current device (stream must belong to it).
 * opt: compute, snapshots and trace as in kdcd_krr_solve; workspace,
 * workspace_bytes, monitor_every, flags and profile must be zero / NULL
 * (UNSUPPORTED otherwise, since each of them allocates).
 * Errors: those of kdcd_krr_solve, and WORKSPACE when
 * kdcd_workspace_bytes(1, A, kernel, b, s, compute) exceeds
 * KDCD_NOALLOC_SCRATCH_BYTES.
 * All calls on one device share the one array: calls that overlap in time on
 * a device (other host threads, or other streams before the previous call
 * returned) race and give undefined results.  Every call rewrites the parts of
 * the array it reads before reading them.
 */
#define KDCD_NOALLOC_SCRATCH_BYTES (32u << 20)
kdcd_status kdcd_krr_solve_noalloc(const kdcd_matrix *A, const double *y,
                                   const kdcd_kernel *kernel, double lambda, int32_t b, int32_t s,
                                   int64_t H, const int32_t *idx, double *alpha,
                                   const kdcd_options *opt, kdcd_stream stream);

/* One problem of a batched solve. */
typedef struct {
    int32_t problem;      /* 0 = K-SVM, 1 = K-RR                                        */
    int32_t loss;         /* K-SVM: 1 = hinge, 2 = squared hinge (0 means 1)             */
    double param;         /* C (K-SVM, > 0) or lambda (K-RR, > 0)                        */
    double sigma;         /* RBF sigma of this problem (> 0); ignored for other kernels  */
    const double *y;      /* device, m: labels (+-1) or targets                          */
    double *alpha;        /* device, m: alpha_0 on entry, alpha_H on exit                */
    double *trace;        /* device or NULL: per-update theta / Delta alpha, H*b entries */
} kdcd_batch_problem;

/*
 * kdcd_batch_solve -- several problems over one matrix and one index
 * sequence, sharing every kernel-block product (the batching of
 * a (lambda, sigma) K-RR sweep and one-vs-rest K-SVMs; the paper's Alg. 2
 * and 4 per problem).  Per outer iteration one launch forms P = A A_S^T once,
 * maps it once per distinct sigma and reduces it against every problem's
 * alpha; one launch forms every sigma's Gram; the recurrences of all problems
 * run in one launch per problem kind.
 * Each problem's result equals its single solve:
 *   K-RR  problem p == kdcd_krr_solve(A, y_p, kernel(sigma_p), lambda_p, b, s, H, idx, alpha_p)
 *   K-SVM problem q == kdcd_ksvm_solve(A, y_q, kernel(sigma_q), C_q, 1, s*b, H*b, idx, alpha_q)
 * (the K-SVM problems take the same s*b indices of each outer iteration as
 * s*b scalar steps), up to the summation order of the shared reduction.
 *   kernel     host: kind, c and degree shared; sigma comes from each problem
 *   b, s, H    as in kdcd_krr_solve (b = 1 allowed); s*b <= 1024; every
 *              b-block of idx distinct when any K-RR problem is present
 *   problems   host array of n_problems (1..32) descriptors; at most 8
 *              distinct sigma values
 *   opt        compute, snapshot-free; workspace / profile as elsewhere
 * Errors: as kdcd_krr_solve / kdcd_ksvm_solve; UNSUPPORTED beyond the limits.
 */
kdcd_status kdcd_batch_solve(const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t b,
                             int32_t s, int64_t H, const int32_t *idx,
                             const kdcd_batch_problem *problems, int32_t n_problems,
                             const kdcd_options *opt, kdcd_stream stream);

/*
 * kdcd_kernel_rhs -- one kernel-block pass on its own (steps 2-5 above):
 *   r[j] = sum_p K(a_p, a_{S_j}) * beta[p] * (beta_scale ? beta_scale[p] : 1)
 *   W[t*sb + j] = K(a_{S_t}, a_{S_j})              (only if W != NULL)
 * This is the quantity U_k^T alpha (K-RR) / U_k^T (y o alpha) (K-SVM) of
 * Algorithms 2 and 4 together with V_k^T U_k.
 *   S        device, sb indices in [0, m); 1 <= sb <= 1024
 *   beta     device, m;  beta_scale device, m or NULL
 *   r        device, sb outputs;  W device, sb*sb outputs or NULL
 *   compute  kdcd_compute of the product (DENSE only for non-F64)
 * Synchronises `stream`.  Errors: INVALID_ARG, UNSUPPORTED, INDEX_RANGE, HIP, ALLOC.
 */
kdcd_status kdcd_kernel_rhs(const kdcd_matrix *A, const kdcd_kernel *kernel, const int32_t *S,
                            int32_t sb, const double *beta, const double *beta_scale, double *r,
                            double *W, int32_t compute, kdcd_stream stream);

/*
 * kdcd_ksvm_eval / kdcd_krr_eval -- matrix-free FP64 evaluation on the
 * device (measurement only; m^2 kernel evaluations).
 *   ksvm: out[0] = f(alpha) = 1/2 a^T Q a - 1^T a (+ ||a||^2/(4C) for loss 2)
 *         out[1] = primal P(alpha) = 1/2 a^T Q a + C sum max(0, 1-(Qa)_i) (squared for loss 2)
 *         out[2] = duality gap P + f;  out[3] = max |projected gradient|
 *   krr:  out[0] = f(alpha) = 1/2 a^T (K/lambda + m I) a - y^T a
 *         out[1] = ||y - (K/lambda + m I) alpha||_2
 *   out is host memory (4 resp. 2 doubles).  Synchronises `stream`.
 */
kdcd_status kdcd_ksvm_eval(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                           double C, int32_t loss, const double *alpha, double *out,
                           kdcd_stream stream);
kdcd_status kdcd_krr_eval(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                          double lambda, const double *alpha, double *out, kdcd_stream stream);

/*
 * kdcd_batch_eval -- kdcd_krr_eval / kdcd_ksvm_eval of every problem of a
 * batch (descriptors as in kdcd_batch_solve), with one shared FP64 kernel
 * pass over A for all problems (measurement only; m^2 kernel evaluations per
 * sigma group).  out (host, 4 doubles per problem): K-RR {f, ||y - M a||, 0,
 * 0}; K-SVM {f, P, gap, max |projected gradient|}.  Synchronises `stream`.
 */
kdcd_status kdcd_batch_eval(const kdcd_matrix *A, const kdcd_kernel *kernel,
                            const kdcd_batch_problem *problems, int32_t n_problems, double *out,
                            kdcd_stream stream);

/* ---------------------------------------------------------------------------
 * Low-rank kernel blocks.  The conclusion proposes approximating the sampled
 * kernel matrix (for instance by the Nystrom method) to cut the cost of the
 * kernel computation and of the Gram correction per outer iteration.  Given a
 * factor Phi (m x r) with K ~ Phi Phi^T, Algorithms 2 and 4 need per outer
 * iteration only Phi_S z and Phi_S Phi_S^T, where z = Phi^T beta is kept
 * current on the device: O((s b)^2 r) work instead of O(m n s b), independent
 * of m, which is what allows large blocks; the price is that the solve
 * converges to the minimiser of the approximated problem.
 * ------------------------------------------------------------------------- */

/*
 * kdcd_nystrom_features -- Nystrom factor from r landmark rows L of A:
 *   phi(x) = C^{-1} [K(x, a_{L_1}), ..., K(x, a_{L_r})]^T,
 *   C C^T = K(A_L, A_L) + jitter I  (Cholesky, C lower with positive diagonal)
 * so phi(x) . phi(x') = k_L(x)^T (K_LL + jitter I)^{-1} k_L(x').
 *   A       device dense matrix, m x n (the training rows)
 *   kernel  host, kernel function
 *   L       device, r landmark rows in [0, m) (repeats need jitter > 0);
 *           1 <= r <= min(m, 4096)
 *   jitter  >= 0, added to the diagonal of K(A_L, A_L)
 *   X       device dense matrix with X->n == A->n whose rows are featurised,
 *           or NULL for the rows of A itself
 *   Phi     device, rows(X) x ldphi row-major (ldphi >= r): row i = phi(x_i)
 * Work: rows(X) * r * (n + r) multiply-adds; workspace r*r doubles plus norms,
 * allocated on `stream`.  Synchronises `stream`.
 * Errors: INVALID_ARG, UNSUPPORTED (CSR, r > 4096), INDEX_RANGE, NOT_SPD (a
 * pivot of the Cholesky <= 0 or non-finite), HIP, ALLOC.
 */
kdcd_status kdcd_nystrom_features(const kdcd_matrix *A, const kdcd_kernel *kernel,
                                  const int32_t *L, int32_t r, double jitter,
                                  const kdcd_matrix *X, double *Phi, int64_t ldphi,
                                  kdcd_stream stream);

/*
 * kdcd_lowrank_solve -- Algorithm 2 (problem 0, K-SVM; b must be 1) or
 * Algorithm 4 (problem 1, K-RR) with the kernel matrix replaced by
 * Phi Phi^T.  The result equals kdcd_ksvm_solve / kdcd_krr_solve on the
 * matrix Phi with the linear kernel, up to the order of the sums.
 *   Phi     device dense matrix m x r (r <= 4096), e.g. from
 *           kdcd_nystrom_features
 *   y, param (C or lambda), b, s, H, idx, alpha   as in kdcd_ksvm_solve /
 *           kdcd_krr_solve
 *   z       device, r doubles, or NULL: on exit Phi^T beta_H with beta =
 *           y o alpha (K-SVM) or alpha (K-RR); phi(x) . z is then the sum
 *           sum_i beta_i phi(x) . phi(a_i) for a new row x
 *   opt     loss, snapshots, trace, profile; compute must be F64 and flags,
 *           monitor_every and workspace zero (UNSUPPORTED otherwise)
 * Per outer iteration: the Gram of Phi_S (lower tiles, mirrored), Phi_S z,
 * the finish and recurrence passes of the full solve, and z += Phi_S^T
 * (c o theta) with c = y_S (K-SVM) or 1 (K-RR), theta the updates.
 * Errors: as kdcd_ksvm_solve / kdcd_krr_solve.
 */
kdcd_status kdcd_lowrank_solve(int32_t problem, const kdcd_matrix *Phi, const double *y,
                               double param, int32_t b, int32_t s, int64_t H, const int32_t *idx,
                               double *alpha, double *z, const kdcd_options *opt,
                               kdcd_stream stream);

/* ---------------------------------------------------------------------------
 * Learned coordinate sampler.  Algorithms 1-4 take their coordinate sequence
 * as an input and the paper draws it uniformly (Section 3); here a small MLP
 * (4 -> 64 -> 64 -> 1, tanh hidden units, FP32) scores every coordinate of a
 * K-SVM from its state x_i = (alpha_i / C, g_i, K_ii, y_i), where
 * g = Q alpha - 1 + omega alpha is the full dual gradient, and the s
 * coordinates of an outer iteration are drawn by Gumbel-top-k over
 * score / tau, a share epsilon of the slots being drawn uniformly.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) with
 * key (seed mod 2^32, seed >> 32); a 32-bit output x gives u = (x + 0.5)/2^32.
 *   coordinate noise of outer iteration k: counter (i, k, 0, 0), Gumbel
 *     G_i = -log(-log u(x0)); key_i = float(score_i / tau + G_i)
 *   slot j of outer iteration k: counter (j, k, 1, 0); the slot is uniform
 *     when u(x0) < epsilon and then takes coordinate floor(x1 * m / 2^32),
 *     otherwise it takes the next best key (keys ranked by value, ties by the
 *     smaller index)
 *   initial weight p: counter (p, 0, 2, 0); Glorot-uniform weights with bound
 *     sqrt(6 / (fan_in + fan_out)), zero biases
 * Parameter layout (KDCD_SAMPLER_NPARAMS floats): W1[64][4], b1[64],
 * W2[64][64], b2[64], w3[64], b3.  Training minimises
 * 1/(2n) sum_i (f(x_i) - t_i)^2 with Adam (Kingma and Ba, 2015; beta1 0.9,
 * beta2 0.999, eps 1e-8), one step per minibatch, minibatches in data order.
 * A model lives on the device that was current at creation; all calls on it
 * must use that device.  Calls on one model must not overlap.
 * ------------------------------------------------------------------------- */
#define KDCD_SAMPLER_NPARAMS 4545
typedef struct kdcd_sampler kdcd_sampler;

/* Allocate a model on the current device with Glorot-uniform weights. */
kdcd_status kdcd_sampler_create(kdcd_sampler **out, uint64_t seed);
void kdcd_sampler_destroy(kdcd_sampler *model);
/* Copy the parameters to / from device memory (KDCD_SAMPLER_NPARAMS floats);
 * set_params also clears the Adam state.  Both synchronise `stream`. */
kdcd_status kdcd_sampler_get_params(const kdcd_sampler *model, float *params, kdcd_stream stream);
kdcd_status kdcd_sampler_set_params(kdcd_sampler *model, const float *params, kdcd_stream stream);
/* out[i] = f(x_i); x device n x 4 row-major, out device n.  Asynchronous. */
kdcd_status kdcd_sampler_forward(const kdcd_sampler *model, const float *x, int64_t n, float *out,
                                 kdcd_stream stream);
/* Loss and its gradient over n samples (1 <= n <= 65536): grad device
 * KDCD_SAMPLER_NPARAMS floats, loss device 1 float.  Asynchronous. */
kdcd_status kdcd_sampler_grad(const kdcd_sampler *model, const float *x, const float *t,
                              int64_t n, float *grad, float *loss, kdcd_stream stream);
/* `epochs` passes over (x, t) in minibatches of `batch` (<= 65536), one Adam
 * step of rate lr each; epoch_loss (device, epochs floats, or NULL) receives
 * each epoch's size-weighted mean minibatch loss.  Synchronises `stream`. */
kdcd_status kdcd_sampler_train(kdcd_sampler *model, const float *x, const float *t, int64_t n,
                               int32_t batch, int32_t epochs, float lr, float *epoch_loss,
                               kdcd_stream stream);
/* keys[i] = float(f(x_i) / tau + G_i) with the noise of outer iteration
 * `outer` (n < 2^31).  Asynchronous. */
kdcd_status kdcd_sampler_keys(const kdcd_sampler *model, const float *x, int64_t n, double tau,
                              uint64_t seed, int64_t outer, float *keys, kdcd_stream stream);
/* The s slots of outer iteration `outer` from caller-given finite keys
 * (device, m): S device, s outputs; 1 <= s <= min(m, 1024).  Errors:
 * NONFINITE (a key), UNSUPPORTED (more than 2048 keys tied at the threshold).
 * Synchronises `stream`. */
kdcd_status kdcd_sampler_select(const float *keys, int64_t m, int32_t s, double epsilon,
                                uint64_t seed, int64_t outer, int32_t *S, kdcd_stream stream);

/* Sampling options of kdcd_ksvm_solve_sampled. */
typedef struct {
    const kdcd_sampler *model; /* NULL: every slot uniform (the paper's draw)        */
    double epsilon;            /* [0, 1]: share of uniform slots (model != NULL)      */
    double tau;                /* > 0: temperature of the Gumbel keys                 */
    uint64_t seed;             /* Philox key                                          */
    int32_t *idx_out;          /* device, H: the realised coordinates (required)      */
    float *features_out;       /* device or NULL: H x 4, x_i of every drawn coordinate
                                  at the start of its outer iteration                 */
    double *grad_out;          /* device or NULL: m, the maintained g on exit         */
    int32_t pool;              /* 0: score every coordinate; s <= pool <= 2048: score
                                  only `pool` candidates per outer iteration, drawn
                                  uniformly from counters (j, k, 3, 0) as
                                  floor(x0 * m / 2^32) and ranked by key, ties by
                                  pool position (duplicates possible)               */
} kdcd_sampling;

/*
 * kdcd_ksvm_solve_sampled -- Algorithm 2 (b = 1) whose s coordinates per
 * outer iteration are drawn on the device, before the kernel block, by the
 * sampler above; the full gradient g is kept current by
 * g += diag(y) U_k diag(y_S) theta + omega * (scatter of theta), with U_k
 * stored by the kernel-block pass.  The result equals kdcd_ksvm_solve with
 * b = 1 on idx_out.  Dense FP64 only; H < 2^32 * s; when model != NULL,
 * s <= m (pool == 0) or s <= pool.  Other arguments as kdcd_ksvm_solve
 * (opt->trace receives theta).
 * Errors: as kdcd_ksvm_solve; UNSUPPORTED for CSR, low precision,
 * KDCD_FLAG_GRAPH or a tie group beyond 2048 keys; NONFINITE for a
 * non-finite score.
 */
kdcd_status kdcd_ksvm_solve_sampled(const kdcd_matrix *A, const double *y,
                                    const kdcd_kernel *kernel, double C, int32_t s, int64_t H,
                                    const kdcd_sampling *sampling, double *alpha,
                                    const kdcd_options *opt, kdcd_stream stream);

/* ---------------------------------------------------------------------------
 * Tuning of the kernel-block products.  The tile configuration of the FP64
 * product and of the single-problem BF16 / F16 / BF16X3 product is chosen per
 * (compute, n, sb) from a process-wide table, else by a built-in rule.
 * Entries come from kdcd_autotune (which times every configuration on the
 * caller's matrix) or kdcd_tune_set, and can be saved to and loaded from a
 * text file.  A launch reads the table once and its finish pass uses the same
 * configuration, so the table may change while solves run (they then take
 * the old or the new entry).
 * ------------------------------------------------------------------------- */
/* compute + KDCD_TUNE_BATCH addresses the table of the batched product
 * (kdcd_batch_solve) computed in `compute`, in every kdcd_tune_* call. */
#define KDCD_TUNE_BATCH 16
/* Number of configurations for `compute` (0 if not tunable); fills up to
 * `max` entries of bm, bn (tile rows x columns) and waves per workgroup
 * (each array may be NULL). */
int32_t kdcd_tune_configs(int32_t compute, int32_t *bm, int32_t *bn, int32_t *waves, int32_t max);
/* Pin configuration `id` for (compute, n, sb); id < 0 removes the entry. */
kdcd_status kdcd_tune_set(int32_t compute, int64_t n, int32_t sb, int32_t id);
/* The configuration a launch with (compute, n, sb) uses now (-1: invalid). */
int32_t kdcd_tune_get(int32_t compute, int64_t n, int32_t sb);
/* Time every configuration on A with sb sampled rows (evenly strided),
 * three rounds of `reps` launches each (a configuration counts with its
 * fastest round), record the fastest for (compute, A->n, sb).  The
 * low-precision products are timed without the FP64 Gram launch.
 * best_id / best_us (host, may be NULL) receive the winner and its mean
 * launch time.  Dense A only.  Synchronises `stream`. */
kdcd_status kdcd_autotune(const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t sb,
                          int32_t compute, int32_t reps, int32_t *best_id, double *best_us,
                          kdcd_stream stream);
/* kdcd_autotune for the batched product of kdcd_batch_solve on these problems
 * (their alpha arrays are read, not changed; sigma groups as in the solve):
 * every configuration of compute + KDCD_TUNE_BATCH is timed with sb evenly
 * strided sampled rows, the product and its Gram included, and the fastest is
 * recorded for (compute + KDCD_TUNE_BATCH, A->n, sb).  Dense A only.
 * Synchronises `stream`. */
kdcd_status kdcd_autotune_batch(const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t sb,
                                const kdcd_batch_problem *problems, int32_t n_problems,
                                int32_t compute, int32_t reps, int32_t *best_id, double *best_us,
                                kdcd_stream stream);
kdcd_status kdcd_tune_save(const char *path);
kdcd_status kdcd_tune_load(const char *path);

/* Destroy every graph cached by KDCD_FLAG_GRAPH calls and free the
 * workspaces they own (no call may be running). */
void kdcd_graph_cache_clear(void);

/* Device workspace a solve needs (problem: 0 = K-SVM, 1 = K-RR). */
size_t kdcd_workspace_bytes(int32_t problem, const kdcd_matrix *A, const kdcd_kernel *kernel,
                            int32_t b, int32_t s, int32_t compute);

/* Static, human-readable text for a status code. */
const char *kdcd_status_string(kdcd_status status);

/* Library version string, e.g. "kdcd 0.1.0 gfx950". */
const char *kdcd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KDCD_H */
