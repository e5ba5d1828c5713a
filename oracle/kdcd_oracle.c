/*
 * kdcd_oracle.c -- plain FP64 CPU oracle for s-step DCD (kernel SVM) and
 * s-step BDCD (kernel ridge regression).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference the HIP path is checked against.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it follows (paper: "Scalable Dual Coordinate Descent for Kernel
 * Methods", Shao & Devarakonda):
 *   - kernel functions: Table 1 definitions, evaluated directly (the RBF
 *     distance is summed as sum_k (x_k - y_k)^2, never by norm expansion;
 *     the polynomial power is repeated multiplication);
 *   - DCD for K-SVM (Algorithms 1 and 2) and BDCD for K-RR (Algorithms 3
 *     and 4 / Eq. (3)) written as what they compute: exact minimisation of
 *     the dual objective over one coordinate (K-SVM, projected onto the box)
 *     or one block of coordinates (K-RR), in the order of the index
 *     sequence, each at the current iterate; the s-step variants form the
 *     kernel columns of s consecutive coordinates (blocks) in one pass over
 *     A and then take the s steps with them;
 *   - the K-SVM dual objectives of Sec. 3.1, the primal of Eq. (1) in hinge
 *     form, and the K-RR dual of Eq. (2).
 *
 * Readings where the paper is ambiguous (each is listed in the design notes):
 *   R1  the dual Hessian is Q_pq = y_p y_q K(a_p, a_q) (Sec. 3.1), so the
 *       kernel is applied to the rows of A and then scaled by the labels;
 *   R2  exactly H inner (block) updates; the last outer iteration holds
 *       H - s*floor(H/s) of them;
 *   R3  omega = 1/(2C) for the squared hinge;
 *   R4  the projected-gradient test is an exact FP64 "!= 0";
 *   R5  eta <= 0 gives theta = 0;
 *   R6  the K-RR objective is 1/2 a^T (K/lambda + m I) a - y^T a (the "+m"
 *       inside the double sum of Eq. (2) is read as m * identity, as in
 *       Algorithm 3's G_k);
 *   R15 G_k is SPD and is solved by an unpivoted Cholesky factorisation.
 *
 * Arithmetic: round-to-nearest, no contraction (-ffp-contract=off), no
 * fast-math; sums over n and over m are Neumaier-compensated; loops over
 * independent rows may run under OpenMP (each row's value is computed
 * exactly as in the serial loop, so results do not depend on thread count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_LINEAR = 0, ORC_POLY = 1, ORC_RBF = 2 };
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NOT_SPD = -5, ORC_ERR_ALLOC = -8 };

/* A is either dense row-major (dense != NULL, leading dimension ld) or CSR
 * with sorted, distinct column indices in every row. */
typedef struct {
    int64_t m, n, ld;
    const double *dense;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} orc_matrix;

typedef struct {
    int32_t kind;
    int32_t degree;
    double sigma;
    double c;
} orc_kernel;

/* ---------------------------------------------------------------- sums -- */

typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(const nsum *a) { return a->s + a->c; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later calls (timing only: results do not depend on it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------ kernel function -- */

/* Table 1: a_p . a_q  (compensated sum over the features) */
static double row_dot(const orc_matrix *A, int64_t p, int64_t q)
{
    nsum acc = {0.0, 0.0};
    if (A->dense) {
        const double *x = A->dense + p * A->ld, *z = A->dense + q * A->ld;
        for (int64_t k = 0; k < A->n; ++k) nadd(&acc, x[k] * z[k]);
    } else {
        int64_t i = A->row_ptr[p], ie = A->row_ptr[p + 1];
        int64_t j = A->row_ptr[q], je = A->row_ptr[q + 1];
        while (i < ie && j < je) {
            if (A->col_idx[i] == A->col_idx[j]) { nadd(&acc, A->val[i] * A->val[j]); ++i; ++j; }
            else if (A->col_idx[i] < A->col_idx[j]) ++i;
            else ++j;
        }
    }
    return nval(&acc);
}

/* Table 1 (RBF): ||a_p - a_q||^2 summed term by term over the features */
static double row_dist2(const orc_matrix *A, int64_t p, int64_t q)
{
    nsum acc = {0.0, 0.0};
    if (A->dense) {
        const double *x = A->dense + p * A->ld, *z = A->dense + q * A->ld;
        for (int64_t k = 0; k < A->n; ++k) { double d = x[k] - z[k]; nadd(&acc, d * d); }
    } else {
        int64_t i = A->row_ptr[p], ie = A->row_ptr[p + 1];
        int64_t j = A->row_ptr[q], je = A->row_ptr[q + 1];
        while (i < ie || j < je) {
            double d;
            if (j >= je || (i < ie && A->col_idx[i] < A->col_idx[j])) { d = A->val[i]; ++i; }
            else if (i >= ie || A->col_idx[j] < A->col_idx[i]) { d = -A->val[j]; ++j; }
            else { d = A->val[i] - A->val[j]; ++i; ++j; }
            nadd(&acc, d * d);
        }
    }
    return nval(&acc);
}

/* K(a_p, a_q) from the Table 1 definitions */
double orc_kernel_eval(const orc_matrix *A, const orc_kernel *k, int64_t p, int64_t q)
{
    switch (k->kind) {
    case ORC_LINEAR:
        return row_dot(A, p, q);
    case ORC_POLY: {
        double base = k->c + row_dot(A, p, q), r = 1.0;
        for (int32_t t = 0; t < k->degree; ++t) r *= base;
        return r;
    }
    case ORC_RBF:
        return exp(-k->sigma * row_dist2(A, p, q));
    }
    return NAN;
}

/* out[r*nc + c] = K(a_rows[r], a_cols[c]) */
void orc_kernel_block(const orc_matrix *A, const orc_kernel *k, const int32_t *rows, int64_t nr,
                      const int32_t *cols, int64_t nc, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nr; ++r)
        for (int64_t c = 0; c < nc; ++c)
            out[r * nc + c] = orc_kernel_eval(A, k, rows[r], cols[c]);
}

/* Column q of K(A, A): out[p] = K(a_p, a_q) for every row p */
static void kernel_column(const orc_matrix *A, const orc_kernel *k, int64_t q, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < A->m; ++p) out[p] = orc_kernel_eval(A, k, p, q);
}

/* r_j = sum_p K(a_p, a_{S_j}) beta_p  -- the right-hand-side product U^T beta */
void orc_kernel_rhs(const orc_matrix *A, const orc_kernel *k, const int32_t *S, int64_t sb,
                    const double *beta, double *r)
{
    double *col = malloc(sizeof(double) * (size_t)A->m);
    for (int64_t j = 0; j < sb; ++j) {
        kernel_column(A, k, S[j], col);
        nsum acc = {0.0, 0.0};
        for (int64_t p = 0; p < A->m; ++p) nadd(&acc, col[p] * beta[p]);
        r[j] = nval(&acc);
    }
    free(col);
}

/* ------------------------------------------------------------- K-SVM --- */

static void svm_constants(int loss, double C, double *nu, double *omega)
{
    if (loss == 2) { *nu = INFINITY; *omega = 1.0 / (2.0 * C); }
    else { *nu = C; *omega = 0.0; }
}

static double clip(double x, double nu) { return fmin(fmax(x, 0.0), nu); }

/* Exact minimiser of rho + t over t of  t g + t^2 eta / 2  with rho + t
 * kept in [0, nu]: the unconstrained step -g/eta, clipped.  When the
 * projected gradient is exactly zero (reading R4) or eta <= 0 (R5) the step
 * is 0. */
static double dcd_theta(double rho, double g, double eta, double nu)
{
    double gt = fabs(clip(rho - g, nu) - rho);
    if (gt != 0.0 && eta > 0.0) return clip(rho - g / eta, nu) - rho;
    return 0.0;
}

/* The dual of Sec. 3.1 restricted to coordinate i is the one-dimensional
 * quadratic  f(alpha + t e_i) = f(alpha) + t g + t^2 eta / 2  with
 * g = (Q alpha)_i - 1 + omega alpha_i  (the i-th partial derivative) and
 * eta = Q_ii + omega, minimised over alpha_i + t in [0, nu].  Both DCD
 * variants take exactly this step; they differ only in when the columns of
 * Q are formed. */
static double ksvm_coordinate_gradient(const double *Qcol, const double *alpha, int64_t m,
                                       int64_t i, double omega)
{
    nsum acc = {0.0, 0.0};
    for (int64_t p = 0; p < m; ++p) nadd(&acc, Qcol[p] * alpha[p]);
    nadd(&acc, -1.0);
    nadd(&acc, omega * alpha[i]);
    return nval(&acc);
}

/* Column i of Q = diag(y) K diag(y) (reading R1): out[p] = y_p y_i K(a_p, a_i) */
static void ksvm_q_column(const orc_matrix *A, const double *y, const orc_kernel *k, int64_t i,
                          double *out)
{
    kernel_column(A, k, i, out);
    for (int64_t p = 0; p < A->m; ++p) out[p] *= y[p] * y[i];
}

/* Algorithm 1 (DCD for K-SVM-L1 with loss 1, K-SVM-L2 with loss 2): one
 * exact coordinate minimisation per entry of idx, each with a freshly formed
 * column of Q.  idx holds i_1..i_H; alpha is alpha_0 on entry and alpha_H on
 * exit; theta (optional, length H) receives each step. */
int orc_dcd_ksvm(const orc_matrix *A, const double *y, const orc_kernel *k, double C, int loss,
                 int64_t H, const int32_t *idx, double *alpha, double *theta)
{
    double nu, omega;
    svm_constants(loss, C, &nu, &omega);
    double *q = malloc(sizeof(double) * (size_t)A->m);
    if (!q) return ORC_ERR_ALLOC;
    for (int64_t it = 0; it < H; ++it) {
        const int64_t i = idx[it];
        ksvm_q_column(A, y, k, i, q);
        const double g = ksvm_coordinate_gradient(q, alpha, A->m, i, omega);
        const double th = dcd_theta(alpha[i], g, q[i] + omega, nu);
        alpha[i] += th;
        if (theta) theta[it] = th;
    }
    free(q);
    return ORC_OK;
}

/* Algorithm 2 (s-step DCD): the coordinates are taken s at a time; the s
 * columns of Q that a group needs are formed together, in one pass over A,
 * at the start of the group, and the group's s coordinate minimisations then
 * run in order, each at the current iterate (the gradient of a later step
 * sees every earlier step of its group, duplicates included).  Same contract
 * as orc_dcd_ksvm. */
int orc_sstep_dcd_ksvm(const orc_matrix *A, const double *y, const orc_kernel *k, double C,
                       int loss, int64_t s, int64_t H, const int32_t *idx, double *alpha,
                       double *theta)
{
    if (s < 1) return ORC_ERR_ARG;
    double nu, omega;
    svm_constants(loss, C, &nu, &omega);
    const int64_t m = A->m;
    double *cols = malloc(sizeof(double) * (size_t)(m * s));   /* column t at cols + t*m */
    if (!cols) return ORC_ERR_ALLOC;
    for (int64_t first = 0; first < H; first += s) {
        const int64_t len = (H - first < s) ? H - first : s;     /* reading R2 */
        const int32_t *grp = idx + first;
        for (int64_t t = 0; t < len; ++t) ksvm_q_column(A, y, k, grp[t], cols + t * m);
        for (int64_t t = 0; t < len; ++t) {
            const int64_t i = grp[t];
            const double *q = cols + t * m;
            const double g = ksvm_coordinate_gradient(q, alpha, m, i, omega);
            const double th = dcd_theta(alpha[i], g, q[i] + omega, nu);
            alpha[i] += th;
            if (theta) theta[first + t] = th;
        }
    }
    free(cols);
    return ORC_OK;
}

/* -------------------------------------------------------------- K-RR --- */

/* Unpivoted Cholesky G = L L^T (lower, in place) and solve G x = rhs. */
static int chol_solve(double *G, int64_t b, double *x)
{
    for (int64_t j = 0; j < b; ++j) {
        double d = G[j * b + j];
        for (int64_t p = 0; p < j; ++p) d -= G[j * b + p] * G[j * b + p];
        if (!(d > 0.0)) return ORC_ERR_NOT_SPD;
        d = sqrt(d);
        G[j * b + j] = d;
        for (int64_t i = j + 1; i < b; ++i) {
            double v = G[i * b + j];
            for (int64_t p = 0; p < j; ++p) v -= G[i * b + p] * G[j * b + p];
            G[i * b + j] = v / d;
        }
    }
    for (int64_t i = 0; i < b; ++i) {            /* L z = rhs */
        double v = x[i];
        for (int64_t p = 0; p < i; ++p) v -= G[i * b + p] * x[p];
        x[i] = v / G[i * b + i];
    }
    for (int64_t i = b - 1; i >= 0; --i) {       /* L^T x = z */
        double v = x[i];
        for (int64_t p = i + 1; p < b; ++p) v -= G[p * b + i] * x[p];
        x[i] = v / G[i * b + i];
    }
    return ORC_OK;
}

/* Exact minimisation of the K-RR dual f(alpha) = 1/2 a^T M a - y^T a,
 * M = K/lambda + m I (reading R6), over the b coordinates of block `blk`
 * with the others held fixed: the step d solves M[blk, blk] d = y[blk] -
 * (M alpha)[blk].  cols holds the b kernel columns K(A, a_{blk_l}) (column l
 * at cols + l*m).  The step is written to d and added to alpha. */
static int krr_block_step(const double *cols, const double *y, double lambda, int64_t m,
                          int64_t b, const int32_t *blk, double *alpha, double *G, double *d)
{
    for (int64_t l = 0; l < b; ++l) {
        const double *kl = cols + l * m;
        for (int64_t q = 0; q < b; ++q)
            G[l * b + q] = kl[blk[q]] / lambda + (l == q ? (double)m : 0.0);
        nsum ka = {0.0, 0.0};                    /* (K alpha)_{blk_l} */
        for (int64_t p = 0; p < m; ++p) nadd(&ka, kl[p] * alpha[p]);
        nsum v = {0.0, 0.0};
        nadd(&v, y[blk[l]]);
        nadd(&v, -nval(&ka) / lambda);
        nadd(&v, -(double)m * alpha[blk[l]]);
        d[l] = nval(&v);
    }
    const int rc = chol_solve(G, b, d);
    if (rc != ORC_OK) return rc;
    for (int64_t l = 0; l < b; ++l) alpha[blk[l]] += d[l];
    return ORC_OK;
}

/* Algorithm 3 (BDCD for K-RR): one exact block minimisation per block of
 * idx (H blocks of b distinct coordinates, block major), each with freshly
 * formed kernel columns.  alpha is alpha_0 on entry and alpha_H on exit;
 * delta (optional, length H*b) receives every block's step. */
int orc_bdcd_krr(const orc_matrix *A, const double *y, const orc_kernel *k, double lambda,
                 int64_t b, int64_t H, const int32_t *idx, double *alpha, double *delta)
{
    const int64_t m = A->m;
    double *cols = malloc(sizeof(double) * (size_t)(m * b));
    double *G = malloc(sizeof(double) * (size_t)(b * b));
    double *d = malloc(sizeof(double) * (size_t)b);
    int rc = ORC_OK;
    if (!cols || !G || !d) { rc = ORC_ERR_ALLOC; goto out; }
    for (int64_t it = 0; it < H && rc == ORC_OK; ++it) {
        const int32_t *blk = idx + it * b;
        for (int64_t l = 0; l < b; ++l) kernel_column(A, k, blk[l], cols + l * m);
        rc = krr_block_step(cols, y, lambda, m, b, blk, alpha, G, d);
        if (rc == ORC_OK && delta) memcpy(delta + it * b, d, sizeof(double) * (size_t)b);
    }
out:
    free(cols); free(G); free(d);
    return rc;
}

/* Algorithm 4 / Eq. (3) (s-step BDCD): blocks are taken s at a time; the
 * s*b kernel columns a group needs are formed together, in one pass over A,
 * at the start of the group, and the group's s block minimisations then run
 * in order, each at the current iterate (so a later block sees the earlier
 * blocks' steps, including on coordinates the blocks share).  Same contract
 * as orc_bdcd_krr. */
int orc_sstep_bdcd_krr(const orc_matrix *A, const double *y, const orc_kernel *k, double lambda,
                       int64_t b, int64_t s, int64_t H, const int32_t *idx, double *alpha,
                       double *delta)
{
    if (s < 1) return ORC_ERR_ARG;
    const int64_t m = A->m;
    double *cols = malloc(sizeof(double) * (size_t)(m * s * b));
    double *G = malloc(sizeof(double) * (size_t)(b * b));
    double *d = malloc(sizeof(double) * (size_t)b);
    int rc = ORC_OK;
    if (!cols || !G || !d) { rc = ORC_ERR_ALLOC; goto out; }
    for (int64_t first = 0; first < H && rc == ORC_OK; first += s) {
        const int64_t len = (H - first < s) ? H - first : s;     /* reading R2 */
        const int32_t *grp = idx + first * b;
        for (int64_t c = 0; c < len * b; ++c) kernel_column(A, k, grp[c], cols + c * m);
        for (int64_t t = 0; t < len && rc == ORC_OK; ++t) {
            rc = krr_block_step(cols + t * b * m, y, lambda, m, b, grp + t * b, alpha, G, d);
            if (rc == ORC_OK && delta)
                memcpy(delta + (first + t) * b, d, sizeof(double) * (size_t)b);
        }
    }
out:
    free(cols); free(G); free(d);
    return rc;
}

/* ------------------------------------------------------- objectives --- */

/* out[p] = (K beta)_p = sum_q K(a_p, a_q) beta_q  (m^2 kernel evaluations) */
void orc_kernel_matvec(const orc_matrix *A, const orc_kernel *k, const double *beta, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < A->m; ++p) {
        nsum acc = {0.0, 0.0};
        for (int64_t q = 0; q < A->m; ++q)
            if (beta[q] != 0.0) nadd(&acc, orc_kernel_eval(A, k, p, q) * beta[q]);
        out[p] = nval(&acc);
    }
}

/* K-SVM quantities at alpha (Sec. 3.1 duals, Eq. (1) primal in hinge form):
 * out[0] = f(alpha)   = 1/2 a^T Q a - 1^T a (+ 1/(4C) ||a||^2 for loss 2)
 * out[1] = P(alpha)   = 1/2 a^T Q a + C sum_i max(0, 1 - (Q a)_i)  (squared for loss 2)
 * out[2] = gap        = P(alpha) + f(alpha)   (>= 0; reading R13)
 * out[3] = max |projected gradient| over the box [0, nu]   (KKT violation)
 * Qa (optional, length m) receives Q alpha. */
void orc_ksvm_eval(const orc_matrix *A, const double *y, const orc_kernel *k, double C, int loss,
                   const double *alpha, double *out, double *Qa_out)
{
    int64_t m = A->m;
    double nu, omega;
    svm_constants(loss, C, &nu, &omega);
    double *beta = malloc(sizeof(double) * (size_t)m);
    double *Qa = malloc(sizeof(double) * (size_t)m);
    for (int64_t p = 0; p < m; ++p) beta[p] = y[p] * alpha[p];
    orc_kernel_matvec(A, k, beta, Qa);
    for (int64_t p = 0; p < m; ++p) Qa[p] *= y[p];
    nsum aQa = {0.0, 0.0}, sa = {0.0, 0.0}, sa2 = {0.0, 0.0}, hinge = {0.0, 0.0};
    double kkt = 0.0;
    for (int64_t p = 0; p < m; ++p) {
        nadd(&aQa, alpha[p] * Qa[p]);
        nadd(&sa, alpha[p]);
        nadd(&sa2, alpha[p] * alpha[p]);
        double xi = fmax(0.0, 1.0 - Qa[p]);
        nadd(&hinge, loss == 2 ? xi * xi : xi);
        double grad = Qa[p] - 1.0 + omega * alpha[p], pg;
        if (alpha[p] <= 0.0) pg = fmin(0.0, grad);
        else if (alpha[p] >= nu) pg = fmax(0.0, grad);
        else pg = grad;
        if (fabs(pg) > kkt) kkt = fabs(pg);
    }
    double f = 0.5 * nval(&aQa) - nval(&sa) + (loss == 2 ? nval(&sa2) / (4.0 * C) : 0.0);
    double P = 0.5 * nval(&aQa) + C * nval(&hinge);
    out[0] = f;
    out[1] = P;
    out[2] = P + f;
    out[3] = kkt;
    if (Qa_out) memcpy(Qa_out, Qa, sizeof(double) * (size_t)m);
    free(beta);
    free(Qa);
}

/* K-RR quantities at alpha (Eq. (2), reading R6), M = K/lambda + m I:
 * out[0] = f(alpha) = 1/2 a^T M a - y^T a
 * out[1] = ||y - M a||_2
 * res (optional, length m) receives y - M alpha. */
void orc_krr_eval(const orc_matrix *A, const double *y, const orc_kernel *k, double lambda,
                  const double *alpha, double *out, double *res)
{
    int64_t m = A->m;
    double *Ka = malloc(sizeof(double) * (size_t)m);
    orc_kernel_matvec(A, k, alpha, Ka);
    nsum aMa = {0.0, 0.0}, ya = {0.0, 0.0}, rr = {0.0, 0.0};
    for (int64_t p = 0; p < m; ++p) {
        double Ma = Ka[p] / lambda + (double)m * alpha[p];
        nadd(&aMa, alpha[p] * Ma);
        nadd(&ya, y[p] * alpha[p]);
        double r = y[p] - Ma;
        nadd(&rr, r * r);
        if (res) res[p] = r;
    }
    out[0] = 0.5 * nval(&aMa) - nval(&ya);
    out[1] = sqrt(nval(&rr));
    free(Ka);
}
