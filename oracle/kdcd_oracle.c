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
 *   - Algorithm 1 (DCD for K-SVM) and Algorithm 2 (s-step DCD), steps in
 *     the paper's order and notation;
 *   - Algorithm 3 (BDCD for K-RR) and Algorithm 4 / Eq. (3) (s-step BDCD);
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

/* The coordinate step shared by Algorithms 1 and 2: given the current value
 * rho of the coordinate, its gradient g and curvature eta, return theta. */
static double dcd_theta(double rho, double g, double eta, double nu)
{
    double gt = fabs(clip(rho - g, nu) - rho);
    if (gt != 0.0 && eta > 0.0) return clip(rho - g / eta, nu) - rho;
    return 0.0;
}

/* Algorithm 1: DCD for K-SVM-L1 (loss 1) / K-SVM-L2 (loss 2).  idx holds the
 * H coordinates i_1..i_H; alpha is alpha_0 on entry and alpha_H on exit.
 * theta (optional, length H) receives every step's theta_k. */
int orc_dcd_ksvm(const orc_matrix *A, const double *y, const orc_kernel *k, double C, int loss,
                 int64_t H, const int32_t *idx, double *alpha, double *theta)
{
    double nu, omega;
    svm_constants(loss, C, &nu, &omega);
    double *u = malloc(sizeof(double) * (size_t)A->m);
    if (!u) return ORC_ERR_ALLOC;
    for (int64_t it = 0; it < H; ++it) {
        int64_t i = idx[it];
        /* u_k = K(Atilde, e_i^T Atilde): Q column i (reading R1) */
        kernel_column(A, k, i, u);
        for (int64_t p = 0; p < A->m; ++p) u[p] *= y[p] * y[i];
        double eta = u[i] + omega;
        nsum acc = {0.0, 0.0};
        for (int64_t p = 0; p < A->m; ++p) nadd(&acc, u[p] * alpha[p]);
        double g = nval(&acc) - 1.0 + omega * alpha[i];
        double th = dcd_theta(alpha[i], g, eta, nu);
        alpha[i] += th;
        if (theta) theta[it] = th;
    }
    free(u);
    return ORC_OK;
}

/* Algorithm 2: s-step DCD for K-SVM.  Same contract as orc_dcd_ksvm. */
int orc_sstep_dcd_ksvm(const orc_matrix *A, const double *y, const orc_kernel *k, double C,
                       int loss, int64_t s, int64_t H, const int32_t *idx, double *alpha,
                       double *theta)
{
    if (s < 1) return ORC_ERR_ARG;
    double nu, omega;
    svm_constants(loss, C, &nu, &omega);
    int64_t m = A->m;
    double *U = malloc(sizeof(double) * (size_t)(m * s));
    double *col = malloc(sizeof(double) * (size_t)m);
    double *G = malloc(sizeof(double) * (size_t)(s * s));
    double *th = malloc(sizeof(double) * (size_t)s);
    if (!U || !col || !G || !th) { free(U); free(col); free(G); free(th); return ORC_ERR_ALLOC; }
    for (int64_t k0 = 0; k0 < H; k0 += s) {
        int64_t sk = (H - k0 < s) ? H - k0 : s;        /* reading R2 */
        const int32_t *I = idx + k0;
        /* U_k = K(Atilde, Atilde_k): columns i_1..i_sk of Q, stored U[p*sk + j] */
        for (int64_t j = 0; j < sk; ++j) {
            kernel_column(A, k, I[j], col);
            for (int64_t p = 0; p < m; ++p) U[p * sk + j] = col[p] * y[p] * y[I[j]];
        }
        /* G_k = V_k^T U_k + omega I ; eta_j = diag(G_k) */
        for (int64_t t = 0; t < sk; ++t)
            for (int64_t j = 0; j < sk; ++j)
                G[t * sk + j] = U[(int64_t)I[t] * sk + j] + (t == j ? omega : 0.0);
        for (int64_t j = 0; j < sk; ++j) {
            /* rho_j = e_{i_j}^T alpha_sk + sum_{t<j, i_t = i_j} theta_t */
            nsum rho = {0.0, 0.0};
            nadd(&rho, alpha[I[j]]);
            for (int64_t t = 0; t < j; ++t)
                if (I[t] == I[j]) nadd(&rho, th[t]);
            /* g_j = (U_k e_j)^T alpha_sk - 1 + omega alpha_{i_j}
             *       + sum_{t<j} (e_{i_t}^T U_k e_j) theta_t
             *       + omega sum_{t<j, i_t = i_j} theta_t */
            nsum g = {0.0, 0.0};
            for (int64_t p = 0; p < m; ++p) nadd(&g, U[p * sk + j] * alpha[p]);
            nadd(&g, -1.0);
            nadd(&g, omega * alpha[I[j]]);
            for (int64_t t = 0; t < j; ++t) nadd(&g, U[(int64_t)I[t] * sk + j] * th[t]);
            for (int64_t t = 0; t < j; ++t)
                if (I[t] == I[j]) nadd(&g, omega * th[t]);
            double eta = G[j * sk + j];
            th[j] = dcd_theta(nval(&rho), nval(&g), eta, nu);
        }
        /* alpha_{sk+s} = alpha_sk + sum_t theta_t e_{i_t}, in t order */
        for (int64_t t = 0; t < sk; ++t) {
            alpha[I[t]] += th[t];
            if (theta) theta[k0 + t] = th[t];
        }
    }
    free(U); free(col); free(G); free(th);
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

/* Algorithm 3: BDCD for K-RR.  idx holds H blocks of b coordinates (block
 * major); alpha is alpha_0 on entry and alpha_H on exit.  delta (optional,
 * length H*b) receives every block's Delta alpha_k. */
int orc_bdcd_krr(const orc_matrix *A, const double *y, const orc_kernel *k, double lambda,
                 int64_t b, int64_t H, const int32_t *idx, double *alpha, double *delta)
{
    int64_t m = A->m;
    double *U = malloc(sizeof(double) * (size_t)(m * b));
    double *col = malloc(sizeof(double) * (size_t)m);
    double *G = malloc(sizeof(double) * (size_t)(b * b));
    double *x = malloc(sizeof(double) * (size_t)b);
    int rc = ORC_OK;
    if (!U || !col || !G || !x) { rc = ORC_ERR_ALLOC; goto out; }
    for (int64_t it = 0; it < H; ++it) {
        const int32_t *S = idx + it * b;
        /* U_k = K(A, V_k^T A) */
        for (int64_t l = 0; l < b; ++l) {
            kernel_column(A, k, S[l], col);
            for (int64_t p = 0; p < m; ++p) U[p * b + l] = col[p];
        }
        /* G_k = (1/lambda) V_k^T U_k + m I */
        for (int64_t l = 0; l < b; ++l)
            for (int64_t q = 0; q < b; ++q)
                G[l * b + q] = U[(int64_t)S[l] * b + q] / lambda + (l == q ? (double)m : 0.0);
        /* rhs = V_k^T y - m V_k^T alpha - (1/lambda) U_k^T alpha */
        for (int64_t l = 0; l < b; ++l) {
            nsum ua = {0.0, 0.0};
            for (int64_t p = 0; p < m; ++p) nadd(&ua, U[p * b + l] * alpha[p]);
            nsum v = {0.0, 0.0};
            nadd(&v, y[S[l]]);
            nadd(&v, -(double)m * alpha[S[l]]);
            nadd(&v, -nval(&ua) / lambda);
            x[l] = nval(&v);
        }
        if ((rc = chol_solve(G, b, x)) != ORC_OK) goto out;
        for (int64_t l = 0; l < b; ++l) {
            alpha[S[l]] += x[l];
            if (delta) delta[it * b + l] = x[l];
        }
    }
out:
    free(U); free(col); free(G); free(x);
    return rc;
}

/* Algorithm 4 / Eq. (3): s-step BDCD for K-RR.  Same contract as orc_bdcd_krr. */
int orc_sstep_bdcd_krr(const orc_matrix *A, const double *y, const orc_kernel *k, double lambda,
                       int64_t b, int64_t s, int64_t H, const int32_t *idx, double *alpha,
                       double *delta)
{
    if (s < 1) return ORC_ERR_ARG;
    int64_t m = A->m, sbmax = s * b;
    double *Q = malloc(sizeof(double) * (size_t)(m * sbmax));
    double *col = malloc(sizeof(double) * (size_t)m);
    double *G = malloc(sizeof(double) * (size_t)(b * b));
    double *D = malloc(sizeof(double) * (size_t)sbmax);
    int rc = ORC_OK;
    if (!Q || !col || !G || !D) { rc = ORC_ERR_ALLOC; goto out; }
    for (int64_t k0 = 0; k0 < H; k0 += s) {
        int64_t sk = (H - k0 < s) ? H - k0 : s;        /* reading R2 */
        int64_t sb = sk * b;
        const int32_t *Om = idx + k0 * b;              /* Omega_k, sk*b coordinates */
        /* Q_k = K(A, Omega_k^T A), stored Q[p*sb + c] */
        for (int64_t c = 0; c < sb; ++c) {
            kernel_column(A, k, Om[c], col);
            for (int64_t p = 0; p < m; ++p) Q[p * sb + c] = col[p];
        }
        for (int64_t j = 0; j < sk; ++j) {
            const int32_t *Sj = Om + j * b;            /* V_{sk+j}; U_{sk+j} = Q_k Psi_j */
            /* G_{sk+j} = (1/lambda) V^T U + m I */
            for (int64_t l = 0; l < b; ++l)
                for (int64_t q = 0; q < b; ++q)
                    G[l * b + q] = Q[(int64_t)Sj[l] * sb + j * b + q] / lambda +
                                   (l == q ? (double)m : 0.0);
            double *x = D + j * b;
            for (int64_t l = 0; l < b; ++l) {
                /* V^T y - m V^T alpha_sk - m sum_t V_j^T V_t Delta_t
                 *  - (1/lambda) U^T alpha_sk - (1/lambda) sum_t U_j^T V_t Delta_t */
                nsum ua = {0.0, 0.0};
                for (int64_t p = 0; p < m; ++p) nadd(&ua, Q[p * sb + j * b + l] * alpha[p]);
                nsum ov = {0.0, 0.0}, uv = {0.0, 0.0};
                for (int64_t t = 0; t < j; ++t)
                    for (int64_t q = 0; q < b; ++q) {
                        int32_t it = Om[t * b + q];
                        if (it == Sj[l]) nadd(&ov, D[t * b + q]);
                        nadd(&uv, Q[(int64_t)it * sb + j * b + l] * D[t * b + q]);
                    }
                nsum v = {0.0, 0.0};
                nadd(&v, y[Sj[l]]);
                nadd(&v, -(double)m * alpha[Sj[l]]);
                nadd(&v, -(double)m * nval(&ov));
                nadd(&v, -nval(&ua) / lambda);
                nadd(&v, -nval(&uv) / lambda);
                x[l] = nval(&v);
            }
            if ((rc = chol_solve(G, b, x)) != ORC_OK) goto out;
        }
        /* alpha_{sk+s} = alpha_sk + sum_t V_t Delta_t, in t order */
        for (int64_t c = 0; c < sb; ++c) {
            alpha[Om[c]] += D[c];
            if (delta) delta[k0 * b + c] = D[c];
        }
    }
out:
    free(Q); free(col); free(G); free(D);
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
