// Support kernels around the kernel-block product:
//   - row norms ||a_p||^2 (once per solve, RBF only);
//   - input validation (index range, labels, box feasibility, finiteness);
//   - the finish pass of every outer iteration: the deterministic reduction
//     of the per-row-group partials into r, and, for K-RR, the inverses of
//     the s diagonal block matrices G_j = W_jj / lambda + m I of Algorithm 4.
#include "common.hpp"

namespace kdcd {
namespace {

// One wave per row; lanes stride over the row (dense) or its stored entries (CSR).
__global__ __launch_bounds__(256) void norms_kernel(const double *__restrict__ vals,
                                                    const int64_t *__restrict__ row_ptr,
                                                    int64_t m, int64_t n, int64_t ld,
                                                    double *__restrict__ norms)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    double s = 0.0;
    if (row_ptr) {
        for (int64_t e = row_ptr[row] + lane; e < row_ptr[row + 1]; e += 64) s += vals[e] * vals[e];
    } else {
        const double *x = vals + row * ld;
        for (int64_t k = lane; k < n; k += 64) s += x[k] * x[k];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) norms[row] = s;
}

// problem 0 (K-SVM): y in {-1,+1}, 0 <= alpha <= nu; problem 1 (K-RR): finite y, alpha.
__global__ __launch_bounds__(256) void validate_kernel(const int32_t *__restrict__ idx,
                                                       int64_t count, int64_t m,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ alpha,
                                                       int64_t mrows, int32_t problem, double nu,
                                                       int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = i; t < count; t += stride) {
        const int32_t v = idx[t];
        if (v < 0 || v >= m) set_status(status, KDCD_ERR_INDEX_RANGE);
    }
    for (int64_t p = i; p < mrows; p += stride) {
        const double yv = y[p], av = alpha[p];
        if (!isfinite(yv) || !isfinite(av)) set_status(status, KDCD_ERR_NONFINITE);
        if (problem == 0) {
            if (yv != 1.0 && yv != -1.0) set_status(status, KDCD_ERR_INVALID_ARG);
            if (!(av >= 0.0 && av <= nu)) set_status(status, KDCD_ERR_INVALID_ARG);
        }
    }
}

// CSR structure: row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz, columns in [0, n).
__global__ __launch_bounds__(256) void validate_csr_kernel(const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col_idx,
                                                           int64_t m, int64_t n, int64_t nnz,
                                                           int32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i == 0 && (row_ptr[0] != 0 || row_ptr[m] != nnz)) set_status(status, KDCD_ERR_INVALID_ARG);
    for (int64_t r = i; r < m; r += stride)
        if (row_ptr[r + 1] < row_ptr[r]) set_status(status, KDCD_ERR_INVALID_ARG);
    for (int64_t e = i; e < nnz; e += stride) {
        const int32_t c = col_idx[e];
        if (c < 0 || c >= n) set_status(status, KDCD_ERR_INVALID_ARG);
    }
}

// Longest row of a CSR matrix (stored entries) into *out (cleared by the caller);
// a decreasing row_ptr gives a huge unsigned length, i.e. no bound.
__global__ __launch_bounds__(256) void csr_row_max_kernel(const int64_t *__restrict__ row_ptr,
                                                          int64_t m, unsigned long long *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long v = 0;
    for (int64_t r = i; r < m; r += stride) {
        const unsigned long long len = (unsigned long long)(row_ptr[r + 1] - row_ptr[r]);
        v = len > v ? len : v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, v);
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void iota_i32_kernel(int32_t *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = (int32_t)i;
}

constexpr int FIN_COLS = 8;     // columns per reduction workgroup
constexpr int FIN_PARTS = 32;   // row-group partitions per column

// Blocks [0, nprob * ceil(sb/8)) reduce r of every problem; the next nkrr * sk
// invert one diagonal block of one K-RR problem each (Gauss-Jordan without
// pivoting, valid for SPD matrices); with dup_S the next ceil(sb/4) copy the
// Gram rows of repeated coordinates (one wave per row); with la_Sc or la_pos
// the last two apply the previous block's updates to alpha and move the
// row -> position table on.
__global__ __launch_bounds__(256) void finish_kernel(const FinishDesc d, int32_t sb, int32_t b,
                                                     int32_t sk, double mdbl, int32_t *status)
{
    __shared__ double sh[kMaxB * kMaxB];
    if (d.stop && *d.stop) return;
    const int tid = threadIdx.x;
    const int per = (sb + FIN_COLS - 1) / FIN_COLS;
    const int n_red = per * d.nprob;
    if ((int)blockIdx.x < n_red) {
        const int p = (int)blockIdx.x / per;
        const int c = tid % FIN_COLS, part = tid / FIN_COLS;
        const int64_t col = (int64_t)((int)blockIdx.x % per) * FIN_COLS + c;
        const double *partial = d.partial[p];
        double s = 0.0;
        if (col < sb)
            for (int64_t g0 = part; g0 < d.groups; g0 += 8 * FIN_PARTS) {
                // eight loads in flight, added in row-group order
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int64_t g = g0 + (int64_t)u * FIN_PARTS;
                    v[u] = g < d.groups ? partial[g * sb + col] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s += v[u];
            }
        if (d.la_Sc && col < sb) {
            // the previous block's updates against the kernel rows of their
            // coordinates (one partition's share of the canonical elements),
            // eight rows in flight, added in row order
            double f = 0.0;
            for (int t0 = part; t0 < d.la_sb; t0 += 8 * FIN_PARTS) {
                double q[8], dc[8];
                int32_t sc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int t = t0 + u * FIN_PARTS;
                    const int tc = t < d.la_sb ? t : d.la_sb - 1;
                    sc[u] = t < d.la_sb ? d.la_Sc[tc] : -1;
                    dc[u] = d.la_Dc[tc];
                    q[u] = d.la_QX[(int64_t)tc * sb + col];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (sc[u] >= 0) f += q[u] * dc[u];
            }
            s += f;
        }
        sh[part * FIN_COLS + c] = s;
        __syncthreads();
        if (part == 0 && col < sb) {
            double t = 0.0;
            for (int q = 0; q < FIN_PARTS; ++q) t += sh[q * FIN_COLS + c];
            d.r[p][col] = t;
        }
        return;
    }
    const int x = (int)blockIdx.x - n_red;
    const int n_inv = d.nkrr * sk;
    // row written for the coordinate of row t (t itself unless t repeats it)
    auto src_row = [&](int64_t t) -> int64_t {
        if (!d.dup_S) return t;
        const int32_t p = d.dup_S[t];
        if (p < 0 || p >= d.m) return t;
        const int32_t w = d.dup_pos[p];
        return (w >= 0 && w < sb) ? w : t;
    };
    const int n_dup = d.dup_S ? (sb + 3) / 4 : 0;
    if (x == n_inv + n_dup) {   // lookahead: the previous block's updates into alpha
        if (!d.la_Sc) return;
        for (int t0 = tid; t0 < d.la_sb; t0 += 4 * (int)blockDim.x) {
            int32_t p[4];
            double dc[4], av[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                p[u] = t < d.la_sb ? d.la_Sc[t] : -1;
                dc[u] = t < d.la_sb ? d.la_Dc[t] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = (p[u] >= 0 && p[u] < d.m) ? d.la_alpha[p[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (p[u] < 0 || p[u] >= d.m) continue;
                const double v = av[u] + dc[u];
                if (!isfinite(v)) set_status(status, KDCD_ERR_NONFINITE);
                d.la_alpha[p[u]] = v;
            }
        }
        return;
    }
    if (x > n_inv + n_dup) {    // lookahead: the row -> position table moves on
        if (!d.la_pos) return;
        for (int t = tid; t < d.la_clear_sb; t += blockDim.x) {
            const int32_t p = d.la_clearS[t];
            if (p >= 0 && p < d.m) d.la_pos[p] = -1;
        }
        __syncthreads();
        // a repeated coordinate keeps its last element, whatever the order
        // of the stores: the lookahead sums depend on which one it is
        for (int t = tid; t < d.la_set_sb; t += blockDim.x) {
            const int32_t p = d.la_setS[t];
            if (p >= 0 && p < d.m) atomicMax(&d.la_pos[p], t);
        }
        return;
    }
    if (x >= n_inv) {   // one wave per row
        if (!d.dup_S) return;
        const int lane = tid & 63;
        const int64_t t = (int64_t)(x - n_inv) * 4 + (tid >> 6);
        if (t >= sb) return;
        const int64_t w = src_row(t);
        if (w == t) return;
        const int32_t St = d.dup_S[t];
        // the whole row is loaded before any store (a load after a store to the
        // same array cannot be moved ahead of it, which left one load latency
        // per 64 columns); lookahead: lambda m at the other elements of the
        // coordinate, so that the recurrence reads G = W' / lambda without
        // comparing coordinates
        constexpr int DUPC = kMaxSB / 64;
        double v[DUPC];
        int32_t sc[DUPC];
#pragma unroll
        for (int u = 0; u < DUPC; ++u) {
            const int64_t c = lane + 64 * u;
            v[u] = c < sb ? d.dup_W[w * sb + c] : 0.0;
            sc[u] = (c < sb && d.la_lm != 0.0) ? d.dup_S[c] : -1;
        }
#pragma unroll
        for (int u = 0; u < DUPC; ++u) {
            const int64_t c = lane + 64 * u;
            if (c < sb) d.dup_W[t * sb + c] = (c != t && sc[u] == St) ? v[u] + d.la_lm : v[u];
        }
        return;
    }
    const int k = x / sk, j = x % sk;
    const double *W = d.W[k];
    const double inv_lambda = d.inv_lambda[k];
    const int bb = b * b;
    const int64_t base = (int64_t)j * b;
    for (int e = tid; e < bb; e += blockDim.x) {
        const int l = e / b, q = e % b;
        sh[e] = W[src_row(base + l) * sb + base + q] * inv_lambda + (l == q ? mdbl : 0.0);
    }
    __syncthreads();
    bool bad = false;
    for (int kk = 0; kk < b; ++kk) {
        const double piv = sh[kk * b + kk];
        if (!(piv > 0.0) || !isfinite(piv)) bad = true;
        const double pinv = 1.0 / piv;
        // every thread reads what it needs of row kk and column kk before anyone writes
        double rowk[kMaxB * kMaxB / 256 + 1], colk[kMaxB * kMaxB / 256 + 1];
        int cnt = 0;
        for (int e = tid; e < bb; e += blockDim.x, ++cnt) {
            const int l = e / b, q = e % b;
            rowk[cnt] = (q == kk) ? 1.0 : sh[kk * b + q];
            colk[cnt] = sh[l * b + kk];
        }
        __syncthreads();
        cnt = 0;
        for (int e = tid; e < bb; e += blockDim.x, ++cnt) {
            const int l = e / b, q = e % b;
            const double nk = rowk[cnt] * pinv;           // new row-kk entry in column q
            if (l == kk) sh[e] = nk;
            else sh[e] = ((q == kk) ? 0.0 : sh[e]) - nk * colk[cnt];
        }
        __syncthreads();
    }
    if (bad && tid == 0) set_status(status, KDCD_ERR_NOT_SPD);
    double *Dinv = d.Dinv[k];
    for (int e = tid; e < bb; e += blockDim.x) Dinv[(int64_t)j * bb + e] = sh[e];
}

}  // namespace

hipError_t launch_norms(const kdcd_matrix *A, double *norms, hipStream_t st)
{
    const unsigned blocks = (unsigned)((A->m + 3) / 4);
    const bool csr = A->format == KDCD_CSR;
    hipLaunchKernelGGL(norms_kernel, dim3(blocks), dim3(256), 0, st, A->values,
                       csr ? A->row_ptr : nullptr, A->m, A->n, A->ld, norms);
    return hipGetLastError();
}

hipError_t launch_validate(const int32_t *idx, int64_t count, int64_t m, const double *y,
                           const double *alpha, int64_t mrows, int32_t problem, double nu,
                           int32_t *status, hipStream_t st)
{
    const int64_t work = count > mrows ? count : mrows;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0, st, idx, count, m,
                       y, alpha, mrows, problem, nu, status);
    return hipGetLastError();
}

hipError_t launch_validate_csr(const kdcd_matrix *A, int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL(validate_csr_kernel, dim3(2048), dim3(256), 0, st, A->row_ptr, A->col_idx,
                       A->m, A->n, A->nnz, status);
    return hipGetLastError();
}

hipError_t launch_csr_row_max(const kdcd_matrix *A, unsigned long long *out, hipStream_t st)
{
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<int32_t *>(out),
                       0, (int64_t)2);
    int64_t blocks = (A->m + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(csr_row_max_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A->row_ptr,
                       A->m, out);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       p, v, count);
    return hipGetLastError();
}

// Graph window of W outer iterations: copies index blocks k0 - 1 .. k0 + W of
// idx (blocks of sb) into the window buffer, k0 read from the device counter,
// and moves the counter on by W.  The caller keeps every window inside idx.
__global__ __launch_bounds__(1024) void window_advance_kernel(const int32_t *__restrict__ idx,
                                                              int64_t *counter,
                                                              int32_t *__restrict__ Swin,
                                                              int32_t W, int32_t sb)
{
    const int64_t k0 = *counter;
    const int64_t n = (int64_t)(W + 2) * sb;
    const int32_t *src = idx + (k0 - 1) * (int64_t)sb;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) Swin[i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0) *counter = k0 + W;
}

hipError_t launch_window_advance(const int32_t *idx, int64_t *counter, int32_t *Swin, int32_t W,
                                 int32_t sb, hipStream_t st)
{
    hipLaunchKernelGGL(window_advance_kernel, dim3(1), dim3(1024), 0, st, idx, counter, Swin, W, sb);
    return hipGetLastError();
}

// A batch descriptor passed by value (kernel arguments) written to device
// memory: as a kernel node of a captured graph, every replay rewrites the copy
// its launches read, whatever another call did to that memory meanwhile.
__global__ void copy_batch_desc_kernel(const BatchDesc d, BatchDesc *dst)
{
    if (threadIdx.x == 0) *dst = d;
}

hipError_t launch_copy_batch_desc(const BatchDesc &d, BatchDesc *dst, hipStream_t st)
{
    hipLaunchKernelGGL(copy_batch_desc_kernel, dim3(1), dim3(64), 0, st, d, dst);
    return hipGetLastError();
}

hipError_t launch_iota_i32(int32_t *p, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(iota_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p,
                       count);
    return hipGetLastError();
}

hipError_t launch_finish(const FinishDesc &d, int32_t sb, int32_t b, int32_t sk, double mdbl,
                         int32_t *status, hipStream_t st)
{
    const int per = (sb + FIN_COLS - 1) / FIN_COLS;
    const int blocks = per * d.nprob + d.nkrr * sk + (d.dup_S ? (sb + 3) / 4 : 0) +
                       ((d.la_Sc || d.la_pos) ? 2 : 0);
    KDCD_TIMED_LAUNCH(finish_kernel, dim3(blocks), dim3(256), 0, st, d, sb, b, sk, mdbl, status);
    return hipGetLastError();
}

}  // namespace kdcd
