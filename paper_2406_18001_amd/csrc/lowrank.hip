// Low-rank kernel blocks (the Nystrom approximation of the sampled kernel
// matrix that the paper's conclusion proposes).
//
// With a factor Phi (m x r) of the approximated kernel matrix, K ~ Phi Phi^T,
// the quantities an outer iteration of Algorithms 2 and 4 needs shrink:
//   U^T beta = Phi_S (Phi^T beta) = Phi_S z       (s*b x r, z kept current)
//   V^T U    = Phi_S Phi_S^T                       (s*b x s*b x r)
// and after the recurrence z += Phi_S^T (c o theta), c = y_S (K-SVM) or 1
// (K-RR): no pass over the m rows.  The factor itself is built once:
//   C C^T = K(A_L, A_L) + jitter I (blocked Cholesky),  Phi = K(X, A_L) C^{-T}
// (blocked forward substitution), every step on the device.
//
// All products go through one gathered FP64 MFMA tile kernel
//   out[i][j] (op)= sum_k A[ra(i)][k] * B[rb(j)][k]
// whose epilogue stores, subtracts, or applies the Table 1 map.
#include <algorithm>

#include "common.hpp"

namespace kdcd {
namespace {

constexpr int GT = 64;      // output tile edge
constexpr int GK = 16;      // K chunk staged through LDS
constexpr int PNB = 64;     // panel width of the Cholesky and the substitution

enum { EPI_STORE = 0, EPI_SUB = 1, EPI_KERNEL = 2 };

struct GemmArgs {
    const double *A;
    int64_t lda;
    const int32_t *ra;   // rows of A used as output rows (null: 0..M-1)
    int64_t rowsA;       // rows of A (gathered indices are clamped into range)
    const double *B;
    int64_t ldb;
    const int32_t *rb;
    int64_t rowsB;
    int64_t M, N, K;
    double *out;
    int64_t ldo;
    int32_t lower;       // only tiles on or below the diagonal
    int32_t mirror;      // lower: also store the transpose of off-diagonal tiles
    KParams kp;          // EPI_KERNEL
    const double *na;    // RBF: squared norms of A's rows (indexed by the gathered row)
    const double *nb;
    int32_t same;        // A and B are the same matrix: equal rows have distance 0
    double diag_add;     // EPI_KERNEL: added where i == j
};

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// Output tile of block t: (ti, tj), lower-triangular enumeration when asked.
__device__ __forceinline__ void tile_of(const GemmArgs &g, int64_t t, int32_t tiles_n, int64_t &ti,
                                        int64_t &tj)
{
    if (g.lower) {
        ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = t / tiles_n;
        tj = t % tiles_n;
    }
}

template <int EPI, int KIND>
__device__ __forceinline__ void epilogue(const GemmArgs &g, int64_t row, int64_t col, double x,
                                         bool diag_tile)
{
    if (row >= g.M || col >= g.N) return;
    if constexpr (EPI == EPI_STORE) {
        g.out[row * g.ldo + col] = x;
        if (g.mirror && !diag_tile) g.out[col * g.ldo + row] = x;
    } else if constexpr (EPI == EPI_SUB) {
        if (g.lower && col > row) return;   // only the lower triangle is live
        g.out[row * g.ldo + col] -= x;
    } else {
        const int64_t gr = g.ra ? clampi(g.ra[row], 0, g.rowsA - 1) : row;
        const int64_t gc = g.rb ? clampi(g.rb[col], 0, g.rowsB - 1) : col;
        const double na = (KIND == KDCD_KERNEL_RBF) ? g.na[gr] : 0.0;
        const double nb = (KIND == KDCD_KERNEL_RBF) ? g.nb[gc] : 0.0;
        double kv = kernel_map<KIND>(x, na, nb, g.same && gr == gc, g.kp);
        if (row == col) kv += g.diag_add;
        g.out[row * g.ldo + col] = kv;
    }
}

// Tile grid: 4 waves in 2 x 2, each wave 2 x 2 MFMA blocks of 16 x 16.
// Operands are staged fragment-major exactly as in the FP64 kernel-block
// product (MFMA step ks takes k = 4*(lane/16) + ks of the chunk); the next
// chunk is loaded into registers while the current one is multiplied.
// blockIdx.y = p > 0 splits K: slice p of `ksl` columns, and with more than
// one slice the raw 64 x 64 tile goes to part[(p * tiles + t) * 4096 + ...]
// for the reduction kernel, which then applies the epilogue.
template <int EPI, int KIND>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g, int32_t tiles_n, int64_t tiles,
                                                      int64_t ksl, double *__restrict__ part)
{
    __shared__ double As[GT * GK];
    __shared__ double Bs[GT * GK];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;

    int64_t ti, tj;
    const int64_t t = blockIdx.x;
    tile_of(g, t, tiles_n, ti, tj);
    const int64_t row0 = ti * GT, col0 = tj * GT;
    const int64_t kbeg = (int64_t)blockIdx.y * ksl;
    const int64_t kend = min(g.K, kbeg + ksl);

    // loader: thread -> (tile row r, quad c) for both operands
    const int r = tid >> 2, c = tid & 3;
    const int64_t ia = clampi(row0 + r, 0, g.M - 1);
    const int64_t jb = clampi(col0 + r, 0, g.N - 1);
    const int64_t rowA = g.ra ? clampi(g.ra[ia], 0, g.rowsA - 1) : ia;
    const int64_t rowB = g.rb ? clampi(g.rb[jb], 0, g.rowsB - 1) : jb;
    const double *pa = g.A + rowA * g.lda + 4 * c;
    const double *pb = g.B + rowB * g.ldb + 4 * c;
    const int sidx = ((r >> 4) * 16 + c) * 16 + (r & 15);

    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    double va[4], vb[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ok = k0 + 4 * c + e < kend;
            va[e] = ok ? pa[k0 + e] : 0.0;
            vb[e] = ok ? pb[k0 + e] : 0.0;
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();   // the previous chunk has been consumed
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            As[sidx + e * 64] = va[e];
            Bs[sidx + e * 64] = vb[e];
        }
        __syncthreads();
        if (k0 + GK < kend) load(k0 + GK);   // in flight during the products below
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            double a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = As[((wm * 2 + q) * 4 + ks) * 64 + lane];
                b[q] = Bs[((wn * 2 + q) * 4 + ks) * 64 + lane];
            }
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
        }
    }

    // item v of lane l is row (l/16) + 4v, column l%16 of its block
    const bool diag_tile = ti == tj;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int lr = (wm * 2 + p) * 16 + (lane >> 4) + 4 * v;
                const int lc = (wn * 2 + q) * 16 + (lane & 15);
                if (part) part[((int64_t)blockIdx.y * tiles + t) * (GT * GT) + lr * GT + lc] = acc[p][q][v];
                else epilogue<EPI, KIND>(g, row0 + lr, col0 + lc, acc[p][q][v], diag_tile);
            }
}

// Sum of the K slices of every tile in slice order, then the epilogue;
// blockIdx.y picks 256 of the tile's 4096 elements.
template <int EPI, int KIND>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, int32_t tiles_n,
                                                          int64_t tiles, int32_t nslices,
                                                          const double *__restrict__ part)
{
    const int64_t t = blockIdx.x;
    int64_t ti, tj;
    tile_of(g, t, tiles_n, ti, tj);
    const int e = blockIdx.y * 256 + threadIdx.x;
    const double *src = part + t * (GT * GT) + e;
    const int64_t stride = tiles * (GT * GT);
    double x = 0.0;
#pragma unroll 8
    for (int p = 0; p < nslices; ++p) x += src[p * stride];
    epilogue<EPI, KIND>(g, ti * GT + e / GT, tj * GT + e % GT, x, ti == tj);
}

// Forward substitution of one row, one wave per row and lane l holding x_l:
// x D^T = b for lower-triangular D (PNB x PNB, identity past the panel edge),
// i.e. x_k = (b_k - sum_{l<k} x_l D[k][l]) / D[k][k], the subtractions in
// the order of l.  Dt holds D transposed (Dt[k][l] = D[l][k]).
__device__ __forceinline__ double solve_row_wave(double x, const double (*Dt)[PNB + 1], int lane)
{
    for (int k = 0; k < PNB; ++k) {
        const double xk = __shfl(x, k) / Dt[k][k];
        if (lane == k) x = xk;
        else if (lane > k) x -= xk * Dt[k][lane];
    }
    return x;
}

// Dt[k][i] = D[i][k] for the diagonal block of panel j0 (upper part zero,
// identity past the panel edge).
__device__ void load_diag_block_t(double (*Dt)[PNB + 1], const double *Cw, int64_t ld, int32_t j0,
                                  int32_t nb)
{
    for (int e = threadIdx.x; e < PNB * PNB; e += blockDim.x) {
        const int i = e / PNB, k = e % PNB;
        double v;
        if (i < nb && k < nb) v = (k <= i) ? Cw[(int64_t)(j0 + i) * ld + j0 + k] : 0.0;
        else v = (i == k) ? 1.0 : 0.0;
        Dt[k][i] = v;
    }
}

// Panel j0 of the right-looking Cholesky of the r x r working matrix Cw
// (lower triangle live): factor the diagonal block D in LDS and write it
// back, and write D^{-1} (row-major, 64 x 64, identity past the panel edge)
// to Dinv, column c of D^{-1} being the solution of D u = e_c.  The rows
// below the block and the rows of Phi are then multiplied by D^{-T} with the
// tile kernel.
__global__ __launch_bounds__(1024) void chol_panel_kernel(double *__restrict__ Cw, int64_t ld,
                                                          int32_t r, int32_t j0,
                                                          double *__restrict__ Dinv,
                                                          int32_t *__restrict__ status)
{
    __shared__ double Dt[PNB][PNB + 1];   // Dt[k][i] = D[i][k]
    const int nb = min(PNB, r - j0);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    load_diag_block_t(Dt, Cw, ld, j0, nb);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            double d = Dt[j][j];
            if (!(d > 0.0) || !isfinite(d)) {   // not positive definite: flag, keep going finitely
                set_status(status, KDCD_ERR_NOT_SPD);
                d = 1.0;
            }
            Dt[j][j] = sqrt(d);
        }
        __syncthreads();
        const double piv = Dt[j][j];
        for (int i = j + 1 + tid; i < nb; i += blockDim.x) Dt[j][i] /= piv;
        __syncthreads();
        const int wd = nb - j - 1;
        for (int e = tid; e < wd * wd; e += blockDim.x) {
            const int i = j + 1 + e / wd, k = j + 1 + e % wd;
            if (k <= i) Dt[k][i] -= Dt[j][i] * Dt[j][k];
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, k = e % nb;
        if (k <= i) Cw[(int64_t)(j0 + i) * ld + j0 + k] = Dt[k][i];
    }
    for (int c = w; c < PNB; c += blockDim.x / 64) {
        const double u = solve_row_wave(lane == c ? 1.0 : 0.0, Dt, lane);
        Dinv[lane * PNB + c] = u;
    }
}

__global__ __launch_bounds__(256) void check_rows_kernel(const int32_t *__restrict__ L, int64_t r,
                                                         int64_t m, int32_t *__restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < r && (L[i] < 0 || L[i] >= m)) set_status(status, KDCD_ERR_INDEX_RANGE);
}

// v[j] = Phi[S_j] . z, one wave per sampled row.
__global__ __launch_bounds__(256) void lr_rhs_kernel(const double *__restrict__ Phi, int64_t ldp,
                                                     int64_t m, int32_t r,
                                                     const int32_t *__restrict__ S, int32_t sb,
                                                     const double *__restrict__ z,
                                                     double *__restrict__ v)
{
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= sb) return;
    const double *row = Phi + clampi(S[j], 0, m - 1) * ldp;
    double s = 0.0;
    for (int c = lane; c < r; c += 64) s += row[c] * z[c];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) v[j] = s;
}

// z[c] += sum_t coef(S_t) theta_t Phi[S_t][c] in two passes: block (cb, q)
// sums the positions t of slice q for 64 columns into part[q][c] (the four
// waves take every fourth t and meet in LDS), then every column adds its
// ZU_SLICES partial sums in slice order.
constexpr int ZU_SLICES = 16;

__global__ __launch_bounds__(256) void lr_z_update_kernel(
    const double *__restrict__ Phi, int64_t ldp, int64_t m, int32_t r,
    const int32_t *__restrict__ S, int32_t sb, const double *__restrict__ theta,
    const double *__restrict__ coef, double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    const int64_t cc = col < r ? col : r - 1;
    const int chunk = (sb + ZU_SLICES - 1) / ZU_SLICES;
    const int t0 = blockIdx.y * chunk, t1 = min(sb, t0 + chunk);
    double s = 0.0;
    for (int t = t0 + w; t < t1; t += 4) {
        const int64_t p = clampi(S[t], 0, m - 1);
        const double d = coef ? coef[p] * theta[t] : theta[t];
        s += d * Phi[p * ldp + cc];
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && col < r)
        part[(int64_t)blockIdx.y * r + col] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void lr_z_add_kernel(const double *__restrict__ part, int32_t r,
                                                       double *__restrict__ z)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= r) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < ZU_SLICES; ++q) s += part[(int64_t)q * r + c];
    z[c] += s;
}

// Partial sums of z = Phi^T beta, beta_p = alpha_p (* coef_p): chunk rc of
// the rows into part[rc][c].
constexpr int ZCHUNKS = 128;

__global__ __launch_bounds__(256) void lr_z_init_kernel(const double *__restrict__ Phi,
                                                        int64_t ldp, int64_t m, int32_t r,
                                                        const double *__restrict__ alpha,
                                                        const double *__restrict__ coef,
                                                        double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    const int rc = blockIdx.y;
    const bool ok = col < r;
    double s = 0.0;
    for (int64_t p = (int64_t)rc * 4 + w; p < m; p += (int64_t)ZCHUNKS * 4) {
        const double bp = coef ? alpha[p] * coef[p] : alpha[p];
        if (ok && bp != 0.0) s += bp * Phi[p * ldp + col];
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && ok) part[(int64_t)rc * r + col] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void lr_z_reduce_kernel(const double *__restrict__ part,
                                                          int32_t r, double *__restrict__ z)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= r) return;
    double s = 0.0;
    for (int q = 0; q < ZCHUNKS; ++q) s += part[(int64_t)q * r + c];
    z[c] = s;
}

template <int EPI, int KIND>
hipError_t gemm_launch(const GemmArgs &g, int32_t tn, int64_t tiles, int32_t P, int64_t ksl,
                       double *part, hipStream_t st)
{
    gemm_nt_kernel<EPI, KIND><<<dim3((unsigned)tiles, (unsigned)P), 256, 0, st>>>(
        g, tn, tiles, ksl, P > 1 ? part : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || P == 1) return e;
    gemm_reduce_kernel<EPI, KIND><<<dim3((unsigned)tiles, GT * GT / 256), 256, 0, st>>>(g, tn, tiles, P,
                                                                                   part);
    return hipGetLastError();
}

// Tiles below about two workgroups per CU split K into slices of at least
// four chunks, as far as the partial-tile buffer (part_bytes) allows.
template <int EPI>
hipError_t gemm_dispatch(const GemmArgs &g, int kind, double *part, size_t part_bytes,
                         hipStream_t st)
{
    const int64_t tm = (g.M + GT - 1) / GT, tn = (g.N + GT - 1) / GT;
    const int64_t tiles = g.lower ? tm * (tm + 1) / 2 : tm * tn;
    if (tiles < 1 || g.K < 1) return hipSuccess;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    int64_t P = 1;
    if (part && tiles < 512) {
        P = std::min<int64_t>((512 + tiles - 1) / tiles, g.K / (4 * GK));
        P = std::min<int64_t>(P, (int64_t)(part_bytes / (sizeof(double) * GT * GT * tiles)));
        P = std::max<int64_t>(std::min<int64_t>(P, 64), 1);
    }
    int64_t ksl = (g.K + P - 1) / P;
    ksl = (ksl + GK - 1) / GK * GK;
    P = (g.K + ksl - 1) / ksl;
    if constexpr (EPI == EPI_KERNEL) {
        if (kind == KDCD_KERNEL_POLY)
            return gemm_launch<EPI, KDCD_KERNEL_POLY>(g, (int32_t)tn, tiles, (int32_t)P, ksl, part, st);
        if (kind == KDCD_KERNEL_RBF)
            return gemm_launch<EPI, KDCD_KERNEL_RBF>(g, (int32_t)tn, tiles, (int32_t)P, ksl, part, st);
    }
    return gemm_launch<EPI, KDCD_KERNEL_LINEAR>(g, (int32_t)tn, tiles, (int32_t)P, ksl, part, st);
}

}  // namespace

int32_t lowrank_zinit_chunks() { return ZCHUNKS; }
size_t lowrank_part_bytes() { return (size_t)32 << 20; }

// K(X, A_L) C^{-T} into Phi (rows of X; X == A when Xv == A->values and the
// row norms coincide).  Cw: r x r scratch; normsA / normsX: squared row norms
// (RBF only).  Errors go to status (INDEX_RANGE, NOT_SPD).
hipError_t launch_nystrom(const double *Av, int64_t lda, int64_t m, int64_t n, const int32_t *L,
                          int32_t r, const KParams &kp, double jitter, const double *normsA,
                          const double *Xv, int64_t ldx, int64_t mx, const double *normsX,
                          bool x_is_a, double *Cw, double *Dinv, double *Phi, int64_t ldp,
                          double *part, size_t part_bytes, int32_t *status, hipStream_t st)
{
    check_rows_kernel<<<(unsigned)((r + 255) / 256), 256, 0, st>>>(L, r, m, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    GemmArgs g{};
    g.A = Av; g.lda = lda; g.ra = L; g.rowsA = m;
    g.B = Av; g.ldb = lda; g.rb = L; g.rowsB = m;
    g.M = r; g.N = r; g.K = n;
    g.out = Cw; g.ldo = r;
    g.kp = kp; g.na = normsA; g.nb = normsA; g.same = 1; g.diag_add = jitter;
    if ((e = gemm_dispatch<EPI_KERNEL>(g, kp.kind, part, part_bytes, st)) != hipSuccess) return e;

    // Cholesky: C C^T = K_LL + jitter I, lower triangle of Cw; panel p's
    // diagonal block inverse goes to Dinv + p * 4096
    for (int32_t j0 = 0; j0 < r; j0 += PNB) {
        const int32_t nb = std::min(PNB, r - j0);
        double *Di = Dinv + (int64_t)(j0 / PNB) * PNB * PNB;
        chol_panel_kernel<<<1, 1024, 0, st>>>(Cw, r, r, j0, Di, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int32_t rest = r - j0 - nb;
        if (rest <= 0) break;
        // rows below the block: L_21 = A_21 D^{-T}, in place (one workgroup per row tile)
        GemmArgs q{};
        q.A = Cw + (int64_t)(j0 + nb) * r + j0; q.lda = r; q.rowsA = rest;
        q.B = Di; q.ldb = PNB; q.rowsB = nb;
        q.M = rest; q.N = nb; q.K = nb;
        q.out = Cw + (int64_t)(j0 + nb) * r + j0; q.ldo = r;
        if ((e = gemm_dispatch<EPI_STORE>(q, 0, nullptr, 0, st)) != hipSuccess) return e;
        GemmArgs u{};
        u.A = q.A; u.lda = r; u.rowsA = rest;
        u.B = q.A; u.ldb = r; u.rowsB = rest;
        u.M = rest; u.N = rest; u.K = nb;
        u.out = Cw + (int64_t)(j0 + nb) * r + j0 + nb; u.ldo = r;
        u.lower = 1;
        if ((e = gemm_dispatch<EPI_SUB>(u, 0, part, part_bytes, st)) != hipSuccess) return e;
    }

    // Phi = K(X, A_L), then Phi C^T = K(X, A_L) by panels
    GemmArgs x{};
    x.A = Xv; x.lda = ldx; x.rowsA = mx;
    x.B = Av; x.ldb = lda; x.rb = L; x.rowsB = m;
    x.M = mx; x.N = r; x.K = n;
    x.out = Phi; x.ldo = ldp;
    x.kp = kp; x.na = normsX; x.nb = normsA; x.same = x_is_a ? 1 : 0; x.diag_add = 0.0;
    if ((e = gemm_dispatch<EPI_KERNEL>(x, kp.kind, part, part_bytes, st)) != hipSuccess) return e;
    for (int32_t j0 = 0; j0 < r; j0 += PNB) {
        const int32_t nb = std::min(PNB, r - j0);
        if (j0 > 0) {
            GemmArgs u{};
            u.A = Phi; u.lda = ldp; u.rowsA = mx;
            u.B = Cw + (int64_t)j0 * r; u.ldb = r; u.rowsB = nb;
            u.M = mx; u.N = nb; u.K = j0;
            u.out = Phi + j0; u.ldo = ldp;
            if ((e = gemm_dispatch<EPI_SUB>(u, 0, part, part_bytes, st)) != hipSuccess) return e;
        }
        GemmArgs q{};
        q.A = Phi + j0; q.lda = ldp; q.rowsA = mx;
        q.B = Dinv + (int64_t)(j0 / PNB) * PNB * PNB; q.ldb = PNB; q.rowsB = nb;
        q.M = mx; q.N = nb; q.K = nb;
        q.out = Phi + j0; q.ldo = ldp;
        if ((e = gemm_dispatch<EPI_STORE>(q, 0, nullptr, 0, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// G = Phi_S Phi_S^T (sb x sb, full, symmetric) and v = Phi_S z.
hipError_t launch_lowrank_block(const double *Phi, int64_t ldp, int64_t m, int32_t r,
                                const int32_t *S, int32_t sb, const double *z, double *W,
                                double *v, double *part, size_t part_bytes, hipStream_t st)
{
    GemmArgs g{};
    g.A = Phi; g.lda = ldp; g.ra = S; g.rowsA = m;
    g.B = Phi; g.ldb = ldp; g.rb = S; g.rowsB = m;
    g.M = sb; g.N = sb; g.K = r;
    g.out = W; g.ldo = sb;
    g.lower = 1; g.mirror = 1;
    hipError_t e = gemm_dispatch<EPI_STORE>(g, 0, part, part_bytes, st);
    if (e != hipSuccess) return e;
    lr_rhs_kernel<<<(unsigned)((sb + 3) / 4), 256, 0, st>>>(Phi, ldp, m, r, S, sb, z, v);
    return hipGetLastError();
}

// part: at least ZU_SLICES x r scratch
hipError_t launch_lowrank_z_update(const double *Phi, int64_t ldp, int64_t m, int32_t r,
                                   const int32_t *S, int32_t sb, const double *theta,
                                   const double *coef, double *part, double *z, hipStream_t st)
{
    lr_z_update_kernel<<<dim3((unsigned)((r + 63) / 64), ZU_SLICES), 256, 0, st>>>(
        Phi, ldp, m, r, S, sb, theta, coef, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    lr_z_add_kernel<<<(unsigned)((r + 255) / 256), 256, 0, st>>>(part, r, z);
    return hipGetLastError();
}

// part: ZCHUNKS x r scratch
hipError_t launch_lowrank_z_init(const double *Phi, int64_t ldp, int64_t m, int32_t r,
                                 const double *alpha, const double *coef, double *part, double *z,
                                 hipStream_t st)
{
    lr_z_init_kernel<<<dim3((unsigned)((r + 63) / 64), ZCHUNKS), 256, 0, st>>>(Phi, ldp, m, r,
                                                                             alpha, coef, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    lr_z_reduce_kernel<<<(unsigned)((r + 255) / 256), 256, 0, st>>>(part, r, z);
    return hipGetLastError();
}

}  // namespace kdcd
