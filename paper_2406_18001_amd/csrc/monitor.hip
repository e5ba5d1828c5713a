// On-device upkeep of the dual gradient and the convergence monitor.
//
// The kernel block U_k = K(A, A_S) of an outer iteration, stored column-major
// in the sample index, updates a maintained m-vector after the recurrence:
//   K-SVM  g   = Q alpha - 1 + omega alpha:  g_i   += y_i sum_t U[t][i] y_{S_t} theta_t
//                                                     + omega (sum of theta_t with S_t = i)
//   K-RR   rho = y - M alpha (M = K/lambda + m I):
//                                          rho_i -= (1/lambda) sum_t U[t][i] Delta_t
//                                                     + m (sum of Delta_t with S_t = i)
// From it the monitor evaluates, in O(m), a certified bound on the relative
// objective error (Sec. 3.1 and 3.3 objectives):
//   K-RR   f = 1/2 a^T M a - y^T a = -1/2 a^T (y + rho);  f - f* <= ||rho||^2 / (2m)
//          (the smallest eigenvalue of M is at least m); rel = bound / (|f| - bound)
//   K-SVM  f = 1/2 a^T g - 1/2 sum a;  (Q a)_i = g_i + 1 - omega a_i;
//          P = 1/2 a^T Q a + C sum max(0, 1 - (Q a)_i) (squared for the squared
//          hinge); f - f* <= P + f (the duality gap); rel = gap / |f|
// and sets the stop word once rel <= tol; every later kernel of the solve then
// returns at once.  All sums run in a fixed order (deterministic).
#include "common.hpp"

namespace kdcd {
namespace {

constexpr int MON_BLOCKS = 256;
constexpr int MON_NT = 256;

__global__ __launch_bounds__(256) void dual_update_kernel(
    const double *__restrict__ U, int64_t m, int32_t sb, const int32_t *__restrict__ S,
    const double *__restrict__ theta, const double *__restrict__ vscale, double uscale,
    const double *__restrict__ wscale, double diag, double *__restrict__ v,
    const int32_t *__restrict__ stop)
{
    __shared__ double w[kMaxSB], th[kMaxSB];
    __shared__ int32_t Sl[kMaxSB];
    if (stop && *stop) return;
    for (int t = threadIdx.x; t < sb; t += blockDim.x) {
        const int32_t j = S[t];
        Sl[t] = j;
        th[t] = theta[t];
        w[t] = (wscale ? wscale[j] : 1.0) * theta[t];
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0, da = 0.0;
        for (int t = 0; t < sb; ++t) {
            acc = fma(U[(int64_t)t * m + i], w[t], acc);
            if (Sl[t] == (int32_t)i) da += th[t];
        }
        v[i] += (vscale ? vscale[i] : 1.0) * uscale * acc + diag * da;
    }
}

// The batched form: one pass over U updates up to DB_MAX problems of a sigma
// group (their weights w_p = wscale_p * theta_p and updates theta_p staged in
// LDS); problems [p0, p0 + n) of the descriptor.
constexpr int DB_MAX = 8;
__global__ __launch_bounds__(256) void dual_update_batch_kernel(
    const double *__restrict__ U, int64_t m, int32_t sb, const int32_t *__restrict__ S,
    const DualBatchDesc d, int32_t p0, int32_t n, const int32_t *__restrict__ stop)
{
    extern __shared__ double dsh[];              // w [n][sb], th [n][sb], then S
    if (stop && *stop) return;
    double *w = dsh, *th = dsh + (size_t)n * sb;
    int32_t *Sl = reinterpret_cast<int32_t *>(th + (size_t)n * sb);
    for (int t = threadIdx.x; t < sb; t += blockDim.x) Sl[t] = S[t];
    for (int x = threadIdx.x; x < n * sb; x += blockDim.x) {
        const int q = x / sb, t = x - q * sb;
        const double tv = d.theta[p0 + q][t];
        th[x] = tv;
        w[x] = (d.wscale[p0 + q] ? d.wscale[p0 + q][S[t]] : 1.0) * tv;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc[DB_MAX], da[DB_MAX];
#pragma unroll
        for (int q = 0; q < DB_MAX; ++q) acc[q] = da[q] = 0.0;
        for (int t = 0; t < sb; ++t) {
            const double u = U[(int64_t)t * m + i];
            const bool hit = Sl[t] == (int32_t)i;
#pragma unroll
            for (int q = 0; q < DB_MAX; ++q) {
                if (q < n) {
                    acc[q] = fma(u, w[q * sb + t], acc[q]);
                    if (hit) da[q] += th[q * sb + t];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < DB_MAX; ++q) {
            if (q >= n) break;
            const int p = p0 + q;
            d.v[p][i] += (d.vscale[p] ? d.vscale[p][i] : 1.0) * d.uscale[p] * acc[q] + d.diag[p] * da[q];
        }
    }
}

// Block tree reduction of NV values per thread into out[blockIdx.x * NV + q].
template <int NV>
__device__ __forceinline__ void block_sums(double (&x)[NV], double *out)
{
    __shared__ double red[NV][MON_NT];
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = x[q];
    __syncthreads();
    for (int h = MON_NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) out[blockIdx.x * NV + q] = red[q][0];
}

// problem 0: K-SVM (v = g), 1: K-RR (v = rho).  Four sums per block.
__global__ __launch_bounds__(MON_NT) void monitor_partial_kernel(
    int32_t problem, int64_t m, const double *__restrict__ alpha, const double *__restrict__ y,
    const double *__restrict__ v, double omega, int32_t loss, double *__restrict__ part,
    const int32_t *__restrict__ stop)
{
    if (stop && *stop) return;
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = alpha[i], vi = v[i];
        if (problem == 1) {
            x[0] += vi * vi;
            x[1] += a * (y[i] + vi);
        } else {
            const double qa = vi + 1.0 - omega * a;   // (Q alpha)_i
            const double xi = fmax(0.0, 1.0 - qa);
            x[0] += a * vi;
            x[1] += a;
            x[2] += a * qa;
            x[3] += loss == 2 ? xi * xi : xi;
        }
    }
    block_sums<4>(x, part);
}

__global__ __launch_bounds__(64) void monitor_final_kernel(int32_t problem, int64_t m, double C,
                                                           double tol, int64_t outer,
                                                           const double *__restrict__ part,
                                                           MonitorState *__restrict__ mon)
{
    if (threadIdx.x != 0 || mon->stop) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < MON_BLOCKS; ++b)
        for (int q = 0; q < 4; ++q) s[q] += part[b * 4 + q];
    double f, rel;
    if (problem == 1) {
        f = -0.5 * s[1];
        const double bound = 0.5 * s[0] / (double)m;
        const double den = fabs(f) - bound;
        rel = den > 0.0 ? bound / den : INFINITY;
    } else {
        f = 0.5 * s[0] - 0.5 * s[1];
        const double P = 0.5 * s[2] + C * s[3];
        const double gap = P + f;
        rel = fabs(f) > 0.0 ? gap / fabs(f) : INFINITY;
    }
    mon->rel = rel;
    mon->f = f;
    mon->outer_done = outer;
    const int64_t i = mon->nlog;
    if (mon->log && i < mon->log_len) {
        double *r = mon->log + 4 * i;
        r[0] = (double)outer;
        r[1] = rel;
        r[2] = f;
        r[3] = (double)(wall_clock64() - mon->t0) * mon->tick;
    }
    mon->nlog = i + 1;
    if (rel <= tol) mon->stop = 1;
}

__global__ __launch_bounds__(64) void monitor_combine_kernel(const MonitorState *__restrict__ mons,
                                                             int32_t n, double tol, int64_t outer,
                                                             MonitorState *__restrict__ mon)
{
    if (threadIdx.x != 0 || mon->stop) return;
    double rel = 0.0, f = 0.0;
    for (int p = 0; p < n; ++p) {
        const double r = mons[p].rel;
        if (!(r <= rel)) rel = r;          // NaN propagates
        f += mons[p].f;
    }
    mon->rel = rel;
    mon->f = f;
    mon->outer_done = outer;
    const int64_t i = mon->nlog;
    if (mon->log && i < mon->log_len) {
        double *r = mon->log + 4 * i;
        r[0] = (double)outer;
        r[1] = rel;
        r[2] = f;
        r[3] = (double)(wall_clock64() - mon->t0) * mon->tick;
    }
    mon->nlog = i + 1;
    if (rel <= tol) mon->stop = 1;
}

__global__ void monitor_start_kernel(MonitorState *mon, double *log, int64_t log_len, double tick)
{
    if (threadIdx.x != 0) return;
    mon->log = log;
    mon->log_len = log ? log_len : 0;
    mon->tick = tick;
    mon->t0 = wall_clock64();
}

// rho = y - Ka / lambda - m a   (Ka = K alpha_0, null when alpha_0 = 0)
__global__ __launch_bounds__(256) void rho_init_kernel(const double *__restrict__ Ka,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ alpha,
                                                       double inv_lambda, double mdbl, int64_t m,
                                                       double *__restrict__ rho)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        rho[i] = y[i] - (Ka ? Ka[i] * inv_lambda : 0.0) - mdbl * alpha[i];
}

unsigned grid_of(int64_t m, int64_t cap)
{
    int64_t b = (m + 255) / 256;
    if (b < 1) b = 1;
    return (unsigned)(b < cap ? b : cap);
}

}  // namespace

hipError_t launch_dual_update(const double *U, int64_t m, int32_t sb, const int32_t *S,
                              const double *theta, const double *vscale, double uscale,
                              const double *wscale, double diag, double *v, const int32_t *stop,
                              hipStream_t st)
{
    hipLaunchKernelGGL(dual_update_kernel, dim3(grid_of(m, 4096)), dim3(256), 0, st, U, m, sb, S,
                       theta, vscale, uscale, wscale, diag, v, stop);
    return hipGetLastError();
}

size_t monitor_partial_bytes() { return sizeof(double) * 4 * MON_BLOCKS; }

hipError_t launch_dual_update_batch(const double *U, int64_t m, int32_t sb, const int32_t *S,
                                    const DualBatchDesc &d, const int32_t *stop, hipStream_t st)
{
    if (d.n < 1 || d.n > kMaxProblems || sb < 1 || sb > kMaxSB) return hipErrorInvalidValue;
    // problems per launch: at most DB_MAX, and their staged values within 64 KiB
    const int fit = (int)((65536 - sizeof(int32_t) * (size_t)sb) / (2 * sizeof(double) * (size_t)sb));
    const int per = std::max(1, std::min(DB_MAX, fit));
    const int64_t blocks = std::min<int64_t>((m + 255) / 256, 2048);
    for (int p0 = 0; p0 < d.n; p0 += per) {
        const int n = std::min(per, d.n - p0);
        const size_t shm = sizeof(double) * 2 * (size_t)n * sb + sizeof(int32_t) * (size_t)sb;
        hipLaunchKernelGGL(dual_update_batch_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)),
                           dim3(256), shm, st, U, m, sb, S, d, p0, n, stop);
    }
    return hipGetLastError();
}

hipError_t launch_monitor_combine(const MonitorState *mons, int32_t n, double tol, int64_t outer,
                                  MonitorState *batch, hipStream_t st)
{
    hipLaunchKernelGGL(monitor_combine_kernel, dim3(1), dim3(64), 0, st, mons, n, tol, outer, batch);
    return hipGetLastError();
}

hipError_t launch_monitor_start(MonitorState *mon, double *log, int64_t log_len, hipStream_t st)
{
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    const double tick = khz > 0 ? 1e-3 / (double)khz : 0.0;
    hipLaunchKernelGGL(monitor_start_kernel, dim3(1), dim3(64), 0, st, mon, log, log_len, tick);
    return hipGetLastError();
}

hipError_t launch_monitor(int32_t problem, int64_t m, const double *alpha, const double *y,
                          const double *v, double omega, int32_t loss, double C, double tol,
                          int64_t outer, double *part, MonitorState *mon, hipStream_t st)
{
    hipLaunchKernelGGL(monitor_partial_kernel, dim3(MON_BLOCKS), dim3(MON_NT), 0, st, problem, m,
                       alpha, y, v, omega, loss, part, &mon->stop);
    hipLaunchKernelGGL(monitor_final_kernel, dim3(1), dim3(64), 0, st, problem, m, C, tol, outer,
                       part, mon);
    return hipGetLastError();
}

hipError_t launch_rho_init(const double *Ka, const double *y, const double *alpha,
                           double inv_lambda, double mdbl, int64_t m, double *rho, hipStream_t st)
{
    hipLaunchKernelGGL(rho_init_kernel, dim3(grid_of(m, 2048)), dim3(256), 0, st, Ka, y, alpha,
                       inv_lambda, mdbl, m, rho);
    return hipGetLastError();
}

}  // namespace kdcd
