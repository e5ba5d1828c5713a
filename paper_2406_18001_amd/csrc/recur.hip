// The s-step inner recurrences, one workgroup per outer iteration, FP64.
//
// K-SVM (Algorithm 2, b = 1).  Thread j owns inner step j of the block:
//   rho_j = alpha_{i_j} + sum_{t<j, i_t = i_j} theta_t
//   g_j   = y_{i_j} r_j - 1 + sum_{t<j} Q_{i_t i_j} theta_t + omega rho_j
//   theta_j from the projected coordinate step with eta_j = Q_{i_j i_j} + omega.
// The sum over t < j is accumulated right-looking.  Steps are processed in
// panels of 64: the wave that owns a panel runs its 64 steps wave-
// synchronously (theta broadcast with readlane, the panel's diagonal 64 x 64
// block of W staged in LDS by the other waves while the previous panel ran),
// then one barrier, then every later thread folds the panel's 64 thetas into
// its accumulators.
//
// K-RR (Algorithm 4 / Eq. (3)).  Thread p owns element p of the sb sampled
// coordinates (block p / b).  With c_p = y_{S_p} - m alpha_{S_p} - r_p/lambda,
// block j solves Delta_j = G_j^{-1} c_j (G_j^{-1} precomputed by the finish
// pass), then every later element subtracts (m [S_p = S_q] + W_qp/lambda)
// Delta_q for q in block j -- one block Gauss-Seidel sweep over the sampled
// system, as the unrolled recurrence prescribes.
//
// Both scatter alpha_{S_t} += update in t order: the last occurrence of each
// coordinate writes alpha_0 + (its running sum), so duplicates accumulate.
#include "common.hpp"

namespace kdcd {
namespace {

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The projected coordinate step of Algorithms 1-2: theta = clip(rho - g/eta, 0, nu) - rho when
// the projected gradient |clip(rho - g, 0, nu) - rho| is non-zero and eta > 0, else 0.
// inv_eta = 1/eta is precomputed (0 when eta <= 0); the selection is branch-free.
__device__ __forceinline__ double dcd_theta(double rho, double g, double inv_eta, double nu)
{
    const double gt = fmin(fmax(rho - g, 0.0), nu) - rho;
    const double th = fmin(fmax(rho - g * inv_eta, 0.0), nu) - rho;
    return (gt != 0.0 && inv_eta > 0.0) ? th : 0.0;
}

// Last-occurrence table of the index block: an open-addressing hash in LDS
// (2 * kMaxSB slots for at most kMaxSB keys, so every probe sequence ends at
// an empty slot).  Each element inserts its coordinate and keeps the largest
// element index per coordinate; after a barrier an element is the last
// occurrence of its coordinate iff the slot holds its own index.
constexpr int kHashSlots = 2 * kMaxSB;

__device__ __forceinline__ void lastocc_clear(int32_t *keys, int32_t *idxs, int tid, int nt)
{
    for (int x = tid; x < kHashSlots; x += nt) {
        keys[x] = -1;
        idxs[x] = -1;
    }
}

__device__ __forceinline__ int lastocc_insert(int32_t *keys, int32_t *idxs, int32_t key, int e)
{
    uint32_t h = ((uint32_t)key * 2654435761u) & (kHashSlots - 1);
    for (;;) {
        const int32_t old = atomicCAS(&keys[h], -1, key);
        if (old == -1 || old == key) break;
        h = (h + 1) & (kHashSlots - 1);
    }
    atomicMax(&idxs[h], e);
    return (int)h;
}

// Stage the 64 x 64 diagonal block of panel q of W into dst (zero outside
// the sb x sb matrix), using threads rank in [0, count): loads are issued in
// batches of 8 before the matching LDS stores.
__device__ __forceinline__ void stage_diag(const double *__restrict__ W, int32_t sb, int q,
                                           double *dst, int rank, int count)
{
    const int Q0 = q * 64;
    constexpr int CH = 8;
    for (int e0 = rank; e0 < 64 * 64; e0 += CH * count) {
        double v[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int e = e0 + c * count;
            const int t = e >> 6, u = e & 63;
            v[c] = (e < 64 * 64 && Q0 + t < sb && Q0 + u < sb) ? W[(int64_t)(Q0 + t) * sb + Q0 + u]
                                                              : 0.0;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int e = e0 + c * count;
            if (e < 64 * 64) dst[e] = v[c];
        }
    }
}

// K-SVM recurrence.  NT threads (512 covers sb <= 512, 1024 covers sb <= 1024);
// PF = W values of the next fold-in phase prefetched into registers.
template <int NT>
__global__ __launch_bounds__(NT) void ksvm_recur_kernel(const KsvmRecurDesc D,
                                                        const int32_t *__restrict__ S, int32_t sb,
                                                        int64_t m, int32_t *status)
{
    if (D.stop && *D.stop) return;             // converged: nothing more to do
    // problem of this workgroup (one workgroup per problem of a batch)
    const int pb = blockIdx.x;
    const double *__restrict__ r = D.r[pb];
    const double *__restrict__ W = D.W[pb];
    const double *__restrict__ y = D.y[pb];
    double *__restrict__ alpha = D.alpha[pb];
    double *__restrict__ trace = D.trace[pb];
    const double nu = D.nu[pb], omega = D.omega[pb];
    constexpr int PF = NT <= 512 ? 64 : 32;
    __shared__ double Wd[2][64 * 64];
    __shared__ double th_l[kMaxSB + 64];       // padded: entries >= sb hold 0 / -1
    __shared__ double y_l[kMaxSB + 64];
    __shared__ __align__(16) int32_t S_l[kMaxSB + 64];
    __shared__ int32_t hkeys[kHashSlots], hidx[kHashSlots];
    const int j = threadIdx.x, lane = j & 63, wid = j >> 6;
    const bool act = j < sb;
    const int64_t Sj = act ? clampi(S[j], 0, m - 1) : -1;
    const double yj = act ? y[Sj] : 0.0;
    double rho = act ? alpha[Sj] : 0.0;
    const double g0 = act ? yj * r[j] - 1.0 : 0.0;
    const double eta = act ? W[(int64_t)j * sb + j] + omega : 1.0;
    const double inv_eta = eta > 0.0 ? 1.0 / eta : 0.0;
    double gacc = 0.0, theta = 0.0;
    S_l[j] = (int32_t)Sj;
    y_l[j] = yj;
    th_l[j] = 0.0;
    if (j < 64) { S_l[NT + j] = -1; y_l[NT + j] = 0.0; th_l[NT + j] = 0.0; }
    lastocc_clear(hkeys, hidx, j, NT);
    stage_diag(W, sb, 0, Wd[0], j, NT);
    lds_barrier();
    const int hslot = act ? lastocc_insert(hkeys, hidx, (int32_t)Sj, j) : 0;

    const int npanels = (sb + 63) / 64;
    for (int p = 0; p < npanels; ++p) {
        const int P0 = p * 64;
        const int plen = (sb - P0) < 64 ? (sb - P0) : 64;
        const int buf = p & 1;
        const bool later = act && wid > p;
        double wpre[PF];
        if (later) {
#pragma unroll
            for (int t = 0; t < PF; ++t) wpre[t] = (t < plen) ? W[(int64_t)(P0 + t) * sb + j] : 0.0;
        }
        if (wid != p && p + 1 < npanels)   // the other waves stage the next diagonal block
            stage_diag(W, sb, p + 1, Wd[buf ^ 1], wid < p ? j : j - 64, NT - 64);
        if (wid == p) {
            const double *wd = Wd[buf];
#pragma unroll
            for (int t = 0; t < 64; ++t) {
                if (t < plen) {
                    // everything but theta_t is independent of the chain and can be issued early
                    const double coef = (lane > t) ? readlane_d(yj, t) * yj * wd[t * 64 + lane] : 0.0;
                    const bool dup = (lane > t) && __builtin_amdgcn_readlane((int)Sj, t) == (int32_t)Sj;
                    const double g = g0 + gacc + omega * rho;
                    const double th = dcd_theta(rho, g, inv_eta, nu);
                    const double tt = readlane_d(th, t);
                    if (lane == t) theta = th;
                    gacc += coef * tt;
                    rho += dup ? tt : 0.0;
                }
            }
            th_l[j] = theta;
        }
        lds_barrier();
        if (later) {
            // branch-free: wpre[t] and th_l[P0 + t] are 0 past the end of S_k
#pragma unroll
            for (int t = 0; t < PF; ++t) {
                const double tt = th_l[P0 + t];
                gacc += y_l[P0 + t] * yj * wpre[t] * tt;
                rho += (S_l[P0 + t] == (int32_t)Sj) ? tt : 0.0;
            }
            for (int t = PF; t < plen; ++t) {
                const double tt = th_l[P0 + t];
                gacc += y_l[P0 + t] * yj * W[(int64_t)(P0 + t) * sb + j] * tt;
                if (S_l[P0 + t] == (int32_t)Sj) rho += tt;
            }
        }
    }
    const bool last = act && hidx[hslot] == j;
    if (act) {
        const double nv = rho + theta;
        if (!isfinite(nv)) set_status(status, KDCD_ERR_NONFINITE);
        if (last) alpha[Sj] = nv;
        if (trace) trace[j] = theta;
    }
}

// K-RR recurrence.  Elements are grouped in panels of PE = floor(64/b)*b
// (whole blocks); panel q lives on lanes [0, PE) of wave q.  Inside a panel
// the wave runs its blocks one after the other (values exchanged between
// lanes with readlane, no workgroup barrier); then one barrier and every
// later element folds in the panel's Delta values.  BMAX bounds b, NT the
// thread count; BX > 0 fixes b = BX at compile time (fully unrolled block
// loops), BX = 0 handles any b <= BMAX.
template <int BMAX, int NT, int BX>
__global__ __launch_bounds__(NT) void krr_recur_kernel(const KrrRecurDesc D,
                                                       const int32_t *__restrict__ S, int32_t b,
                                                       int32_t sk, int64_t m, double mdbl,
                                                       int32_t *status)
{
    if (D.stop && *D.stop) return;             // converged: nothing more to do
    // problem of this workgroup (one workgroup per problem of a batch)
    const int pb = blockIdx.x;
    const double *__restrict__ r = D.r[pb];
    const double *__restrict__ W = D.W[pb];
    const double *__restrict__ Dinv = D.Dinv[pb];
    const double *__restrict__ y = D.y[pb];
    double *__restrict__ alpha = D.alpha[pb];
    double *__restrict__ trace = D.trace[pb];
    const double lambda = D.lambda[pb];
    constexpr int PF = NT > 512 ? 16 : ((BMAX >= 32 || BX == 0) ? 32 : 64);
    __shared__ double Wd[2][64 * 64];
    __shared__ double c_l[kMaxSB + 64];        // padded: entries past the last panel hold 0 / -1
    __shared__ double d_l[kMaxSB + 64];
    __shared__ __align__(16) int32_t S_l[kMaxSB + 64];
    __shared__ int32_t hkeys[kHashSlots], hidx[kHashSlots];
    if (BX > 0) b = BX;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int sb = sk * b;
    const int PE = (64 / b) * b;
    const int npanels = (sb + PE - 1) / PE;
    const int e = wid * PE + lane;                    // element owned by this thread
    const bool act = lane < PE && e < sb;
    const int64_t Sp = act ? clampi(S[e], 0, m - 1) : -1;
    const double a0 = act ? alpha[Sp] : 0.0;
    const double inv_lambda = 1.0 / lambda;
    double c = act ? y[Sp] - mdbl * a0 - r[e] / lambda : 0.0;
    const int myblk = act ? e / b : sk;
    const int ll = act ? e % b : 0;
    const int lblk = lane / b;                        // block index inside the panel
    for (int x = tid; x < kMaxSB + 64; x += NT) {   // every slot without an owner: S = -1, d = 0
        S_l[x] = -1;
        d_l[x] = 0.0;
    }
    lastocc_clear(hkeys, hidx, tid, NT);
    lds_barrier();
    if (act) {
        S_l[e] = (int32_t)Sp;
        c_l[e] = c;
    }
    double dv[BMAX];
#pragma unroll
    for (int q = 0; q < BMAX; ++q)
        dv[q] = (act && q < b) ? Dinv[((int64_t)myblk * b + ll) * b + q] : 0.0;

    // diagonal PE x PE block of panel q, stored with row stride 64
    auto stage = [&](int q, double *dst, int rank, int count) {
        const int Q0 = q * PE;
        constexpr int CH = 8;
        for (int e0 = rank; e0 < 64 * 64; e0 += CH * count) {
            double v[CH];
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int x = e0 + cc * count, t = x >> 6, u = x & 63;
                v[cc] = (x < 64 * 64 && t < PE && u < PE && Q0 + t < sb && Q0 + u < sb)
                            ? W[(int64_t)(Q0 + t) * sb + Q0 + u] : 0.0;
            }
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int x = e0 + cc * count;
                if (x < 64 * 64) dst[x] = v[cc];
            }
        }
    };
    stage(0, Wd[0], tid, NT);
    lds_barrier();
    const int hslot = act ? lastocc_insert(hkeys, hidx, (int32_t)Sp, e) : 0;
    if (act) {
        const int q0 = myblk * b;
        for (int q = q0; q < q0 + b; ++q)
            if (q != e && S_l[q] == (int32_t)Sp) set_status(status, KDCD_ERR_INDEX_DUPLICATE);
    }

    double delta = 0.0, dsum = 0.0;   // dsum: updates of earlier repeats of this coordinate, in order
    for (int p = 0; p < npanels; ++p) {
        const int P0 = p * PE;
        const int plen = (sb - P0) < PE ? (sb - P0) : PE;
        const int buf = p & 1;
        const bool later = act && wid > p;
        double wpre[PF];
        if (later) {
#pragma unroll
            for (int t = 0; t < PF; ++t) wpre[t] = (t < plen) ? W[(int64_t)(P0 + t) * sb + e] : 0.0;
        }
        if (wid != p && p + 1 < npanels) stage(p + 1, Wd[buf ^ 1], wid < p ? tid : tid - 64, NT - 64);
        if (wid == p) {
            const double *wd = Wd[buf];
            const int nbl = plen / b;
            constexpr int QN = BX > 0 ? BX : BMAX;
            for (int bl = 0; bl < nbl; ++bl) {
                const int l0 = bl * b;                 // first lane of block bl
                // coefficients of the fold-in, independent of the chain: fetched first
                double coef[QN];
#pragma unroll
                for (int q = 0; q < QN; ++q) {
                    if (BX > 0 || q < b) {
                        const int32_t Sq = __builtin_amdgcn_readlane((int)Sp, l0 + q);
                        coef[q] = (Sq == (int32_t)Sp ? mdbl : 0.0) + wd[(l0 + q) * 64 + lane] * inv_lambda;
                    }
                }
                // Delta for block bl: lanes of the block combine the block's c values
                double dl = 0.0;
#pragma unroll
                for (int q = 0; q < QN; ++q)
                    if (BX > 0 || q < b) dl += dv[q] * readlane_d(c, l0 + q);
                if (lblk == bl) delta = dl;
                // every later lane of the panel subtracts (m [S_e = S_q] + W_qe / lambda) Delta_q
                double acc = 0.0, dup_acc = 0.0;
                bool any_dup = false;
#pragma unroll
                for (int q = 0; q < QN; ++q) {
                    if (BX > 0 || q < b) {
                        const double dq = readlane_d(dl, l0 + q);
                        const bool dup = __builtin_amdgcn_readlane((int)Sp, l0 + q) == (int32_t)Sp;
                        acc += coef[q] * dq;
                        dup_acc += dup ? dq : 0.0;
                        any_dup |= dup;
                    }
                }
                if (act && lblk > bl) {
                    c -= acc;
                    if (any_dup) dsum += dup_acc;
                }
            }
            if (act) d_l[e] = delta;
        }
        lds_barrier();
        if (later) {
            // branch-free: wpre[t] and d_l[P0 + t] are 0 past the end of the panel
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < PF; ++t) {
                const bool dup = S_l[P0 + t] == (int32_t)Sp;
                const double dt = d_l[P0 + t];
                acc += ((dup ? mdbl : 0.0) + wpre[t] * inv_lambda) * dt;
                dsum += dup ? dt : 0.0;
            }
            for (int t = PF; t < plen; ++t) {
                const bool dup = S_l[P0 + t] == (int32_t)Sp;
                const double dt = d_l[P0 + t];
                acc += ((dup ? mdbl : 0.0) + W[(int64_t)(P0 + t) * sb + e] * inv_lambda) * dt;
                if (dup) dsum += dt;
            }
            c -= acc;
            c_l[e] = c;
        }
    }
    // scatter: the last occurrence of a coordinate writes alpha_0 plus all of
    // its updates (earlier repeats were folded into dsum in order)
    const bool last = act && hidx[hslot] == e;
    const double v = a0 + (dsum + delta);
    if (act) {
        if (last) {
            if (!isfinite(v)) set_status(status, KDCD_ERR_NONFINITE);
            alpha[Sp] = v;
        }
        if (trace) trace[e] = delta;
    }
}

}  // namespace

// Threads of a K-RR recurrence launch: one wave per panel of floor(64/b)*b elements.
int krr_recur_threads(int32_t b, int32_t sk)
{
    const int PE = (64 / b) * b;
    const int waves = (sk * b + PE - 1) / PE;
    return waves * 64;
}

hipError_t launch_ksvm_recur(const KsvmRecurDesc &d, int32_t nprob, const int32_t *S, int32_t sb,
                             int64_t m, int32_t *status, hipStream_t st)
{
    if (sb <= 512)
        KDCD_TIMED_LAUNCH((ksvm_recur_kernel<512>), dim3(nprob), dim3(512), 0, st, d, S, sb, m,
                          status);
    else
        KDCD_TIMED_LAUNCH((ksvm_recur_kernel<1024>), dim3(nprob), dim3(1024), 0, st, d, S, sb, m,
                          status);
    return hipGetLastError();
}

hipError_t launch_krr_recur(const KrrRecurDesc &d, int32_t nprob, const int32_t *S, int32_t b,
                            int32_t sk, int64_t m, double mdbl, int32_t *status, hipStream_t st)
{
    const int nt = krr_recur_threads(b, sk);
    if (nt > 1024 || b > kMaxB) return hipErrorInvalidValue;
#define KDCD_KRR(BM_, NT_, BX_)                                                                 \
    KDCD_TIMED_LAUNCH((krr_recur_kernel<BM_, NT_, BX_>), dim3(nprob), dim3(NT_), 0, st, d, S, b, \
                      sk, m, mdbl, status)
    if (nt <= 512) {
        switch (b) {
        case 1: KDCD_KRR(1, 512, 1); break;
        case 2: KDCD_KRR(2, 512, 2); break;
        case 4: KDCD_KRR(4, 512, 4); break;
        case 8: KDCD_KRR(8, 512, 8); break;
        case 16: KDCD_KRR(16, 512, 16); break;
        case 32: KDCD_KRR(32, 512, 32); break;
        default:
            if (b <= 8) KDCD_KRR(8, 512, 0);
            else if (b <= 16) KDCD_KRR(16, 512, 0);
            else KDCD_KRR(32, 512, 0);
        }
    } else {
        switch (b) {
        case 1: KDCD_KRR(1, 1024, 1); break;
        case 2: KDCD_KRR(2, 1024, 2); break;
        case 4: KDCD_KRR(4, 1024, 4); break;
        case 8: KDCD_KRR(8, 1024, 8); break;
        case 16: KDCD_KRR(16, 1024, 16); break;
        default:
            if (b <= 8) KDCD_KRR(8, 1024, 0);
            else if (b <= 16) KDCD_KRR(16, 1024, 0);
            else return hipErrorInvalidValue;
        }
    }
#undef KDCD_KRR
    return hipGetLastError();
}

}  // namespace kdcd
