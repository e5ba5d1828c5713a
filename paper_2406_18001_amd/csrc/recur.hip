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

// A double in the constant address space: loads through it may be scalar.
typedef const double __attribute__((address_space(4))) ConstF64;

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

// K-RR recurrence (Algorithm 4's inner loop).  Elements are grouped in panels
// of PE = floor(64/b)*b (whole blocks); panel q lives on lanes [0, PE) of wave
// q.  With G[t][u] = W[t][u]/lambda + m [S_t = S_u] the block step for block j
// of a panel is Delta_j = D_j^{-1} c_j, and every later element u of the panel
// subtracts sum_q G[j_q][u] Delta_{j_q}.  Both are linear in c_j, so the
// coefficients K[r][u] = (D_j^{-1})[u][r] (u in block j) or
// sum_q G[j_q][u] (D_j^{-1})[q][r] (u later) are formed for the whole panel
// before it starts, by the waves that do not own the running panel; the owner
// then spends one b-term chain per block: x_u = sum_r K[r][u] c_{j_r}.  After
// the panel, one barrier, and every later element folds in the panel's Delta
// values.  Repeated coordinates (a coordinate sampled in several blocks) add
// the m-term to G and their updates to the running sum of the coordinate; each
// panel keeps the list of its elements whose coordinate comes again later, so
// the folds visit only those for that term.  BMAX bounds b, NT the
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
    constexpr int NW = NT / 64;
    constexpr int QN = BX > 0 ? BX : BMAX;
    constexpr int RC = QN < 8 ? QN : 8;        // coefficient rows per work item
    __shared__ double Kd[2][64 * 64];          // block-step coefficients of a panel, [row][lane]
    __shared__ double d_l[kMaxSB + 64];        // padded: entries past the last panel hold 0 / -1
    __shared__ __align__(16) int32_t S_l[kMaxSB + 64];
    __shared__ int32_t hkeys[kHashSlots], hidx[kHashSlots];
    __shared__ int32_t rep_l[NW * 64];         // panel q: rep_l[64 q, 64 q + rep_n[q]), ascending
    __shared__ int32_t rep_n[NW];
    __shared__ double c_bc[QN];                // PIPE: c of the owner wave's running block
    if (BX > 0) b = BX;
    // wid through readfirstlane: the compiler then treats it (and what depends on it) as
    // wave-uniform, so per-block coefficients and branches on the panel owner are scalar
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    const int lblk = lane / b;                        // block index inside the panel
    constexpr bool PIPE = BX > 0 && BX <= 8 && NT <= 512;
    constexpr int DVN = PIPE ? QN : 1;
    double dv[DVN];                                   // PIPE: this element's row of D_j^{-1}
#pragma unroll
    for (int t = 0; t < DVN; ++t)
        dv[t] = (PIPE && act) ? Dinv[((int64_t)myblk * b + e % b) * b + t] : 0.0;
    for (int x = tid; x < kMaxSB + 64; x += NT) {   // every slot without an owner: S = -1, d = 0
        S_l[x] = -1;
        d_l[x] = 0.0;
    }
    lastocc_clear(hkeys, hidx, tid, NT);
    lds_barrier();
    if (act) S_l[e] = (int32_t)Sp;
    const int hslot = act ? lastocc_insert(hkeys, hidx, (int32_t)Sp, e) : 0;

    // Coefficients of panel q: work items are (block, chunk of RC rows); lane u
    // computes column u.  An item's loads are issued first (k_load) and turned
    // into coefficients later (k_finish).  PIPE (b <= 8 fixed at compile time,
    // 512 threads): the rows of a block's own lanes (its D_j^{-1} rows) are
    // written by the owner wave when the panel starts, so only blocks with later
    // lanes are items, and each wave loads its items of panel q + 2 while panel
    // q runs: the coefficients of panel q + 1 are then formed from registers
    // whose loads are long done.  Otherwise items also write the own rows and
    // are loaded and finished in the panel before their use.
    auto k_items = [&](int q) {
        const int qlen = (sb - q * PE) < PE ? (sb - q * PE) : PE;
        return (qlen / b - (PIPE ? 1 : 0)) * ((b + RC - 1) / RC);
    };
    auto k_load = [&](int q, int it, double (&x)[QN], double (&dvo)[RC]) {
        const int Q0 = q * PE;
        const int qlen = (sb - Q0) < PE ? (sb - Q0) : PE;
        const int nrc = (b + RC - 1) / RC;
        const int l0 = (it / nrc) * b;
        // a clamped, valid column for every lane (no per-load branch); rows
        // Q0 + l0 + t < Q0 + qlen as the block has later lanes
        const int64_t ucol = Q0 + (lane < qlen ? lane : qlen - 1);
#pragma unroll
        for (int t = 0; t < QN; ++t)
            if (BX > 0 || t < b) x[t] = W[(int64_t)(Q0 + l0 + t) * sb + ucol];
        if constexpr (!PIPE) {   // this lane's D_j^{-1} row, if the lane is in the block
            const int r0 = (it % nrc) * RC;
            const bool own = lane >= l0 && lane < l0 + b;
            const int64_t urow = (Q0 + l0) + (own ? lane - l0 : 0);
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
                if (r0 + rr < b) dvo[rr] = Dinv[urow * b + r0 + rr];
        }
    };
    auto k_finish = [&](int q, int it, double (&x)[QN], const double (&dvo)[RC], double *dst) {
        const int Q0 = q * PE;
        const int qlen = (sb - Q0) < PE ? (sb - Q0) : PE;
        const int nrc = (b + RC - 1) / RC;
        const int l0 = (it / nrc) * b, r0 = (it % nrc) * RC;
        const int u = lane;
        const int32_t Su = S_l[Q0 + u];
        const bool lat = u >= l0 + b && u < qlen;
#pragma unroll
        for (int t = 0; t < QN; ++t) {
            if (BX > 0 || t < b) {
                const double g = x[t] * inv_lambda + (S_l[Q0 + l0 + t] == Su ? mdbl : 0.0);
                x[t] = lat ? g : 0.0;
            }
        }
        // D_j^{-1} is read-only during the launch and its addresses are uniform:
        // through the constant address space its rows come in by scalar loads
        const ConstF64 *Db = (const ConstF64 *)(Dinv + (int64_t)(Q0 + l0) * b);
        double kacc[RC];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) kacc[rr] = 0.0;
        if constexpr (PIPE && QN == 8) {
            // two halves of four columns: each half's 8 x 4 entries are fetched
            // as one batch of scalar loads before its FMAs (two waits per item)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double dd[8][4];
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int c = 0; c < 4; ++c) dd[t][c] = Db[t * 8 + h * 4 + c];
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int c = 0; c < 4; ++c) kacc[h * 4 + c] += x[t] * dd[t][c];
            }
        } else {
#pragma unroll
            for (int t = 0; t < QN; ++t) {
                if (BX > 0 || t < b) {
#pragma unroll
                    for (int rr = 0; rr < RC; ++rr)
                        if (r0 + rr < b) kacc[rr] += x[t] * Db[t * b + r0 + rr];
                }
            }
        }
        const bool own = u >= l0 && u < l0 + b;
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) {
            if (r0 + rr < b) {
                if (!PIPE) dst[(l0 + r0 + rr) * 64 + u] = own ? dvo[rr] : kacc[rr];
                else if (!own) dst[(l0 + r0 + rr) * 64 + u] = kacc[rr];   // own rows: the owner's
            }
        }
    };
    // items per wave held in registers between k_load and k_finish
    constexpr int KI = PIPE ? ((64 / QN - 1) + NW - 2) / (NW - 1) : 1;
    double xp[KI][PIPE ? QN : 1], dvp[PIPE ? RC : 1];
    // the waves other than wave q - 1 form panel q's coefficients; rank among them
    auto k_rank = [&](int q) { return wid < q - 1 ? wid : wid - 1; };
    auto k_direct = [&](int q, double *dst, int rank, int count) {
        const int items = k_items(q);
        for (int it = rank; it < items; it += count) {
            double x[QN], dvo[RC];
            k_load(q, it, x, dvo);
            k_finish(q, it, x, dvo, dst);
        }
    };
    lds_barrier();
    if (act) {
        const int q0 = myblk * b;
        for (int q = q0; q < q0 + b; ++q)
            if (q != e && S_l[q] == (int32_t)Sp) set_status(status, KDCD_ERR_INDEX_DUPLICATE);
    }
    {   // elements of this wave's panel whose coordinate comes again later
        const bool rl = act && hidx[hslot] != e;
        const uint64_t bal = __ballot(rl);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (rl) rep_l[wid * 64 + below] = e;
        if (lane == 0) rep_n[wid] = __popcll(bal);
    }
    k_direct(0, Kd[0], wid, NW);
    if constexpr (PIPE) {
        if (wid != 0 && 1 < npanels) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                const int it = k_rank(1) + k * (NW - 1);
                if (it < k_items(1)) k_load(1, it, xp[k], dvp);
            }
        }
    }
    lds_barrier();

    double delta = 0.0, dsum = 0.0;   // dsum: updates of earlier repeats of this coordinate, in order
    for (int p = 0; p < npanels; ++p) {
        const int P0 = p * PE;
        const int plen = (sb - P0) < PE ? (sb - P0) : PE;
        const int buf = p & 1;
        const bool later = act && wid > p;
        // the fold's W values: with PIPE issued after the coefficient work, so
        // that its waits do not cover them
        double wpre[PF];
        auto fold_loads = [&]() {
            if (later) {
#pragma unroll
                for (int t = 0; t < PF; ++t)
                    wpre[t] = (t < plen) ? W[(int64_t)(P0 + t) * sb + e] : 0.0;
            }
        };
        // the next owner's fold loads go first (its fold is on the critical path)
        if (!PIPE || wid == p + 1) fold_loads();
        if (wid != p && p + 1 < npanels) {
            if constexpr (PIPE) {
#pragma unroll
                for (int k = 0; k < KI; ++k) {
                    const int it = k_rank(p + 1) + k * (NW - 1);
                    if (it < k_items(p + 1)) k_finish(p + 1, it, xp[k], dvp, Kd[buf ^ 1]);
                }
            } else {
                k_direct(p + 1, Kd[buf ^ 1], k_rank(p + 1), NW - 1);
            }
        }
        if constexpr (PIPE) {
            if (wid != p + 1 && p + 2 < npanels) {
#pragma unroll
                for (int k = 0; k < KI; ++k) {
                    const int it = k_rank(p + 2) + k * (NW - 1);
                    if (it < k_items(p + 2)) k_load(p + 2, it, xp[k], dvp);
                }
            }
        }
        if (PIPE && wid != p + 1) fold_loads();
        if (wid == p) {
            double *kd = Kd[buf];
            if (PIPE && act) {   // this lane's row of its block's D_j^{-1}
#pragma unroll
                for (int t = 0; t < DVN; ++t) kd[(lblk * b + t) * 64 + lane] = dv[t];
            }
            const int nbl = plen / b;
            for (int bl = 0; bl < nbl; ++bl) {
                const int l0 = bl * b;
                double kc[QN];
#pragma unroll
                for (int t = 0; t < QN; ++t)
                    if (BX > 0 || t < b) kc[t] = kd[(l0 + t) * 64 + lane];
                double x = 0.0;
                if constexpr (PIPE) {
                    // the block's lanes publish their c through LDS and every lane
                    // reads the b values back: one LDS round trip is shorter than 2b
                    // dependent lane reads
                    if (lblk == bl) c_bc[lane - l0] = c;
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int t = 0; t < QN; ++t) x += kc[t] * c_bc[t];
                    __builtin_amdgcn_wave_barrier();
                } else {
#pragma unroll
                    for (int t = 0; t < QN; ++t)
                        if (BX > 0 || t < b) x += kc[t] * readlane_d(c, l0 + t);
                }
                if (lblk == bl) delta = x;
                if (act && lblk > bl) c -= x;
            }
            if (act) d_l[e] = delta;
        }
        lds_barrier();
        const int nrep = rep_n[p];
        if (wid == p && act) {
            // repeats of this coordinate in the earlier blocks of the panel, in order
            for (int k = 0; k < nrep; ++k) {
                const int t = rep_l[p * 64 + k];
                if (t < P0 + lblk * b && S_l[t] == (int32_t)Sp) dsum += d_l[t];
            }
        }
        if (later) {
            // wpre[t] and d_l[P0 + t] are 0 past the end of the panel
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < PF; ++t) acc += wpre[t] * d_l[P0 + t];
            for (int t = PF; t < plen; ++t) acc += W[(int64_t)(P0 + t) * sb + e] * d_l[P0 + t];
            c -= acc * inv_lambda;
            for (int k = 0; k < nrep; ++k) {          // repeats of this coordinate in the panel
                const int t = rep_l[p * 64 + k];
                if (S_l[t] == (int32_t)Sp) {
                    c -= mdbl * d_l[t];
                    dsum += d_l[t];
                }
            }
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
    if (D.pos) {   // the next product's row -> position table: clear S_k, then mark S_next
        if (act) D.pos[Sp] = -1;
        __syncthreads();
        for (int t = tid; t < D.sb_next; t += NT) {
            const int32_t q = D.S_next[t];
            if (q >= 0 && q < m) D.pos[q] = t;
        }
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
