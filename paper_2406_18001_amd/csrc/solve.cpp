// Host driver of the kdcd C-ABI: argument validation, workspace, the outer
// loop of Algorithms 2 and 4 (kernel block -> finish -> recurrence per outer
// iteration), status reporting and optional stage timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "sampler.hpp"

using namespace kdcd;

namespace kdcd {
hipError_t launch_kblock_mixed(const KBlockArgs &a, hipStream_t st);
hipError_t launch_kblock_csr(const KBlockArgs &a, hipStream_t st);
int64_t kblock_csr_row_groups(const kdcd_matrix *A, int32_t sb);
int64_t kblock_csr_max_row_groups(int64_t m);
hipError_t launch_convert_lowp(const kdcd_matrix *A, int32_t compute, void *hi, void *lo,
                               int64_t ldlow, float *normlow, hipStream_t st);
int krr_recur_threads(int32_t b, int32_t sk);
int32_t lowrank_zinit_chunks();
size_t lowrank_part_bytes();
hipError_t launch_nystrom(const double *Av, int64_t lda, int64_t m, int64_t n, const int32_t *L,
                          int32_t r, const KParams &kp, double jitter, const double *normsA,
                          const double *Xv, int64_t ldx, int64_t mx, const double *normsX,
                          bool x_is_a, double *Cw, double *Dinv, double *Phi, int64_t ldp,
                          double *part, size_t part_bytes, int32_t *status, hipStream_t st);
hipError_t launch_lowrank_block(const double *Phi, int64_t ldp, int64_t m, int32_t r,
                                const int32_t *S, int32_t sb, const double *z, double *W,
                                double *v, double *part, size_t part_bytes, hipStream_t st);
hipError_t launch_lowrank_z_update(const double *Phi, int64_t ldp, int64_t m, int32_t r,
                                   const int32_t *S, int32_t sb, const double *theta,
                                   const double *coef, double *part, double *z, hipStream_t st);
hipError_t launch_lowrank_z_init(const double *Phi, int64_t ldp, int64_t m, int32_t r,
                                 const double *alpha, const double *coef, double *part, double *z,
                                 hipStream_t st);
}  // namespace kdcd

namespace {

constexpr int64_t kMaxGroups = 1024;   // upper bound on row groups of any kernel-block launch

// Upper bound on the row groups (rows of the partial column sums) of any
// kernel-block launch on A.
int64_t max_row_groups(const kdcd_matrix *A)
{
    if (A->format == KDCD_CSR) return kblock_csr_max_row_groups(A->m);
    return std::min<int64_t>(kMaxGroups, (A->m + 63) / 64);   // dense tiles are >= 64 rows
}
// From this block width on, the Gram rows come from the U-part (two small
// launches per outer iteration) instead of tiles of their own, which at
// these widths add a round of workgroups.
constexpr int64_t kGatherMinSB = 256;
// Tile configuration of the FP64 Gram-only launches that follow a
// low-precision product: 128 x 16 (four waves) spreads an s*b-row Gram over
// the most workgroups; with its long K loop and few tiles that launch is bound
// by latency, not by the tile's MFMA rate (C2's 1024 x 512 lookahead Gram:
// 29.8 us against 34.3 for the 64 x 64 tile, 40.3 for 128 x 32).
constexpr int32_t kGramCfg = 0;
// Largest rank of a low-rank factor (Nystrom landmarks, columns of Phi).
constexpr int64_t kMaxRank = 4096;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

kdcd_status check_matrix(const kdcd_matrix *A)
{
    if (!A || !A->values || A->m < 1 || A->n < 1) return KDCD_ERR_INVALID_ARG;
    if (A->m > INT32_MAX) return KDCD_ERR_UNSUPPORTED;
    if (A->format == KDCD_DENSE) {
        if (A->ld < A->n) return KDCD_ERR_INVALID_ARG;
    } else if (A->format == KDCD_CSR) {
        if (!A->row_ptr || !A->col_idx || A->nnz < 0 || A->n > INT32_MAX) return KDCD_ERR_INVALID_ARG;
    } else {
        return KDCD_ERR_INVALID_ARG;
    }
    return KDCD_OK;
}

kdcd_status check_kernel(const kdcd_kernel *k)
{
    if (!k) return KDCD_ERR_INVALID_ARG;
    switch (k->kind) {
    case KDCD_KERNEL_LINEAR: return KDCD_OK;
    case KDCD_KERNEL_POLY:
        return (std::isfinite(k->c) && k->c >= 0.0 && k->degree >= 1 && k->degree <= 64)
                   ? KDCD_OK : KDCD_ERR_INVALID_ARG;
    case KDCD_KERNEL_RBF: return finite_pos(k->sigma) ? KDCD_OK : KDCD_ERR_INVALID_ARG;
    default: return KDCD_ERR_INVALID_ARG;
    }
}

kdcd_status check_compute(const kdcd_matrix *A, int32_t compute)
{
    if (compute < KDCD_F64 || compute > KDCD_BF16X3) return KDCD_ERR_INVALID_ARG;
    if (compute != KDCD_F64 && A->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    return KDCD_OK;
}

// The product's tile configuration is looked up once (into kb.cfg) and the
// finish pass sums the row groups of that same configuration, so a change of
// the tuning table between the two cannot pair a launch with the wrong count.
// Uses kb.A, kb.sb and kb.compute; returns the row-group count.
int64_t bind_config(KBlockArgs &kb, bool batch = false)
{
    const kdcd_matrix *A = kb.A;
    kb.cfg = -1;
    if (A->format == KDCD_CSR) return kblock_csr_row_groups(A, kb.sb);
    if (kb.compute == KDCD_F64) {
        kb.cfg = batch ? f64_batch_config_id(A->n, kb.sb) : f64_config_id(A->n, kb.sb);
        return kblock_f64_row_groups(kb.cfg, A->m, A->n, kb.sb, batch);
    }
    if (!batch && kb.compute != KDCD_F32) {
        kb.cfg = lowp_config_id(kb.compute, A->n, kb.sb);
        return kblock_lowp_row_groups(kb.cfg, A->m);
    }
    if (batch) kb.cfg = mixed_batch_config_id(kb.compute, A->n, kb.sb);
    return kblock_mixed_row_groups(kb.cfg, A->m, A->n, kb.sb, kb.compute, batch);
}

// One kernel-block pass.  Mixed precisions produce the U-part only; their
// Gram W comes from the FP64 kernel run on the Gram tiles alone.
hipError_t launch_kblock(const KBlockArgs &a, hipStream_t st)
{
    if (a.A->format == KDCD_CSR) return launch_kblock_csr(a, st);
    if (a.compute == KDCD_F64) return launch_kblock_f64(a, st);
    hipError_t e = launch_kblock_mixed(a, st);
    if (e != hipSuccess || !a.W) return e;
    KBlockArgs w = a;
    w.compute = KDCD_F64;
    w.w_only = 1;
    w.cfg = kGramCfg;    // (a.cfg names a low-precision tile)
    w.U = nullptr;       // the stored kernel block is the low-precision product's
    return launch_kblock_f64(w, st);
}

size_t lowp_elem_bytes(int32_t compute) { return compute == KDCD_F32 ? 4 : 2; }

// Workspace regions of one solve.
struct Layout {
    size_t status, norms, partial, r, W, Dinv, iota, hi, lo, normlow, pos, carry, panel, total;
    // K-RR lookahead (la_ok): second row table and Gram, the kernel rows of the
    // previous block's coordinates, its summed updates and their coordinates
    bool la_ok;
    size_t pos2, W2, QX, la_dc, la_sc;
    int64_t ldlow;
    // convergence monitor (0 when off): state, partial sums, maintained
    // gradient / residual (m), stored kernel block (s*b x m), updates (s*b),
    // scratch m-vector
    size_t mon, mon_part, mon_v, mon_U, mon_th, mon_tmp;
    // second stored kernel block for the lookahead loop with the monitor (0: none)
    size_t mon_U2;
};

void add_monitor(Layout &L, int64_t m, int64_t sbmax)
{
    size_t off = L.total;
    L.mon = off; off += 256;
    L.mon_part = off; off += align256(monitor_partial_bytes());
    L.mon_v = off; off += align256(sizeof(double) * (size_t)m);
    L.mon_U = off; off += align256(sizeof(double) * (size_t)(sbmax * m));
    L.mon_th = off; off += align256(sizeof(double) * (size_t)sbmax);
    L.mon_tmp = off; off += align256(sizeof(double) * (size_t)m);
    L.total = off;
}

Layout make_layout(int32_t problem, const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t b,
                   int32_t s, int32_t compute)
{
    Layout L{};
    const int64_t sb = (int64_t)s * b;
    size_t off = 0;
    L.status = off; off += 256;
    L.norms = off; off += align256(sizeof(double) * (size_t)A->m);
    L.partial = off; off += align256(sizeof(double) * (size_t)(max_row_groups(A) * sb));
    L.r = off; off += align256(sizeof(double) * (size_t)sb);
    L.W = off; off += align256(sizeof(double) * (size_t)(sb * sb));
    L.Dinv = off; off += (problem == 1) ? align256(sizeof(double) * (size_t)(sb * b)) : 0;
    L.iota = off; off += (problem == 2) ? align256(sizeof(int32_t) * (size_t)A->m) : 0;
    L.pos = off; off += align256(sizeof(int32_t) * (size_t)A->m);   // row -> position in S
    const bool la_compute = compute == KDCD_F64 || compute == KDCD_F32 ||
                            compute == KDCD_BF16 || compute == KDCD_F16 ||
                            compute == KDCD_BF16X3;
    L.la_ok = problem == 1 && A->format == KDCD_DENSE && la_compute && sb >= kGatherMinSB &&
              b <= kLaMaxB && sb <= kLaEPT * 256;
    // FP64: second Gram and QX; low precision: one buffer of two Grams' rows
    // (QX of the previous block, then the block's Gram)
    const size_t gram = align256(sizeof(double) * (size_t)(sb * sb));
    L.pos2 = off; off += L.la_ok ? align256(sizeof(int32_t) * (size_t)A->m) : 0;
    L.W2 = off; off += L.la_ok ? (compute == KDCD_F64 ? gram : 2 * gram) : 0;
    L.QX = off; off += (L.la_ok && compute == KDCD_F64) ? gram : 0;
    L.la_dc = off; off += L.la_ok ? align256(sizeof(double) * (size_t)sb) : 0;
    L.la_sc = off; off += L.la_ok ? align256(sizeof(int32_t) * (size_t)sb) : 0;
    L.carry = off;   // CSR: partial dot products of sampled rows longer than the panel
    off += (A->format == KDCD_CSR) ? align256(sizeof(double) * (size_t)(A->m + sb)) : 0;
    L.panel = off;   // CSR: the dense-head panel of a chunk of sampled rows
    off += (A->format == KDCD_CSR) ? align256(kblock_csr_panel_bytes(A->n)) : 0;
    L.ldlow = 0;
    L.hi = L.lo = L.normlow = off;
    if (compute != KDCD_F64) {
        L.ldlow = (A->n + 63) / 64 * 64;   // pad K to whole stages of every product tile
        const size_t bytes = align256(lowp_elem_bytes(compute) * (size_t)(A->m * L.ldlow));
        L.hi = off; off += bytes;
        L.lo = off; off += (compute == KDCD_BF16X3) ? bytes : 0;
        L.normlow = off; off += align256(sizeof(float) * (size_t)A->m);
    }
    (void)kernel;
    L.total = off;
    return L;
}

// Device workspace: caller-provided or allocated on the stream.
struct Workspace {
    char *base = nullptr;
    bool owned = false;
    hipStream_t st = nullptr;
    ~Workspace()
    {
        if (owned && base) {
            (void)hipFreeAsync(base, st);
            (void)hipStreamSynchronize(st);
        }
    }
    template <class T> T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
};

kdcd_status acquire(Workspace &ws, const Layout &L, const kdcd_options *opt, hipStream_t st)
{
    ws.st = st;
    if (opt && opt->workspace) {
        if (opt->workspace_bytes < L.total) return KDCD_ERR_WORKSPACE;
        if (reinterpret_cast<uintptr_t>(opt->workspace) & 255) return KDCD_ERR_INVALID_ARG;
        ws.base = static_cast<char *>(opt->workspace);
        return KDCD_OK;
    }
    void *p = nullptr;
    if (hipMallocAsync(&p, L.total, st) != hipSuccess || !p) return KDCD_ERR_ALLOC;
    ws.base = static_cast<char *>(p);
    ws.owned = true;
    return KDCD_OK;
}

}  // namespace

namespace kdcd {
ArmedEvents &armed_events()
{
    static thread_local ArmedEvents ev{nullptr, nullptr};
    return ev;
}
}  // namespace kdcd

namespace {

// Event pairs of the launches of one stage: recorded around the launches
// (begin / end), or inside a kernel's own dispatch (arm).
// Timing events are kept per host thread and device and reused by later
// solves (a solve reads its timings before it returns); timers that are alive
// at the same time take disjoint ranges of the pool.
struct EventPool {
    int device = -1;
    size_t in_use = 0;
    std::vector<hipEvent_t> ev;
};

EventPool &event_pool()
{
    static thread_local EventPool p;
    return p;
}

struct StageTimer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
    hipEvent_t first = nullptr;   // alias of the first recorded event
    bool pooled = false;
    size_t pool_base = 0;
    std::vector<hipEvent_t> own;  // events made outside the pool (another device)
    ~StageTimer()
    {
        if (pooled) event_pool().in_use = pool_base;
        for (hipEvent_t e : own) (void)hipEventDestroy(e);
    }
    hipEvent_t mk()
    {
        EventPool &p = event_pool();
        int dev = -1;
        if (!pooled) {
            (void)hipGetDevice(&dev);
            if (p.device != dev && p.in_use == 0) {
                for (hipEvent_t e : p.ev) (void)hipEventDestroy(e);
                p.ev.clear();
                p.device = dev;
            }
            if (p.device == dev) {
                pooled = true;
                pool_base = p.in_use;
            }
        }
        hipEvent_t e = nullptr;
        if (!pooled) {
            (void)hipEventCreate(&e);
            own.push_back(e);
            return e;
        }
        if (p.in_use == p.ev.size()) {
            (void)hipEventCreate(&e);
            p.ev.push_back(e);
        }
        return p.ev[p.in_use++];
    }
    void begin(int stage, hipStream_t st)
    {
        if (!on) return;
        ev[stage].push_back({mk(), mk()});
        (void)hipEventRecord(ev[stage].back().first, st);
        if (!first) { first = ev[stage].back().first; }
    }
    void end(int stage, hipStream_t st)
    {
        if (!on) return;
        (void)hipEventRecord(ev[stage].back().second, st);
    }
    // The next KDCD_TIMED_LAUNCH of this thread records a new pair of `stage`
    // inside its own dispatch; disarm() after the launcher returns, so that a
    // launcher that started nothing leaves no pair armed.
    void arm(int stage)
    {
        if (!on) return;
        ev[stage].push_back({mk(), mk()});
        if (!first) { first = ev[stage].back().first; }
        armed_events() = ArmedEvents{ev[stage].back().first, ev[stage].back().second};
    }
    void disarm()
    {
        if (on) armed_events() = ArmedEvents{nullptr, nullptr};
    }
    void report(kdcd_profile *p)
    {
        if (!on || !p) return;
        double ms[3] = {0, 0, 0};
        for (int s = 0; s < 3; ++s)
            for (auto &e : ev[s]) {
                float t = 0.f;
                (void)hipEventElapsedTime(&t, e.first, e.second);
                ms[s] += t;
            }
        p->kblock_ms = ms[0]; p->kblock_launches = (int64_t)ev[0].size();
        p->finish_ms = ms[1]; p->finish_launches = (int64_t)ev[1].size();
        p->recur_ms = ms[2]; p->recur_launches = (int64_t)ev[2].size();
        p->total_ms = 0.0;
        hipEvent_t lastev = nullptr;
        for (int s = 2; s >= 0 && !lastev; --s)
            if (!ev[s].empty()) lastev = ev[s].back().second;
        if (first && lastev) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, first, lastev);
            p->total_ms = t;
        }
    }
};

kdcd_status read_status(int32_t *dstatus, hipStream_t st)
{
    int32_t hs = 0;
    if (hipMemcpyAsync(&hs, dstatus, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return KDCD_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return KDCD_ERR_HIP;
    return (kdcd_status)hs;
}

KParams to_params(const kdcd_kernel *k) { return KParams{k->kind, k->degree, k->sigma, k->c}; }

struct SolveArgs {
    int32_t problem;   // 0 = K-SVM, 1 = K-RR
    const kdcd_matrix *A;
    const double *y;
    const kdcd_kernel *kernel;
    double C, lambda;
    int32_t b, s;
    int64_t H;
    const int32_t *idx;
    double *alpha;
    kdcd_options opt;
    hipStream_t st;
    int64_t csr_max_row = -1;   // CSR: longest row of A, when measured (-1: unknown)
};

kdcd_status prepare_lowp(const KBlockArgs &base, const Layout &L, Workspace &ws, hipStream_t st,
                         KBlockArgs &a, bool convert = true)
{
    a = base;
    if (base.compute == KDCD_F64 || base.A->format != KDCD_DENSE) return KDCD_OK;
    a.Alow = ws.at<void>(L.hi);
    a.Alow2 = ws.at<void>(L.lo);
    a.ldlow = L.ldlow;
    a.normlow = ws.at<float>(L.normlow);
    if (convert)
        KDCD_HIP_TRY(launch_convert_lowp(base.A, base.compute, ws.at<void>(L.hi), ws.at<void>(L.lo),
                                         L.ldlow, ws.at<float>(L.normlow), st));
    return KDCD_OK;
}

}  // namespace

static kdcd_status kernel_matvec(const kdcd_matrix *A, const kdcd_kernel *kernel,
                                 const double *beta, std::vector<double> *host, double *dev,
                                 hipStream_t st);

namespace {

// Sigma groups and problem lists of a batch (shared by the solve and the tuner).
kdcd_status describe_batch(const kdcd_kernel *kernel, const kdcd_batch_problem *problems,
                           int32_t n_problems, BatchDesc &bd, std::vector<int> &krr,
                           std::vector<int> &svm)
{
    const bool rbf = kernel->kind == KDCD_KERNEL_RBF;
    kdcd_status rc = KDCD_OK;
    bd = BatchDesc{};
    bd.nprob = n_problems;
    for (int p = 0; p < n_problems; ++p) {
        const kdcd_batch_problem &q = problems[p];
        kdcd_kernel kp = *kernel;
        kp.sigma = q.sigma;
        if ((rc = check_kernel(&kp)) != KDCD_OK) return rc;
        if (!q.y || !q.alpha || !finite_pos(q.param)) return KDCD_ERR_INVALID_ARG;
        if (q.problem == 1) {
            krr.push_back(p);
        } else if (q.problem == 0) {
            if (q.loss != 0 && q.loss != 1 && q.loss != 2) return KDCD_ERR_INVALID_ARG;
            svm.push_back(p);
        } else {
            return KDCD_ERR_INVALID_ARG;
        }
        int g = 0;
        if (rbf) {
            while (g < bd.ngroups && bd.sigma[g] != q.sigma) ++g;
            if (g == bd.ngroups) {
                if (bd.ngroups == kMaxSigmas) return KDCD_ERR_UNSUPPORTED;
                bd.sigma[bd.ngroups++] = q.sigma;
            }
        } else {
            bd.ngroups = 1;
            bd.sigma[0] = kernel->sigma;
        }
        bd.group[p] = g;
        bd.beta[p] = q.alpha;
        bd.bscale[p] = q.problem == 0 ? q.y : nullptr;
    }
    return KDCD_OK;
}

// The maintained dual vector at the start: K-SVM g = Q a0 - 1 + omega a0,
// K-RR rho = y - M a0; the kernel product only runs for a nonzero a0 (one
// host round trip to find out).
kdcd_status init_dual_vector(int32_t problem, const kdcd_matrix *A, const kdcd_kernel *kernel,
                             const double *y, const double *alpha, double omega, double lambda,
                             double *v, double *tmp, int32_t *flag, hipStream_t st)
{
    const int64_t m = A->m;
    KDCD_HIP_TRY(launch_fill_i32(flag, 0, 1, st));
    if (problem == 0) KDCD_HIP_TRY(launch_product(y, alpha, m, tmp, flag, st));
    else KDCD_HIP_TRY(launch_product(alpha, alpha, m, tmp, flag, st));
    int32_t nonzero = 0;
    KDCD_HIP_TRY(hipMemcpyAsync(&nonzero, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    KDCD_HIP_TRY(hipStreamSynchronize(st));
    kdcd_status rc = KDCD_OK;
    if (nonzero && (rc = kernel_matvec(A, kernel, problem == 0 ? tmp : alpha, nullptr, v, st)) != KDCD_OK)
        return rc;
    if (problem == 0) KDCD_HIP_TRY(launch_grad_init(nonzero ? v : nullptr, y, alpha, omega, m, v, st));
    else KDCD_HIP_TRY(launch_rho_init(nonzero ? v : nullptr, y, alpha, 1.0 / lambda, (double)m, m, v, st));
    return KDCD_OK;
}

// Host side of an early stop: after every monitor evaluation the stop word is
// copied to pinned host memory and an event recorded; before enqueuing the
// next period the host waits for the copy of LAG periods earlier and stops
// enqueuing once it reads 1.  The host so runs at most LAG periods ahead of
// a stop instead of enqueuing every planned outer iteration.
struct StopPoller {
    static constexpr int LAG = 2;
    int32_t *host = nullptr;           // pinned, one word per monitor period
    hipEvent_t ev[LAG + 1] = {};
    int64_t periods = 0;
    bool ok = false;
    explicit StopPoller(int64_t n_periods) : periods(n_periods)
    {
        if (hipHostMalloc(reinterpret_cast<void **>(&host), sizeof(int32_t) * (size_t)(periods + 1)) !=
            hipSuccess)
            return;
        for (auto &e : ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
        ok = true;
    }
    ~StopPoller()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (host) (void)hipHostFree(host);
    }
    // after the monitor launch of period j (a final evaluation before the
    // first whole period comes as j = -1 and is not recorded)
    hipError_t post(int64_t j, const MonitorState *mon, hipStream_t st)
    {
        if (!ok || j < 0 || j > periods) return hipSuccess;
        hipError_t e = hipMemcpyAsync(host + j, &mon->stop, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(ev[j % (LAG + 1)], st);
        return e;
    }
    // before enqueuing period j + 1: true when the device had stopped at period j - LAG
    bool stopped(int64_t j)
    {
        if (!ok || j < LAG) return false;
        if (hipEventSynchronize(ev[(j - LAG) % (LAG + 1)]) != hipSuccess) return false;
        return host[j - LAG] != 0;
    }
};

// A part of a solve: outer iterations [k_begin, k_end) (k_end < 0: to the
// end), with or without the set-up launches (validation, norms, conversions,
// tables).  With S_base the index blocks come from a window buffer instead of
// idx: block k_begin - 1 at S_base, block k at S_base + (k - k_begin + 1) s b
// (every block of the range and the one after it full).
struct SolveRange {
    int64_t k_begin = 0, k_end = -1;
    bool setup = true;
    const int32_t *S_base = nullptr;
};

// Work (2 m n s b flops per product) from which the lookahead loop is the
// default: the product then takes well over 100 us, several times the
// recurrence it hides.
constexpr double kLaMinFlops = 4e9;

// Whether a K-RR solve runs the lookahead loop (see LookaheadArgs): dense FP64
// with a gathered Gram, b <= 8, 256 <= s*b <= 512, whole product tiles along
// K, no snapshots (the monitor only with the second stored kernel block), the
// whole solve in one call.
bool lookahead_use(const SolveArgs &sa, const Layout &L, const KBlockArgs &kb,
                   const SolveRange &R)
{
    const kdcd_matrix *A = sa.A;
    const bool f64 = sa.opt.compute == KDCD_F64;
    if (!L.la_ok || sa.problem != 1 || sa.b > kLaMaxB || (f64 && !kb.pos)) return false;
    if (sa.opt.flags & KDCD_FLAG_SERIAL) return false;
    if (sa.opt.monitor_every > 0 && (!f64 || L.mon_U2 == 0)) return false;
    if (sa.opt.snapshot_every > 0 && sa.opt.snapshots) return false;
    if (R.k_begin != 0 || R.k_end >= 0 || R.S_base || !R.setup) return false;
    const int64_t n_outer = (sa.H + sa.s - 1) / sa.s;
    if (n_outer < 2) return false;
    const bool aligned = (A->ld % 2 == 0) && ((reinterpret_cast<uintptr_t>(A->values) & 15) == 0);
    if (f64 && (!aligned || A->n % 16 != 0)) return false;
    // every product configuration has at least 256 threads, so the recurrence
    // fits whichever configuration a launch resolves
    const int64_t sb_full = (int64_t)sa.s * sa.b;
    if (sb_full > (int64_t)kLaEPT * 256) return false;
    if (sa.opt.flags & KDCD_FLAG_LOOKAHEAD) return true;
    return 2.0 * (double)A->m * (double)A->n * (double)sb_full >= kLaMinFlops;
}

// The lookahead loop of a K-RR solve.  Per outer iteration k: the finish pass
// of block k (r_k from the partial sums plus the kernel rows of block k-1's
// coordinates times their updates, D_j^{-1}, repeated Gram rows; block k-1's
// updates added to alpha; the row table of block k+1), then one launch with
// the recurrence of block k and the product of block k+1 (the last block's
// recurrence runs alone and writes alpha itself).  Row tables and Grams
// alternate between two copies: block k uses copy k % 2, which stays untouched
// until the finish pass of block k+1 has run.  With the monitor the stored
// kernel blocks alternate too; block k-1's dual update and the evaluation
// after k outer iterations run between the finish pass of block k (alpha then
// holds block k-1's updates) and the next launch (which overwrites the
// updates of block k-1 and the stored kernel block k-1).
kdcd_status enqueue_lookahead(const SolveArgs &sa, const Layout &L, Workspace &ws, KBlockArgs kb,
                              StageTimer &timer, bool product_only, bool sampled,
                              MonitorState *mon, double *dual, StopPoller *poll)
{
    const kdcd_matrix *A = sa.A;
    const hipStream_t st = sa.st;
    int32_t *status = ws.at<int32_t>(L.status);
    double *r = ws.at<double>(L.r);
    double *Dinv = ws.at<double>(L.Dinv);
    int32_t *P[2] = {ws.at<int32_t>(L.pos), ws.at<int32_t>(L.pos2)};
    double *Wb[2] = {ws.at<double>(L.W), ws.at<double>(L.W2)};
    double *QX = ws.at<double>(L.QX);
    double *Dc = ws.at<double>(L.la_dc);
    int32_t *Sc = ws.at<int32_t>(L.la_sc);
    const int64_t n_outer = (sa.H + sa.s - 1) / sa.s;
    auto block = [&](int64_t k, int32_t &sk, int32_t &sb) -> const int32_t * {
        const int64_t done = k * sa.s;
        sk = (int32_t)std::min<int64_t>(sa.s, sa.H - done);
        sb = sk * sa.b;
        return sa.idx + done * sa.b;
    };
    const bool monitor = mon != nullptr;
    const int32_t *stop = monitor ? &mon->stop : nullptr;
    double *Ub[2] = {monitor ? ws.at<double>(L.mon_U) : nullptr,
                     monitor ? ws.at<double>(L.mon_U2) : nullptr};
    auto trace_of = [&](int64_t k) -> double * {
        if (sa.opt.trace) return sa.opt.trace + k * sa.s * sa.b;
        return monitor ? ws.at<double>(L.mon_th) : nullptr;
    };
    const int64_t every = monitor ? sa.opt.monitor_every : 0;
    // block k's dual update, then the evaluation after k + 1 outer iterations
    // when one is due
    auto monitor_after = [&](int64_t k, bool last) -> kdcd_status {
        int32_t skk = 0, sbk = 0;
        const int32_t *Sk = block(k, skk, sbk);
        KDCD_HIP_TRY(launch_dual_update(Ub[k & 1], A->m, sbk, Sk, trace_of(k), nullptr,
                                        -1.0 / sa.lambda, nullptr, -(double)A->m, dual, stop, st));
        if ((k + 1) % every == 0 || last) {
            KDCD_HIP_TRY(launch_monitor(sa.problem, A->m, sa.alpha, sa.y, dual, 0.0, sa.opt.loss,
                                        sa.C, sa.opt.tol, k + 1, ws.at<double>(L.mon_part), mon,
                                        st));
            KDCD_HIP_TRY(poll->post((k + 1) / every - 1, mon, st));
        }
        return KDCD_OK;
    };

    KDCD_HIP_TRY(launch_fill_i32(P[1], -1, A->m, st));   // copy 0 was cleared by the set-up
    int32_t sk0 = 0, sb0 = 0;
    kb.S = block(0, sk0, sb0);
    kb.sb = sb0;
    kb.prevS = nullptr;
    kb.prev_sb = 0;
    kb.pos = P[0];
    kb.W = Wb[0];
    kb.la = nullptr;
    kb.U = Ub[0];
    kb.stop = stop;
    int64_t groups = bind_config(kb);
    KDCD_HIP_TRY(launch_kblock_f64_pre(kb, st));   // row table of block 0
    timer.arm(0);
    {
        const hipError_t e = launch_kblock_f64_main(kb, st);
        timer.disarm();
        KDCD_HIP_TRY(e);
    }
    for (int64_t k = 0; k < n_outer; ++k) {
        // the evaluation after k - 1 outer iterations is the last one posted
        if (monitor && k >= 2 && (k - 1) % every == 0 && poll->stopped((k - 1) / every - 1))
            return KDCD_OK;
        int32_t sk = 0, sb = 0, sk1 = 0, sb1 = 0, skp = 0, sbp = 0;
        const int32_t *S = block(k, sk, sb);
        const int32_t *S1 = k + 1 < n_outer ? block(k + 1, sk1, sb1) : nullptr;
        const int32_t *Sp = k > 0 ? block(k - 1, skp, sbp) : nullptr;
        FinishDesc fd{};
        fd.nprob = 1;
        fd.nkrr = 1;
        fd.groups = (int32_t)groups;
        fd.partial[0] = ws.at<double>(L.partial);
        fd.r[0] = r;
        fd.W[0] = Wb[k & 1];
        fd.Dinv[0] = Dinv;
        fd.inv_lambda[0] = 1.0 / sa.lambda;
        fd.stop = stop;
        fd.dup_S = S;
        fd.dup_pos = P[k & 1];
        fd.dup_W = Wb[k & 1];
        fd.m = A->m;
        if (k > 0) {
            fd.la_QX = QX;
            fd.la_Dc = Dc;
            fd.la_Sc = Sc;
            fd.la_sb = sbp;
            fd.la_alpha = sa.alpha;
        }
        fd.la_pos = P[(k + 1) & 1];
        fd.la_clearS = Sp;
        fd.la_clear_sb = sbp;
        fd.la_setS = S1;
        fd.la_set_sb = sb1;
        // the Gram of block k feeds the lookahead recurrence unless k is the last
        fd.la_lm = k + 1 < n_outer ? sa.lambda * (double)A->m : 0.0;
        if (!product_only) timer.arm(1);
        {
            const hipError_t e = launch_finish(fd, sb, sa.b, sk, (double)A->m, status, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        }
        if (monitor && k > 0) {
            const kdcd_status mrc = monitor_after(k - 1, false);
            if (mrc != KDCD_OK) return mrc;
        }
        if (k + 1 < n_outer) {
            LookaheadArgs la{};
            la.S = S;
            la.sb = sb;
            la.b = sa.b;
            la.sk = sk;
            la.r = r;
            la.W = Wb[k & 1];
            la.Dinv = Dinv;
            la.y = sa.y;
            la.alpha = sa.alpha;
            la.lambda = sa.lambda;
            la.mdbl = (double)A->m;
            la.pos = P[k & 1];
            la.Dc = Dc;
            la.Sc = Sc;
            la.trace = trace_of(k);
            la.status = status;
            la.m = A->m;
            la.QX = QX;
            kb.S = S1;
            kb.sb = sb1;
            kb.pos = P[(k + 1) & 1];
            kb.W = Wb[(k + 1) & 1];
            kb.U = Ub[(k + 1) & 1];
            kb.la = &la;
            groups = bind_config(kb);
            if (!sampled || (k + 1) % 8 == 0) timer.arm(0);
            const hipError_t e = launch_kblock_f64_main(kb, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        } else {
            KrrRecurDesc rd{};
            rd.r[0] = r;
            rd.W[0] = Wb[k & 1];
            rd.Dinv[0] = Dinv;
            rd.y[0] = sa.y;
            rd.alpha[0] = sa.alpha;
            rd.trace[0] = trace_of(k);
            rd.lambda[0] = sa.lambda;
            rd.stop = stop;
            if (!product_only) timer.arm(2);
            const hipError_t e =
                launch_krr_recur(rd, 1, S, sa.b, sk, A->m, (double)A->m, status, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
            if (monitor) {
                const kdcd_status mrc = monitor_after(k, true);
                if (mrc != KDCD_OK) return mrc;
            }
        }
    }
    return KDCD_OK;
}

// The lookahead loop with a low-precision product (f32, bf16, f16, bf16x3).  As the
// FP64 loop, but the product stores no Gram rows: after each lookahead launch
// an FP64 Gram launch takes the rows of index blocks k and k+1, which lie back
// to back in idx, against block k+1's columns, giving in one buffer the kernel
// rows of block k's coordinates (QX, here in FP64) followed by block k+1's
// Gram.  The buffer is overwritten only after the launch whose recurrence read
// block k's Gram and the finish pass that read block k's QX.
kdcd_status enqueue_lookahead_lowp(const SolveArgs &sa, const Layout &L, Workspace &ws,
                                   KBlockArgs kb, StageTimer &timer, bool product_only,
                                   bool sampled)
{
    const kdcd_matrix *A = sa.A;
    const hipStream_t st = sa.st;
    int32_t *status = ws.at<int32_t>(L.status);
    double *r = ws.at<double>(L.r);
    double *Dinv = ws.at<double>(L.Dinv);
    int32_t *P[2] = {ws.at<int32_t>(L.pos), ws.at<int32_t>(L.pos2)};
    double *Wx = ws.at<double>(L.W2);
    double *Dc = ws.at<double>(L.la_dc);
    int32_t *Sc = ws.at<int32_t>(L.la_sc);
    const int64_t n_outer = (sa.H + sa.s - 1) / sa.s;
    auto block = [&](int64_t k, int32_t &sk, int32_t &sb) -> const int32_t * {
        const int64_t done = k * sa.s;
        sk = (int32_t)std::min<int64_t>(sa.s, sa.H - done);
        sb = sk * sa.b;
        return sa.idx + done * sa.b;
    };
    auto trace_of = [&](int64_t k) -> double * {
        return sa.opt.trace ? sa.opt.trace + k * sa.s * sa.b : nullptr;
    };
    // the Gram of block k (after the QX rows of block k - 1, when there is one)
    auto gram_of = [&](int64_t k) -> double * {
        int32_t skk = 0, sbk = 0, skp = 0, sbp = 0;
        block(k, skk, sbk);
        if (k > 0) block(k - 1, skp, sbp);
        return Wx + (int64_t)sbp * sbk;
    };
    auto gram_launch = [&](int64_t k) -> kdcd_status {
        int32_t skk = 0, sbk = 0, skp = 0, sbp = 0;
        const int32_t *Sk = block(k, skk, sbk);
        if (k > 0) block(k - 1, skp, sbp);
        KBlockArgs w = kb;
        w.compute = KDCD_F64;
        w.w_only = 1;
        w.cfg = kGramCfg;
        w.U = nullptr;
        w.pos = nullptr;
        w.la = nullptr;
        w.S = Sk;
        w.sb = sbk;
        w.W = Wx;
        w.w_row0 = -sbp;          // block k - 1's indices precede block k's in idx
        w.w_rows = sbp + sbk;
        KDCD_HIP_TRY(launch_kblock_f64(w, st));
        return KDCD_OK;
    };

    KDCD_HIP_TRY(launch_fill_i32(P[0], -1, A->m, st));
    KDCD_HIP_TRY(launch_fill_i32(P[1], -1, A->m, st));
    int32_t sk0 = 0, sb0 = 0;
    const int32_t *S0 = block(0, sk0, sb0);
    {   // row table of block 0 (the positions of its coordinates)
        KBlockArgs t = kb;
        t.S = S0;
        t.sb = sb0;
        t.W = Wx;
        t.pos = P[0];
        t.prevS = nullptr;
        t.prev_sb = 0;
        t.w_only = 0;
        KDCD_HIP_TRY(launch_kblock_f64_pre(t, st));
    }
    kb.S = S0;
    kb.sb = sb0;
    kb.pos = nullptr;
    kb.la = nullptr;
    int64_t groups = bind_config(kb);
    timer.arm(0);
    {
        const hipError_t e = launch_kblock_mixed(kb, st);
        timer.disarm();
        KDCD_HIP_TRY(e);
    }
    kdcd_status rc = gram_launch(0);
    if (rc != KDCD_OK) return rc;
    for (int64_t k = 0; k < n_outer; ++k) {
        int32_t sk = 0, sb = 0, sk1 = 0, sb1 = 0, skp = 0, sbp = 0;
        const int32_t *S = block(k, sk, sb);
        const int32_t *S1 = k + 1 < n_outer ? block(k + 1, sk1, sb1) : nullptr;
        const int32_t *Sp = k > 0 ? block(k - 1, skp, sbp) : nullptr;
        double *Wk = gram_of(k);
        FinishDesc fd{};
        fd.nprob = 1;
        fd.nkrr = 1;
        fd.groups = (int32_t)groups;
        fd.partial[0] = ws.at<double>(L.partial);
        fd.r[0] = r;
        fd.W[0] = Wk;
        fd.Dinv[0] = Dinv;
        fd.inv_lambda[0] = 1.0 / sa.lambda;
        fd.dup_S = S;
        fd.dup_pos = P[k & 1];
        fd.dup_W = Wk;
        fd.m = A->m;
        if (k > 0) {
            fd.la_QX = Wx;            // block k - 1's rows against block k's columns
            fd.la_Dc = Dc;
            fd.la_Sc = Sc;
            fd.la_sb = sbp;
            fd.la_alpha = sa.alpha;
        }
        fd.la_pos = P[(k + 1) & 1];
        fd.la_clearS = Sp;
        fd.la_clear_sb = sbp;
        fd.la_setS = S1;
        fd.la_set_sb = sb1;
        fd.la_lm = k + 1 < n_outer ? sa.lambda * (double)A->m : 0.0;
        if (!product_only) timer.arm(1);
        {
            const hipError_t e = launch_finish(fd, sb, sa.b, sk, (double)A->m, status, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        }
        if (k + 1 < n_outer) {
            LookaheadArgs la{};
            la.S = S;
            la.sb = sb;
            la.b = sa.b;
            la.sk = sk;
            la.r = r;
            la.W = Wk;
            la.Dinv = Dinv;
            la.y = sa.y;
            la.alpha = sa.alpha;
            la.lambda = sa.lambda;
            la.mdbl = (double)A->m;
            la.pos = P[k & 1];
            la.Dc = Dc;
            la.Sc = Sc;
            la.trace = trace_of(k);
            la.status = status;
            la.m = A->m;
            la.QX = nullptr;          // the Gram launch after it stores them
            kb.S = S1;
            kb.sb = sb1;
            kb.la = &la;
            groups = bind_config(kb);
            if (!sampled || (k + 1) % 8 == 0) timer.arm(0);
            const hipError_t e = launch_kblock_mixed(kb, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
            kb.la = nullptr;
            if ((rc = gram_launch(k + 1)) != KDCD_OK) return rc;
        } else {
            KrrRecurDesc rd{};
            rd.r[0] = r;
            rd.W[0] = Wk;
            rd.Dinv[0] = Dinv;
            rd.y[0] = sa.y;
            rd.alpha[0] = sa.alpha;
            rd.trace[0] = trace_of(k);
            rd.lambda[0] = sa.lambda;
            if (!product_only) timer.arm(2);
            const hipError_t e =
                launch_krr_recur(rd, 1, S, sa.b, sk, A->m, (double)A->m, status, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        }
    }
    return KDCD_OK;
}

// Everything a solve (or a part of it) puts on its stream, in the workspace at
// `base`, without the final status read (the status word is at offset L.status).
kdcd_status enqueue_solve(const SolveArgs &sa, const Layout &L, char *wsbase, StageTimer &timer,
                          const SolveRange &R = SolveRange{})
{
    const kdcd_matrix *A = sa.A;
    const hipStream_t st = sa.st;
    Workspace ws;            // a view: not owned, never freed here
    ws.base = wsbase;
    kdcd_status rc = KDCD_OK;
    int32_t *status = ws.at<int32_t>(L.status);
    double *norms = ws.at<double>(L.norms);
    double *partial = ws.at<double>(L.partial);
    double *r = ws.at<double>(L.r);
    double *W = ws.at<double>(L.W);
    double *Dinv = sa.problem == 1 ? ws.at<double>(L.Dinv) : nullptr;

    const bool svm = sa.problem == 0;
    const bool product_only = (sa.opt.flags & KDCD_FLAG_TIME_PRODUCT) != 0;
    const bool sampled = product_only && (sa.opt.flags & KDCD_FLAG_TIME_SAMPLE) != 0;
    const double nu = svm ? (sa.opt.loss == 2 ? INFINITY : sa.C) : 0.0;
    const double omega = (svm && sa.opt.loss == 2) ? 1.0 / (2.0 * sa.C) : 0.0;

    if (R.setup) {
        KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
        if (A->format == KDCD_CSR) KDCD_HIP_TRY(launch_validate_csr(A, status, st));
        KDCD_HIP_TRY(launch_validate(sa.idx, sa.H * sa.b, A->m, sa.y, sa.alpha, A->m, sa.problem,
                                     nu, status, st));
        if (sa.kernel->kind == KDCD_KERNEL_RBF) KDCD_HIP_TRY(launch_norms(A, norms, st));
    }

    KBlockArgs base{};
    base.A = A;
    base.norms = norms;
    base.kp = to_params(sa.kernel);
    base.beta = sa.alpha;
    base.beta_scale = svm ? sa.y : nullptr;
    base.partial = partial;
    base.W = W;
    base.status = status;
    base.compute = sa.opt.compute;
    if (A->format == KDCD_DENSE && sa.opt.compute == KDCD_F64 &&
        (int64_t)sa.s * sa.b >= kGatherMinSB) {
        base.pos = ws.at<int32_t>(L.pos);
        if (R.setup) KDCD_HIP_TRY(launch_fill_i32(base.pos, -1, A->m, st));
    }
    if (A->format == KDCD_CSR) {
        base.carry = ws.at<double>(L.carry);
        base.csr_panel = ws.at<void>(L.panel);
        base.csr_max_row = sa.csr_max_row;
        if (R.setup) KDCD_HIP_TRY(launch_csr_panel_init(A, base.csr_panel, st));
    }
    KBlockArgs kb;
    rc = prepare_lowp(base, L, ws, st, kb, R.setup);
    if (rc != KDCD_OK) return rc;

    const bool monitor = sa.opt.monitor_every > 0;
    MonitorState *mon = monitor ? ws.at<MonitorState>(L.mon) : nullptr;
    const int32_t *stop = monitor ? &mon->stop : nullptr;
    double *dual = monitor ? ws.at<double>(L.mon_v) : nullptr;
    if (monitor) {
        KDCD_HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(mon),
                                     0, (int64_t)(sizeof(MonitorState) / 4), st));
        KDCD_HIP_TRY(launch_monitor_start(mon, sa.opt.monitor_log, sa.opt.monitor_log_len, st));
        rc = init_dual_vector(sa.problem, A, sa.kernel, sa.y, sa.alpha, omega, sa.lambda, dual,
                              ws.at<double>(L.mon_tmp), &mon->pad, st);
        if (rc != KDCD_OK) return rc;
        kb.U = ws.at<double>(L.mon_U);
        kb.stop = stop;
    }

    const int64_t n_outer = (sa.H + sa.s - 1) / sa.s;
    int64_t snap = 0;
    std::unique_ptr<StopPoller> poll;
    if (monitor) poll.reset(new StopPoller(n_outer / sa.opt.monitor_every + 1));
    if (lookahead_use(sa, L, kb, R)) {
        if (sa.opt.compute != KDCD_F64)
            return enqueue_lookahead_lowp(sa, L, ws, kb, timer, product_only, sampled);
        return enqueue_lookahead(sa, L, ws, kb, timer, product_only, sampled, mon, dual,
                                 poll.get());
    }

    int64_t k = R.k_begin;
    const int64_t k_end = R.k_end < 0 ? n_outer : R.k_end;
    const int64_t sb_full = (int64_t)sa.s * sa.b;
    if (k > 0) {              // the block before the range (full): prevS of its first iteration
        kb.S = R.S_base ? R.S_base : sa.idx + (k - 1) * sb_full;
        kb.sb = (int32_t)sb_full;
    }
    for (; k < k_end; ++k) {
        if (monitor && k > 0 && k % sa.opt.monitor_every == 0 &&
            poll->stopped(k / sa.opt.monitor_every - 1))
            break;
        const int64_t done = k * sa.s;
        const int32_t sk = (int32_t)std::min<int64_t>(sa.s, sa.H - done);
        const int32_t sb = sk * sa.b;
        const int32_t *S = R.S_base ? R.S_base + (k - R.k_begin + 1) * sb_full : sa.idx + done * sa.b;
        kb.prevS = kb.S;          // the previous block (null before the first)
        kb.prev_sb = kb.sb;
        kb.S = S;
        kb.sb = sb;
        // K-RR with a gathered Gram: the finish launch copies the repeated rows
        // and each recurrence prepares the row -> position table of the next
        // block, so only the first block needs the separate update launch
        const bool fused = !svm && kb.W && kb.pos && !kb.w_only;
        const int64_t groups = bind_config(kb);
        if (A->format == KDCD_DENSE && sa.opt.compute == KDCD_F64) {
            // the product kernel times itself (the row-position update and
            // the repeated-row copies of the gathered Gram are not timed)
            if (k == 0 || !fused) KDCD_HIP_TRY(launch_kblock_f64_pre(kb, st));
            if (!sampled || k % 8 == 0) timer.arm(0);
            const hipError_t e = launch_kblock_f64_main(kb, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
            if (!fused) KDCD_HIP_TRY(launch_kblock_f64_post(kb, st));
        } else if (product_only && A->format == KDCD_CSR) {
            // the CSR product (with its Gram part) timed in its own dispatch
            if (!sampled || k % 8 == 0) timer.arm(0);
            const hipError_t e = launch_kblock_csr(kb, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        } else if (product_only && A->format == KDCD_DENSE) {
            // low-precision product timed in its own dispatch; the FP64 Gram
            // launch after it is not timed
            if (!sampled || k % 8 == 0) timer.arm(0);
            const hipError_t e = launch_kblock_mixed(kb, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
            KBlockArgs w = kb;
            w.compute = KDCD_F64;
            w.w_only = 1;
            w.cfg = kGramCfg;
            KDCD_HIP_TRY(launch_kblock_f64(w, st));
        } else {
            timer.begin(0, st);
            KDCD_HIP_TRY(launch_kblock(kb, st));
            timer.end(0, st);
        }
        FinishDesc fd{};
        fd.nprob = 1;
        fd.nkrr = svm ? 0 : 1;
        fd.groups = (int32_t)groups;
        fd.partial[0] = partial;
        fd.r[0] = r;
        fd.W[0] = W;
        fd.Dinv[0] = Dinv;
        fd.inv_lambda[0] = svm ? 0.0 : 1.0 / sa.lambda;
        fd.stop = stop;
        if (fused) {
            fd.dup_S = S;
            fd.dup_pos = kb.pos;
            fd.dup_W = W;
            fd.m = A->m;
        }
        if (!product_only) timer.arm(1);
        {
            const hipError_t e = launch_finish(fd, sb, sa.b, sk, (double)A->m, status, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        }
        double *tr = sa.opt.trace ? sa.opt.trace + done * sa.b
                                  : (monitor ? ws.at<double>(L.mon_th) : nullptr);
        if (svm) {
            KsvmRecurDesc kd{};
            kd.r[0] = r;
            kd.W[0] = W;
            kd.y[0] = sa.y;
            kd.alpha[0] = sa.alpha;
            kd.trace[0] = tr;
            kd.nu[0] = nu;
            kd.omega[0] = omega;
            kd.stop = stop;
            if (!product_only) timer.arm(2);
            const hipError_t e = launch_ksvm_recur(kd, 1, S, sb, A->m, status, st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        } else {
            KrrRecurDesc rd{};
            rd.r[0] = r;
            rd.W[0] = W;
            rd.Dinv[0] = Dinv;
            rd.y[0] = sa.y;
            rd.alpha[0] = sa.alpha;
            rd.trace[0] = tr;
            rd.lambda[0] = sa.lambda;
            rd.stop = stop;
            if (fused) {
                rd.pos = kb.pos;
                if (k + 1 < n_outer) {
                    rd.S_next = S + sb;
                    rd.sb_next = (int32_t)std::min<int64_t>(sa.s, sa.H - done - sk) * sa.b;
                }
            }
            if (!product_only) timer.arm(2);
            const hipError_t e = launch_krr_recur(rd, 1, S, sa.b, sk, A->m, (double)A->m, status,
                                                  st);
            timer.disarm();
            KDCD_HIP_TRY(e);
        }
        if (monitor) {
            if (svm)
                KDCD_HIP_TRY(launch_dual_update(kb.U, A->m, sb, S, tr, sa.y, 1.0, sa.y, omega,
                                                dual, stop, st));
            else
                KDCD_HIP_TRY(launch_dual_update(kb.U, A->m, sb, S, tr, nullptr, -1.0 / sa.lambda,
                                                nullptr, -(double)A->m, dual, stop, st));
            if ((k + 1) % sa.opt.monitor_every == 0 || k + 1 == n_outer) {
                KDCD_HIP_TRY(launch_monitor(sa.problem, A->m, sa.alpha, sa.y, dual, omega,
                                            sa.opt.loss, sa.C, sa.opt.tol, k + 1,
                                            ws.at<double>(L.mon_part), mon, st));
                KDCD_HIP_TRY(poll->post((k + 1) / sa.opt.monitor_every - 1, mon, st));
            }
        }
        if (sa.opt.snapshot_every > 0 && sa.opt.snapshots &&
            ((k + 1) % sa.opt.snapshot_every == 0 || k + 1 == n_outer)) {
            KDCD_HIP_TRY(hipMemcpyAsync(sa.opt.snapshots + snap * A->m, sa.alpha,
                                        sizeof(double) * (size_t)A->m, hipMemcpyDeviceToDevice,
                                        st));
            ++snap;
        }
    }
    // stopped early: the snapshots not yet taken all hold the final iterate
    if (R.k_end < 0 && k < n_outer && sa.opt.snapshot_every > 0 && sa.opt.snapshots) {
        const int64_t rows = (n_outer + sa.opt.snapshot_every - 1) / sa.opt.snapshot_every;
        for (; snap < rows; ++snap)
            KDCD_HIP_TRY(hipMemcpyAsync(sa.opt.snapshots + snap * A->m, sa.alpha,
                                        sizeof(double) * (size_t)A->m, hipMemcpyDeviceToDevice,
                                        st));
    }
    return KDCD_OK;
}

// ------------------------------------------------------------ graph replay
// KDCD_FLAG_GRAPH: the whole enqueue sequence of a call is captured once on a
// private stream of the device into a hipGraph, instantiated and kept in a
// small process-wide cache keyed by every argument of the call; identical
// later calls launch the instantiated graph on the caller's stream.  A cache
// entry owns its workspace unless the caller passed one.  Device memory is
// cleared by kernels, never by memset nodes.  Calls in graph mode are
// serialised by one mutex, held until the call's status is read.

struct GraphEntry {
    std::string key;
    int device = -1;
    hipGraphExec_t exec = nullptr;
    char *ws = nullptr;
    bool owned = false;
    uint64_t used = 0;
};

struct GraphCache {
    std::mutex mu;
    std::vector<GraphEntry> entries;
    hipStream_t capture[64] = {};
    uint64_t tick = 0;
};

GraphCache &graph_cache()
{
    static GraphCache c;
    return c;
}

constexpr size_t kGraphCacheSize = 8;

void drop_entry(GraphEntry &e)
{
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.owned && e.ws) (void)hipFree(e.ws);
    e.exec = nullptr;
    e.ws = nullptr;
}

struct KeyBuilder {
    std::string k;
    template <class T> void add(const T &v) { k.append(reinterpret_cast<const char *>(&v), sizeof(T)); }
    void matrix(const kdcd_matrix *A)
    {
        add(A->format); add(A->m); add(A->n); add(A->ld); add(A->nnz);
        add(A->values); add(A->row_ptr); add(A->col_idx);
    }
    void kernel(const kdcd_kernel *k) { add(k->kind); add(k->degree); add(k->sigma); add(k->c); }
    void options(const kdcd_options &o)
    {
        add(o.compute); add(o.loss); add(o.snapshot_every); add(o.snapshots); add(o.trace);
        add(o.workspace); add(o.workspace_bytes);
    }
};

// The cache entry of `key` on the current device, captured and instantiated
// on first use (with c.mu held): prepare(base) is synchronous set-up before
// the capture (host-to-device copies of data the graph reads); enqueue(base,
// stream) is the work to capture.
GraphEntry *graph_entry(GraphCache &c, const std::string &key, size_t bytes,
                        const kdcd_options &opt,
                        const std::function<kdcd_status(char *)> &prepare,
                        const std::function<kdcd_status(char *, hipStream_t)> &enqueue,
                        kdcd_status &rc)
{
    rc = KDCD_OK;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        rc = KDCD_ERR_HIP;
        return nullptr;
    }
    for (auto &x : c.entries)
        if (x.device == dev && x.key == key) {
            x.used = ++c.tick;
            return &x;
        }
    if (!c.capture[dev] &&
        hipStreamCreateWithFlags(&c.capture[dev], hipStreamNonBlocking) != hipSuccess) {
        rc = KDCD_ERR_HIP;
        return nullptr;
    }
    GraphEntry ne;
    ne.key = key;
    ne.device = dev;
    if (opt.workspace) {
        if (opt.workspace_bytes < bytes) rc = KDCD_ERR_WORKSPACE;
        else if (reinterpret_cast<uintptr_t>(opt.workspace) & 255) rc = KDCD_ERR_INVALID_ARG;
        else ne.ws = static_cast<char *>(opt.workspace);
        if (rc != KDCD_OK) return nullptr;
    } else {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess || !p) {
            rc = KDCD_ERR_ALLOC;
            return nullptr;
        }
        ne.ws = static_cast<char *>(p);
        ne.owned = true;
    }
    rc = prepare ? prepare(ne.ws) : KDCD_OK;
    hipGraph_t g = nullptr;
    if (rc == KDCD_OK) {
        if (hipStreamBeginCapture(c.capture[dev], hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = KDCD_ERR_HIP;
        } else {
            rc = enqueue(ne.ws, c.capture[dev]);
            const hipError_t ce = hipStreamEndCapture(c.capture[dev], &g);
            if (rc == KDCD_OK && ce != hipSuccess) rc = KDCD_ERR_HIP;
        }
    }
    if (rc == KDCD_OK && hipGraphInstantiate(&ne.exec, g, nullptr, nullptr, 0) != hipSuccess)
        rc = KDCD_ERR_HIP;
    if (g) (void)hipGraphDestroy(g);
    if (rc != KDCD_OK) {
        drop_entry(ne);
        return nullptr;
    }
    if (c.entries.size() >= kGraphCacheSize) {   // least recently used goes
        size_t lru = 0;
        for (size_t i = 1; i < c.entries.size(); ++i)
            if (c.entries[i].used < c.entries[lru].used) lru = i;
        drop_entry(c.entries[lru]);
        c.entries.erase(c.entries.begin() + (std::ptrdiff_t)lru);
    }
    ne.used = ++c.tick;
    c.entries.push_back(ne);
    return &c.entries.back();
}

// A whole call captured as one graph and replayed by calls with identical
// arguments.
kdcd_status run_graph(const std::string &key, size_t bytes, const kdcd_options &opt,
                      hipStream_t st, const std::function<kdcd_status(char *)> &prepare,
                      const std::function<kdcd_status(char *, hipStream_t)> &enqueue)
{
    GraphCache &c = graph_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    kdcd_status rc = KDCD_OK;
    GraphEntry *e = graph_entry(c, key, bytes, opt, prepare, enqueue, rc);
    if (!e) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (opt.profile) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, st);
    }
    if (hipGraphLaunch(e->exec, st) != hipSuccess) return KDCD_ERR_HIP;
    if (opt.profile) (void)hipEventRecord(e1, st);
    rc = read_status(reinterpret_cast<int32_t *>(e->ws), st);
    if (opt.profile) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *opt.profile = kdcd_profile{};
        opt.profile->total_ms = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return rc;
}

// Host copy of the monitor's outcome into the caller's outputs.
kdcd_status report_monitor(const kdcd_options &o, const MonitorState *dmon, int64_t n_outer,
                           hipStream_t st)
{
    MonitorState h{};
    KDCD_HIP_TRY(hipMemcpyAsync(&h, dmon, sizeof(MonitorState), hipMemcpyDeviceToHost, st));
    KDCD_HIP_TRY(hipStreamSynchronize(st));
    if (o.outer_done) *o.outer_done = h.stop ? h.outer_done : n_outer;
    if (o.rel_err) *o.rel_err = h.rel;
    return KDCD_OK;
}

kdcd_status check_monitor(const kdcd_matrix *A, const kdcd_options &o)
{
    if (o.monitor_every < 0) return KDCD_ERR_INVALID_ARG;
    if (o.monitor_every == 0) return KDCD_OK;
    if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return KDCD_ERR_INVALID_ARG;
    if (o.monitor_log_len < 0 || (o.monitor_log_len > 0 && !o.monitor_log))
        return KDCD_ERR_INVALID_ARG;
    if (o.flags & KDCD_FLAG_GRAPH) return KDCD_ERR_UNSUPPORTED;
    // the U store of the product: FP64 (dense or CSR) and the single-problem
    // low-precision products; not the FP32 product
    if (A->format == KDCD_CSR ? o.compute != KDCD_F64 : o.compute == KDCD_F32)
        return KDCD_ERR_UNSUPPORTED;
    return KDCD_OK;
}

// Graph replay by windows of kGraphWindow outer iterations: one graph holds a
// window -- a kernel that copies the window's index blocks from idx into a
// buffer, the block index taken from a counter in device memory and moved on
// by the same kernel, then the window's launches reading that buffer -- and
// is replayed window after window; the set-up, the first outer iteration and
// the iterations after the last whole window (the ragged one included) run
// eagerly around the replays, in the graph's own workspace.  The graph does
// not depend on H or on the index values, so calls that differ only in those
// share it.  Used for solves without trace or snapshots and with at least
// kGraphWindow + 2 whole blocks; returns KDCD_ERR_UNSUPPORTED otherwise (the
// whole call is then captured instead).
constexpr int32_t kGraphWindow = 16;

kdcd_status run_graph_windowed(const SolveArgs &sa, const Layout &L)
{
    const int64_t sbw = (int64_t)sa.s * sa.b;
    const int64_t n_full = sa.H / sa.s;
    if (sa.opt.trace || sa.opt.snapshot_every > 0 || sa.opt.workspace || sa.opt.profile ||
        n_full < kGraphWindow + 2)
        return KDCD_ERR_UNSUPPORTED;
    const int64_t nwin = (n_full - 2) / kGraphWindow;
    const size_t o_cnt = L.total;
    const size_t o_win = o_cnt + 256;
    const size_t bytes = o_win + align256(sizeof(int32_t) * (size_t)((kGraphWindow + 2) * sbw));
    KeyBuilder kb;
    kb.add('W');
    kb.add(sa.problem);
    kb.matrix(sa.A);
    kb.add(sa.y);
    kb.kernel(sa.kernel);
    kb.add(sa.C); kb.add(sa.lambda); kb.add(sa.b); kb.add(sa.s);
    kb.add(sa.idx); kb.add(sa.alpha);
    kb.options(sa.opt);
    GraphCache &c = graph_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    kdcd_status rc = KDCD_OK;
    GraphEntry *e = graph_entry(
        c, kb.k, bytes, sa.opt, nullptr,
        [&](char *base, hipStream_t cs) {
            int64_t *cnt = reinterpret_cast<int64_t *>(base + o_cnt);
            int32_t *win = reinterpret_cast<int32_t *>(base + o_win);
            KDCD_HIP_TRY(launch_window_advance(sa.idx, cnt, win, kGraphWindow, (int32_t)sbw, cs));
            SolveArgs g = sa;
            g.st = cs;
            StageTimer off;
            SolveRange R;
            R.k_begin = 1;
            R.k_end = 1 + kGraphWindow;
            R.setup = false;
            R.S_base = win;
            return enqueue_solve(g, L, base, off, R);
        },
        rc);
    if (!e) return rc;
    StageTimer off;
    SolveRange head;                       // set-up and the first outer iteration
    head.k_end = 1;
    if ((rc = enqueue_solve(sa, L, e->ws, off, head)) != KDCD_OK) return rc;
    int32_t *cnt = reinterpret_cast<int32_t *>(e->ws + o_cnt);   // the counter's two words: 1, 0
    KDCD_HIP_TRY(launch_fill_i32(cnt, 1, 1, sa.st));
    KDCD_HIP_TRY(launch_fill_i32(cnt + 1, 0, 1, sa.st));
    for (int64_t w = 0; w < nwin; ++w)
        if (hipGraphLaunch(e->exec, sa.st) != hipSuccess) return KDCD_ERR_HIP;
    SolveRange tail;
    tail.k_begin = 1 + nwin * kGraphWindow;
    tail.setup = false;
    if ((rc = enqueue_solve(sa, L, e->ws, off, tail)) != KDCD_OK) return rc;
    return read_status(reinterpret_cast<int32_t *>(e->ws + L.status), sa.st);
}

kdcd_status run_solve(const SolveArgs &sa)
{
    kdcd_status rc = check_monitor(sa.A, sa.opt);
    if (rc != KDCD_OK) return rc;
    Layout L = make_layout(sa.problem, sa.A, sa.kernel, sa.b, sa.s, sa.opt.compute);
    if (sa.opt.monitor_every > 0) {
        add_monitor(L, sa.A->m, (int64_t)sa.s * sa.b);
        // the lookahead loop keeps two stored kernel blocks (not in a caller's
        // workspace, whose size kdcd_workspace_bytes gives without it)
        if (L.la_ok && !sa.opt.workspace && !(sa.opt.flags & KDCD_FLAG_SERIAL)) {
            L.mon_U2 = L.total;
            L.total += align256(sizeof(double) * (size_t)((int64_t)sa.s * sa.b * sa.A->m));
        }
    }
    if (sa.opt.flags & KDCD_FLAG_GRAPH) {
        rc = run_graph_windowed(sa, L);
        if (rc != KDCD_ERR_UNSUPPORTED) return rc;
        KeyBuilder kb;
        kb.add('S');
        kb.add(sa.problem);
        kb.matrix(sa.A);
        kb.add(sa.y);
        kb.kernel(sa.kernel);
        kb.add(sa.C); kb.add(sa.lambda); kb.add(sa.b); kb.add(sa.s); kb.add(sa.H);
        kb.add(sa.idx); kb.add(sa.alpha);
        kb.options(sa.opt);
        return run_graph(kb.k, L.total, sa.opt, sa.st, nullptr,
                         [&](char *base, hipStream_t cs) {
                             SolveArgs g = sa;
                             g.st = cs;
                             StageTimer off;
                             return enqueue_solve(g, L, base, off);
                         });
    }
    Workspace ws;
    if ((rc = acquire(ws, L, &sa.opt, sa.st)) != KDCD_OK) return rc;
    SolveArgs sx = sa;
    if (sa.A->format == KDCD_CSR && sa.A->m > 0) {
        // the longest row (one reduction and a wait at the start of the call),
        // so that chunks which cannot overflow the dense-head panel skip the
        // gated broadcast launch (kept by graph calls, which cannot wait)
        unsigned long long *dmax = reinterpret_cast<unsigned long long *>(ws.at<char>(L.status) + 8);
        unsigned long long hmax = ~0ull;
        KDCD_HIP_TRY(launch_csr_row_max(sa.A, dmax, sa.st));
        KDCD_HIP_TRY(hipMemcpyAsync(&hmax, dmax, sizeof(hmax), hipMemcpyDeviceToHost, sa.st));
        KDCD_HIP_TRY(hipStreamSynchronize(sa.st));
        if (hmax <= (unsigned long long)sa.A->n) sx.csr_max_row = (int64_t)hmax;
    }
    StageTimer timer;
    timer.on = sa.opt.profile != nullptr;
    rc = enqueue_solve(sx, L, ws.base, timer);
    if (rc != KDCD_OK) {
        (void)hipStreamSynchronize(sa.st);
        return rc;
    }
    rc = read_status(ws.at<int32_t>(L.status), sa.st);
    timer.report(sa.opt.profile);
    if (rc == KDCD_OK && sa.opt.monitor_every > 0)
        rc = report_monitor(sa.opt, ws.at<MonitorState>(L.mon), (sa.H + sa.s - 1) / sa.s, sa.st);
    return rc;
}

kdcd_status common_checks(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                          int32_t b, int32_t s, int64_t H, const int32_t *idx, double *alpha,
                          const kdcd_options *opt)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if (!y || !idx || !alpha) return KDCD_ERR_INVALID_ARG;
    if (b < 1 || s < 1 || H < 1) return KDCD_ERR_INVALID_ARG;
    if (b > A->m) return KDCD_ERR_INVALID_ARG;
    if (opt) {
        if ((rc = check_compute(A, opt->compute)) != KDCD_OK) return rc;
        if (opt->snapshot_every < 0) return KDCD_ERR_INVALID_ARG;
        if (opt->snapshot_every > 0 && !opt->snapshots) return KDCD_ERR_INVALID_ARG;
        if (opt->flags & ~(KDCD_FLAG_GRAPH | KDCD_FLAG_TIME_PRODUCT | KDCD_FLAG_TIME_SAMPLE |
                           KDCD_FLAG_LOOKAHEAD | KDCD_FLAG_SERIAL))
            return KDCD_ERR_INVALID_ARG;
    }
    if ((int64_t)s * b > kMaxSB) return KDCD_ERR_UNSUPPORTED;
    return KDCD_OK;
}

kdcd_options defaults(const kdcd_options *opt)
{
    kdcd_options o{};
    if (opt) o = *opt;
    if (o.loss == 0) o.loss = 1;
    return o;
}

}  // namespace

extern "C" {

void kdcd_graph_cache_clear(void)
{
    GraphCache &c = graph_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto &e : c.entries) drop_entry(e);
    c.entries.clear();
}

kdcd_status kdcd_ksvm_solve(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                            double C, int32_t b, int32_t s, int64_t H, const int32_t *idx,
                            double *alpha, const kdcd_options *opt, kdcd_stream stream)
{
    kdcd_status rc = common_checks(A, y, kernel, b, s, H, idx, alpha, opt);
    if (rc != KDCD_OK) return rc;
    if (!finite_pos(C)) return KDCD_ERR_INVALID_ARG;
    if (b != 1) return KDCD_ERR_INVALID_ARG;
    kdcd_options o = defaults(opt);
    if (o.loss != 1 && o.loss != 2) return KDCD_ERR_INVALID_ARG;
    SolveArgs sa{0, A, y, kernel, C, 0.0, b, s, H, idx, alpha, o, (hipStream_t)stream};
    return run_solve(sa);
}

kdcd_status kdcd_krr_solve(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                           double lambda, int32_t b, int32_t s, int64_t H, const int32_t *idx,
                           double *alpha, const kdcd_options *opt, kdcd_stream stream)
{
    kdcd_status rc = common_checks(A, y, kernel, b, s, H, idx, alpha, opt);
    if (rc != KDCD_OK) return rc;
    if (!finite_pos(lambda)) return KDCD_ERR_INVALID_ARG;
    if (b > kMaxB) return KDCD_ERR_UNSUPPORTED;
    // one recurrence wave per panel of floor(64/b)*b elements; wide blocks keep <= 512 threads
    const int nt = krr_recur_threads(b, s);
    if (nt > 1024 || (b > 16 && nt > 512)) return KDCD_ERR_UNSUPPORTED;
    kdcd_options o = defaults(opt);
    SolveArgs sa{1, A, y, kernel, 0.0, lambda, b, s, H, idx, alpha, o, (hipStream_t)stream};
    return run_solve(sa);
}

kdcd_status kdcd_batch_solve(const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t b,
                             int32_t s, int64_t H, const int32_t *idx,
                             const kdcd_batch_problem *problems, int32_t n_problems,
                             const kdcd_options *opt, kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if (!kernel || kernel->kind < KDCD_KERNEL_LINEAR || kernel->kind > KDCD_KERNEL_RBF)
        return KDCD_ERR_INVALID_ARG;
    if (!idx || !problems || n_problems < 1 || b < 1 || s < 1 || H < 1 || b > A->m)
        return KDCD_ERR_INVALID_ARG;
    if (n_problems > kMaxProblems || (int64_t)s * b > kMaxSB) return KDCD_ERR_UNSUPPORTED;
    kdcd_options o = defaults(opt);
    if ((rc = check_compute(A, o.compute)) != KDCD_OK) return rc;
    if (A->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    if (o.snapshot_every != 0 || o.trace) return KDCD_ERR_INVALID_ARG;   // per problem instead
    if ((rc = check_monitor(A, o)) != KDCD_OK) return rc;
    const bool monitor = o.monitor_every > 0;
    if (monitor && o.compute != KDCD_F64) return KDCD_ERR_UNSUPPORTED;   // FP64 stores U

    // sigma groups and problem lists
    BatchDesc bd{};
    std::vector<int> krr, svm;
    if ((rc = describe_batch(kernel, problems, n_problems, bd, krr, svm)) != KDCD_OK) return rc;
    const bool rbf = kernel->kind == KDCD_KERNEL_RBF;
    if (!krr.empty()) {
        if (b > kMaxB) return KDCD_ERR_UNSUPPORTED;
        const int nt = krr_recur_threads(b, s);
        if (nt > 1024 || (b > 16 && nt > 512)) return KDCD_ERR_UNSUPPORTED;
    }

    // workspace: single-problem layout plus the per-problem / per-sigma buffers
    const hipStream_t st = (hipStream_t)stream;
    const int64_t sbmax = (int64_t)s * b;
    Layout L = make_layout(0, A, kernel, b, s, o.compute);
    size_t off = L.total;
    const size_t o_bd = off; off += align256(sizeof(BatchDesc));
    const int64_t max_groups = max_row_groups(A);
    const size_t o_part = off; off += align256(sizeof(double) * (size_t)(n_problems * max_groups * sbmax));
    const size_t o_r = off; off += align256(sizeof(double) * (size_t)(n_problems * sbmax));
    const size_t o_W = off; off += align256(sizeof(double) * (size_t)(bd.ngroups * sbmax * sbmax));
    const size_t o_D = off; off += align256(sizeof(double) * (size_t)(krr.size() * sbmax * b + 1));
    // monitor: U per sigma group, per problem the dual vector, the updates, a
    // state and partial sums; the batch's state; an m-vector of scratch
    size_t o_U = 0, o_v = 0, o_th = 0, o_mons = 0, o_mpart = 0, o_mon = 0, o_tmp = 0;
    const int64_t m = A->m;
    if (monitor) {
        o_U = off; off += align256(sizeof(double) * (size_t)(bd.ngroups * sbmax * m));
        o_v = off; off += align256(sizeof(double) * (size_t)(n_problems * m));
        o_th = off; off += align256(sizeof(double) * (size_t)(n_problems * sbmax));
        o_mons = off; off += align256(sizeof(MonitorState) * (size_t)n_problems);
        o_mpart = off; off += align256(monitor_partial_bytes() * (size_t)n_problems);
        o_mon = off; off += 256;
        o_tmp = off; off += align256(sizeof(double) * (size_t)m);
    }
    L.total = off;

    // the work of the call on stream cs in the workspace at wsbase (the
    // descriptor is written by a kernel, so a captured graph rewrites it on
    // every replay)
    auto enqueue = [&](char *wsbase, hipStream_t cs, bool graph, StageTimer &timer) -> kdcd_status {
    const hipStream_t st = cs;
    Workspace ws;            // a view: not owned
    ws.base = wsbase;
    kdcd_status rc = KDCD_OK;
    int32_t *status = ws.at<int32_t>(L.status);
    double *norms = ws.at<double>(L.norms);
    BatchDesc *dbd = ws.at<BatchDesc>(o_bd);
    double *partial = ws.at<double>(o_part);
    double *r = ws.at<double>(o_r);
    double *W = ws.at<double>(o_W);
    double *Dinv = ws.at<double>(o_D);

    (void)graph;
    KDCD_HIP_TRY(launch_copy_batch_desc(bd, dbd, st));
    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    KDCD_HIP_TRY(launch_validate(idx, H * b, A->m, nullptr, nullptr, 0, 0, 0.0, status, st));
    for (int p = 0; p < n_problems; ++p) {
        const kdcd_batch_problem &q = problems[p];
        const double nu = q.problem == 0 ? (q.loss == 2 ? INFINITY : q.param) : 0.0;
        KDCD_HIP_TRY(launch_validate(idx, 0, A->m, q.y, q.alpha, A->m, q.problem == 0 ? 0 : 1, nu,
                                     status, st));
    }
    if (rbf) KDCD_HIP_TRY(launch_norms(A, norms, st));

    KBlockArgs base{};
    base.A = A;
    base.norms = norms;
    base.kp = to_params(kernel);
    base.beta = problems[0].alpha;
    base.partial = partial;
    base.W = W;
    base.status = status;
    base.compute = o.compute;
    base.batch = dbd;
    KBlockArgs kb;
    if ((rc = prepare_lowp(base, L, ws, st, kb)) != KDCD_OK) return rc;

    const int64_t n_outer = (H + s - 1) / s;
    MonitorState *mons = monitor ? ws.at<MonitorState>(o_mons) : nullptr;
    MonitorState *bmon = monitor ? ws.at<MonitorState>(o_mon) : nullptr;
    double *mon_th = monitor ? ws.at<double>(o_th) : nullptr;
    std::unique_ptr<StopPoller> poll;
    if (monitor) {
        KDCD_HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(mons), 0,
                                     (int64_t)(sizeof(MonitorState) / 4) * n_problems, st));
        KDCD_HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(bmon), 0,
                                     (int64_t)(sizeof(MonitorState) / 4), st));
        KDCD_HIP_TRY(launch_monitor_start(bmon, o.monitor_log, o.monitor_log_len, st));
        for (int p = 0; p < n_problems; ++p) {
            const kdcd_batch_problem &q = problems[p];
            kdcd_kernel kp = *kernel;
            kp.sigma = q.sigma;
            const double om = (q.problem == 0 && q.loss == 2) ? 1.0 / (2.0 * q.param) : 0.0;
            rc = init_dual_vector(q.problem == 0 ? 0 : 1, A, &kp, q.y, q.alpha, om, q.param,
                                  ws.at<double>(o_v) + (int64_t)p * m, ws.at<double>(o_tmp),
                                  &bmon->pad, st);
            if (rc != KDCD_OK) return rc;
        }
        kb.U = ws.at<double>(o_U);
        kb.u_gstride = sbmax * m;
        kb.stop = &bmon->stop;
        poll.reset(new StopPoller(n_outer / o.monitor_every + 1));
    }
    const int32_t *stop = monitor ? &bmon->stop : nullptr;
    int64_t k = 0;
    for (; k < n_outer; ++k) {
        if (monitor && k > 0 && k % o.monitor_every == 0 && poll->stopped(k / o.monitor_every - 1))
            break;
        const int64_t done = k * s;
        const int32_t sk = (int32_t)std::min<int64_t>(s, H - done);
        const int32_t sb = sk * b;
        const int32_t *S = idx + done * b;
        kb.S = S;
        kb.sb = sb;
        const int32_t groups = (int32_t)bind_config(kb, true);
        timer.begin(0, st);
        KDCD_HIP_TRY(launch_kblock(kb, st));
        timer.end(0, st);

        timer.begin(1, st);
        FinishDesc fd{};
        fd.nprob = n_problems;
        fd.nkrr = (int32_t)krr.size();
        fd.groups = groups;
        fd.stop = stop;
        for (int p = 0; p < n_problems; ++p) {
            fd.partial[p] = partial + (int64_t)p * groups * sb;
            fd.r[p] = r + (int64_t)p * sb;
        }
        for (size_t kk = 0; kk < krr.size(); ++kk) {
            const int p = krr[kk];
            fd.W[kk] = W + (int64_t)bd.group[p] * sb * sb;
            fd.Dinv[kk] = Dinv + (int64_t)kk * sb * b;
            fd.inv_lambda[kk] = 1.0 / problems[p].param;
        }
        KDCD_HIP_TRY(launch_finish(fd, sb, b, sk, (double)A->m, status, st));
        timer.end(1, st);

        timer.begin(2, st);
        if (!krr.empty()) {
            KrrRecurDesc rd{};
            for (size_t kk = 0; kk < krr.size(); ++kk) {
                const int p = krr[kk];
                rd.r[kk] = r + (int64_t)p * sb;
                rd.W[kk] = W + (int64_t)bd.group[p] * sb * sb;
                rd.Dinv[kk] = Dinv + (int64_t)kk * sb * b;
                rd.y[kk] = problems[p].y;
                rd.alpha[kk] = problems[p].alpha;
                rd.trace[kk] = problems[p].trace ? problems[p].trace + done * b
                                                 : (monitor ? mon_th + (int64_t)p * sbmax : nullptr);
                rd.lambda[kk] = problems[p].param;
            }
            rd.stop = stop;
            KDCD_HIP_TRY(launch_krr_recur(rd, (int32_t)krr.size(), S, b, sk, A->m, (double)A->m,
                                          status, st));
        }
        if (!svm.empty()) {
            KsvmRecurDesc kd{};
            for (size_t qq = 0; qq < svm.size(); ++qq) {
                const int p = svm[qq];
                const kdcd_batch_problem &q = problems[p];
                kd.r[qq] = r + (int64_t)p * sb;
                kd.W[qq] = W + (int64_t)bd.group[p] * sb * sb;
                kd.y[qq] = q.y;
                kd.alpha[qq] = q.alpha;
                kd.trace[qq] = q.trace ? q.trace + done * b
                                       : (monitor ? mon_th + (int64_t)p * sbmax : nullptr);
                kd.nu[qq] = q.loss == 2 ? INFINITY : q.param;
                kd.omega[qq] = q.loss == 2 ? 1.0 / (2.0 * q.param) : 0.0;
            }
            kd.stop = stop;
            KDCD_HIP_TRY(launch_ksvm_recur(kd, (int32_t)svm.size(), S, sb, A->m, status, st));
        }
        timer.end(2, st);
        if (monitor) {
            // every sigma group's problems from one pass over its stored block
            for (int g = 0; g < bd.ngroups; ++g) {
                DualBatchDesc dd{};
                for (int p = 0; p < n_problems; ++p) {
                    if (bd.group[p] != g) continue;
                    const kdcd_batch_problem &q = problems[p];
                    const int i = dd.n++;
                    dd.theta[i] = q.trace ? q.trace + done * b : mon_th + (int64_t)p * sbmax;
                    dd.v[i] = ws.at<double>(o_v) + (int64_t)p * m;
                    if (q.problem == 0) {
                        dd.vscale[i] = q.y;
                        dd.wscale[i] = q.y;
                        dd.uscale[i] = 1.0;
                        dd.diag[i] = q.loss == 2 ? 1.0 / (2.0 * q.param) : 0.0;
                    } else {
                        dd.uscale[i] = -1.0 / q.param;
                        dd.diag[i] = -(double)m;
                    }
                }
                if (dd.n > 0)
                    KDCD_HIP_TRY(launch_dual_update_batch(ws.at<double>(o_U) + (int64_t)g * sbmax * m,
                                                          m, sb, S, dd, stop, st));
            }
            if ((k + 1) % o.monitor_every == 0 || k + 1 == n_outer) {
                for (int p = 0; p < n_problems; ++p) {
                    const kdcd_batch_problem &q = problems[p];
                    const double om = (q.problem == 0 && q.loss == 2) ? 1.0 / (2.0 * q.param) : 0.0;
                    // each problem's bound (never its own stop); the batch stops on the largest
                    KDCD_HIP_TRY(launch_monitor(q.problem == 0 ? 0 : 1, m, q.alpha, q.y,
                                                ws.at<double>(o_v) + (int64_t)p * m, om,
                                                q.loss == 2 ? 2 : 1, q.param, -1.0, k + 1,
                                                reinterpret_cast<double *>(ws.at<char>(o_mpart) +
                                                                           monitor_partial_bytes() * p),
                                                mons + p, st));
                }
                KDCD_HIP_TRY(launch_monitor_combine(mons, n_problems, o.tol, k + 1, bmon, st));
                KDCD_HIP_TRY(poll->post((k + 1) / o.monitor_every - 1, bmon, st));
            }
        }
    }
    if (monitor) rc = report_monitor(o, bmon, n_outer, st);
    return rc;
    };

    if (o.flags & KDCD_FLAG_GRAPH) {
        KeyBuilder key;
        key.add('B');
        key.matrix(A);
        key.kernel(kernel);
        key.add(b); key.add(s); key.add(H); key.add(idx); key.add(n_problems);
        for (int p = 0; p < n_problems; ++p) {
            const kdcd_batch_problem &q = problems[p];
            key.add(q.problem); key.add(q.loss); key.add(q.param); key.add(q.sigma);
            key.add(q.y); key.add(q.alpha); key.add(q.trace);
        }
        key.options(o);
        return run_graph(
            key.k, L.total, o, st, nullptr,
            [&](char *wsbase, hipStream_t cs) {
                StageTimer off;
                return enqueue(wsbase, cs, true, off);
            });
    }
    Workspace ws;
    if ((rc = acquire(ws, L, &o, st)) != KDCD_OK) return rc;
    StageTimer timer;
    timer.on = o.profile != nullptr;
    if ((rc = enqueue(ws.base, st, false, timer)) != KDCD_OK) return rc;
    rc = read_status(ws.at<int32_t>(L.status), st);
    timer.report(o.profile);
    return rc;
}

}  // extern "C"

static kdcd_status kernel_matvec(const kdcd_matrix *A, const kdcd_kernel *kernel,
                                 const double *beta, std::vector<double> *host, double *dev,
                                 hipStream_t st);

extern "C" {

kdcd_status kdcd_ksvm_solve_sampled(const kdcd_matrix *A, const double *y,
                                    const kdcd_kernel *kernel, double C, int32_t s, int64_t H,
                                    const kdcd_sampling *smp, double *alpha,
                                    const kdcd_options *opt, kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if (!y || !alpha || !smp || !smp->idx_out || !finite_pos(C) || s < 1 || H < 1)
        return KDCD_ERR_INVALID_ARG;
    kdcd_options o = defaults(opt);
    if (o.loss != 1 && o.loss != 2) return KDCD_ERR_INVALID_ARG;
    if (o.snapshot_every < 0 || (o.snapshot_every > 0 && !o.snapshots)) return KDCD_ERR_INVALID_ARG;
    if ((rc = check_compute(A, o.compute)) != KDCD_OK) return rc;
    if (A->format != KDCD_DENSE || o.compute != KDCD_F64) return KDCD_ERR_UNSUPPORTED;
    if (s > kMaxSB || A->m >= ((int64_t)1 << 31)) return KDCD_ERR_UNSUPPORTED;
    if (o.flags & KDCD_FLAG_GRAPH) return KDCD_ERR_UNSUPPORTED;   // host-side decisions inside
    if ((rc = check_monitor(A, o)) != KDCD_OK) return rc;
    const bool monitor = o.monitor_every > 0;
    const int64_t m = A->m;
    const int64_t n_outer = (H + s - 1) / s;
    if (n_outer > (int64_t)0xFFFFFFFF) return KDCD_ERR_UNSUPPORTED;
    const bool learned = smp->model != nullptr;
    if (learned) {
        if (!(smp->tau > 0.0) || !std::isfinite(smp->tau) ||
            !(smp->epsilon >= 0.0 && smp->epsilon <= 1.0))
            return KDCD_ERR_INVALID_ARG;
        if (smp->pool == 0 ? s > m : (smp->pool < s || smp->pool > SMP_MAX_POOL))
            return KDCD_ERR_INVALID_ARG;
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev != smp->model->device)
            return KDCD_ERR_INVALID_ARG;
    }
    const hipStream_t st = (hipStream_t)stream;
    const double nu = o.loss == 2 ? INFINITY : C;
    const double omega = o.loss == 2 ? 1.0 / (2.0 * C) : 0.0;

    Layout L = make_layout(0, A, kernel, 1, s, KDCD_F64);
    size_t off = L.total;
    const size_t o_g = off; off += align256(sizeof(double) * (size_t)m);
    const size_t o_U = off; off += align256(sizeof(double) * (size_t)(s * m));
    const size_t o_th = off; off += align256(sizeof(double) * (size_t)s);
    const size_t o_tmp = off; off += align256(sizeof(double) * (size_t)m);
    const size_t o_flag = off; off += 256;
    const size_t o_sel = off; off += align256(select_workspace_bytes(m));
    const size_t o_mon = off; off += 256;
    const size_t o_monp = off; off += align256(monitor_partial_bytes());
    L.total = off;
    Workspace ws;
    if ((rc = acquire(ws, L, &o, st)) != KDCD_OK) return rc;
    int32_t *status = ws.at<int32_t>(L.status);
    double *norms = ws.at<double>(L.norms);
    double *partial = ws.at<double>(L.partial);
    double *r = ws.at<double>(L.r);
    double *W = ws.at<double>(L.W);
    double *g = smp->grad_out ? smp->grad_out : ws.at<double>(o_g);
    double *U = ws.at<double>(o_U);
    double *theta = ws.at<double>(o_th);
    double *tmp = ws.at<double>(o_tmp);
    int32_t *flag = ws.at<int32_t>(o_flag);
    const SelectWs sel = select_workspace(ws.at<char>(o_sel), m);
    const KParams kp = to_params(kernel);
    MonitorState *mon = ws.at<MonitorState>(o_mon);
    const int32_t *stop = monitor ? &mon->stop : nullptr;
    KDCD_HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(mon), 0,
                                 (int64_t)(sizeof(MonitorState) / 4), st));
    KDCD_HIP_TRY(launch_monitor_start(mon, o.monitor_log, o.monitor_log_len, st));

    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    KDCD_HIP_TRY(launch_fill_i32(flag, 0, 1, st));
    KDCD_HIP_TRY(launch_validate(nullptr, 0, m, y, alpha, m, 0, nu, status, st));
    KDCD_HIP_TRY(launch_norms(A, norms, st));
    // g = Q alpha_0 - 1 + omega alpha_0; the kernel product only for a nonzero alpha_0
    KDCD_HIP_TRY(launch_product(y, alpha, m, tmp, flag, st));
    int32_t nonzero = 0;
    KDCD_HIP_TRY(hipMemcpyAsync(&nonzero, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    KDCD_HIP_TRY(hipStreamSynchronize(st));
    if (nonzero) {
        if ((rc = kernel_matvec(A, kernel, tmp, nullptr, g, st)) != KDCD_OK) return rc;
        KDCD_HIP_TRY(launch_grad_init(g, y, alpha, omega, m, g, st));
    } else {
        KDCD_HIP_TRY(launch_grad_init(nullptr, y, alpha, omega, m, g, st));
    }
    KDCD_HIP_TRY(launch_select_reset(sel, st));

    KBlockArgs kb{};
    kb.A = A;
    kb.norms = norms;
    kb.kp = kp;
    kb.beta = alpha;
    kb.beta_scale = y;
    kb.partial = partial;
    kb.W = W;
    kb.status = status;
    kb.compute = KDCD_F64;
    kb.U = U;
    kb.stop = stop;
    if (s >= kGatherMinSB) {
        kb.pos = ws.at<int32_t>(L.pos);
        KDCD_HIP_TRY(launch_fill_i32(kb.pos, -1, m, st));
    }

    StageTimer timer;
    timer.on = o.profile != nullptr;
    int64_t snap = 0;
    std::unique_ptr<StopPoller> poll;
    if (monitor) poll.reset(new StopPoller(n_outer / o.monitor_every + 1));
    int64_t k = 0;
    for (; k < n_outer; ++k) {
        if (monitor && k > 0 && k % o.monitor_every == 0 && poll->stopped(k / o.monitor_every - 1))
            break;
        const int64_t done = k * s;
        const int32_t sk = (int32_t)std::min<int64_t>(s, H - done);
        int32_t *S = smp->idx_out + done;
        timer.begin(2, st);
        SelectArgs a{};
        a.ws = sel;
        a.m = m;
        a.ns = sk;
        a.topk = learned;
        a.pool = learned ? smp->pool : 0;
        a.epsilon = smp->epsilon;
        a.tau = smp->tau;
        a.seed = smp->seed;
        a.outer = (uint32_t)k;
        a.params = learned ? smp->model->params : nullptr;
        a.alpha = alpha;
        a.g = g;
        a.norms = norms;
        a.y = y;
        a.kp = kp;
        a.invC = 1.0 / C;
        a.S = S;
        a.status = status;
        KDCD_HIP_TRY(launch_select(a, st));
        if (smp->features_out)
            KDCD_HIP_TRY(launch_features(S, sk, alpha, g, norms, y, kp, 1.0 / C,
                                         smp->features_out + 4 * done, st));
        timer.end(2, st);
        kb.prevS = kb.S;
        kb.prev_sb = kb.sb;
        kb.S = S;
        kb.sb = sk;
        const int64_t groups = bind_config(kb);
        timer.begin(0, st);
        KDCD_HIP_TRY(launch_kblock(kb, st));
        timer.end(0, st);
        timer.begin(1, st);
        FinishDesc fd{};
        fd.nprob = 1;
        fd.groups = (int32_t)groups;
        fd.partial[0] = partial;
        fd.r[0] = r;
        fd.stop = stop;
        KDCD_HIP_TRY(launch_finish(fd, sk, 1, sk, (double)m, status, st));
        timer.end(1, st);
        timer.begin(2, st);
        KsvmRecurDesc kd{};
        kd.r[0] = r;
        kd.W[0] = W;
        kd.y[0] = y;
        kd.alpha[0] = alpha;
        kd.trace[0] = theta;
        kd.nu[0] = nu;
        kd.omega[0] = omega;
        kd.stop = stop;
        KDCD_HIP_TRY(launch_ksvm_recur(kd, 1, S, sk, m, status, st));
        KDCD_HIP_TRY(launch_dual_update(U, m, sk, S, theta, y, 1.0, y, omega, g, stop, st));
        if (monitor && ((k + 1) % o.monitor_every == 0 || k + 1 == n_outer)) {
            KDCD_HIP_TRY(launch_monitor(0, m, alpha, y, g, omega, o.loss, C, o.tol, k + 1,
                                        ws.at<double>(o_monp), mon, st));
            KDCD_HIP_TRY(poll->post((k + 1) / o.monitor_every - 1, mon, st));
        }
        timer.end(2, st);
        if (o.trace)
            KDCD_HIP_TRY(hipMemcpyAsync(o.trace + done, theta, sizeof(double) * (size_t)sk,
                                        hipMemcpyDeviceToDevice, st));
        if (o.snapshot_every > 0 && ((k + 1) % o.snapshot_every == 0 || k + 1 == n_outer)) {
            KDCD_HIP_TRY(hipMemcpyAsync(o.snapshots + snap * m, alpha, sizeof(double) * (size_t)m,
                                        hipMemcpyDeviceToDevice, st));
            ++snap;
        }
    }
    if (k < n_outer && o.snapshot_every > 0) {   // stopped early: the rest hold the final iterate
        const int64_t rows = (n_outer + o.snapshot_every - 1) / o.snapshot_every;
        for (; snap < rows; ++snap)
            KDCD_HIP_TRY(hipMemcpyAsync(o.snapshots + snap * m, alpha, sizeof(double) * (size_t)m,
                                        hipMemcpyDeviceToDevice, st));
    }
    rc = read_status(status, st);
    timer.report(o.profile);
    if (rc == KDCD_OK && monitor) rc = report_monitor(o, mon, n_outer, st);
    return rc;
}

kdcd_status kdcd_autotune(const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t sb,
                          int32_t compute, int32_t reps, int32_t *best_id, double *best_us,
                          kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if (A->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    const int ncfg = kdcd_tune_configs(compute, nullptr, nullptr, nullptr, 0);
    if (ncfg == 0) return KDCD_ERR_UNSUPPORTED;
    if (sb < 1 || sb > kMaxSB || sb > A->m || reps < 1) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    Layout L = make_layout(0, A, kernel, 1, sb, compute);
    const size_t o_S = L.total;
    L.total += align256(sizeof(int32_t) * (size_t)sb);
    Workspace ws;
    if ((rc = acquire(ws, L, nullptr, st)) != KDCD_OK) return rc;
    int32_t *S = ws.at<int32_t>(o_S);
    std::vector<int32_t> hS((size_t)sb);
    for (int32_t j = 0; j < sb; ++j) hS[(size_t)j] = (int32_t)(((int64_t)j * A->m) / sb);
    KDCD_HIP_TRY(hipMemcpyAsync(S, hS.data(), sizeof(int32_t) * (size_t)sb, hipMemcpyHostToDevice, st));
    double *norms = ws.at<double>(L.norms);
    KDCD_HIP_TRY(launch_fill_i32(ws.at<int32_t>(L.status), 0, 1, st));
    KDCD_HIP_TRY(launch_norms(A, norms, st));
    KBlockArgs kb{};
    kb.A = A;
    kb.S = S;
    kb.sb = sb;
    kb.norms = norms;
    kb.kp = to_params(kernel);
    kb.beta = norms;                 // any finite m-vector
    kb.partial = ws.at<double>(L.partial);
    kb.status = ws.at<int32_t>(L.status);
    kb.compute = compute;
    // the low-precision products are timed alone (their Gram comes from the
    // FP64 kernel whatever the configuration)
    kb.W = compute == KDCD_F64 ? ws.at<double>(L.W) : nullptr;
    if (compute != KDCD_F64) {
        KBlockArgs low;
        if ((rc = prepare_lowp(kb, L, ws, st, low)) != KDCD_OK) return rc;
        kb = low;
    } else if (sb >= kGatherMinSB) {       // W from the U rows, as in the solves
        kb.pos = ws.at<int32_t>(L.pos);
        KDCD_HIP_TRY(launch_fill_i32(kb.pos, -1, A->m, st));
        kb.prevS = S;                      // every launch re-marks the same block
        kb.prev_sb = sb;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return KDCD_ERR_HIP;
    // three interleaved rounds; a configuration's time is its fastest round
    std::vector<double> tmin((size_t)ncfg, 0.0);
    rc = KDCD_OK;
    for (int round = 0; round < 3 && rc == KDCD_OK; ++round) {
        for (int id = 0; id < ncfg && rc == KDCD_OK; ++id) {
            kb.cfg = id;                   // timed by id; the table changes only at the end
            float ms = 0.f;
            if (launch_kblock(kb, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) {
                rc = KDCD_ERR_HIP;
                break;
            }
            for (int r = 0; r < reps && rc == KDCD_OK; ++r)
                if (launch_kblock(kb, st) != hipSuccess) rc = KDCD_ERR_HIP;
            if (rc != KDCD_OK || hipEventRecord(e1, st) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = KDCD_ERR_HIP;
                break;
            }
            const double t = 1e3 * (double)ms / reps;
            if (round == 0 || t < tmin[(size_t)id]) tmin[(size_t)id] = t;
        }
    }
    int best = -1;
    double best_t = 0.0;
    for (int id = 0; id < ncfg; ++id)
        if (best < 0 || tmin[(size_t)id] < best_t) {
            best = id;
            best_t = tmin[(size_t)id];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != KDCD_OK) return rc;
    tune_store(compute, A->n, sb, best);
    if ((rc = read_status(ws.at<int32_t>(L.status), st)) != KDCD_OK) return rc;
    if (best_id) *best_id = best;
    if (best_us) *best_us = best_t;
    return KDCD_OK;
}

kdcd_status kdcd_autotune_batch(const kdcd_matrix *A, const kdcd_kernel *kernel, int32_t sb,
                                const kdcd_batch_problem *problems, int32_t n_problems,
                                int32_t compute, int32_t reps, int32_t *best_id, double *best_us,
                                kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if (!kernel || kernel->kind < KDCD_KERNEL_LINEAR || kernel->kind > KDCD_KERNEL_RBF)
        return KDCD_ERR_INVALID_ARG;
    if (A->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    if ((rc = check_compute(A, compute)) != KDCD_OK) return rc;
    if (!problems || n_problems < 1 || sb < 1 || sb > A->m || reps < 1)
        return KDCD_ERR_INVALID_ARG;
    if (n_problems > kMaxProblems || sb > kMaxSB) return KDCD_ERR_UNSUPPORTED;
    const int32_t key = compute + KDCD_TUNE_BATCH;
    const int ncfg = kdcd_tune_configs(key, nullptr, nullptr, nullptr, 0);
    if (ncfg == 0) return KDCD_ERR_UNSUPPORTED;
    BatchDesc bd{};
    std::vector<int> krr, svm;
    if ((rc = describe_batch(kernel, problems, n_problems, bd, krr, svm)) != KDCD_OK) return rc;
    const hipStream_t st = (hipStream_t)stream;
    Layout L = make_layout(0, A, kernel, 1, sb, compute);
    size_t off = L.total;
    const size_t o_bd = off; off += align256(sizeof(BatchDesc));
    const int64_t max_groups = max_row_groups(A);
    const size_t o_part = off; off += align256(sizeof(double) * (size_t)(n_problems * max_groups * sb));
    const size_t o_W = off; off += align256(sizeof(double) * (size_t)(bd.ngroups * sb * sb));
    const size_t o_S = off; off += align256(sizeof(int32_t) * (size_t)sb);
    L.total = off;
    Workspace ws;
    if ((rc = acquire(ws, L, nullptr, st)) != KDCD_OK) return rc;
    int32_t *S = ws.at<int32_t>(o_S);
    std::vector<int32_t> hS((size_t)sb);
    for (int32_t j = 0; j < sb; ++j) hS[(size_t)j] = (int32_t)(((int64_t)j * A->m) / sb);
    KDCD_HIP_TRY(hipMemcpyAsync(S, hS.data(), sizeof(int32_t) * (size_t)sb, hipMemcpyHostToDevice, st));
    KDCD_HIP_TRY(hipMemcpyAsync(ws.at<BatchDesc>(o_bd), &bd, sizeof(BatchDesc),
                                hipMemcpyHostToDevice, st));
    KDCD_HIP_TRY(hipStreamSynchronize(st));          // bd and hS are host locals
    double *norms = ws.at<double>(L.norms);
    KDCD_HIP_TRY(launch_fill_i32(ws.at<int32_t>(L.status), 0, 1, st));
    if (kernel->kind == KDCD_KERNEL_RBF) KDCD_HIP_TRY(launch_norms(A, norms, st));
    KBlockArgs kb{};
    kb.A = A;
    kb.S = S;
    kb.sb = sb;
    kb.norms = norms;
    kb.kp = to_params(kernel);
    kb.beta = problems[0].alpha;
    kb.partial = ws.at<double>(o_part);
    kb.W = ws.at<double>(o_W);
    kb.status = ws.at<int32_t>(L.status);
    kb.compute = compute;
    kb.batch = ws.at<BatchDesc>(o_bd);
    KBlockArgs low;
    if ((rc = prepare_lowp(kb, L, ws, st, low)) != KDCD_OK) return rc;
    kb = low;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return KDCD_ERR_HIP;
    std::vector<double> tmin((size_t)ncfg, 0.0);
    for (int round = 0; round < 3 && rc == KDCD_OK; ++round) {
        for (int id = 0; id < ncfg && rc == KDCD_OK; ++id) {
            kb.cfg = id;
            float ms = 0.f;
            if (launch_kblock(kb, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess) {
                rc = KDCD_ERR_HIP;
                break;
            }
            for (int r = 0; r < reps && rc == KDCD_OK; ++r)
                if (launch_kblock(kb, st) != hipSuccess) rc = KDCD_ERR_HIP;
            if (rc != KDCD_OK || hipEventRecord(e1, st) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = KDCD_ERR_HIP;
                break;
            }
            const double t = 1e3 * (double)ms / reps;
            if (round == 0 || t < tmin[(size_t)id]) tmin[(size_t)id] = t;
        }
    }
    int best = -1;
    double best_t = 0.0;
    for (int id = 0; id < ncfg; ++id)
        if (best < 0 || tmin[(size_t)id] < best_t) {
            best = id;
            best_t = tmin[(size_t)id];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != KDCD_OK) return rc;
    if ((rc = read_status(ws.at<int32_t>(L.status), st)) != KDCD_OK) return rc;
    tune_store(key, A->n, sb, best);
    if (best_id) *best_id = best;
    if (best_us) *best_us = best_t;
    return KDCD_OK;
}

kdcd_status kdcd_kernel_rhs(const kdcd_matrix *A, const kdcd_kernel *kernel, const int32_t *S,
                            int32_t sb, const double *beta, const double *beta_scale, double *r,
                            double *W, int32_t compute, kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if ((rc = check_compute(A, compute)) != KDCD_OK) return rc;
    if (!S || !beta || !r || sb < 1) return KDCD_ERR_INVALID_ARG;
    if (sb > kMaxSB) return KDCD_ERR_UNSUPPORTED;
    const hipStream_t st = (hipStream_t)stream;
    const Layout L = make_layout(0, A, kernel, 1, sb, compute);
    Workspace ws;
    if ((rc = acquire(ws, L, nullptr, st)) != KDCD_OK) return rc;
    int32_t *status = ws.at<int32_t>(L.status);
    double *norms = ws.at<double>(L.norms);
    double *partial = ws.at<double>(L.partial);
    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    if (A->format == KDCD_CSR) KDCD_HIP_TRY(launch_validate_csr(A, status, st));
    KDCD_HIP_TRY(launch_validate(S, sb, A->m, nullptr, nullptr, 0, 0, 0.0, status, st));
    if (kernel->kind == KDCD_KERNEL_RBF) KDCD_HIP_TRY(launch_norms(A, norms, st));
    KBlockArgs base{};
    base.A = A;
    base.S = S;
    base.sb = sb;
    base.norms = norms;
    base.kp = to_params(kernel);
    base.beta = beta;
    base.beta_scale = beta_scale;
    base.partial = partial;
    base.W = W;
    base.status = status;
    base.compute = compute;
    if (W && A->format == KDCD_DENSE && compute == KDCD_F64 && sb >= kGatherMinSB) {
        base.pos = ws.at<int32_t>(L.pos);
        KDCD_HIP_TRY(launch_fill_i32(base.pos, -1, A->m, st));
    }
    if (A->format == KDCD_CSR) {
        base.carry = ws.at<double>(L.carry);
        base.csr_panel = ws.at<void>(L.panel);
        KDCD_HIP_TRY(launch_csr_panel_init(A, base.csr_panel, st));
    }
    KBlockArgs kb;
    if ((rc = prepare_lowp(base, L, ws, st, kb)) != KDCD_OK) return rc;
    const int64_t groups = bind_config(kb);
    KDCD_HIP_TRY(launch_kblock(kb, st));
    FinishDesc fd{};
    fd.nprob = 1;
    fd.groups = (int32_t)groups;
    fd.partial[0] = partial;
    fd.r[0] = r;
    KDCD_HIP_TRY(launch_finish(fd, sb, 1, 0, 0.0, status, st));
    return read_status(status, st);
}

// (K beta) for all rows, FP64, in column chunks of kMaxSB through the kernel-block path.
// The result goes to host memory (host != nullptr) or to device memory (dev).
static kdcd_status kernel_matvec(const kdcd_matrix *A, const kdcd_kernel *kernel,
                                 const double *beta, std::vector<double> *host, double *dev,
                                 hipStream_t st)
{
    const int64_t m = A->m;
    const int32_t chunk = kMaxSB;
    const Layout L = make_layout(2, A, kernel, 1, chunk, KDCD_F64);
    Workspace ws;
    kdcd_status rc = acquire(ws, L, nullptr, st);
    if (rc != KDCD_OK) return rc;
    int32_t *status = ws.at<int32_t>(L.status);
    double *norms = ws.at<double>(L.norms);
    double *partial = ws.at<double>(L.partial);
    double *r = ws.at<double>(L.r);
    int32_t *iota = ws.at<int32_t>(L.iota);
    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    if (A->format == KDCD_CSR) KDCD_HIP_TRY(launch_validate_csr(A, status, st));
    KDCD_HIP_TRY(launch_iota_i32(iota, m, st));
    if (kernel->kind == KDCD_KERNEL_RBF) KDCD_HIP_TRY(launch_norms(A, norms, st));
    if (host) host->assign((size_t)m, 0.0);
    for (int64_t c0 = 0; c0 < m; c0 += chunk) {
        const int32_t sb = (int32_t)std::min<int64_t>(chunk, m - c0);
        KBlockArgs a{};
        a.A = A;
        a.S = iota + c0;
        a.sb = sb;
        a.norms = norms;
        a.kp = to_params(kernel);
        a.beta = beta;
        a.partial = partial;
        a.W = nullptr;
        a.status = status;
        a.compute = KDCD_F64;
        if (A->format == KDCD_CSR) {
            a.carry = ws.at<double>(L.carry);
            a.csr_panel = ws.at<void>(L.panel);
            if (c0 == 0) KDCD_HIP_TRY(launch_csr_panel_init(A, a.csr_panel, st));
        }
        const int64_t groups = bind_config(a);
        KDCD_HIP_TRY(launch_kblock(a, st));
        FinishDesc fd{};
        fd.nprob = 1;
        fd.groups = (int32_t)groups;
        fd.partial[0] = partial;
        fd.r[0] = r;
        KDCD_HIP_TRY(launch_finish(fd, sb, 1, 0, 0.0, status, st));
        if (host)
            KDCD_HIP_TRY(hipMemcpyAsync(host->data() + c0, r, sizeof(double) * (size_t)sb,
                                        hipMemcpyDeviceToHost, st));
        else
            KDCD_HIP_TRY(hipMemcpyAsync(dev + c0, r, sizeof(double) * (size_t)sb,
                                        hipMemcpyDeviceToDevice, st));
    }
    return read_status(status, st);
}

static void copy_to_host(std::vector<double> &h, const double *d, int64_t m, hipStream_t st)
{
    h.assign((size_t)m, 0.0);
    (void)hipMemcpyAsync(h.data(), d, sizeof(double) * (size_t)m, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
}

kdcd_status kdcd_ksvm_eval(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                           double C, int32_t loss, const double *alpha, double *out,
                           kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if (!y || !alpha || !out || !finite_pos(C) || (loss != 1 && loss != 2)) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    std::vector<double> hy, ha;
    copy_to_host(hy, y, A->m, st);
    copy_to_host(ha, alpha, A->m, st);
    std::vector<double> beta((size_t)A->m);
    for (int64_t p = 0; p < A->m; ++p) beta[p] = hy[p] * ha[p];
    double *dbeta = nullptr;
    if (hipMalloc(&dbeta, sizeof(double) * (size_t)A->m) != hipSuccess) return KDCD_ERR_ALLOC;
    (void)hipMemcpy(dbeta, beta.data(), sizeof(double) * (size_t)A->m, hipMemcpyHostToDevice);
    std::vector<double> Kb;
    rc = kernel_matvec(A, kernel, dbeta, &Kb, nullptr, st);
    (void)hipFree(dbeta);
    if (rc != KDCD_OK) return rc;
    const double nu = loss == 2 ? INFINITY : C, omega = loss == 2 ? 1.0 / (2.0 * C) : 0.0;
    long double aQa = 0, sa = 0, sa2 = 0, hinge = 0;
    double kkt = 0.0;
    for (int64_t p = 0; p < A->m; ++p) {
        const double Qa = hy[p] * Kb[p];
        aQa += (long double)ha[p] * Qa;
        sa += ha[p];
        sa2 += (long double)ha[p] * ha[p];
        const double xi = std::max(0.0, 1.0 - Qa);
        hinge += loss == 2 ? (long double)xi * xi : xi;
        const double g = Qa - 1.0 + omega * ha[p];
        const double pg = ha[p] <= 0.0 ? std::min(0.0, g) : (ha[p] >= nu ? std::max(0.0, g) : g);
        kkt = std::max(kkt, std::fabs(pg));
    }
    const double f = (double)(0.5L * aQa - sa + (loss == 2 ? sa2 / (4.0L * C) : 0.0L));
    const double P = (double)(0.5L * aQa + (long double)C * hinge);
    out[0] = f;
    out[1] = P;
    out[2] = P + f;
    out[3] = kkt;
    return KDCD_OK;
}

kdcd_status kdcd_batch_eval(const kdcd_matrix *A, const kdcd_kernel *kernel,
                            const kdcd_batch_problem *problems, int32_t n_problems, double *out,
                            kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if (!kernel || kernel->kind < KDCD_KERNEL_LINEAR || kernel->kind > KDCD_KERNEL_RBF)
        return KDCD_ERR_INVALID_ARG;
    if (!problems || !out || n_problems < 1) return KDCD_ERR_INVALID_ARG;
    if (n_problems > kMaxProblems) return KDCD_ERR_UNSUPPORTED;
    if (A->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    BatchDesc bd{};
    std::vector<int> krr, svm;
    if ((rc = describe_batch(kernel, problems, n_problems, bd, krr, svm)) != KDCD_OK) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const int64_t m = A->m;
    const int32_t chunk = kMaxSB;
    Layout L = make_layout(2, A, kernel, 1, chunk, KDCD_F64);
    size_t off = L.total;
    const size_t o_bd = off; off += align256(sizeof(BatchDesc));
    const int64_t max_groups = max_row_groups(A);
    const size_t o_part = off; off += align256(sizeof(double) * (size_t)(n_problems * max_groups * chunk));
    const size_t o_r = off; off += align256(sizeof(double) * (size_t)(n_problems * chunk));
    L.total = off;
    Workspace ws;
    if ((rc = acquire(ws, L, nullptr, st)) != KDCD_OK) return rc;
    int32_t *status = ws.at<int32_t>(L.status);
    double *norms = ws.at<double>(L.norms);
    double *partial = ws.at<double>(o_part);
    double *r = ws.at<double>(o_r);
    int32_t *iota = ws.at<int32_t>(L.iota);
    BatchDesc *dbd = ws.at<BatchDesc>(o_bd);
    KDCD_HIP_TRY(hipMemcpyAsync(dbd, &bd, sizeof(BatchDesc), hipMemcpyHostToDevice, st));
    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    KDCD_HIP_TRY(launch_iota_i32(iota, m, st));
    if (kernel->kind == KDCD_KERNEL_RBF) KDCD_HIP_TRY(launch_norms(A, norms, st));
    // (K_p beta_p) for every problem: K_p is its sigma group's kernel, beta_p =
    // alpha_p (K-RR) or y_p o alpha_p (K-SVM); row chunks of the symmetric K
    std::vector<double> Kb((size_t)(n_problems * m), 0.0);
    std::vector<double> hr((size_t)(n_problems * chunk));
    for (int64_t c0 = 0; c0 < m; c0 += chunk) {
        const int32_t sb = (int32_t)std::min<int64_t>(chunk, m - c0);
        KBlockArgs a{};
        a.A = A;
        a.S = iota + c0;
        a.sb = sb;
        a.norms = norms;
        a.kp = to_params(kernel);
        a.beta = problems[0].alpha;
        a.partial = partial;
        a.W = nullptr;
        a.status = status;
        a.compute = KDCD_F64;
        a.batch = dbd;
        const int64_t groups = bind_config(a, true);
        KDCD_HIP_TRY(launch_kblock(a, st));
        FinishDesc fd{};
        fd.nprob = n_problems;
        fd.groups = (int32_t)groups;
        for (int p = 0; p < n_problems; ++p) {
            fd.partial[p] = partial + (int64_t)p * groups * sb;
            fd.r[p] = r + (int64_t)p * sb;
        }
        KDCD_HIP_TRY(launch_finish(fd, sb, 1, 0, 0.0, status, st));
        KDCD_HIP_TRY(hipMemcpyAsync(hr.data(), r, sizeof(double) * (size_t)(n_problems * sb),
                                    hipMemcpyDeviceToHost, st));
        KDCD_HIP_TRY(hipStreamSynchronize(st));
        for (int p = 0; p < n_problems; ++p)
            std::copy(hr.begin() + (int64_t)p * sb, hr.begin() + (int64_t)(p + 1) * sb,
                      Kb.begin() + (int64_t)p * m + c0);
    }
    if ((rc = read_status(status, st)) != KDCD_OK) return rc;
    for (int p = 0; p < n_problems; ++p) {
        const kdcd_batch_problem &q = problems[p];
        std::vector<double> hy, ha;
        copy_to_host(hy, q.y, m, st);
        copy_to_host(ha, q.alpha, m, st);
        const double *kb = Kb.data() + (int64_t)p * m;
        double *o = out + 4 * p;
        if (q.problem == 1) {
            long double aMa = 0, ya = 0, rr = 0;
            for (int64_t i = 0; i < m; ++i) {
                const double Ma = kb[i] / q.param + (double)m * ha[i];
                aMa += (long double)ha[i] * Ma;
                ya += (long double)hy[i] * ha[i];
                const double res = hy[i] - Ma;
                rr += (long double)res * res;
            }
            o[0] = (double)(0.5L * aMa - ya);
            o[1] = std::sqrt((double)rr);
            o[2] = o[3] = 0.0;
        } else {
            const int loss = q.loss == 2 ? 2 : 1;
            const double C = q.param;
            const double nu = loss == 2 ? INFINITY : C, omega = loss == 2 ? 1.0 / (2.0 * C) : 0.0;
            long double aQa = 0, sa = 0, sa2 = 0, hinge = 0;
            double kkt = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                const double Qa = hy[i] * kb[i];
                aQa += (long double)ha[i] * Qa;
                sa += ha[i];
                sa2 += (long double)ha[i] * ha[i];
                const double xi = std::max(0.0, 1.0 - Qa);
                hinge += loss == 2 ? (long double)xi * xi : xi;
                const double g = Qa - 1.0 + omega * ha[i];
                const double pg = ha[i] <= 0.0 ? std::min(0.0, g) : (ha[i] >= nu ? std::max(0.0, g) : g);
                kkt = std::max(kkt, std::fabs(pg));
            }
            const double f = (double)(0.5L * aQa - sa + (loss == 2 ? sa2 / (4.0L * C) : 0.0L));
            const double P = (double)(0.5L * aQa + (long double)C * hinge);
            o[0] = f;
            o[1] = P;
            o[2] = P + f;
            o[3] = kkt;
        }
    }
    return KDCD_OK;
}

kdcd_status kdcd_krr_eval(const kdcd_matrix *A, const double *y, const kdcd_kernel *kernel,
                          double lambda, const double *alpha, double *out, kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if (!y || !alpha || !out || !finite_pos(lambda)) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    std::vector<double> Ka, hy, ha;
    if ((rc = kernel_matvec(A, kernel, alpha, &Ka, nullptr, st)) != KDCD_OK) return rc;
    copy_to_host(hy, y, A->m, st);
    copy_to_host(ha, alpha, A->m, st);
    long double aMa = 0, ya = 0, rr = 0;
    const double m = (double)A->m;
    for (int64_t p = 0; p < A->m; ++p) {
        const double Ma = Ka[p] / lambda + m * ha[p];
        aMa += (long double)ha[p] * Ma;
        ya += (long double)hy[p] * ha[p];
        const double res = hy[p] - Ma;
        rr += (long double)res * res;
    }
    out[0] = (double)(0.5L * aMa - ya);
    out[1] = std::sqrt((double)rr);
    return KDCD_OK;
}

// ------------------------------------------------------------ low rank
// Nystrom factor and solves on an explicit factor Phi (K ~ Phi Phi^T).

kdcd_status kdcd_nystrom_features(const kdcd_matrix *A, const kdcd_kernel *kernel,
                                  const int32_t *L, int32_t r, double jitter,
                                  const kdcd_matrix *X, double *Phi, int64_t ldphi,
                                  kdcd_stream stream)
{
    kdcd_status rc = check_matrix(A);
    if (rc != KDCD_OK) return rc;
    if ((rc = check_kernel(kernel)) != KDCD_OK) return rc;
    if (A->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    if (X) {
        if ((rc = check_matrix(X)) != KDCD_OK) return rc;
        if (X->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
        if (X->n != A->n) return KDCD_ERR_INVALID_ARG;
    }
    if (!L || !Phi || r < 1 || r > A->m || ldphi < r) return KDCD_ERR_INVALID_ARG;
    if (r > kMaxRank) return KDCD_ERR_UNSUPPORTED;
    if (!std::isfinite(jitter) || jitter < 0.0) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    const kdcd_matrix *Xm = X ? X : A;
    const bool rbf = kernel->kind == KDCD_KERNEL_RBF;
    size_t off = 0;
    const size_t o_status = off; off += 256;
    const size_t o_na = off; off += rbf ? align256(sizeof(double) * (size_t)A->m) : 0;
    const size_t o_nx = off; off += (rbf && X) ? align256(sizeof(double) * (size_t)Xm->m) : 0;
    const size_t o_cw = off; off += align256(sizeof(double) * (size_t)r * (size_t)r);
    const size_t o_dinv = off; off += align256(sizeof(double) * 4096 * (size_t)((r + 63) / 64));
    const size_t o_part = off; off += lowrank_part_bytes();
    Layout L0{};
    L0.total = off;
    Workspace ws;
    if ((rc = acquire(ws, L0, nullptr, st)) != KDCD_OK) return rc;
    int32_t *status = ws.at<int32_t>(o_status);
    double *na = rbf ? ws.at<double>(o_na) : nullptr;
    double *nx = rbf ? (X ? ws.at<double>(o_nx) : na) : nullptr;
    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    if (rbf) {
        KDCD_HIP_TRY(launch_norms(A, na, st));
        if (X) KDCD_HIP_TRY(launch_norms(X, nx, st));
    }
    KDCD_HIP_TRY(launch_nystrom(A->values, A->ld, A->m, A->n, L, r, to_params(kernel), jitter, na,
                                Xm->values, Xm->ld, Xm->m, nx, X == nullptr, ws.at<double>(o_cw),
                                ws.at<double>(o_dinv), Phi, ldphi, ws.at<double>(o_part), lowrank_part_bytes(), status,
                                st));
    return read_status(status, st);
}

kdcd_status kdcd_lowrank_solve(int32_t problem, const kdcd_matrix *Phi, const double *y,
                               double param, int32_t b, int32_t s, int64_t H, const int32_t *idx,
                               double *alpha, double *z, const kdcd_options *opt,
                               kdcd_stream stream)
{
    if (problem != 0 && problem != 1) return KDCD_ERR_INVALID_ARG;
    kdcd_status rc = check_matrix(Phi);
    if (rc != KDCD_OK) return rc;
    if (Phi->format != KDCD_DENSE) return KDCD_ERR_UNSUPPORTED;
    if (Phi->n > kMaxRank) return KDCD_ERR_UNSUPPORTED;
    if (!y || !idx || !alpha || b < 1 || s < 1 || H < 1 || b > Phi->m) return KDCD_ERR_INVALID_ARG;
    if (!finite_pos(param)) return KDCD_ERR_INVALID_ARG;
    kdcd_options o = defaults(opt);
    if (o.snapshot_every < 0 || (o.snapshot_every > 0 && !o.snapshots)) return KDCD_ERR_INVALID_ARG;
    if (o.compute != KDCD_F64 || o.flags != 0 || o.monitor_every != 0 || o.workspace)
        return KDCD_ERR_UNSUPPORTED;
    if ((int64_t)s * b > kMaxSB) return KDCD_ERR_UNSUPPORTED;
    const bool svm = problem == 0;
    if (svm) {
        if (b != 1 || (o.loss != 1 && o.loss != 2)) return KDCD_ERR_INVALID_ARG;
    } else {
        if (b > kMaxB) return KDCD_ERR_UNSUPPORTED;
        const int nt = krr_recur_threads(b, s);
        if (nt > 1024 || (b > 16 && nt > 512)) return KDCD_ERR_UNSUPPORTED;
    }
    const hipStream_t st = (hipStream_t)stream;
    const int64_t m = Phi->m;
    const int32_t r = (int32_t)Phi->n;
    const int64_t sbmax = (int64_t)s * b;
    size_t off = 0;
    const size_t o_status = off; off += 256;
    const size_t o_v = off; off += align256(sizeof(double) * (size_t)sbmax);
    const size_t o_r = off; off += align256(sizeof(double) * (size_t)sbmax);
    const size_t o_W = off; off += align256(sizeof(double) * (size_t)(sbmax * sbmax));
    const size_t o_D = off; off += svm ? 0 : align256(sizeof(double) * (size_t)(sbmax * b));
    const size_t o_th = off; off += align256(sizeof(double) * (size_t)sbmax);
    const size_t o_z = off; off += align256(sizeof(double) * (size_t)r);
    const size_t o_zp = off; off += align256(sizeof(double) * (size_t)lowrank_zinit_chunks() * r);
    // partial Gram tiles of a split-K product: at most 64 slices of the lower tiles
    const int64_t gt = (sbmax + 63) / 64;
    const size_t part_bytes =
        std::min(lowrank_part_bytes(), sizeof(double) * 4096 * (size_t)(64 * gt * (gt + 1) / 2));
    const size_t o_part = off; off += align256(part_bytes);
    Layout L0{};
    L0.total = off;
    Workspace ws;
    if ((rc = acquire(ws, L0, nullptr, st)) != KDCD_OK) return rc;
    int32_t *status = ws.at<int32_t>(o_status);
    double *v = ws.at<double>(o_v), *rr = ws.at<double>(o_r), *W = ws.at<double>(o_W);
    double *Dinv = svm ? nullptr : ws.at<double>(o_D);
    double *zz = z ? z : ws.at<double>(o_z);
    const double nu = svm ? (o.loss == 2 ? INFINITY : param) : 0.0;
    const double omega = (svm && o.loss == 2) ? 1.0 / (2.0 * param) : 0.0;
    const double *coef = svm ? y : nullptr;

    StageTimer timer;
    timer.on = o.profile != nullptr;
    KDCD_HIP_TRY(launch_fill_i32(status, 0, 1, st));
    KDCD_HIP_TRY(launch_validate(idx, H * b, m, y, alpha, m, problem, nu, status, st));
    KDCD_HIP_TRY(launch_lowrank_z_init(Phi->values, Phi->ld, m, r, alpha, coef,
                                       ws.at<double>(o_zp), zz, st));
    const int64_t n_outer = (H + s - 1) / s;
    int64_t snap = 0;
    for (int64_t k = 0; k < n_outer; ++k) {
        const int64_t done = k * s;
        const int32_t sk = (int32_t)std::min<int64_t>(s, H - done);
        const int32_t sb = sk * b;
        const int32_t *S = idx + done * b;
        timer.begin(0, st);
        KDCD_HIP_TRY(launch_lowrank_block(Phi->values, Phi->ld, m, r, S, sb, zz, W, v,
                                          ws.at<double>(o_part), part_bytes, st));
        timer.end(0, st);
        timer.begin(1, st);
        FinishDesc fd{};
        fd.nprob = 1;
        fd.nkrr = svm ? 0 : 1;
        fd.groups = 1;
        fd.partial[0] = v;
        fd.r[0] = rr;
        fd.W[0] = W;
        fd.Dinv[0] = Dinv;
        fd.inv_lambda[0] = svm ? 0.0 : 1.0 / param;
        KDCD_HIP_TRY(launch_finish(fd, sb, b, sk, (double)m, status, st));
        timer.end(1, st);
        timer.begin(2, st);
        double *th = o.trace ? o.trace + done * b : ws.at<double>(o_th);
        if (svm) {
            KsvmRecurDesc kd{};
            kd.r[0] = rr;
            kd.W[0] = W;
            kd.y[0] = y;
            kd.alpha[0] = alpha;
            kd.trace[0] = th;
            kd.nu[0] = nu;
            kd.omega[0] = omega;
            KDCD_HIP_TRY(launch_ksvm_recur(kd, 1, S, sb, m, status, st));
        } else {
            KrrRecurDesc rd{};
            rd.r[0] = rr;
            rd.W[0] = W;
            rd.Dinv[0] = Dinv;
            rd.y[0] = y;
            rd.alpha[0] = alpha;
            rd.trace[0] = th;
            rd.lambda[0] = param;
            KDCD_HIP_TRY(launch_krr_recur(rd, 1, S, b, sk, m, (double)m, status, st));
        }
        KDCD_HIP_TRY(launch_lowrank_z_update(Phi->values, Phi->ld, m, r, S, sb, th, coef,
                                             ws.at<double>(o_zp), zz, st));
        timer.end(2, st);
        if (o.snapshot_every > 0 && ((k + 1) % o.snapshot_every == 0 || k + 1 == n_outer)) {
            KDCD_HIP_TRY(hipMemcpyAsync(o.snapshots + snap * m, alpha, sizeof(double) * (size_t)m,
                                        hipMemcpyDeviceToDevice, st));
            ++snap;
        }
    }
    rc = read_status(status, st);
    timer.report(o.profile);
    return rc;
}

size_t kdcd_workspace_bytes(int32_t problem, const kdcd_matrix *A, const kdcd_kernel *kernel,
                            int32_t b, int32_t s, int32_t compute)
{
    if (!A || b < 1 || s < 1 || (problem != 0 && problem != 1)) return 0;
    return make_layout(problem, A, kernel, b, s, compute).total;
}

const char *kdcd_status_string(kdcd_status st)
{
    switch (st) {
    case KDCD_OK: return "ok";
    case KDCD_ERR_INVALID_ARG: return "invalid argument";
    case KDCD_ERR_UNSUPPORTED: return "unsupported configuration";
    case KDCD_ERR_INDEX_RANGE: return "coordinate index out of range";
    case KDCD_ERR_INDEX_DUPLICATE: return "duplicate coordinate inside a K-RR block";
    case KDCD_ERR_NOT_SPD: return "block matrix not symmetric positive definite";
    case KDCD_ERR_NONFINITE: return "non-finite value";
    case KDCD_ERR_HIP: return "HIP runtime error";
    case KDCD_ERR_ALLOC: return "device allocation failed";
    case KDCD_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

const char *kdcd_version(void) { return "kdcd 0.1.0 gfx950"; }

}  // extern "C"
