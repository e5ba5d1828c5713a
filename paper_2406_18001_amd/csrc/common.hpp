// Internal declarations shared by the kdcd HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>

#include "kdcd.h"

namespace kdcd {

constexpr int kMaxSB = 1024;   // s*b limit: one recurrence workgroup holds a whole S_k
constexpr int kMaxB = 32;      // K-RR block size limit (block inverses live in LDS)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Kernel parameters as the device sees them.
struct KParams {
    int32_t kind;
    int32_t degree;
    double sigma;
    double c;
};

// Device status word: the first error code written wins.
__device__ inline void set_status(int32_t *status, int32_t code)
{
    if (status) atomicCAS(status, 0, code);
}

// Table 1 map applied to one inner product P = a_p . a_q.
//   na, nb: ||a_p||^2 and ||a_q||^2 (RBF only); same: p and q are the same
//   row, so the distance is exactly zero.
template <int KIND>
__device__ __forceinline__ double kernel_map(double P, double na, double nb, bool same,
                                             const KParams &kp)
{
    if constexpr (KIND == KDCD_KERNEL_LINEAR) {
        return P;
    } else if constexpr (KIND == KDCD_KERNEL_POLY) {
        double base = kp.c + P, r = base;
        for (int t = 1; t < kp.degree; ++t) r *= base;
        return r;
    } else {
        double d2 = same ? 0.0 : fmax(na + nb - 2.0 * P, 0.0);
        return exp(-kp.sigma * d2);
    }
}

template <int KIND>
__device__ __forceinline__ float kernel_map_f32(float P, float na, float nb, bool same,
                                                const KParams &kp)
{
    if constexpr (KIND == KDCD_KERNEL_LINEAR) {
        return P;
    } else if constexpr (KIND == KDCD_KERNEL_POLY) {
        float base = (float)kp.c + P, r = base;
        for (int t = 1; t < kp.degree; ++t) r *= base;
        return r;
    } else {
        float d2 = same ? 0.0f : fmaxf(na + nb - 2.0f * P, 0.0f);
        return expf(-(float)kp.sigma * d2);
    }
}

// Workgroup barrier that orders LDS only: outstanding global loads stay in
// flight across it (a plain __syncthreads() also waits for every global load).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders LDS accesses of one wave (its lanes exchange values through LDS).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__device__ __forceinline__ double wave_sum_xor16_32(double v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// ------------------------------------------------------------------ host side

// Kernel timing without marker packets: a profiled solve arms a start / stop
// event pair for the calling thread, and the next kernel started through
// KDCD_TIMED_LAUNCH records both in its own dispatch (hipExtLaunchKernelGGL);
// unarmed launches are plain hipLaunchKernelGGL launches.
struct ArmedEvents {
    hipEvent_t start;
    hipEvent_t stop;
};
ArmedEvents &armed_events();   // per host thread

#define KDCD_TIMED_LAUNCH(kernel, grid, block, shmem, st, ...)                                 \
    do {                                                                                        \
        ::kdcd::ArmedEvents &ev_ = ::kdcd::armed_events();                                      \
        if (ev_.start) {                                                                        \
            hipEvent_t a_ = ev_.start, b_ = ev_.stop;                                           \
            ev_.start = ev_.stop = nullptr;                                                     \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, a_, b_, 0, __VA_ARGS__);      \
        } else {                                                                                \
            hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                    \
        }                                                                                       \
    } while (0)

#define KDCD_HIP_TRY(expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return KDCD_ERR_HIP;           \
    } while (0)

constexpr int kMaxProblems = 32;   // problems of one batched solve
constexpr int kMaxSigmas = 8;      // distinct RBF widths of one batched solve

// Problems sharing one kernel block (passed by value to the kernel-block
// launch).  Problem p reduces K_{group[p]} against beta[p] (* bscale[p]);
// group g maps P with sigma[g].  partial is laid out [p][row group][sb], the
// Gram W [g][sb][sb].
struct BatchDesc {
    int32_t nprob;
    int32_t ngroups;
    double sigma[kMaxSigmas];
    const double *beta[kMaxProblems];
    const double *bscale[kMaxProblems];
    int32_t group[kMaxProblems];
};

// Arguments of one kernel-block launch (dense or CSR, any compute type).
struct LookaheadArgs;

struct KBlockArgs {
    const kdcd_matrix *A;
    const void *Alow;        // low-precision copy of A (F32/BF16/F16), or hi part (BF16X3)
    const void *Alow2;       // lo part (BF16X3)
    int64_t ldlow;           // leading dimension of the low-precision copies
    const float *normlow;    // row norms of the rounded data (mixed RBF)
    const int32_t *S;        // sb sampled rows
    int32_t sb;
    const double *norms;     // m row norms ||a_p||^2 (RBF), FP64
    KParams kp;
    const double *beta;      // m
    const double *beta_scale;// m or nullptr
    double *partial;         // [n_row_groups][sb]
    double *W;               // sb x sb or nullptr
    int32_t *status;
    int32_t compute;
    int32_t w_only;          // FP64 kernel: compute the Gram tiles only (no U-part)
    const BatchDesc *batch;  // non-null: batched epilogue (dense F64 and mixed kernels)
    double *U;               // dense F64 only: non-null stores K(a_p, a_{S_j}) at U[j*m + p]
    const int32_t *stop;     // dense F64 only: non-null and set -> the launch does nothing
    // dense F64 only: when non-null, W is taken from the U-part rows of the
    // sampled rows (no W tiles).  pos[p] is the position t of row p in S (one
    // of them for repeated rows) or -1; it must hold -1 everywhere except the
    // entries of prevS (the previous index block, prev_sb entries), which the
    // launch resets before marking S; rows of repeated indices are copied after.
    int32_t *pos;
    const int32_t *prevS;
    int32_t prev_sb;
    // CSR only: m + s*b doubles of scratch for sampled rows longer than the
    // LDS panel (their dot products are summed over pieces); null refuses them
    double *carry;
    // batched FP64 with the monitor: U of sigma group g at U + g * u_gstride
    int64_t u_gstride = 0;
    // CSR only: the dense-head panel (kblock_csr_panel_bytes(n) bytes, prepared
    // once with launch_csr_panel_init); null keeps the broadcast kernels
    void *csr_panel = nullptr;
    // CSR: the longest row of A (stored entries) when the caller knows it, else
    // -1; a chunk of sampled rows that cannot exceed the dense-head panel then
    // skips the broadcast launch that would only run for an overflowing chunk
    int64_t csr_max_row = -1;
    // dense single-problem FP64 product: tile configuration, resolved once by
    // the caller together with the row-group count the finish pass sums
    // (-1: looked up in the tuning table at launch)
    int32_t cfg = -1;
    // dense single-problem FP64 product with a gathered Gram: non-null runs the
    // K-RR lookahead launch described by *la (the recurrence of the previous
    // block in workgroup 0, the product storing QX)
    const LookaheadArgs *la = nullptr;
    // dense FP64 Gram tiles: their rows are S[w_row0 .. w_row0 + w_rows) (w_rows
    // <= 0: the sb rows of S), W is then w_rows x sb; the batched launch ignores it
    int32_t w_row0 = 0;
    int32_t w_rows = 0;
};

// K-RR lookahead (one problem, dense FP64, gathered Gram).  The recurrence of
// index block k needs nothing of the product of block k+1 and the product
// needs the iterate only through r_{k+1} = U_{k+1}^T alpha, which is linear in
// alpha.  So one launch runs both: workgroup 0 runs the recurrence of block k
// (Algorithm 4's inner loop, updates kept apart from alpha), the other
// workgroups the product of block k+1 against the iterate before those
// updates, storing as well the kernel rows of S_k's coordinates (QX).  The
// finish pass of block k+1 then adds QX^T (updates) to r_{k+1} and the updates
// to alpha.
constexpr int kLaMaxB = 8;   // largest block size b of the lookahead recurrence
constexpr int kLaEPT = 2;    // elements of S_k per recurrence thread: s*b <= 2 * threads
constexpr int kLaLead = 8;   // leading workgroups of a lookahead launch (one per XCD)
struct LookaheadArgs {
    const int32_t *S;        // S_k, sb entries
    int32_t sb, b, sk;
    const double *r;         // r_k, final
    const double *W;         // Gram of S_k, [sb][sb], repeated rows copied with lambda m added
    const double *Dinv;      // inverses of the diagonal blocks, [sk][b][b]
    const double *y;
    const double *alpha;     // iterate before block k (read only during the launch)
    double lambda, mdbl;
    // row -> position table of S_k: element t of a coordinate is its canonical
    // element when pos[S_t] == t (the coordinate's last element: the tables
    // are marked with atomicMax, so the canonical element, and with it the
    // order of the finish pass's sums, is the same in every run); the product
    // stores row QX[t] for it
    const int32_t *pos;
    double *Dc;              // per element: summed update of its coordinate (canonical), else 0
    int32_t *Sc;             // per element: its coordinate (canonical), else -1
    double *trace;           // per-element updates, or null
    int32_t *status;
    int64_t m;
    double *QX;              // [sb][sb of the product]: kernel rows of canonical elements
};

// Launchers (return hipError_t of the launch).
// Row groups of a dense FP64 launch with configuration cfg (single problem;
// cfg < 0: the tuning table's choice for (n, sb)) or of a batched launch.
int64_t kblock_f64_row_groups(int cfg, int64_t m, int64_t n, int32_t sb, bool batch = false);
// Tile configurations of the FP64 product and the process-wide tuning table.
int f64_config_count();
void f64_config_shape(int id, int *bm, int *bn, int *waves);
int f64_config_id(int64_t n, int32_t sb);
int tune_lookup(int32_t compute, int64_t n, int32_t sb);   // -1: no entry
void tune_store(int32_t compute, int64_t n, int32_t sb, int id);   // id < 0 removes
size_t kblock_csr_panel_bytes(int64_t n);
hipError_t launch_csr_panel_init(const kdcd_matrix *A, void *panel, hipStream_t st);
int64_t kblock_mixed_row_groups(int cfg, int64_t m, int64_t n, int32_t sb, int32_t compute,
                                bool batch);
// Tile configurations of the batched products, tuned under compute + KDCD_TUNE_BATCH.
int f64_batch_config_count();
void f64_batch_config_shape(int id, int *bm, int *bn, int *waves);
int f64_batch_config_id(int64_t n, int32_t sb);
int mixed_batch_config_count();
void mixed_batch_config_shape(int id, int *bm, int *bn, int *waves);
int mixed_batch_config_id(int32_t compute, int64_t n, int32_t sb);
// Single-problem bf16 / fp16 / bf16x3 product (32 x 32 x 16 MFMA tiles) and
// its tile configurations (tuning table entries under the compute id).
int lowp_config_count();
void lowp_config_shape(int id, int *bm, int *bn, int *waves);
int lowp_config_id(int32_t compute, int64_t n, int32_t sb);
int64_t kblock_lowp_row_groups(int cfg, int64_t m);
hipError_t launch_kblock_lowp(const KBlockArgs &a, hipStream_t st);
hipError_t launch_kblock_f64(const KBlockArgs &a, hipStream_t st);
// launch_kblock_f64 = pre (row positions of the gathered Gram) + main (the
// product) + post (repeated Gram rows); pre and post do nothing outside the
// gathered single-problem mode.
hipError_t launch_kblock_f64_pre(const KBlockArgs &a, hipStream_t st);
hipError_t launch_kblock_f64_main(const KBlockArgs &a, hipStream_t st);
hipError_t launch_kblock_f64_post(const KBlockArgs &a, hipStream_t st);
hipError_t launch_norms(const kdcd_matrix *A, double *norms, hipStream_t st);
// Per-problem arguments of the finish pass and of the recurrences; one entry
// per workgroup-problem (blockIdx.x), passed by value.
struct FinishDesc {
    int32_t nprob;          // problems whose r is reduced
    int32_t nkrr;           // K-RR problems whose diagonal blocks are inverted
    int32_t groups;         // row groups of the partial sums
    const double *partial[kMaxProblems];   // [groups][sb] each
    double *r[kMaxProblems];               // [sb] each
    const double *W[kMaxProblems];         // Gram of K-RR problem k, [sb][sb]
    double *Dinv[kMaxProblems];            // inverses of K-RR problem k, [sk][b][b]
    double inv_lambda[kMaxProblems];
    const int32_t *stop;    // non-null and set: the solve has converged, do nothing
    // Gathered Gram of one problem (dup_S non-null): the product wrote one row
    // per coordinate (row dup_pos[S_t]); rows of repeated coordinates are
    // copied from it by extra blocks, and the inversions read such rows'
    // diagonal entries from it
    const int32_t *dup_S;   // S_k, [sb]
    const int32_t *dup_pos; // row -> position table of S_k
    double *dup_W;          // the Gram, [sb][sb]
    int64_t m;
    // K-RR lookahead (la_Sc non-null): r also receives sum_t QX[t][j] Dc[t]
    // over the canonical elements t of the previous block (la_sb of them),
    // whose summed updates one extra workgroup then adds to alpha; the same
    // workgroup moves the row -> position table la_pos on (clears the entries
    // of la_clearS, then marks la_setS), when la_pos is non-null
    const double *la_QX;
    const double *la_Dc;
    const int32_t *la_Sc;
    int32_t la_sb;
    double *la_alpha;
    int32_t *la_pos;
    const int32_t *la_clearS;
    int32_t la_clear_sb;
    const int32_t *la_setS;
    int32_t la_set_sb;
    // non-zero: the copied Gram rows (the coordinates that come again later)
    // also get la_lm = lambda m at the columns of their coordinate's other
    // elements, the m term of G for the lookahead recurrence
    double la_lm;
};

struct KsvmRecurDesc {
    const double *r[kMaxProblems];
    const double *W[kMaxProblems];
    const double *y[kMaxProblems];
    double *alpha[kMaxProblems];
    double *trace[kMaxProblems];
    double nu[kMaxProblems];
    double omega[kMaxProblems];
    const int32_t *stop;
};

struct KrrRecurDesc {
    const double *r[kMaxProblems];
    const double *W[kMaxProblems];
    const double *Dinv[kMaxProblems];
    const double *y[kMaxProblems];
    double *alpha[kMaxProblems];
    double *trace[kMaxProblems];
    double lambda[kMaxProblems];
    const int32_t *stop;
    // One problem with a gathered Gram (pos non-null): after the scatter the
    // launch clears the row -> position table for its block and marks S_next
    // (sb_next entries; none after the last block) for the next product
    int32_t *pos;
    const int32_t *S_next;
    int32_t sb_next;
};

// Convergence monitor state (device): stop word first, so that &stop can be
// handed to kernels as a plain int32 pointer.
struct MonitorState {
    int32_t stop;
    int32_t pad;
    int64_t outer_done;   // outer iterations done at the last evaluation
    double rel;           // last certified relative objective error
    double f;             // last objective value
    uint64_t t0;          // device wall clock at the set-up
    double tick;          // seconds per wall-clock tick
    double *log;          // optional records {outer, rel, f, seconds} per evaluation
    int64_t log_len;
    int64_t nlog;         // evaluations so far
};

// Set-up after the state is zero-filled: start clock and the optional log.
hipError_t launch_monitor_start(MonitorState *mon, double *log, int64_t log_len, hipStream_t st);

hipError_t launch_dual_update(const double *U, int64_t m, int32_t sb, const int32_t *S,
                              const double *theta, const double *vscale, double uscale,
                              const double *wscale, double diag, double *v, const int32_t *stop,
                              hipStream_t st);
size_t monitor_partial_bytes();
// Batched gradient upkeep: one pass over U (sb x m, one sigma group) updates
// the dual vectors of every problem of the group, each with its own
// parameters (as launch_dual_update).
struct DualBatchDesc {
    int32_t n;
    const double *theta[kMaxProblems];
    const double *vscale[kMaxProblems];
    const double *wscale[kMaxProblems];
    double uscale[kMaxProblems];
    double diag[kMaxProblems];
    double *v[kMaxProblems];
};
hipError_t launch_dual_update_batch(const double *U, int64_t m, int32_t sb, const int32_t *S,
                                    const DualBatchDesc &d, const int32_t *stop, hipStream_t st);
// Batched monitor: the batch state takes the largest of the problems' last
// bounds (their states at mons[0 .. n)), stops once it is <= tol, and logs.
hipError_t launch_monitor_combine(const MonitorState *mons, int32_t n, double tol, int64_t outer,
                                  MonitorState *batch, hipStream_t st);
hipError_t launch_monitor(int32_t problem, int64_t m, const double *alpha, const double *y,
                          const double *v, double omega, int32_t loss, double C, double tol,
                          int64_t outer, double *part, MonitorState *mon, hipStream_t st);
hipError_t launch_rho_init(const double *Ka, const double *y, const double *alpha,
                           double inv_lambda, double mdbl, int64_t m, double *rho, hipStream_t st);

// r[j] += sum over the first occurrences t in prevS of X[t][j] * beta(prevS_t),
hipError_t launch_finish(const FinishDesc &d, int32_t sb, int32_t b, int32_t sk, double mdbl,
                         int32_t *status, hipStream_t st);
hipError_t launch_ksvm_recur(const KsvmRecurDesc &d, int32_t nprob, const int32_t *S, int32_t sb,
                             int64_t m, int32_t *status, hipStream_t st);
hipError_t launch_krr_recur(const KrrRecurDesc &d, int32_t nprob, const int32_t *S, int32_t b,
                            int32_t sk, int64_t m, double mdbl, int32_t *status, hipStream_t st);
hipError_t launch_validate(const int32_t *idx, int64_t count, int64_t m, const double *y,
                           const double *alpha, int64_t mrows, int32_t problem, double nu,
                           int32_t *status, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st);
hipError_t launch_copy_batch_desc(const BatchDesc &d, BatchDesc *dst, hipStream_t st);
hipError_t launch_window_advance(const int32_t *idx, int64_t *counter, int32_t *Swin, int32_t W,
                                 int32_t sb, hipStream_t st);
hipError_t launch_validate_csr(const kdcd_matrix *A, int32_t *status, hipStream_t st);
hipError_t launch_csr_row_max(const kdcd_matrix *A, unsigned long long *out, hipStream_t st);
hipError_t launch_iota_i32(int32_t *p, int64_t count, hipStream_t st);

}  // namespace kdcd
