// Dense FP64 kernel block on gfx950 MFMA (v_mfma_f64_16x16x4f64).
//
// One launch computes, for the index block S (sb sampled rows):
//   U-tiles:  P = A A_S^T (m x sb), the Table 1 map K = map(P) in the
//             epilogue, and the column sums partial[g][j] = sum_{p in group g}
//             K(a_p, a_{S_j}) beta_p -- the right-hand side U^T beta of
//             Algorithms 2 and 4 -- without ever writing U;
//   W-tiles:  W = K(A_S, A_S) (sb x sb), the sampled Gram V^T U; with a row
//             range (w_row0, w_rows) the rows are S[w_row0 .. w_row0 + w_rows)
//             instead (W then w_rows x sb: index blocks stored back to back
//             give the Gram of one block against the next in one launch).
// Both read the sampled rows straight from A through S (no gather pass).
//
// Tiling: a workgroup of WM x WN waves owns a BM x BN tile; each wave owns
// TM x TN MFMA blocks of 16 x 16.  K is walked in chunks of 16 doubles that
// are staged through LDS in "fragment-major" order, so every MFMA operand
// fetch is one contiguous 512-byte ds_read_b64 per wave.  Inside a chunk,
// MFMA step ks uses k = 4*(lane/16) + ks for both operands; any bijection of
// k works as long as A and B agree, and this one makes a thread's 4 doubles
// of a row contiguous in global memory.
#include "common.hpp"
#include "la_recur.hpp"

namespace kdcd {
namespace {

constexpr int BK = 16;

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// Logical tile id from the hardware block id: consecutive logical ids land
// on the same XCD (workgroups are dealt round-robin over the 8 XCDs), so the
// column tiles that share one row group of A share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int total)
{
    const int per = total / 8, rem = total % 8;
    const int x = bid % 8, w = bid / 8;
    return x < rem ? x * (per + 1) + w : rem * (per + 1) + (x - rem) * per + w;
}

// BATCH: several problems share the product (descriptor bd in device memory):
// the map runs once per sigma group, every problem reduces its own beta, and
// the Gram tiles are written once per group.  partial is then [p][group][sb]
// and W is [g][sb][sb].
// FULL: rows 16-byte aligned and n a multiple of BK, so every chunk is loaded
// with unconditional 16-byte loads (no per-element bounds branches, which also
// lets the compiler keep the next chunks' loads in flight across the stores).
// The batched epilogue keeps one row of kernel values per sigma group live; left
// to itself the compiler then settles on one wave per SIMD, so the batched
// variants ask for two (they still fit without spilling).  OCC > 0 asks for
// OCC waves per SIMD (the 64 x 64 tile at three: three 4-wave workgroups per
// CU, so that one's prologue and epilogue overlap the others' MFMA loops).
// LA: a lookahead launch (workgroup 0 runs la_recur for the previous block,
// workgroups 1 .. kLaLead - 1 return, the product's tiles follow; the product
// also stores the rows of la.pos's coordinates into la.QX).
template <int WM, int WN, int TM, int TN, int KIND, bool BATCH, bool FULL, int OCC, bool LA>
__global__ __launch_bounds__(64 * WM * WN)
__attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : (BATCH ? 2 : 1))))
void kblock_f64_kernel(
    const double *__restrict__ A, int64_t lda, int64_t m, int64_t n,
    const int32_t *__restrict__ S, int32_t sb, const double *__restrict__ norms, KParams kp,
    const double *__restrict__ beta, const double *__restrict__ bscale,
    double *__restrict__ partial, double *__restrict__ W, int32_t n_u_tiles,
    int32_t n_row_groups, int32_t n_w_tiles, int32_t n_tiles_n, int32_t aligned,
    const BatchDesc *__restrict__ bd, double *__restrict__ U, const int32_t *__restrict__ stop,
    const int32_t *__restrict__ pos, int64_t u_gstride, int32_t w_row0, int32_t w_rows,
    const LookaheadArgs la)
{
    if (stop && *stop) return;   // the solve has converged
    constexpr int NT = 64 * WM * WN;
    constexpr int BM = 16 * TM * WM;
    constexpr int BN = 16 * TN * WN;
    constexpr int SEGA = (BM * 4 + NT - 1) / NT;
    constexpr int SEGB = (BN * 4 + NT - 1) / NT;

    __shared__ double As[2][BM * BK];
    __shared__ double Bs[2][BN * BK];
    __shared__ double red[WM][BN];
    __shared__ double redb[BATCH ? kMaxProblems : 1][WM][BN];   // batched column sums

    if constexpr (LA) {
        static_assert(2 * BM * BK * 8 >= 24 * NT + 8 * (2 * kLaMaxB + 256) + NT / 4,
                      "the lookahead recurrence's LDS must fit the A buffers");
        if (blockIdx.x < kLaLead) {
            if (blockIdx.x == 0 && la.sb > 0) {
                char *smem = reinterpret_cast<char *>(&As[0][0]);
                if (la.b == 8) la_recur<NT, 8>(la, smem);
                else la_recur<NT, 0>(la, smem);
            }
            return;
        }
    }
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int total = n_tiles_n * (n_row_groups + n_w_tiles);
    // the leading workgroups of a lookahead launch are a multiple of 8, so
    // bid % 8 is still the XCD of the workgroup
    const int bid = LA ? (int)blockIdx.x - kLaLead : (int)blockIdx.x;
    const int L = xcd_remap(bid, total);
    const int cn = L % n_tiles_n;
    const int rg = L / n_tiles_n;
    const bool is_w = rg >= n_row_groups;
    if (is_w && W == nullptr) return;
    const int col0 = cn * BN;

    // sampled rows feeding the B operand (clamped so that every load is in bounds)
    const double *bptr[SEGB];
#pragma unroll
    for (int i = 0; i < SEGB; ++i) {
        const int seg = tid + i * NT;
        const int r = (seg < BN * 4) ? (seg >> 2) : 0;
        const int c = seg & 3;
        const int64_t j = clampi(col0 + r, 0, sb - 1);
        const int64_t row = clampi(S[j], 0, m - 1);
        bptr[i] = A + row * lda + 4 * c;
    }
    // per-lane output columns of this wave
    int64_t Sc[TN];
    double nb[TN];
    bool colok[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const int64_t gcol = col0 + (wn * TN + tn) * 16 + (lane & 15);
        colok[tn] = gcol < sb;
        Sc[tn] = clampi(S[clampi(gcol, 0, sb - 1)], 0, m - 1);
        nb[tn] = (KIND == KDCD_KERNEL_RBF) ? norms[Sc[tn]] : 0.0;
    }

    double colsum[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) colsum[tn] = 0.0;
    if constexpr (BATCH) {
        for (int x = tid; x < kMaxProblems * WM * BN; x += NT) (&redb[0][0][0])[x] = 0.0;
        __syncthreads();
    }

    const int rt_first = is_w ? rg - n_row_groups : rg;
    const int rt_end = is_w ? rt_first + 1 : n_u_tiles;
    const int rt_step = is_w ? 1 : n_row_groups;
    const int64_t nK = (n + BK - 1) / BK;

    for (int rt = rt_first; rt < rt_end; rt += rt_step) {
        const int64_t row0 = (int64_t)rt * BM;
        const double *aptr[SEGA];
#pragma unroll
        for (int i = 0; i < SEGA; ++i) {
            const int seg = tid + i * NT;
            const int r = (seg < BM * 4) ? (seg >> 2) : 0;
            const int c = seg & 3;
            int64_t row;
            if (is_w) row = clampi(S[w_row0 + clampi(row0 + r, 0, w_rows - 1)], 0, m - 1);
            else row = clampi(row0 + r, 0, m - 1);
            aptr[i] = A + row * lda + 4 * c;
        }

        d4 acc[TM][TN];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = d4{0.0, 0.0, 0.0, 0.0};

        // Two register stages: while chunk kc is multiplied out of one LDS buffer,
        // chunk kc+1 waits in registers for its turn to be stored into the other
        // buffer and chunk kc+2 is already in flight from memory.
        double ra0[SEGA][4], rb0[SEGB][4], ra1[SEGA][4], rb1[SEGB][4];
        auto load = [&](int64_t kc, double (&ra)[SEGA][4], double (&rb)[SEGB][4]) {
            const int64_t k0 = kc * BK;
#pragma unroll
            for (int i = 0; i < SEGA; ++i) {
                const int seg = tid + i * NT;
                const int64_t kk = k0 + 4 * (seg & 3);
                if (FULL || (aligned && kk + 4 <= n)) {
                    const d2 *p = reinterpret_cast<const d2 *>(aptr[i] + k0);
                    d2 x = p[0], y = p[1];
                    ra[i][0] = x[0]; ra[i][1] = x[1]; ra[i][2] = y[0]; ra[i][3] = y[1];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) ra[i][e] = (kk + e < n) ? aptr[i][k0 + e] : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < SEGB; ++i) {
                const int seg = tid + i * NT;
                const int64_t kk = k0 + 4 * (seg & 3);
                if (FULL || (aligned && kk + 4 <= n)) {
                    const d2 *p = reinterpret_cast<const d2 *>(bptr[i] + k0);
                    d2 x = p[0], y = p[1];
                    rb[i][0] = x[0]; rb[i][1] = x[1]; rb[i][2] = y[0]; rb[i][3] = y[1];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) rb[i][e] = (kk + e < n) ? bptr[i][k0 + e] : 0.0;
                }
            }
        };
        auto store = [&](int buf, const double (&ra)[SEGA][4], const double (&rb)[SEGB][4]) {
#pragma unroll
            for (int i = 0; i < SEGA; ++i) {
                const int seg = tid + i * NT;
                if (seg < BM * 4) {
                    const int r = seg >> 2, c = seg & 3;
                    double *dst = &As[buf][((r >> 4) * 16 + c) * 16 + (r & 15)];
#pragma unroll
                    for (int e = 0; e < 4; ++e) dst[e * 64] = ra[i][e];
                }
            }
#pragma unroll
            for (int i = 0; i < SEGB; ++i) {
                const int seg = tid + i * NT;
                if (seg < BN * 4) {
                    const int r = seg >> 2, c = seg & 3;
                    double *dst = &Bs[buf][((r >> 4) * 16 + c) * 16 + (r & 15)];
#pragma unroll
                    for (int e = 0; e < 4; ++e) dst[e * 64] = rb[i][e];
                }
            }
        };
        auto compute = [&](int buf) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                double a[TM], b[TN];
#pragma unroll
                for (int tm = 0; tm < TM; ++tm) a[tm] = As[buf][((wm * TM + tm) * 4 + ks) * 64 + lane];
#pragma unroll
                for (int tn = 0; tn < TN; ++tn) b[tn] = Bs[buf][((wn * TN + tn) * 4 + ks) * 64 + lane];
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn)
                        acc[tm][tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[tm], b[tn], acc[tm][tn], 0, 0, 0);
            }
        };

        if constexpr (FULL) {
            // Loads are unconditional (chunk indices clamped to the last chunk,
            // which is then read again and ignored): a conditional load would
            // make the compiler copy the stage registers around it and wait for
            // every load in flight, including the chunk just issued.
            // Whole pairs of chunks in the loop and an odd last chunk after it:
            // one loop exit, so the accumulators keep their registers across
            // the back-edge (a break between the two halves made the compiler
            // copy all of them, after waiting for the MFMA results, every pair).
            const int64_t last = nK - 1;
            load(0, ra0, rb0);
            load(last < 1 ? last : 1, ra1, rb1);
            store(0, ra0, rb0);
            lds_barrier();
            const int64_t npairs = nK / 2;
            for (int64_t pk = 0; pk < npairs; ++pk) {
                const int64_t kc = 2 * pk;
                load(kc + 2 < last ? kc + 2 : last, ra0, rb0);
                compute(0);
                store(1, ra1, rb1);          // chunk kc + 1 < nK
                lds_barrier();
                load(kc + 3 < last ? kc + 3 : last, ra1, rb1);
                compute(1);
                if (kc + 2 < nK) store(0, ra0, rb0);
                lds_barrier();
            }
            if (nK & 1) {                    // chunk nK - 1, in buffer 0
                compute(0);
                lds_barrier();
            }
        } else {
            // the same pair structure (one loop exit) with bounds-checked loads
            load(0, ra0, rb0);
            if (nK > 1) load(1, ra1, rb1);
            store(0, ra0, rb0);
            lds_barrier();
            const int64_t npairs = nK / 2;
            for (int64_t pk = 0; pk < npairs; ++pk) {
                const int64_t kc = 2 * pk;
                if (kc + 2 < nK) load(kc + 2, ra0, rb0);
                compute(0);
                store(1, ra1, rb1);          // chunk kc + 1 < nK
                lds_barrier();
                if (kc + 3 < nK) load(kc + 3, ra1, rb1);
                compute(1);
                if (kc + 2 < nK) store(0, ra0, rb0);
                lds_barrier();
            }
            if (nK & 1) {                    // chunk nK - 1, in buffer 0
                compute(0);
                lds_barrier();
            }
        }

        // epilogue: item v of MFMA output lane l is row (l/16) + 4v, column l%16 of its block
        if constexpr (BATCH) {
            const int ng = bd->ngroups, np = bd->nprob;
            // beta (times its scale) of every problem for this tile's rows, staged
            // once in the A operand buffers (free after the loop's last barrier)
            // instead of one round of global loads per problem
            static_assert(kMaxProblems * BM <= 2 * BM * BK, "staged beta must fit the A buffers");
            double *bsh = &As[0][0];
            if (!is_w) {
                for (int x = tid; x < np * BM; x += NT) {
                    const int p = x / BM;
                    const int64_t grow = row0 + (x - p * BM);
                    double bval = 0.0;
                    if (grow < m) {
                        bval = bd->beta[p][grow];
                        if (bd->bscale[p]) bval *= bd->bscale[p][grow];
                    }
                    bsh[x] = bval;
                }
                __syncthreads();
            }
            double na[TM][4];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t grow = row0 + (wm * TM + tm) * 16 + (lane >> 4) + 4 * v;
                    const int64_t rr = is_w ? clampi(S[clampi(grow, 0, sb - 1)], 0, m - 1)
                                            : clampi(grow, 0, m - 1);
                    na[tm][v] = (KIND == KDCD_KERNEL_RBF) ? norms[rr] : 0.0;
                }
            for (int g = 0; g < ng; ++g) {
                KParams kg = kp;
                kg.sigma = bd->sigma[g];
                double kv[TM][4][TN];
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t grow = row0 + (wm * TM + tm) * 16 + (lane >> 4) + 4 * v;
                        const int64_t rr = is_w ? clampi(S[clampi(grow, 0, sb - 1)], 0, m - 1) : grow;
                        const bool rok = is_w ? grow < sb : grow < m;
#pragma unroll
                        for (int tn = 0; tn < TN; ++tn)
                            kv[tm][v][tn] = (rok && colok[tn])
                                                ? kernel_map<KIND>(acc[tm][tn][v], na[tm][v], nb[tn],
                                                                   rr == Sc[tn], kg)
                                                : 0.0;
                    }
                if (is_w) {
#pragma unroll
                    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t grow = row0 + (wm * TM + tm) * 16 + (lane >> 4) + 4 * v;
#pragma unroll
                            for (int tn = 0; tn < TN; ++tn) {
                                const int64_t gcol = col0 + (wn * TN + tn) * 16 + (lane & 15);
                                if (grow < sb && colok[tn])
                                    W[((int64_t)g * sb + grow) * sb + gcol] = kv[tm][v][tn];
                            }
                        }
                    continue;
                }
                if (U) {             // the monitor's stored kernel block of group g
#pragma unroll
                    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t grow = row0 + (wm * TM + tm) * 16 + (lane >> 4) + 4 * v;
#pragma unroll
                            for (int tn = 0; tn < TN; ++tn) {
                                const int64_t gcol = col0 + (wn * TN + tn) * 16 + (lane & 15);
                                if (grow < m && colok[tn])
                                    U[(int64_t)g * u_gstride + gcol * m + grow] = kv[tm][v][tn];
                            }
                        }
                }
                for (int p = 0; p < np; ++p) {
                    if (bd->group[p] != g) continue;
                    double bv[TM][4];
#pragma unroll
                    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            bv[tm][v] = bsh[p * BM + (wm * TM + tm) * 16 + (lane >> 4) + 4 * v];
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn) {
                        double acc_p = 0.0;
#pragma unroll
                        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc_p += bv[tm][v] * kv[tm][v][tn];
                        acc_p = wave_sum_xor16_32(acc_p);
                        if (lane < 16) redb[p][wm][(wn * TN + tn) * 16 + lane] += acc_p;
                    }
                }
            }
            if (!is_w) __syncthreads();   // the staged beta is read before the next tile reuses As
        } else {
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t lrow = (wm * TM + tm) * 16 + (lane >> 4) + 4 * v;
                    const int64_t grow = row0 + lrow;
                    if (!is_w) {
                        if (grow < m) {
                            double bval = beta[grow];
                            if (bscale) bval *= bscale[grow];
                            const double na = (KIND == KDCD_KERNEL_RBF) ? norms[grow] : 0.0;
                            const int32_t wrow = pos ? pos[grow] : -1;   // row of W, if sampled
                            // row of QX, if the row is a coordinate of the previous block
                            const int32_t xrow = LA ? la.pos[grow] : -1;
#pragma unroll
                            for (int tn = 0; tn < TN; ++tn)
                                if (colok[tn]) {
                                    const double kv = kernel_map<KIND>(acc[tm][tn][v], na, nb[tn],
                                                                       grow == Sc[tn], kp);
                                    const int64_t gcol = col0 + (wn * TN + tn) * 16 + (lane & 15);
                                    colsum[tn] += bval * kv;
                                    if (U) U[gcol * m + grow] = kv;
                                    if (wrow >= 0 && wrow < sb) W[(int64_t)wrow * sb + gcol] = kv;
                                    if (LA && xrow >= 0 && xrow < la.sb)
                                        la.QX[(int64_t)xrow * sb + gcol] = kv;
                                }
                        }
                    } else if (grow < w_rows) {
                        const int64_t St = clampi(S[w_row0 + grow], 0, m - 1);
                        const double na = (KIND == KDCD_KERNEL_RBF) ? norms[St] : 0.0;
#pragma unroll
                        for (int tn = 0; tn < TN; ++tn) {
                            const int64_t gcol = col0 + (wn * TN + tn) * 16 + (lane & 15);
                            if (colok[tn])
                                W[grow * sb + gcol] = kernel_map<KIND>(acc[tm][tn][v], na, nb[tn],
                                                                       St == Sc[tn], kp);
                        }
                    }
                }
            }
        }
    }
    if (is_w) return;

    if constexpr (BATCH) {   // every problem: waves -> one partial row per group
        __syncthreads();
        const int np = bd->nprob;
        for (int x = tid; x < np * BN; x += NT) {
            const int p = x / BN, c = x % BN;
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < WM; ++w) s += redb[p][w][c];
            if (col0 + c < sb) partial[((int64_t)p * n_row_groups + rg) * sb + col0 + c] = s;
        }
        return;
    }
    // deterministic column reduction: lanes -> waves -> one partial row per group
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const double v = wave_sum_xor16_32(colsum[tn]);
        if (lane < 16) red[wm][(wn * TN + tn) * 16 + lane] = v;
    }
    __syncthreads();
    for (int c = tid; c < BN; c += NT) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WM; ++w) s += red[w][c];
        if (col0 + c < sb) partial[(int64_t)rg * sb + col0 + c] = s;
    }
}

// pos[] upkeep: clear the previous block's entries, then mark the new one
// (one workgroup, so the clears are ordered before the marks; the marks of a
// repeated row keep its largest position, so the table does not depend on the
// order of the stores).
__global__ __launch_bounds__(1024) void pos_set_kernel(int32_t *__restrict__ pos, int64_t m,
                                                       const int32_t *__restrict__ prevS,
                                                       int32_t prev_sb,
                                                       const int32_t *__restrict__ S, int32_t sb,
                                                       const int32_t *__restrict__ stop)
{
    if (stop && *stop) return;
    for (int t = threadIdx.x; t < prev_sb; t += blockDim.x) {
        const int32_t p = prevS[t];
        if (p >= 0 && p < m) pos[p] = -1;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < sb; t += blockDim.x) {   // a repeated row keeps its last t
        const int32_t p = S[t];
        if (p >= 0 && p < m) atomicMax(&pos[p], t);
    }
}

// Rows of W for repeated indices: row t copies the row written for S_t.
__global__ __launch_bounds__(256) void w_dup_kernel(double *__restrict__ W, int64_t m,
                                                    const int32_t *__restrict__ S, int32_t sb,
                                                    const int32_t *__restrict__ pos,
                                                    const int32_t *__restrict__ stop)
{
    if (stop && *stop) return;
    const int t = blockIdx.x;
    const int32_t p = S[t];
    if (p < 0 || p >= m) return;
    const int32_t r = pos[p];
    if (r == t || r < 0) return;
    for (int j = threadIdx.x; j < sb; j += blockDim.x)
        W[(int64_t)t * sb + j] = W[(int64_t)r * sb + j];
}

struct Cfg {
    int bm, bn;
};

constexpr int64_t kMaxRowGroups = 1024;

template <int WM, int WN, int TM, int TN, bool BATCH, int OCC = 0>
hipError_t launch_cfg(const KBlockArgs &a, hipStream_t st)
{
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    const kdcd_matrix *A = a.A;
    const int64_t n_u = a.w_only ? 0 : (A->m + BM - 1) / BM;
    const int64_t groups = n_u < kMaxRowGroups ? n_u : kMaxRowGroups;
    const int32_t w_rows = a.w_rows > 0 ? a.w_rows : a.sb;
    const int64_t n_w = (a.W && !a.pos) ? (w_rows + BM - 1) / BM : 0;
    if (groups + n_w == 0) return hipSuccess;
    const int64_t n_n = (a.sb + BN - 1) / BN;
    const int aligned = (A->ld % 2 == 0) && ((reinterpret_cast<uintptr_t>(A->values) & 15) == 0);
    const bool full = aligned && A->n % BK == 0;
    const bool la = !BATCH && a.la != nullptr;
    if (la && !(full && a.pos && a.la->b <= kLaMaxB && a.la->sb <= kLaEPT * 64 * WM * WN))
        return hipErrorInvalidValue;   // the caller checks lookahead_supported first
    const int64_t blocks = n_n * (groups + n_w) + (la ? kLaLead : 0);
    const LookaheadArgs lav = la ? *a.la : LookaheadArgs{};
    dim3 grid((unsigned)blocks), block(64 * WM * WN);
#define KDCD_LAUNCH_F(KIND, FULL, LA)                                                          \
    KDCD_TIMED_LAUNCH((kblock_f64_kernel<WM, WN, TM, TN, KIND, BATCH, FULL, OCC, LA>), grid, block, 0, \
                       st, A->values, A->ld, A->m, A->n, a.S, a.sb, a.norms, a.kp, a.beta,      \
                       a.beta_scale, a.partial, a.W, (int32_t)n_u, (int32_t)groups,            \
                       (int32_t)n_w, (int32_t)n_n, aligned, a.batch, a.U, a.stop,              \
                       BATCH ? nullptr : a.pos, a.u_gstride, a.w_row0, w_rows, lav)
#define KDCD_LAUNCH(KIND)                                                                      \
    do {                                                                                        \
        if (la) {                                                                               \
            if constexpr (!BATCH) KDCD_LAUNCH_F(KIND, true, true);                              \
        } else if (full) KDCD_LAUNCH_F(KIND, true, false);                                      \
        else KDCD_LAUNCH_F(KIND, false, false);                                                 \
    } while (0)
    switch (a.kp.kind) {
    case KDCD_KERNEL_LINEAR: KDCD_LAUNCH(KDCD_KERNEL_LINEAR); break;
    case KDCD_KERNEL_POLY: KDCD_LAUNCH(KDCD_KERNEL_POLY); break;
    default: KDCD_LAUNCH(KDCD_KERNEL_RBF); break;
    }
#undef KDCD_LAUNCH
#undef KDCD_LAUNCH_F
    return hipGetLastError();
}

}  // namespace

// Configurations of the batched launch (WM, WN, TM, TN): the mapped values of
// every sigma group stay in registers while the problems of the group are
// reduced, so the tiles stay small.
struct F64Cfg {
    int wm, wn, tm, tn;
};
constexpr F64Cfg kF64BatchCfgs[] = {
    {4, 1, 2, 1},   // 0: 128 x 16, 4 waves
    {4, 1, 2, 2},   // 1: 128 x 32, 4 waves
    {2, 2, 2, 2},   // 2: 64 x 64, 4 waves
    {4, 2, 2, 2},   // 3: 128 x 64, 8 waves
    {2, 2, 2, 1},   // 4: 64 x 32, 4 waves
};
constexpr int kF64BatchNumCfgs = sizeof(kF64BatchCfgs) / sizeof(kF64BatchCfgs[0]);

int f64_batch_default_id(int32_t sb)
{
    if (sb <= 16) return 0;
    if (sb <= 32) return 1;
    return 2;
}

// Configurations of the single-problem launch: (WM, WN, TM, TN).  The 8-wave
// shapes keep the 64 x 128 / 128 x 64 tile at two waves per SIMD.
constexpr F64Cfg kF64Cfgs[] = {
    {4, 1, 2, 1},   // 0: 128 x 16, 4 waves
    {4, 1, 2, 2},   // 1: 128 x 32, 4 waves
    {2, 2, 2, 2},   // 2: 64 x 64, 4 waves
    {2, 2, 2, 4},   // 3: 64 x 128, 4 waves
    {2, 4, 2, 2},   // 4: 64 x 128, 8 waves
    {4, 2, 2, 2},   // 5: 128 x 64, 8 waves
    {2, 2, 2, 2},   // 6: 64 x 64, 4 waves, built for three waves per SIMD
};
constexpr int kF64NumCfgs = sizeof(kF64Cfgs) / sizeof(kF64Cfgs[0]);

int f64_config_count() { return kF64NumCfgs; }

void f64_config_shape(int id, int *bm, int *bn, int *waves)
{
    const F64Cfg &c = kF64Cfgs[id];
    *bm = 16 * c.tm * c.wm;
    *bn = 16 * c.tn * c.wn;
    *waves = c.wm * c.wn;
}

// Built-in rule, used when the tuning table has no entry for (n, sb).
static int f64_default_id(int32_t sb)
{
    if (sb <= 16) return 0;
    if (sb <= 32) return 1;
    if (sb <= 64) return 2;
    return 6;
}

int f64_config_id(int64_t n, int32_t sb)
{
    const int id = tune_lookup(KDCD_F64, n, sb);
    return (id >= 0 && id < kF64NumCfgs) ? id : f64_default_id(sb);
}

int f64_batch_config_count() { return kF64BatchNumCfgs; }

void f64_batch_config_shape(int id, int *bm, int *bn, int *waves)
{
    const F64Cfg &c = kF64BatchCfgs[id >= 0 && id < kF64BatchNumCfgs ? id : 2];
    *bm = 16 * c.tm * c.wm;
    *bn = 16 * c.tn * c.wn;
    *waves = c.wm * c.wn;
}

int f64_batch_config_id(int64_t n, int32_t sb)
{
    const int id = tune_lookup(KDCD_F64 + KDCD_TUNE_BATCH, n, sb);
    return (id >= 0 && id < kF64BatchNumCfgs) ? id : f64_batch_default_id(sb);
}

int64_t kblock_f64_row_groups(int cfg, int64_t m, int64_t n, int32_t sb, bool batch)
{
    int bm;
    if (batch) {
        int bn, w;
        f64_batch_config_shape(cfg >= 0 && cfg < kF64BatchNumCfgs ? cfg : f64_batch_config_id(n, sb),
                               &bm, &bn, &w);
    } else {
        int bn, w;
        f64_config_shape(cfg >= 0 && cfg < kF64NumCfgs ? cfg : f64_config_id(n, sb), &bm, &bn, &w);
    }
    const int64_t n_u = (m + bm - 1) / bm;
    return n_u < kMaxRowGroups ? n_u : kMaxRowGroups;
}

// The three parts of a single-problem launch: the row-position update of the
// gathered-Gram mode, the product, and the copies of repeated Gram rows.
hipError_t launch_kblock_f64_pre(const KBlockArgs &a, hipStream_t st)
{
    if (a.batch || !(a.W && a.pos && !a.w_only)) return hipSuccess;
    hipLaunchKernelGGL(pos_set_kernel, dim3(1), dim3(1024), 0, st, a.pos, a.A->m, a.prevS,
                       a.prevS ? a.prev_sb : 0, a.S, a.sb, a.stop);
    return hipGetLastError();
}

hipError_t launch_kblock_f64_main(const KBlockArgs &a, hipStream_t st)
{
    if (a.batch) {
        switch (a.cfg >= 0 && a.cfg < kF64BatchNumCfgs ? a.cfg : f64_batch_config_id(a.A->n, a.sb)) {
        case 0: return launch_cfg<4, 1, 2, 1, true>(a, st);
        case 1: return launch_cfg<4, 1, 2, 2, true>(a, st);
        case 3: return launch_cfg<4, 2, 2, 2, true>(a, st);
        case 4: return launch_cfg<2, 2, 2, 1, true>(a, st);
        default: return launch_cfg<2, 2, 2, 2, true>(a, st);
        }
    }
    KBlockArgs b = a;
    if (!(a.W && a.pos && !a.w_only)) b.pos = nullptr;
    switch (a.cfg >= 0 && a.cfg < kF64NumCfgs ? a.cfg : f64_config_id(a.A->n, a.sb)) {
    case 0: return launch_cfg<4, 1, 2, 1, false>(b, st);
    case 1: return launch_cfg<4, 1, 2, 2, false>(b, st);
    case 2: return launch_cfg<2, 2, 2, 2, false>(b, st);
    case 3: return launch_cfg<2, 2, 2, 4, false>(b, st);
    case 4: return launch_cfg<2, 4, 2, 2, false>(b, st);
    case 6: return launch_cfg<2, 2, 2, 2, false, 3>(b, st);
    default: return launch_cfg<4, 2, 2, 2, false>(b, st);
    }
}

hipError_t launch_kblock_f64_post(const KBlockArgs &a, hipStream_t st)
{
    if (a.batch || !(a.W && a.pos && !a.w_only)) return hipSuccess;
    hipLaunchKernelGGL(w_dup_kernel, dim3((unsigned)a.sb), dim3(256), 0, st, a.W, a.A->m, a.S, a.sb,
                       a.pos, a.stop);
    return hipGetLastError();
}

hipError_t launch_kblock_f64(const KBlockArgs &a, hipStream_t st)
{
    hipError_t e = launch_kblock_f64_pre(a, st);
    if (e == hipSuccess) e = launch_kblock_f64_main(a, st);
    if (e == hipSuccess) e = launch_kblock_f64_post(a, st);
    return e;
}

}  // namespace kdcd
