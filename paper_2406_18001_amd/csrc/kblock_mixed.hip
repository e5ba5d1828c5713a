// Mixed-precision kernel block on gfx950 MFMA: P = A A_S^T with FP32 or
// 16-bit operands and FP32 accumulation, for the U-part only (the Gram W of
// the sampled rows always comes from the FP64 kernel).
//
//   F32     v_mfma_f32_16x16x4_f32   on an FP32 copy of A
//   BF16    v_mfma_f32_16x16x32_bf16 on a bf16 copy of A
//   F16     v_mfma_f32_16x16x32_f16  on an fp16 copy of A
//   BF16X3  A = hi + lo (both bf16, lo = bf16(A - hi)); P = hi.hi + hi.lo + lo.hi,
//           three bf16 MFMAs into the same FP32 accumulators (the dropped lo.lo
//           term is below FP32 rounding of P)
//
// The low-precision copies and the row norms of the rounded data (so that
// ||x||^2 + ||z||^2 - 2 x.z is consistent for the RBF map) are made once per
// solve by convert_kernel.  The map runs in FP32; beta, the column sums and r
// stay in FP64.
//
// Operands travel in 16-byte segments (4 floats or 8 halves of one row).  A
// chunk of K is 4 segments per row; LDS holds each tile in fragment-major
// order [16-row block][segment q][row i], so lane l = 16 q + i fetches its
// whole MFMA fragment with one ds_read_b128.  As in the FP64 kernel, k-slot
// assignment inside a chunk is the same for A and B, which is all the
// contraction needs.  Output item v of lane l is row 4 (l/16) + v, column l%16.
#include "common.hpp"
#include "la_recur.hpp"

namespace kdcd {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ int xcd_remap(int bid, int total)
{
    const int per = total / 8, rem = total % 8;
    const int x = bid % 8, w = bid / 8;
    return x < rem ? x * (per + 1) + w : rem * (per + 1) + (x - rem) * per + w;
}

// One 16-byte segment pair -> accumulator update.
template <int CMP>
__device__ __forceinline__ f4 mfma_seg(u4 a, u4 b, f4 acc)
{
    if constexpr (CMP == KDCD_F32) {
        const f4 af = __builtin_bit_cast(f4, a), bf = __builtin_bit_cast(f4, b);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[e], bf[e], acc, 0, 0, 0);
        return acc;
    } else if constexpr (CMP == KDCD_F16) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                      __builtin_bit_cast(h8, b), acc, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                       __builtin_bit_cast(bf8, b), acc, 0, 0, 0);
    }
}

// Elements per 16-byte segment.
template <int CMP> constexpr int seg_elems() { return CMP == KDCD_F32 ? 4 : 8; }

// BATCH: several problems share the product (see the FP64 kernel): the map
// runs once per sigma group and every problem reduces its own beta;
// partial is then [p][row group][sb].
// Every variant asks for at least two waves per SIMD (all fit without
// spilling; the 128 x 64 single-problem tile reaches three): left to itself the
// compiler runs the batched variants at one.
// LAH (single problem): a K-RR lookahead launch: workgroup 0 runs la_recur for
// the previous block, workgroups 1 .. kLaLead - 1 return, the tiles follow.
template <int CMP, int WM, int WN, int TM, int TN, int KIND, bool BATCH, bool LAH>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(2)))
void kblock_mixed_kernel(
    const u4 *__restrict__ Ahi, const u4 *__restrict__ Alo, int64_t ldseg, int64_t m,
    int64_t nseg, const float *__restrict__ normlow, const int32_t *__restrict__ S, int32_t sb,
    KParams kp, const double *__restrict__ beta, const double *__restrict__ bscale,
    double *__restrict__ partial, int32_t n_u_tiles, int32_t n_row_groups, int32_t n_tiles_n,
    const BatchDesc *__restrict__ bd, const LookaheadArgs la)
{
    constexpr bool X3 = CMP == KDCD_BF16X3;
    constexpr int NT = 64 * WM * WN;
    constexpr int BM = 16 * TM * WM;
    constexpr int BN = 16 * TN * WN;
    constexpr int SEGA = (BM * 4 + NT - 1) / NT;
    constexpr int SEGB = (BN * 4 + NT - 1) / NT;
    constexpr int NL = X3 ? 2 : 1;                 // hi (and lo) copies

    __shared__ u4 As[2][NL][BM * 4];
    __shared__ u4 Bs[2][NL][BN * 4];
    __shared__ double red[WM][BN];
    __shared__ double redb[BATCH ? kMaxProblems : 1][WM][BN];

    if constexpr (LAH) {
        static_assert((int)sizeof(As) >= 24 * NT + 8 * (2 * kLaMaxB + 256) + NT / 4,
                      "the lookahead recurrence's LDS must fit the A buffers");
        if (blockIdx.x < kLaLead) {
            if (blockIdx.x == 0 && la.sb > 0) {
                char *smem = reinterpret_cast<char *>(&As[0][0][0]);
                if (la.b == 8) la_recur<NT, 8>(la, smem);
                else la_recur<NT, 0>(la, smem);
            }
            return;
        }
    }
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int total = n_tiles_n * n_row_groups;
    // the leading workgroups of a lookahead launch are a multiple of 8, so
    // bid % 8 is still the XCD of the workgroup
    const int bid = LAH ? (int)blockIdx.x - kLaLead : (int)blockIdx.x;
    const int L = xcd_remap(bid, total);
    const int cn = L % n_tiles_n;
    const int rg = L / n_tiles_n;
    const int col0 = cn * BN;

    int64_t boff[SEGB];
#pragma unroll
    for (int i = 0; i < SEGB; ++i) {
        const int seg = tid + i * NT;
        const int r = (seg < BN * 4) ? (seg >> 2) : 0;
        const int64_t row = clampi(S[clampi(col0 + r, 0, sb - 1)], 0, m - 1);
        boff[i] = row * ldseg + (seg & 3);
    }
    int64_t Sc[TN];
    float nb[TN];
    bool colok[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const int64_t gcol = col0 + (wn * TN + tn) * 16 + (lane & 15);
        colok[tn] = gcol < sb;
        Sc[tn] = clampi(S[clampi(gcol, 0, sb - 1)], 0, m - 1);
        nb[tn] = (KIND == KDCD_KERNEL_RBF) ? normlow[Sc[tn]] : 0.0f;
    }
    double colsum[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) colsum[tn] = 0.0;
    if constexpr (BATCH) {
        for (int x = tid; x < kMaxProblems * WM * BN; x += NT) (&redb[0][0][0])[x] = 0.0;
        __syncthreads();
    }

    const int64_t nK = (nseg + 3) / 4;            // chunks of 4 segments per row
    for (int rt = rg; rt < n_u_tiles; rt += n_row_groups) {
        const int64_t row0 = (int64_t)rt * BM;
        int64_t aoff[SEGA];
#pragma unroll
        for (int i = 0; i < SEGA; ++i) {
            const int seg = tid + i * NT;
            const int r = (seg < BM * 4) ? (seg >> 2) : 0;
            aoff[i] = clampi(row0 + r, 0, m - 1) * ldseg + (seg & 3);
        }
        f4 acc[TM][TN];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = f4{0.f, 0.f, 0.f, 0.f};

        u4 ra0[NL][SEGA], rb0[NL][SEGB], ra1[NL][SEGA], rb1[NL][SEGB];
        auto load = [&](int64_t kc, u4 (&ra)[NL][SEGA], u4 (&rb)[NL][SEGB]) {
            const int64_t s0 = kc * 4;
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const u4 *src = h == 0 ? Ahi : Alo;
#pragma unroll
                for (int i = 0; i < SEGA; ++i) {
                    const int seg = tid + i * NT;
                    (void)seg;
                    ra[h][i] = src[aoff[i] + s0];
                }
#pragma unroll
                for (int i = 0; i < SEGB; ++i) {
                    const int seg = tid + i * NT;
                    (void)seg;
                    rb[h][i] = src[boff[i] + s0];
                }
            }
        };
        auto store = [&](int buf, const u4 (&ra)[NL][SEGA], const u4 (&rb)[NL][SEGB]) {
#pragma unroll
            for (int h = 0; h < NL; ++h) {
#pragma unroll
                for (int i = 0; i < SEGA; ++i) {
                    const int seg = tid + i * NT;
                    if (seg < BM * 4) {
                        const int r = seg >> 2, q = seg & 3;
                        As[buf][h][((r >> 4) * 4 + q) * 16 + (r & 15)] = ra[h][i];
                    }
                }
#pragma unroll
                for (int i = 0; i < SEGB; ++i) {
                    const int seg = tid + i * NT;
                    if (seg < BN * 4) {
                        const int r = seg >> 2, q = seg & 3;
                        Bs[buf][h][((r >> 4) * 4 + q) * 16 + (r & 15)] = rb[h][i];
                    }
                }
            }
        };
        auto compute = [&](int buf) {
            u4 a[NL][TM], b[NL][TN];
#pragma unroll
            for (int h = 0; h < NL; ++h) {
#pragma unroll
                for (int tm = 0; tm < TM; ++tm) a[h][tm] = As[buf][h][(wm * TM + tm) * 64 + lane];
#pragma unroll
                for (int tn = 0; tn < TN; ++tn) b[h][tn] = Bs[buf][h][(wn * TN + tn) * 64 + lane];
            }
#pragma unroll
            for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                for (int tn = 0; tn < TN; ++tn) {
                    acc[tm][tn] = mfma_seg<CMP>(a[0][tm], b[0][tn], acc[tm][tn]);
                    if constexpr (X3) {
                        acc[tm][tn] = mfma_seg<CMP>(a[0][tm], b[1][tn], acc[tm][tn]);
                        acc[tm][tn] = mfma_seg<CMP>(a[1][tm], b[0][tn], acc[tm][tn]);
                    }
                }
        };

        // The rounded copies are padded to whole chunks, so every chunk is
        // loaded unconditionally; chunk indices past the end are clamped to the
        // last chunk (read again, never stored), which keeps the compiler from
        // copying the stage registers around conditional loads and waiting for
        // every load in flight.
        // Whole pairs of chunks in the loop and an odd last chunk after it: one
        // loop exit, so the accumulators keep their registers across the
        // back-edge (as in the FP64 kernel).
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
            store(1, ra1, rb1);              // chunk kc + 1 < nK
            lds_barrier();
            load(kc + 3 < last ? kc + 3 : last, ra1, rb1);
            compute(1);
            if (kc + 2 < nK) store(0, ra0, rb0);
            lds_barrier();
        }
        if (nK & 1) {                        // chunk nK - 1, in buffer 0
            compute(0);
            lds_barrier();
        }

        // epilogue: item v of lane l is row 4 (l/16) + v, column l%16 of its block
        if constexpr (BATCH) {
            const int ng = bd->ngroups, np = bd->nprob;
            // beta (times its scale) of every problem for this tile's rows, staged
            // once in the A operand buffers (free after the loop's last barrier)
            // when they hold all problems (always for bf16x3, up to 16 problems
            // otherwise); else one round of global loads per problem
            constexpr int BSH_CAP = (int)(sizeof(As) / sizeof(double)) / BM;
            double *bsh = reinterpret_cast<double *>(&As[0][0][0]);
            const bool staged = np <= BSH_CAP;
            if (staged) {
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
            for (int g = 0; g < ng; ++g) {
                KParams kg = kp;
                kg.sigma = bd->sigma[g];
                float kv[TM][4][TN];
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t grow = row0 + (wm * TM + tm) * 16 + 4 * (lane >> 4) + v;
                        const float na = (KIND == KDCD_KERNEL_RBF) ? normlow[clampi(grow, 0, m - 1)] : 0.0f;
#pragma unroll
                        for (int tn = 0; tn < TN; ++tn)
                            kv[tm][v][tn] = (grow < m && colok[tn])
                                                ? kernel_map_f32<KIND>(acc[tm][tn][v], na, nb[tn],
                                                                       grow == Sc[tn], kg)
                                                : 0.0f;
                    }
                for (int p = 0; p < np; ++p) {
                    if (bd->group[p] != g) continue;
                    const double *bp = bd->beta[p];
                    const double *sp = bd->bscale[p];
                    double bv[TM][4];
                    if (staged) {
#pragma unroll
                        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                bv[tm][v] = bsh[p * BM + (wm * TM + tm) * 16 + 4 * (lane >> 4) + v];
                    } else {
#pragma unroll
                        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int64_t grow = row0 + (wm * TM + tm) * 16 + 4 * (lane >> 4) + v;
                                double x = 0.0;
                                if (grow < m) {
                                    x = bp[grow];
                                    if (sp) x *= sp[grow];
                                }
                                bv[tm][v] = x;
                            }
                    }
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn) {
                        double acc_p = 0.0;
#pragma unroll
                        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc_p += bv[tm][v] * (double)kv[tm][v][tn];
                        acc_p = wave_sum_xor16_32(acc_p);
                        if (lane < 16) redb[p][wm][(wn * TN + tn) * 16 + lane] += acc_p;
                    }
                }
            }
            if (staged) __syncthreads();   // the staged beta is read before the next tile reuses As
        } else {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t grow = row0 + (wm * TM + tm) * 16 + 4 * (lane >> 4) + v;
                if (grow < m) {
                    double bval = beta[grow];
                    if (bscale) bval *= bscale[grow];
                    const float na = (KIND == KDCD_KERNEL_RBF) ? normlow[grow] : 0.0f;
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn)
                        if (colok[tn])
                            colsum[tn] += bval * (double)kernel_map_f32<KIND>(acc[tm][tn][v], na, nb[tn],
                                                                              grow == Sc[tn], kp);
                }
            }
        }
        }
    }

    if constexpr (BATCH) {
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

// FP64 -> low-precision copy with the row padded to ldlow elements (zeros),
// and FP32 norms of the rounded rows.  One wave per row.
template <int CMP>
__global__ __launch_bounds__(256) void convert_kernel(const double *__restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n, int64_t ldlow,
                                                      void *__restrict__ hi, void *__restrict__ lo,
                                                      float *__restrict__ normlow)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const double *x = A + row * lda;
    double s = 0.0;
    for (int64_t k = lane; k < ldlow; k += 64) {
        const double v = k < n ? x[k] : 0.0;
        double rv;
        if constexpr (CMP == KDCD_F32) {
            const float f = (float)v;
            static_cast<float *>(hi)[row * ldlow + k] = f;
            rv = (double)f;
        } else if constexpr (CMP == KDCD_F16) {
            const _Float16 f = (_Float16)v;
            static_cast<_Float16 *>(hi)[row * ldlow + k] = f;
            rv = (double)f;
        } else {
            const __bf16 h = (__bf16)(float)v;
            static_cast<__bf16 *>(hi)[row * ldlow + k] = h;
            rv = (double)(float)h;
            if constexpr (CMP == KDCD_BF16X3) {
                const __bf16 l = (__bf16)(float)(v - rv);
                static_cast<__bf16 *>(lo)[row * ldlow + k] = l;
                rv += (double)(float)l;
            }
        }
        s += rv * rv;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) normlow[row] = (float)s;
}

constexpr int64_t kMaxRowGroups = 1024;

struct Cfg {
    int bm, bn;
};

Cfg pick_cfg(int32_t sb)
{
    if (sb <= 16) return {128, 16};
    if (sb <= 32) return {128, 32};
    return {128, 64};
}

template <int CMP, int WM, int WN, int TM, int TN, bool BATCH>
hipError_t launch_cfg(const KBlockArgs &a, hipStream_t st)
{
    constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
    const kdcd_matrix *A = a.A;
    const int64_t n_u = (A->m + BM - 1) / BM;
    const int64_t groups = n_u < kMaxRowGroups ? n_u : kMaxRowGroups;
    const int64_t n_n = (a.sb + BN - 1) / BN;
    const int64_t esz = CMP == KDCD_F32 ? 4 : 2;
    const int64_t ldseg = a.ldlow * esz / 16;
    const int64_t nseg = (A->n * esz + 15) / 16;
    const bool la = !BATCH && a.la != nullptr;
    if (la && !(a.la->b <= kLaMaxB && a.la->sb <= kLaEPT * 64 * WM * WN))
        return hipErrorInvalidValue;   // the caller checks lookahead_use first
    const LookaheadArgs lav = la ? *a.la : LookaheadArgs{};
    dim3 grid((unsigned)(n_n * groups + (la ? kLaLead : 0))), block(64 * WM * WN);
#define KDCD_LAUNCH_L(KIND, LAH)                                                                \
    KDCD_TIMED_LAUNCH((kblock_mixed_kernel<CMP, WM, WN, TM, TN, KIND, BATCH, LAH>), grid, block, \
                       0, st, static_cast<const u4 *>(a.Alow), static_cast<const u4 *>(a.Alow2), \
                       ldseg, A->m, nseg, a.normlow, a.S, a.sb, a.kp, a.beta, a.beta_scale,      \
                       a.partial, (int32_t)n_u, (int32_t)groups, (int32_t)n_n, a.batch, lav)
#define KDCD_LAUNCH(KIND)                                                                       \
    do {                                                                                        \
        if (la) {                                                                               \
            if constexpr (!BATCH) KDCD_LAUNCH_L(KIND, true);                                    \
        } else KDCD_LAUNCH_L(KIND, false);                                                      \
    } while (0)
    switch (a.kp.kind) {
    case KDCD_KERNEL_LINEAR: KDCD_LAUNCH(KDCD_KERNEL_LINEAR); break;
    case KDCD_KERNEL_POLY: KDCD_LAUNCH(KDCD_KERNEL_POLY); break;
    default: KDCD_LAUNCH(KDCD_KERNEL_RBF); break;
    }
#undef KDCD_LAUNCH
#undef KDCD_LAUNCH_L
    return hipGetLastError();
}

// Batched launches use at most a 128 x 64 tile (mapped values of a sigma group
// stay in registers while its problems are reduced): (WM, WN, TM, TN).
struct MixedCfg {
    int wm, wn, tm, tn;
};
constexpr MixedCfg kMixedBatchCfgs[] = {
    {4, 1, 2, 1},   // 0: 128 x 16
    {4, 1, 2, 2},   // 1: 128 x 32
    {2, 2, 4, 2},   // 2: 128 x 64
    {2, 2, 2, 2},   // 3: 64 x 64
};
constexpr int kMixedBatchNumCfgs = sizeof(kMixedBatchCfgs) / sizeof(kMixedBatchCfgs[0]);

int mixed_batch_default_id(int32_t sb)
{
    if (sb <= 16) return 0;
    if (sb <= 32) return 1;
    return 2;
}

int mixed_batch_valid(int id) { return id >= 0 && id < kMixedBatchNumCfgs; }

template <int CMP>
hipError_t launch_for(const KBlockArgs &a, hipStream_t st)
{
    if (a.batch) {
        switch (mixed_batch_valid(a.cfg) ? a.cfg
                                         : mixed_batch_config_id(a.compute, a.A->n, a.sb)) {
        case 0: return launch_cfg<CMP, 4, 1, 2, 1, true>(a, st);
        case 1: return launch_cfg<CMP, 4, 1, 2, 2, true>(a, st);
        case 3: return launch_cfg<CMP, 2, 2, 2, 2, true>(a, st);
        default: return launch_cfg<CMP, 2, 2, 4, 2, true>(a, st);
        }
    }
    const Cfg c = pick_cfg(a.sb);
    if (c.bn == 16) return launch_cfg<CMP, 4, 1, 2, 1, false>(a, st);
    if (c.bn == 32) return launch_cfg<CMP, 4, 1, 2, 2, false>(a, st);
    // wider blocks also take the 128 x 64 tile: it runs at three waves per
    // SIMD (the 128 x 128 one at two, one for bf16x3), which measured faster
    return launch_cfg<CMP, 2, 2, 4, 2, false>(a, st);
}

}  // namespace

int mixed_batch_config_count() { return kMixedBatchNumCfgs; }

void mixed_batch_config_shape(int id, int *bm, int *bn, int *waves)
{
    const MixedCfg &c = kMixedBatchCfgs[mixed_batch_valid(id) ? id : 2];
    *bm = 16 * c.tm * c.wm;
    *bn = 16 * c.tn * c.wn;
    *waves = c.wm * c.wn;
}

int mixed_batch_config_id(int32_t compute, int64_t n, int32_t sb)
{
    const int id = tune_lookup(compute + KDCD_TUNE_BATCH, n, sb);
    return mixed_batch_valid(id) ? id : mixed_batch_default_id(sb);
}

// Row groups of the launches of this file: the batched product (configuration
// cfg, or the table's choice when cfg < 0) and the single-problem FP32 product.
int64_t kblock_mixed_row_groups(int cfg, int64_t m, int64_t n, int32_t sb, int32_t compute,
                                bool batch)
{
    int bm = pick_cfg(sb).bm;
    if (batch) {
        int bn, w;
        mixed_batch_config_shape(mixed_batch_valid(cfg) ? cfg
                                                        : mixed_batch_config_id(compute, n, sb),
                                 &bm, &bn, &w);
    }
    const int64_t n_u = (m + bm - 1) / bm;
    return n_u < kMaxRowGroups ? n_u : kMaxRowGroups;
}

hipError_t launch_kblock_mixed(const KBlockArgs &a, hipStream_t st)
{
    if (!a.batch && a.compute != KDCD_F32) return launch_kblock_lowp(a, st);
    switch (a.compute) {
    case KDCD_F32: return launch_for<KDCD_F32>(a, st);
    case KDCD_BF16: return launch_for<KDCD_BF16>(a, st);
    case KDCD_F16: return launch_for<KDCD_F16>(a, st);
    case KDCD_BF16X3: return launch_for<KDCD_BF16X3>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_convert_lowp(const kdcd_matrix *A, int32_t compute, void *hi, void *lo,
                               int64_t ldlow, float *normlow, hipStream_t st)
{
    const dim3 grid((unsigned)((A->m + 3) / 4)), block(256);
    switch (compute) {
    case KDCD_F32:
        hipLaunchKernelGGL(convert_kernel<KDCD_F32>, grid, block, 0, st, A->values, A->ld, A->m,
                           A->n, ldlow, hi, lo, normlow);
        break;
    case KDCD_BF16:
        hipLaunchKernelGGL(convert_kernel<KDCD_BF16>, grid, block, 0, st, A->values, A->ld, A->m,
                           A->n, ldlow, hi, lo, normlow);
        break;
    case KDCD_F16:
        hipLaunchKernelGGL(convert_kernel<KDCD_F16>, grid, block, 0, st, A->values, A->ld, A->m,
                           A->n, ldlow, hi, lo, normlow);
        break;
    case KDCD_BF16X3:
        hipLaunchKernelGGL(convert_kernel<KDCD_BF16X3>, grid, block, 0, st, A->values, A->ld, A->m,
                           A->n, ldlow, hi, lo, normlow);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kdcd
