// Low-precision kernel block on gfx950 MFMA, 32 x 32 x 16 shape: P = A A_S^T
// with bf16 or fp16 operands (or the bf16x3 split) and FP32 accumulation, the
// Table 1 map in FP32, and the right-hand side r = U^T beta summed in FP64 --
// the U-part of the kernel-block pass of Algorithms 2 and 4 without writing U.
//
//   BF16    v_mfma_f32_32x32x16_bf16 on the bf16 copy of A
//   F16     v_mfma_f32_32x32x16_f16  on the fp16 copy
//   BF16X3  A = hi + lo (bf16 each), P = hi.hi + hi.lo + lo.hi: three MFMAs
//           per k-step into the same accumulators
//
// Tile: 256 x 256 per workgroup of 4 waves (2 x 2), 128 x 128 per wave as
// 4 x 4 MFMA blocks of 32 x 32 (256 accumulator registers per lane).  K is
// walked in chunks of BK elements, staged through LDS in fragment-major
// order: block b (32 rows) and k-step ks (16 elements) form one 1 KiB
// fragment in which lane l holds row l%32, elements 8(l/32)..8(l/32)+7, so
// every operand fetch is one contiguous ds_read_b128 per wave.  A and B use
// the same lane -> k-slot assignment, which is all the contraction needs.
// Output: item v of lane l of a block is row 8(v/4) + 4(l/32) + v%4,
// column l%32.
//
// Each output element gets the same MFMA sequence (chunks in order, k-steps
// in order, hi.hi, hi.lo, lo.hi) whatever the tile, so the batched variant's
// kernel values are bit for bit those of the single-problem launch.
#include "common.hpp"
#include "la_recur.hpp"

namespace kdcd {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;       // 4 waves, 2 x 2

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

template <int CMP>
__device__ __forceinline__ f16v mfma32(u4 a, u4 b, f16v acc)
{
    if constexpr (CMP == KDCD_F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a),
                                                      __builtin_bit_cast(h8, b), acc, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a),
                                                       __builtin_bit_cast(bf8, b), acc, 0, 0, 0);
}

// The Table 1 map in FP32 from the MFMA sum p.  RBF: nab = -sigma log2(e)
// (||a||^2 + ||b||^2) of the rounded rows and s2 = 2 sigma log2(e), so that
// K = exp2(min(p s2 + nab, 0)) = exp(-sigma max(||a - b||^2, 0)).
template <int KIND>
__device__ __forceinline__ float lowp_map(float p, float nab, float s2, float c, int degree)
{
    if constexpr (KIND == KDCD_KERNEL_LINEAR) {
        return p;
    } else if constexpr (KIND == KDCD_KERNEL_POLY) {
        const float base = c + p;
        float r = base;
        for (int t = 1; t < degree; ++t) r *= base;
        return r;
    } else {
        return __builtin_amdgcn_exp2f(fminf(fmaf(p, s2, nab), 0.0f));
    }
}

// BK: elements of K per LDS stage (32, or 16 for bf16x3 whose stages hold two
// layers).  Loads run two stages ahead of the MFMAs (two register stages).
// LAH: a K-RR lookahead launch: workgroup 0 runs la_recur for the previous
// block, workgroups 1 .. kLaLead - 1 return, the tiles follow (the kernel rows
// of the previous block's coordinates come from the FP64 Gram launch).
template <int CMP, int KIND, int BK, int TM, int TN, int OCC, bool STORE_U, bool LAH>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(OCC)))
void kblock_lowp_kernel(
    const u4 *__restrict__ Ahi, const u4 *__restrict__ Alo, int64_t ldseg, int64_t m,
    int64_t nchunks, const float *__restrict__ normlow, const int32_t *__restrict__ S, int32_t sb,
    KParams kp, const double *__restrict__ beta, const double *__restrict__ bscale,
    double *__restrict__ partial, int32_t n_u_tiles, int32_t n_row_groups, int32_t n_tiles_n,
    double *__restrict__ U, const int32_t *__restrict__ stop, const LookaheadArgs la)
{
    if (stop && *stop) return;
    constexpr bool X3 = CMP == KDCD_BF16X3;
    constexpr int NL = X3 ? 2 : 1;
    constexpr int SEGS = BK / 8;                  // 16-byte segments per row per stage
    constexpr int KSTEPS = BK / 16;
    // A fragment takes FRAG 16-byte slots: lanes 0-31 at slots 0-31, lanes
    // 32-63 at HOFF..HOFF+31.  The padding makes the stage stores conflict-free:
    // 16 consecutive threads store 16/SEGS rows x SEGS segments, and segment q
    // of row r lands in 16-byte bank group (q * 16/SEGS + r) mod 16.
    constexpr int HOFF = 32 + 16 / SEGS;
    constexpr int FRAG = 72;
    constexpr int BM = 64 * TM, BN = 64 * TN;     // workgroup tile
    constexpr int SA = BM / 32 * KSTEPS * FRAG;   // u4 per stage and layer
    constexpr int SB = BN / 32 * KSTEPS * FRAG;
    constexpr int LA = BM * SEGS / kThreads;      // segments per thread and layer
    constexpr int LB = BN * SEGS / kThreads;

    __shared__ u4 As[2][NL][SA];
    __shared__ u4 Bs[2][NL][SB];
    __shared__ double red[2][BN];

    if constexpr (LAH) {
        static_assert((int)sizeof(As) >= 24 * kThreads + 8 * (2 * kLaMaxB + 256) + kThreads / 4,
                      "the lookahead recurrence's LDS must fit the A buffers");
        if (blockIdx.x < kLaLead) {
            if (blockIdx.x == 0 && la.sb > 0) {
                char *smem = reinterpret_cast<char *>(&As[0][0][0]);
                if (la.b == 8) la_recur<kThreads, 8>(la, smem);
                else la_recur<kThreads, 0>(la, smem);
            }
            return;
        }
    }
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int lslot = (lane >> 5) * HOFF + (lane & 31);   // this lane's slot in a fragment
    const int total = n_tiles_n * n_row_groups;
    // the leading workgroups of a lookahead launch are a multiple of 8, so
    // bid % 8 is still the XCD of the workgroup
    const int bid = LAH ? (int)blockIdx.x - kLaLead : (int)blockIdx.x;
    const int L = xcd_remap(bid, total);
    const int cn = L % n_tiles_n;
    const int rg = L / n_tiles_n;
    const int col0 = cn * BN;

    // segment i of this thread in a stage: e = tid + 256 i -> row e / SEGS,
    // segment e % SEGS of the chunk; offsets in 16-byte units fit 32 bits
    // (m * ldlow < 2^34 elements)
    uint32_t boff[LB];
#pragma unroll
    for (int i = 0; i < LB; ++i) {
        const int e = tid + kThreads * i;
        const int64_t row = clampi(S[clampi(col0 + e / SEGS, 0, sb - 1)], 0, m - 1);
        boff[i] = (uint32_t)(row * ldseg + e % SEGS);
    }
    auto lds_off = [&](int i) {
        const int e = tid + kThreads * i;
        const int r = e / SEGS, q = e % SEGS;
        return ((r >> 5) * KSTEPS + (q >> 1)) * FRAG + (q & 1) * HOFF + (r & 31);
    };

    const float sig2 = (KIND == KDCD_KERNEL_RBF) ? (float)(kp.sigma * 1.4426950408889634) : 0.0f;
    float nbj[TN];               // -sigma log2(e) ||b_j||^2 of this lane's columns
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const int64_t j = clampi(col0 + (wn * TN + tn) * 32 + (lane & 31), 0, sb - 1);
        nbj[tn] = (KIND == KDCD_KERNEL_RBF) ? -sig2 * normlow[clampi(S[j], 0, m - 1)] : 0.0f;
    }
    double colsum[TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) colsum[tn] = 0.0;

    float *rowc = reinterpret_cast<float *>(&As[0][0][0]);          // staged per tile:
    double *rowb = reinterpret_cast<double *>(&Bs[0][0][0]);        // map term, beta

    for (int rt = rg; rt < n_u_tiles; rt += n_row_groups) {
        const int64_t row0 = (int64_t)rt * BM;
        uint32_t aoff[LA];
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + kThreads * i;
            aoff[i] = (uint32_t)(clampi(row0 + e / SEGS, 0, m - 1) * ldseg + e % SEGS);
        }
        f16v acc[TM][TN];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[tm][tn][v] = 0.0f;

        u4 ra0[NL][LA], rb0[NL][LB], ra1[NL][LA], rb1[NL][LB];
        auto load = [&](int64_t kc, u4 (&ra)[NL][LA], u4 (&rb)[NL][LB]) {
            const uint32_t s0 = (uint32_t)(kc * SEGS);
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const u4 *src = h == 0 ? Ahi : Alo;
#pragma unroll
                for (int i = 0; i < LA; ++i) ra[h][i] = src[aoff[i] + s0];
#pragma unroll
                for (int i = 0; i < LB; ++i) rb[h][i] = src[boff[i] + s0];
            }
        };
        auto store = [&](int buf, const u4 (&ra)[NL][LA], const u4 (&rb)[NL][LB]) {
#pragma unroll
            for (int h = 0; h < NL; ++h) {
#pragma unroll
                for (int i = 0; i < LA; ++i) As[buf][h][lds_off(i)] = ra[h][i];
#pragma unroll
                for (int i = 0; i < LB; ++i) Bs[buf][h][lds_off(i)] = rb[h][i];
            }
        };
        auto compute = [&](int buf) {
#pragma unroll
            for (int ks = 0; ks < KSTEPS; ++ks) {
                u4 a[NL][TM], b[NL][TN];
#pragma unroll
                for (int h = 0; h < NL; ++h) {
#pragma unroll
                    for (int t = 0; t < TM; ++t)
                        a[h][t] = As[buf][h][((wm * TM + t) * KSTEPS + ks) * FRAG + lslot];
#pragma unroll
                    for (int t = 0; t < TN; ++t)
                        b[h][t] = Bs[buf][h][((wn * TN + t) * KSTEPS + ks) * FRAG + lslot];
                }
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn) {
                        acc[tm][tn] = mfma32<CMP>(a[0][tm], b[0][tn], acc[tm][tn]);
                        if constexpr (X3) {
                            acc[tm][tn] = mfma32<CMP>(a[0][tm], b[1][tn], acc[tm][tn]);
                            acc[tm][tn] = mfma32<CMP>(a[1][tm], b[0][tn], acc[tm][tn]);
                        }
                    }
            }
        };

        // The rounded copies are padded to whole chunks: every chunk is loaded
        // unconditionally, chunk indices past the end clamped to the last one.  Whole pairs of chunks per loop
        // iteration and an odd last chunk after it keep one loop exit.
        const int64_t last = nchunks - 1;
        load(0, ra0, rb0);
        load(last < 1 ? last : 1, ra1, rb1);
        store(0, ra0, rb0);
        lds_barrier();
        const int64_t npairs = nchunks / 2;
        for (int64_t pk = 0; pk < npairs; ++pk) {
            const int64_t kc = 2 * pk;
            // the scheduling barriers keep each chunk's loads ahead of the MFMAs
            // of the chunk before (left alone, the compiler issued them after
            // those MFMAs and waited on them one phase later)
            load(kc + 2 < last ? kc + 2 : last, ra0, rb0);
            __builtin_amdgcn_sched_barrier(0);
            compute(0);
            store(1, ra1, rb1);
            lds_barrier();
            load(kc + 3 < last ? kc + 3 : last, ra1, rb1);
            __builtin_amdgcn_sched_barrier(0);
            compute(1);
            // unconditional: past the end it stores the clamped last chunk into a
            // buffer nothing reads any more (a conditional store let the compiler
            // sink the loads feeding it to just before it, waiting on them at once)
            store(0, ra0, rb0);
            lds_barrier();
        }
        if (nchunks & 1) {
            compute(0);
            lds_barrier();
        }

        // epilogue: per-row map term and beta staged in LDS (the operand
        // buffers are free after the loop's last barrier)
        for (int t = tid; t < BM; t += kThreads) {
            const int64_t grow = row0 + t;
            float c = 0.0f;
            double bv = 0.0;
            if (grow < m) {
                if (KIND == KDCD_KERNEL_RBF) c = -sig2 * normlow[grow];
                bv = beta[grow];
                if (bscale) bv *= bscale[grow];
            }
            rowc[t] = c;
            rowb[t] = bv;
        }
        __syncthreads();
        const float cpoly = (float)kp.c;
        // one block row at a time; the 16 rows of a block that a lane holds come
        // in groups of 4 consecutive rows (8 g + 4 (l/32) + 0..3), read as
        // float4 / double2 vectors
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            const int lb = (wm * TM + tm) * 32 + (lane >> 5) * 4;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const float4 c4 = *reinterpret_cast<const float4 *>(&rowc[lb + g * 8]);
                const double2 b01 = *reinterpret_cast<const double2 *>(&rowb[lb + g * 8]);
                const double2 b23 = *reinterpret_cast<const double2 *>(&rowb[lb + g * 8 + 2]);
                const float cv[4] = {c4.x, c4.y, c4.z, c4.w};
                const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn) {
                        const float kv = lowp_map<KIND>(acc[tm][tn][g * 4 + u], cv[u] + nbj[tn],
                                                        2.0f * sig2, cpoly, kp.degree);
                        colsum[tn] = fma(bv[u], (double)kv, colsum[tn]);
                        if constexpr (STORE_U) {
                            const int64_t grow = row0 + lb + g * 8 + u;
                            const int64_t gcol = col0 + (wn * TN + tn) * 32 + (lane & 31);
                            if (grow < m && gcol < sb) U[gcol * m + grow] = (double)kv;
                        }
                    }
                }
            }
        }
        __syncthreads();    // rowc / rowb are read before the next tile's stores
    }

    // lanes l and l ^ 32 hold the same column: lanes -> waves -> one partial row
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
        const double v = colsum[tn] + __shfl_xor(colsum[tn], 32);
        if (lane < 32) red[wm][(wn * TN + tn) * 32 + lane] = v;
    }
    __syncthreads();
    for (int c = tid; c < BN; c += kThreads) {
        const double s = red[0][c] + red[1][c];
        if (col0 + c < sb) partial[(int64_t)rg * sb + col0 + c] = s;
    }
}

constexpr int64_t kMaxRowGroups = 1024;

// Tile configurations of the single-problem launch: TM x TN MFMA blocks of
// 32 x 32 per wave (2 x 2 waves, tile 64 TM x 64 TN) and BK elements of K per
// LDS stage (bf16x3 stages hold two layers and take BK / 2).
struct LowpCfg {
    int tm, tn, bk, occ;
};
constexpr LowpCfg kLowpCfgs[] = {
    {2, 4, 32, 1},   // 0: 128 x 256
    {2, 4, 64, 1},   // 1: 128 x 256, longer stages
    {4, 2, 32, 1},   // 2: 256 x 128
    {4, 2, 64, 1},   // 3: 256 x 128, longer stages
    {4, 2, 16, 2},   // 4: 256 x 128, short stages, two workgroups per CU
    {2, 4, 16, 2},   // 5: 128 x 256, short stages, two workgroups per CU
    {4, 2, 32, 2},   // 6: 256 x 128, two workgroups per CU
};
constexpr int kLowpNumCfgs = sizeof(kLowpCfgs) / sizeof(kLowpCfgs[0]);
// Built-in choice: the 256 x 128 tile at two workgroups per CU with 32-element
// stages (measured fastest of the table on C4, 200000 x 1024 at s*b = 512, for
// bf16 and bf16x3).
constexpr int kLowpDefault = 6;


template <int CMP, int BK, int TM, int TN, int OCC, bool STORE_U>
hipError_t launch_u(const KBlockArgs &a, hipStream_t st)
{
    constexpr int BM = 64 * TM, BN = 64 * TN;
    const kdcd_matrix *A = a.A;
    const int64_t n_u = (A->m + BM - 1) / BM;
    const int64_t groups = n_u < kMaxRowGroups ? n_u : kMaxRowGroups;
    const int64_t n_n = (a.sb + BN - 1) / BN;
    const int64_t ldseg = a.ldlow * 2 / 16;
    if (a.ldlow % BK != 0 || a.ldlow < BK) return hipErrorInvalidValue;   // whole stages only
    const int64_t nchunks = a.ldlow / BK;          // ldlow is a multiple of 64
    const bool la = a.la != nullptr;
    if (la && !(a.la->b <= kLaMaxB && a.la->sb <= kLaEPT * kThreads))
        return hipErrorInvalidValue;   // the caller checks lookahead_use first
    const LookaheadArgs lav = la ? *a.la : LookaheadArgs{};
    dim3 grid((unsigned)(n_n * groups + (la ? kLaLead : 0))), block(kThreads);
#define KDCD_LAUNCH_L(KIND, LAH)                                                                  \
    KDCD_TIMED_LAUNCH((kblock_lowp_kernel<CMP, KIND, BK, TM, TN, OCC, STORE_U, LAH>), grid,       \
                      block, 0, st, static_cast<const u4 *>(a.Alow),                              \
                      static_cast<const u4 *>(a.Alow2), ldseg, A->m, nchunks, a.normlow, a.S,     \
                      a.sb, a.kp, a.beta, a.beta_scale, a.partial, (int32_t)n_u, (int32_t)groups, \
                      (int32_t)n_n, a.U, a.stop, lav)
#define KDCD_LAUNCH(KIND)                                                                         \
    do {                                                                                          \
        if (la) KDCD_LAUNCH_L(KIND, true);                                                        \
        else KDCD_LAUNCH_L(KIND, false);                                                          \
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

template <int CMP, int BK, int TM, int TN, int OCC>
hipError_t launch_cfg(const KBlockArgs &a, hipStream_t st)
{
    constexpr int B = (CMP == KDCD_BF16X3 && BK > 16) ? BK / 2 : BK;
    return a.U ? launch_u<CMP, B, TM, TN, OCC, true>(a, st)
               : launch_u<CMP, B, TM, TN, OCC, false>(a, st);
}

template <int CMP>
hipError_t launch_for(const KBlockArgs &a, hipStream_t st, int id)
{
    switch (id) {
    case 1: return launch_cfg<CMP, 64, 2, 4, 1>(a, st);
    case 2: return launch_cfg<CMP, 32, 4, 2, 1>(a, st);
    case 3: return launch_cfg<CMP, 64, 4, 2, 1>(a, st);
    case 4: return launch_cfg<CMP, 16, 4, 2, 2>(a, st);
    case 5: return launch_cfg<CMP, 16, 2, 4, 2>(a, st);
    case 6: return launch_cfg<CMP, 32, 4, 2, 2>(a, st);
    default: return launch_cfg<CMP, 32, 2, 4, 1>(a, st);
    }
}

int lowp_valid(int id) { return id >= 0 && id < kLowpNumCfgs; }

}  // namespace

int lowp_config_count() { return kLowpNumCfgs; }

void lowp_config_shape(int id, int *bm, int *bn, int *waves)
{
    const LowpCfg &c = kLowpCfgs[lowp_valid(id) ? id : kLowpDefault];
    *bm = 64 * c.tm;
    *bn = 64 * c.tn;
    *waves = 4;
}

int lowp_config_id(int32_t compute, int64_t n, int32_t sb)
{
    const int id = tune_lookup(compute, n, sb);
    return lowp_valid(id) ? id : kLowpDefault;
}

int64_t kblock_lowp_row_groups(int cfg, int64_t m)
{
    int bm, bn, w;
    lowp_config_shape(cfg, &bm, &bn, &w);
    const int64_t n_u = (m + bm - 1) / bm;
    return n_u < kMaxRowGroups ? n_u : kMaxRowGroups;
}

hipError_t launch_kblock_lowp(const KBlockArgs &a, hipStream_t st)
{
    const int id = lowp_valid(a.cfg) ? a.cfg : lowp_config_id(a.compute, a.A->n, a.sb);
    switch (a.compute) {
    case KDCD_BF16: return launch_for<KDCD_BF16>(a, st, id);
    case KDCD_F16: return launch_for<KDCD_F16>(a, st, id);
    case KDCD_BF16X3: return launch_for<KDCD_BF16X3>(a, st, id);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace kdcd
