// CSR kernel block on gfx950 (vector ALU, no MFMA): for sparse A the product
// P = A A_S^T has about nnz(A) * (hit rate) useful multiply-adds and is bound
// by streaming the CSR arrays from HBM, so it is written for memory-level
// parallelism, not for matrix cores.
//
// One launch computes, like the dense kernel block:
//   U-part: the column sums partial[g][j] = sum_p K(a_p, a_{S_j}) beta_p over
//           the rows p of row group g (the map of Table 1 is applied to each
//           P_pj in registers; U is never stored);
//   W-part: W = K(A_S, A_S) (sb x sb).
//
// Sampled-row panel.  For each chunk of at most 32 (or 64) sampled rows, every
// workgroup builds in LDS an open-addressing hash keyed by column id: slot h
// holds the column, a bit mask of the sampled rows that store it, and the
// offset of their values in a compact value array (values of one column are
// stored in sampled-row order).  Column ids are only ever hash keys, never
// addresses.  The table lives in LDS, so nothing has to be cleared between
// outer iterations.
//
// Rows.  A wave processes RPW rows at once, LPR = 64/RPW lanes per row, lane
// jl <-> sampled row j0 + jl; RPW in {1, 2, 4, 8} is picked from s*b and the
// average row length.  The lanes of a row first look up one stored
// entry each; the entries' (value, mask, offset) are then broadcast to the
// row's lanes in storage order, and lane jl accumulates a * B[c][jl] whenever
// its bit is set.  Every sum runs in a fixed order: results are deterministic.
#include <type_traits>

#include "common.hpp"

namespace kdcd {
namespace {

constexpr int CSR_NT = 512;           // threads per workgroup (8 waves)
constexpr int CSR_VMAX = 3072;        // stored entries of one chunk of sampled rows
static_assert(CSR_VMAX <= 32767, "value offsets are 16-bit");
constexpr int CSR_HS = 4096;          // hash slots (power of two, > CSR_VMAX)
constexpr int CSR_MAXGROUPS = 512;    // row groups of the U-part
constexpr double kCsrWaveMinAvg = 128.0;   // average row length from which rows get a wave each

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ uint32_t hash_col(int32_t c)
{
    return ((uint32_t)c * 2654435761u) & (CSR_HS - 1);
}

// Membership filter in front of the table: one bit per value of a second
// hash of the column, so that most columns absent from the panel cost one
// LDS read instead of a probe sequence (at a table load of 3/4, unsuccessful
// linear probing averages 8.5 reads).
constexpr int CSR_FBITS = 32768;
__device__ __forceinline__ uint32_t filt_col(int32_t c)
{
    return ((uint32_t)c * 2246822519u) >> 17;   // 15 bits
}

// Probe for column c; returns the slot or -1 when c is not in the table.
__device__ __forceinline__ int hash_find(const int32_t *keys, const uint32_t *filt, int32_t c)
{
    const uint32_t f = filt_col(c);
    if (!((filt[f >> 5] >> (f & 31)) & 1u)) return -1;
    uint32_t h = hash_col(c);
    for (;;) {
        const int32_t k = keys[h];
        if (k == c) return (int)h;
        if (k == -1) return -1;
        h = (h + 1) & (CSR_HS - 1);
    }
}

__device__ __forceinline__ uint64_t shfl_mask(uint64_t v, int src)
{
    const uint32_t lo = __shfl((int)(uint32_t)v, src), hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int popc(uint64_t v) { return __popcll(v); }
__device__ __forceinline__ int popc(uint32_t v) { return __popc(v); }
__device__ __forceinline__ void atomic_or_mask(uint64_t *p, uint64_t v)
{
    atomicOr((unsigned long long *)p, (unsigned long long)v);
}
__device__ __forceinline__ void atomic_or_mask(uint32_t *p, uint32_t v)
{
    atomicOr((unsigned int *)p, (unsigned int)v);
}

// Entries a lane loads per batch of a row walk (one batch in flight while the
// previous one is multiplied out); sized so that the kernel stays within 128
// VGPRs (four waves per SIMD, two workgroups per CU) without spilling.
template <int KIND, int RPW>
constexpr int csr_nbatch() { return KIND == KDCD_KERNEL_RBF ? 2 : (RPW == 8 ? 3 : 4); }

// The sampled-row panel of the chunk starting at j0: at most LPR sampled rows
// whose stored entries fit CSR_VMAX, hashed by column in LDS (slot: column,
// bit mask of the chunk's rows that store it, offset of their values), the
// values of one column stored in sampled-row order.  Returns the end j1 of
// the chunk, or -2 when the sampled row j0 alone exceeds the panel; such a row
// is then hashed in pieces of CSR_VMAX consecutive entries (piece >= 0: the
// panel holds entries [piece * CSR_VMAX, ...) of row j0 only).  Called by
// every thread of the workgroup; ends with a barrier.
template <class MaskT, int LPR>
__device__ int build_panel(int j0, int piece, const int64_t *__restrict__ row_ptr,
                           const int32_t *__restrict__ col_idx, const double *__restrict__ val,
                           int64_t m, int64_t nnz, const int32_t *__restrict__ S, int32_t sb,
                           int32_t *hkey, uint32_t *hfilt, MaskT *hmask, int16_t *hbase,
                           double *hval,
                           int32_t *rowoff, int32_t *scan, int32_t *status)
{
    const int tid = threadIdx.x;
    auto rp = [&](int64_t r) { return clampi(row_ptr[clampi(r, 0, m)], 0, nnz); };
    int j1 = j0, tot = 0;
    int64_t skip = 0;                     // entries of the row before this piece
    if (piece >= 0) {
        const int64_t r = clampi(S[j0], 0, m - 1);
        skip = (int64_t)piece * CSR_VMAX;
        const int64_t rest = rp(r + 1) - rp(r) - skip;
        tot = (int)(rest < CSR_VMAX ? (rest > 0 ? rest : 0) : CSR_VMAX);
        j1 = j0 + 1;
        if (tid == 0) {
            rowoff[0] = 0;
            rowoff[1] = tot;
        }
    } else {
        if (tid == 0) rowoff[0] = 0;
        while (j1 < sb && j1 - j0 < LPR) {
            const int64_t r = clampi(S[j1], 0, m - 1);
            const int len = (int)(rp(r + 1) - rp(r));
            if (tot + len > CSR_VMAX) break;
            tot += len;
            ++j1;
            if (tid == 0) rowoff[j1 - j0] = tot;
        }
        if (j1 == j0) return -2;          // one sampled row alone exceeds the panel
    }
    for (int x = tid; x < CSR_HS; x += CSR_NT) {
        hkey[x] = -1;
        hmask[x] = 0;
    }
    for (int x = tid; x < CSR_FBITS / 32; x += CSR_NT) hfilt[x] = 0u;
    __syncthreads();
    // 1. insert every stored entry's column, mark which sampled row holds it
    for (int f = tid; f < tot; f += CSR_NT) {
        int jj = 0;
        while (rowoff[jj + 1] <= f) ++jj;
        const int64_t r = clampi(S[j0 + jj], 0, m - 1);
        const int64_t e = clampi(rp(r) + skip + (f - rowoff[jj]), 0, nnz - 1);
        const int32_t c = col_idx[e];
        uint32_t h = hash_col(c);
        for (;;) {
            const int32_t old = atomicCAS(&hkey[h], -1, c);
            if (old == -1 || old == c) break;
            h = (h + 1) & (CSR_HS - 1);
        }
        atomic_or_mask(&hmask[h], (MaskT)1 << jj);
        const uint32_t fb = filt_col(c);
        atomicOr(&hfilt[fb >> 5], 1u << (fb & 31));
    }
    __syncthreads();
    // 2. offsets of each column's values: exclusive scan of popcounts over the slots
    constexpr int PER = CSR_HS / CSR_NT;
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) cnt += popc(hmask[tid * PER + q]);
    scan[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < CSR_NT; off <<= 1) {   // Hillis-Steele inclusive scan
        const int v = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    int base = scan[tid] - cnt;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        hbase[tid * PER + q] = (int16_t)base;
        base += popc(hmask[tid * PER + q]);
    }
    __syncthreads();
    // 3. place the values, in sampled-row order inside each column
    for (int f = tid; f < tot; f += CSR_NT) {
        int jj = 0;
        while (rowoff[jj + 1] <= f) ++jj;
        const int64_t r = clampi(S[j0 + jj], 0, m - 1);
        const int64_t e = clampi(rp(r) + skip + (f - rowoff[jj]), 0, nnz - 1);
        const int h = hash_find(hkey, hfilt, col_idx[e]);
        if (h >= 0) {
            const MaskT msk = hmask[h];
            hval[hbase[h] + popc((MaskT)(msk & (((MaskT)1 << jj) - 1)))] = val[e];
        }
    }
    __syncthreads();
    return j1;
}

template <int RPW, int KIND>
__global__ __launch_bounds__(CSR_NT) __attribute__((amdgpu_waves_per_eu(RPW > 1 ? 4 : 2))) void kblock_csr_kernel(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const double *__restrict__ val, int64_t m, int64_t nnz, const int32_t *__restrict__ S,
    int32_t sb, const double *__restrict__ norms, KParams kp, const double *__restrict__ beta,
    const double *__restrict__ bscale, double *__restrict__ partial, double *__restrict__ W,
    int32_t n_row_groups, double *__restrict__ carry, int32_t *status)
{
    constexpr int LPR = 64 / RPW;                  // lanes per row = sampled rows per chunk
    constexpr int NW = CSR_NT / 64;
    constexpr int ROWS = NW * RPW;                 // rows per workgroup step
    // one bit per sampled row of a chunk; 32-bit masks keep the panel small
    // enough for two workgroups per CU
    using MaskT = typename std::conditional<(LPR > 32), uint64_t, uint32_t>::type;
    __shared__ int32_t hkey[CSR_HS];
    __shared__ MaskT hmask[CSR_HS];
    __shared__ int16_t hbase[CSR_HS];      // value offsets (< CSR_VMAX)
    __shared__ uint32_t hfilt[CSR_FBITS / 32];
    __shared__ double hval[CSR_VMAX];
    __shared__ int32_t rowoff[LPR + 1];            // entry offsets of the chunk's sampled rows
    // Per-wave scratch of SW doubles.  SCATTER (at most 16 sampled rows per
    // chunk): the rows' sums over their sampled rows, to which every lane adds
    // its entries' products (LDS atomic adds; a wave's atomics on one address
    // apply in lane order).  STAGE (32): the broadcast stages each position's
    // entries here (value, and mask | offset << 32).  The panel build's prefix
    // sums and the cross-wave column sums use the same memory at other times.
    constexpr int SW = 128;
    constexpr bool SCATTER = LPR <= 16;              // few sampled rows per chunk
    constexpr bool STAGE = LPR == 32;
    __shared__ double wbuf[NW * SW];
    int32_t *scan = reinterpret_cast<int32_t *>(wbuf);   // CSR_NT ints
    static_assert(CSR_NT * sizeof(int32_t) <= NW * SW * sizeof(double), "scan fits");
    static_assert(RPW * LPR <= SW, "column sums fit");
    auto red = [&](int w, int j) -> double & { return wbuf[(w / RPW) * SW + (w % RPW) * LPR + j]; };

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int rslot = lane / LPR, jl = lane % LPR;
    const bool is_w = (int)blockIdx.x >= n_row_groups;
    if (is_w && W == nullptr) return;
    const int wblk = (int)blockIdx.x - n_row_groups;   // W-part: sampled rows [wblk*ROWS, +ROWS)
    auto rp = [&](int64_t r) { return clampi(row_ptr[clampi(r, 0, m)], 0, nnz); };

    for (int j0 = 0; j0 < sb;) {
        int j1 = build_panel<MaskT, LPR>(j0, -1, row_ptr, col_idx, val, m, nnz, S, sb, hkey, hfilt,
                                          hmask, hbase, hval, rowoff, scan, status);
        int npieces = 1;
        if (j1 == -2) {                  // a sampled row longer than the panel: in pieces
            if (!carry) {
                if (tid == 0) set_status(status, KDCD_ERR_UNSUPPORTED);
                return;
            }
            const int64_t r = clampi(S[j0], 0, m - 1);
            npieces = (int)((rp(r + 1) - rp(r) + CSR_VMAX - 1) / CSR_VMAX);
            j1 = j0 + 1;
        }
        const int nj = j1 - j0;

        // 4. rows: sparse row i against the panel, map, reduce or store
        const bool jok = jl < nj;
        const int64_t Sj = clampi(S[j0 + (jok ? jl : 0)], 0, m - 1);
        const double nb = (KIND == KDCD_KERNEL_RBF) ? norms[Sj] : 0.0;
        const MaskT below = ((MaskT)1 << jl) - 1;
        double colsum = 0.0;
        for (int pc = 0; pc < npieces; ++pc) {
        if (npieces > 1) {
            // the dot products of a long row are summed over its pieces in
            // carry[] (data rows of the U-part at [row], sampled rows of the
            // Gram part at [m + t]) before the map
            __syncthreads();             // every wave is done with the previous piece
            build_panel<MaskT, LPR>(j0, pc, row_ptr, col_idx, val, m, nnz, S, sb, hkey, hfilt, hmask,
                                    hbase, hval, rowoff, scan, status);
        }
        const bool last = pc + 1 == npieces;
        // SCATTER: the row's sums over its sampled rows live in this wave's
        // scratch (the panel build above used the same memory for its scan)
        double *rsum = wbuf + wid * SW + rslot * LPR;
        if constexpr (SCATTER) {
            rsum[jl] = 0.0;
            wave_lds_sync();
        }
        const int64_t nsteps = is_w ? 1 : (m + ROWS - 1) / ROWS;
        for (int64_t st = is_w ? 0 : blockIdx.x; st < nsteps; st += is_w ? 1 : n_row_groups) {
            const int64_t rix = (is_w ? (int64_t)wblk * ROWS : st * ROWS) + wid * RPW + rslot;
            const bool rok = is_w ? rix < sb : rix < m;
            const int64_t row = is_w ? clampi(S[clampi(rix, 0, sb - 1)], 0, m - 1) : clampi(rix, 0, m - 1);
            const int64_t e_beg = rok ? rp(row) : 0, e_end = rok ? rp(row + 1) : 0;
            double acc = 0.0;
            // all rows of the wave step through their entries together, LPR at a time
            int64_t len = e_end - e_beg;
            int64_t lmax = len;
            for (int o = LPR; o < 64; o <<= 1) {
                const int64_t other = __shfl_xor(lmax, o);
                lmax = other > lmax ? other : lmax;
            }
            // entries are loaded CSR_NBATCH per lane at a time, the next batch
            // in flight while the current one is multiplied out
            constexpr int CSR_NBATCH = csr_nbatch<KIND, RPW>();
            int32_t cb[CSR_NBATCH], nc[CSR_NBATCH];
            double vb[CSR_NBATCH], nv[CSR_NBATCH];
            auto load_batch = [&](int64_t eb, int32_t (&c)[CSR_NBATCH], double (&v)[CSR_NBATCH]) {
#pragma unroll
                for (int u = 0; u < CSR_NBATCH; ++u) {
                    const int64_t off = eb + (int64_t)u * LPR + jl;
                    const int64_t ec = clampi(e_beg + off, 0, nnz - 1);
                    const bool ok = off < len;
                    c[u] = ok ? col_idx[ec] : -1;
                    v[u] = ok ? val[ec] : 0.0;
                }
            };
            constexpr int64_t STEP = (int64_t)CSR_NBATCH * LPR;
            if (lmax > 0) load_batch(0, cb, vb);
            for (int64_t eb = 0; eb < lmax; eb += STEP) {
                if (eb + STEP < lmax) load_batch(eb + STEP, nc, nv);
#pragma unroll
                for (int u = 0; u < CSR_NBATCH; ++u) {
                    if (eb + (int64_t)u * LPR >= lmax) break;   // uniform over the wave
                    double a = 0.0;
                    MaskT msk = 0;
                    int bs = 0;
                    if (cb[u] >= 0) {
                        const int h = hash_find(hkey, hfilt, cb[u]);
                        if (h >= 0) {
                            a = vb[u];
                            msk = hmask[h];
                            bs = hbase[h];
                        }
                    }
                    if constexpr (SCATTER) {
                        // every lane adds its entry's products into the row's LDS
                        // sums, one sampled row (set bit) per step
                        MaskT mm = msk;
                        int k = 0;
                        while (__ballot(mm != 0)) {
                            if (mm) {
                                const int j = __builtin_ctz((uint32_t)mm);
                                mm &= mm - 1;
                                atomicAdd(&rsum[j], a * hval[bs + k]);
                                ++k;
                            }
                        }
                    } else {
                        // positions t whose entry hits the panel in some row of the wave
                        // (a position that misses everywhere would add nothing)
                        const uint64_t hits = __ballot(msk != 0);
                        uint64_t pos = 0;
#pragma unroll
                        for (int g = 0; g < RPW; ++g) pos |= (hits >> (g * LPR));
                        if constexpr (LPR < 64) pos &= (1ull << LPR) - 1;
                        if constexpr (STAGE) {
                        double *sa = wbuf + wid * SW;
                        uint64_t *sp = reinterpret_cast<uint64_t *>(wbuf + wid * SW + 64);
                        wave_lds_sync();          // the previous position's reads are done
                        sa[lane] = a;
                        sp[lane] = (uint64_t)(uint32_t)msk | ((uint64_t)(uint32_t)bs << 32);
                        wave_lds_sync();
                        while (pos) {
                            const int t = __builtin_ctzll(pos);
                            pos &= pos - 1;
                            const int src = rslot * LPR + t;
                            const double at = sa[src];
                            const uint64_t pk = sp[src];
                            const MaskT mt = (MaskT)(uint32_t)pk;
                            const int bt = (int)(pk >> 32);
                            if ((mt >> jl) & 1) acc += at * hval[bt + popc((MaskT)(mt & below))];
                        }
                        } else {
                        while (pos) {
                            const int t = __builtin_ctzll(pos);
                            pos &= pos - 1;
                            const int src = rslot * LPR + t;
                            const double at = __shfl(a, src);
                            const MaskT mt = shfl_mask(msk, src);
                            const int bt = __shfl(bs, src);
                            if ((mt >> jl) & 1) acc += at * hval[bt + popc((MaskT)(mt & below))];
                        }
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < CSR_NBATCH; ++u) {
                    cb[u] = nc[u];
                    vb[u] = nv[u];
                }
            }
            if constexpr (SCATTER) {
                wave_lds_sync();                  // every lane's additions are done
                acc = rsum[jl];
                rsum[jl] = 0.0;
                wave_lds_sync();
            }
            if (rok && jok) {
                if (npieces > 1) {
                    const int64_t ci = is_w ? m + rix : row;
                    if (pc > 0) acc += carry[ci];
                    if (!last) carry[ci] = acc;
                }
                if (last) {
                    const double na = (KIND == KDCD_KERNEL_RBF) ? norms[row] : 0.0;
                    const double kv = kernel_map<KIND>(acc, na, nb, row == Sj, kp);
                    if (is_w) {
                        W[rix * sb + j0 + jl] = kv;
                    } else {
                        double bv = beta[row];
                        if (bscale) bv *= bscale[row];
                        colsum += bv * kv;
                    }
                }
            }
        }
        }   // pieces
        if (!is_w) {
            red(wid * RPW + rslot, jl) = colsum;
            __syncthreads();
            if (tid < nj) {
                double s = 0.0;
                for (int w = 0; w < NW * RPW; ++w) s += red(w, tid);
                partial[(int64_t)blockIdx.x * sb + j0 + tid] = s;
            }
        }
        __syncthreads();
        j0 = j1;
    }
}

// Long rows (chunks of at most WJ = 8 sampled rows): one wave walks one data
// row, 64 stored entries at a time (coalesced loads), each lane keeping its
// own partial sums for the chunk's sampled rows; the lanes' sums meet in a
// fixed xor tree at the end of the row, so the result is deterministic.
constexpr int WJ = 8;

template <int KIND>
__global__ __launch_bounds__(CSR_NT) __attribute__((amdgpu_waves_per_eu(4))) void kblock_csr_wave_kernel(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const double *__restrict__ val, int64_t m, int64_t nnz, const int32_t *__restrict__ S,
    int32_t sb, const double *__restrict__ norms, KParams kp, const double *__restrict__ beta,
    const double *__restrict__ bscale, double *__restrict__ partial, double *__restrict__ W,
    int32_t n_row_groups, double *__restrict__ carry, int32_t *status)
{
    constexpr int NW = CSR_NT / 64;
    constexpr int NB = KIND == KDCD_KERNEL_RBF ? 2 : 4;   // entries per lane per batch
    using MaskT = uint32_t;
    __shared__ int32_t hkey[CSR_HS];
    __shared__ MaskT hmask[CSR_HS];
    __shared__ int16_t hbase[CSR_HS];      // value offsets (< CSR_VMAX)
    __shared__ uint32_t hfilt[CSR_FBITS / 32];
    __shared__ double hval[CSR_VMAX];
    __shared__ int32_t rowoff[WJ + 1];
    __shared__ int32_t scan[CSR_NT];
    __shared__ double red[NW][WJ];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool is_w = (int)blockIdx.x >= n_row_groups;
    if (is_w && W == nullptr) return;
    const int wblk = (int)blockIdx.x - n_row_groups;   // W-part: sampled rows [wblk*NW, +NW)
    auto rp = [&](int64_t r) { return clampi(row_ptr[clampi(r, 0, m)], 0, nnz); };

    for (int j0 = 0; j0 < sb;) {
        int j1 = build_panel<MaskT, WJ>(j0, -1, row_ptr, col_idx, val, m, nnz, S, sb, hkey, hfilt,
                                        hmask, hbase, hval, rowoff, scan, status);
        int npieces = 1;
        if (j1 == -2) {                  // a sampled row longer than the panel: in pieces
            if (!carry) {
                if (tid == 0) set_status(status, KDCD_ERR_UNSUPPORTED);
                return;
            }
            const int64_t r = clampi(S[j0], 0, m - 1);
            npieces = (int)((rp(r + 1) - rp(r) + CSR_VMAX - 1) / CSR_VMAX);
            j1 = j0 + 1;
        }
        const int nj = j1 - j0;
        // lane j < nj owns sampled row j0 + j for the map and the reduction
        const bool jok = lane < nj;
        const int64_t Sj = clampi(S[j0 + (jok ? lane : 0)], 0, m - 1);
        const double nbj = (KIND == KDCD_KERNEL_RBF) ? norms[Sj] : 0.0;
        double colsum = 0.0;
        for (int pc = 0; pc < npieces; ++pc) {
        if (npieces > 1) {               // dot products summed over the pieces in carry[]
            __syncthreads();
            build_panel<MaskT, WJ>(j0, pc, row_ptr, col_idx, val, m, nnz, S, sb, hkey, hfilt, hmask,
                                   hbase, hval, rowoff, scan, status);
        }
        const bool last = pc + 1 == npieces;
        const int64_t r_first = is_w ? (int64_t)wblk * NW + wid : (int64_t)blockIdx.x * NW + wid;
        const int64_t r_end = is_w ? min((int64_t)sb, (int64_t)(wblk + 1) * NW) : m;
        const int64_t r_step = is_w ? NW : (int64_t)n_row_groups * NW;
        for (int64_t rix = r_first; rix < r_end; rix += r_step) {
            const int64_t row = is_w ? clampi(S[rix], 0, m - 1) : rix;
            const int64_t e_beg = rp(row), len = rp(row + 1) - e_beg;
            double acc[WJ];
#pragma unroll
            for (int j = 0; j < WJ; ++j) acc[j] = 0.0;
            int32_t cb[NB], nc[NB];
            double vb[NB], nv[NB];
            auto load_batch = [&](int64_t eb, int32_t (&c)[NB], double (&v)[NB]) {
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int64_t off = eb + (int64_t)u * 64 + lane;
                    const int64_t ec = clampi(e_beg + off, 0, nnz - 1);
                    const bool ok = off < len;
                    c[u] = ok ? col_idx[ec] : -1;
                    v[u] = ok ? val[ec] : 0.0;
                }
            };
            constexpr int64_t STEP = (int64_t)NB * 64;
            if (len > 0) load_batch(0, cb, vb);
            for (int64_t eb = 0; eb < len; eb += STEP) {
                if (eb + STEP < len) load_batch(eb + STEP, nc, nv);
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    if (cb[u] >= 0) {
                        const int h = hash_find(hkey, hfilt, cb[u]);
                        if (h >= 0) {
                            const MaskT msk = hmask[h];
                            const int bs = hbase[h];
                            const double a = vb[u];
#pragma unroll
                            for (int j = 0; j < WJ; ++j)
                                if ((msk >> j) & 1u)
                                    acc[j] += a * hval[bs + popc((MaskT)(msk & ((1u << j) - 1u)))];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    cb[u] = nc[u];
                    vb[u] = nv[u];
                }
            }
            double mine = 0.0;
#pragma unroll
            for (int j = 0; j < WJ; ++j) {
                double v = acc[j];
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
                if (lane == j) mine = v;
            }
            if (jok) {
                if (npieces > 1) {
                    const int64_t ci = is_w ? m + rix : row;
                    if (pc > 0) mine += carry[ci];
                    if (!last) carry[ci] = mine;
                }
                if (last) {
                    const double na = (KIND == KDCD_KERNEL_RBF) ? norms[row] : 0.0;
                    const double kv = kernel_map<KIND>(mine, na, nbj, row == Sj, kp);
                    if (is_w) {
                        W[rix * sb + j0 + lane] = kv;
                    } else {
                        double bv = beta[row];
                        if (bscale) bv *= bscale[row];
                        colsum += bv * kv;
                    }
                }
            }
        }
        }   // pieces
        if (!is_w) {
            if (lane < WJ) red[wid][lane] = colsum;
            __syncthreads();
            if (tid < nj) {
                double t = 0.0;
                for (int w = 0; w < NW; ++w) t += red[w][tid];
                partial[(int64_t)blockIdx.x * sb + j0 + tid] = t;
            }
        }
        __syncthreads();
        j0 = j1;
    }
}

int64_t groups_for(int64_t m)
{
    const int64_t steps = (m + 15) / 16;
    return steps < CSR_MAXGROUPS ? steps : CSR_MAXGROUPS;
}

}  // namespace

int64_t kblock_csr_row_groups(int64_t m, int32_t sb)
{
    (void)sb;
    return groups_for(m);
}

// Lanes per row (LPR = 64 / RPW): no more than the sampled rows need, and
// few enough that a chunk of LPR average-length sampled rows fits the panel
// (long rows: narrow chunks, several data rows per wave).
int csr_rows_per_wave(const kdcd_matrix *A, int32_t sb)
{
    int lpr = sb <= 8 ? 8 : (sb <= 16 ? 16 : (sb <= 32 ? 32 : 64));
    const double avg = A->m > 0 ? (double)A->nnz / (double)A->m : 0.0;
    while (lpr > 8 && avg * lpr > CSR_VMAX) lpr >>= 1;
    return 64 / lpr;
}

hipError_t launch_kblock_csr(const KBlockArgs &a, hipStream_t st)
{
    const kdcd_matrix *A = a.A;
    const int rpw = csr_rows_per_wave(A, a.sb);
    // long rows: one wave per data row and per-lane sums (chunks of <= 8 rows)
    const bool wave = rpw == 8 && (double)A->nnz >= kCsrWaveMinAvg * (double)A->m;
    const int rows_per_wg = (CSR_NT / 64) * (wave ? 1 : rpw);
    const int64_t groups = groups_for(A->m);
    const int64_t n_w = a.W ? (a.sb + rows_per_wg - 1) / rows_per_wg : 0;
    dim3 grid((unsigned)(groups + n_w)), block(CSR_NT);
#define KDCD_CSR(RPW, KIND)                                                                   \
    hipLaunchKernelGGL((kblock_csr_kernel<RPW, KIND>), grid, block, 0, st, A->row_ptr,         \
                       A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms, a.kp, a.beta,  \
                       a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status)
#define KDCD_CSR_KIND(RPW)                                                                    \
    switch (a.kp.kind) {                                                                      \
    case KDCD_KERNEL_LINEAR: KDCD_CSR(RPW, KDCD_KERNEL_LINEAR); break;                        \
    case KDCD_KERNEL_POLY: KDCD_CSR(RPW, KDCD_KERNEL_POLY); break;                            \
    default: KDCD_CSR(RPW, KDCD_KERNEL_RBF); break;                                           \
    }
    if (wave) {
        switch (a.kp.kind) {
        case KDCD_KERNEL_LINEAR:
            hipLaunchKernelGGL((kblock_csr_wave_kernel<KDCD_KERNEL_LINEAR>), grid, block, 0, st,
                               A->row_ptr, A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms,
                               a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status);
            break;
        case KDCD_KERNEL_POLY:
            hipLaunchKernelGGL((kblock_csr_wave_kernel<KDCD_KERNEL_POLY>), grid, block, 0, st,
                               A->row_ptr, A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms,
                               a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status);
            break;
        default:
            hipLaunchKernelGGL((kblock_csr_wave_kernel<KDCD_KERNEL_RBF>), grid, block, 0, st,
                               A->row_ptr, A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms,
                               a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status);
            break;
        }
        return hipGetLastError();
    }
    switch (rpw) {
    case 1: KDCD_CSR_KIND(1) break;
    case 2: KDCD_CSR_KIND(2) break;
    case 4: KDCD_CSR_KIND(4) break;
    default: KDCD_CSR_KIND(8) break;
    }
#undef KDCD_CSR_KIND
#undef KDCD_CSR
    return hipGetLastError();
}

}  // namespace kdcd
