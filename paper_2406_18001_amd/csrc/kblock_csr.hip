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
template <class MaskT, int LPR, int NT = CSR_NT>
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
        // the lengths of sampled rows j0 .. j0 + LPR - 1 are loaded in parallel by
        // the first wave; the chunk takes the longest prefix that fits the panel
        static_assert(LPR <= 64, "one wave covers the chunk");
        if (tid < 64) {
            const int lane = tid;
            const bool ok = lane < LPR && j0 + lane < sb;
            int len = 0;
            if (ok) {
                const int64_t r = clampi(S[j0 + lane], 0, m - 1);
                len = (int)(rp(r + 1) - rp(r));
            }
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int up = __shfl_up(incl, o, 64);
                if (lane >= o) incl += up;
            }
            // incl is nondecreasing and ok a prefix, so the rows that fit form a prefix
            const int nrows = __popcll(__ballot(ok && incl <= CSR_VMAX));
            if (lane < nrows) rowoff[lane + 1] = incl;
            if (lane == 0) {
                rowoff[0] = 0;
                scan[0] = nrows;
            }
        }
        __syncthreads();
        const int nrows = scan[0];
        __syncthreads();                  // scan[] is reused below
        if (nrows == 0) return -2;        // one sampled row alone exceeds the panel
        j1 = j0 + nrows;
        tot = rowoff[nrows];
    }
    for (int x = tid; x < CSR_HS; x += NT) {
        hkey[x] = -1;
        hmask[x] = 0;
    }
    for (int x = tid; x < CSR_FBITS / 32; x += NT) hfilt[x] = 0u;
    __syncthreads();
    // 1. insert every stored entry's column, mark which sampled row holds it
    for (int f = tid; f < tot; f += NT) {
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
    constexpr int PER = CSR_HS / NT;
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) cnt += popc(hmask[tid * PER + q]);
    scan[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {   // Hillis-Steele inclusive scan
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
    for (int f = tid; f < tot; f += NT) {
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
    int32_t n_row_groups, double *__restrict__ carry, int32_t *status, int32_t jbeg,
    int32_t jend, const int32_t *__restrict__ gate, double *__restrict__ U)
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

    if (gate && *gate == 0) return;   // the dense-head pass handled this chunk
    for (int j0 = jbeg; j0 < jend;) {
        int j1 = build_panel<MaskT, LPR>(j0, -1, row_ptr, col_idx, val, m, nnz, S, jend, hkey, hfilt,
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
            build_panel<MaskT, LPR>(j0, pc, row_ptr, col_idx, val, m, nnz, S, jend, hkey, hfilt, hmask,
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
                        if (U) U[(int64_t)(j0 + jl) * m + row] = kv;
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
    int32_t n_row_groups, double *__restrict__ carry, int32_t *status, int32_t jbeg,
    int32_t jend, const int32_t *__restrict__ gate, double *__restrict__ U)
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

    if (gate && *gate == 0) return;
    for (int j0 = jbeg; j0 < jend;) {
        int j1 = build_panel<MaskT, WJ>(j0, -1, row_ptr, col_idx, val, m, nnz, S, jend, hkey, hfilt,
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
            build_panel<MaskT, WJ>(j0, pc, row_ptr, col_idx, val, m, nnz, S, jend, hkey, hfilt, hmask,
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
                        if (U) U[(int64_t)(j0 + lane) * m + row] = kv;
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

// ---------------------------------------------------------------- dense head
// Chunks of up to 32 sampled rows, short data rows.  The panel's most shared
// columns -- those stored by at least t* of the chunk's sampled rows, t* the
// smallest count that keeps them <= HD_HEAD -- carry most of the multiply-adds
// (on the C3 workload the 50-odd columns stored by four or more of the 32
// sampled rows carry over nine tenths).  For them a dense HD_HEAD x 32 block
// Bh of the sampled rows' values is kept; every wave scatters the head entries
// of 16 data rows into a dense 16 x HD_HEAD tile X in LDS and forms X Bh^T on
// v_mfma_f64_16x16x4.  Entries in the other panel columns (a few sampled rows
// each) are added to per-row sums Pt in LDS with atomics.  Each wave owns its
// rows' X and Pt, and one wave's atomics apply in lane and instruction order,
// so every sum has a fixed order.
//
// The panel is built once per chunk by csr_panel_build_kernel (one workgroup,
// an LDS hash of the chunk's columns) into workspace memory: a 16-byte record
// per column of A, the tail values and Bh.  A record holds a code word -- the
// build's epoch, a head flag, and the head position or the offset of the
// column's values in tval -- the sampled rows that store the column, and the
// first of its values.  A data entry needs one record load, and most tail
// entries (one sampled row) nothing more.  Records of other epochs are not in
// the panel, so nothing is cleared between builds.  A chunk of more than
// HD_CAP stored entries is left to the broadcast kernel (the build raises a
// flag that gates both passes).
constexpr int HD_NT = 128;                 // 2 waves
constexpr int HD_NJ = 32;                  // sampled rows per chunk
constexpr int HD_HEAD = 64;                // largest dense head
constexpr int HD_RB = 16;                  // data rows per wave block (one MFMA row block)
constexpr int HD_XLD = HD_HEAD + 1;        // padded row of X (rows land in different banks)
constexpr int HD_PLD = HD_NJ + 1;          // padded row of Pt
constexpr int HD_MAXGROUPS = 2048;         // eight workgroups per CU
constexpr int HD_FBGROUPS = 128;           // row groups of the broadcast fallback
constexpr int HD_BUILD_NT = 1024;
constexpr int HD_EPT = 4;                  // stored entries per build thread
constexpr int HD_CAP = HD_BUILD_NT * HD_EPT;   // stored entries of one chunk
constexpr int HD_HS = 2 * HD_CAP;          // build hash slots (power of two)
// code word: epoch << HD_EPOCH_SHIFT | HD_HEADBIT (head) | position or offset
constexpr int HD_EPOCH_SHIFT = 13;
constexpr uint32_t HD_HEADBIT = 1u << 12;
constexpr uint32_t HD_VALMASK = HD_HEADBIT - 1u;
constexpr uint32_t HD_EPOCH_END = 1u << (32 - HD_EPOCH_SHIFT);   // epochs 1 .. END-1
static_assert(HD_CAP <= (int)HD_HEADBIT, "tail offsets fit the code word");
static_assert(HD_HEAD <= (int)HD_HEADBIT, "head positions fit the code word");

// A tail column of the current chunk's panel.
struct __align__(16) TailRec {
    uint32_t mask;       // the sampled rows (bits) that store the column
    uint32_t pad;
    double v0;           // value of the first of them (also at tval[offset])
};

struct PanelMeta {
    uint32_t epoch;      // epoch of the last build (0: none since the init)
    int32_t nh;          // head columns
    int32_t fallback;    // 1: the chunk exceeds HD_CAP, the broadcast kernel runs it
    int32_t pad;
};

struct PanelPtrs {
    PanelMeta *meta;
    uint32_t *code;      // n: code word of every column (another epoch: not in the panel)
    TailRec *tail;       // n: set for the tail columns of the current chunk
    double *tval;        // HD_CAP tail values, per column in sampled-row order
    double *Bh;          // HD_HEAD x HD_NJ
};

__host__ __device__ inline size_t hd_al(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline PanelPtrs panel_ptrs(void *base, int64_t n)
{
    char *p = static_cast<char *>(base);
    PanelPtrs q;
    q.meta = reinterpret_cast<PanelMeta *>(p); p += 256;
    q.code = reinterpret_cast<uint32_t *>(p); p += hd_al(sizeof(uint32_t) * (size_t)n);
    q.tail = reinterpret_cast<TailRec *>(p); p += hd_al(sizeof(TailRec) * (size_t)n);
    q.tval = reinterpret_cast<double *>(p); p += hd_al(sizeof(double) * HD_CAP);
    q.Bh = reinterpret_cast<double *>(p);
    return q;
}

inline size_t panel_bytes(int64_t n)
{
    return 256 + hd_al(sizeof(uint32_t) * (size_t)n) + hd_al(sizeof(TailRec) * (size_t)n) +
           hd_al(sizeof(double) * HD_CAP) +
           hd_al(sizeof(double) * HD_HEAD * HD_NJ);
}

__global__ __launch_bounds__(256) void csr_panel_init_kernel(void *base, int64_t n)
{
    const PanelPtrs q = panel_ptrs(base, n);
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256)
        q.code[c] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *q.meta = PanelMeta{0u, 0, 0, 0};
}

__device__ __forceinline__ uint32_t hd_hash(int32_t c)
{
    return ((uint32_t)c * 2654435761u) & (HD_HS - 1);
}

// The panel of sampled rows S[0 .. nj) (nj <= HD_NJ), one workgroup.  Entry f
// of the chunk (its rows' stored entries concatenated in sampled-row order) is
// held by thread f % HD_BUILD_NT; the first entry of a column numbers it, so
// head positions and tail offsets follow the chunk's order and do not depend
// on the order of the hash inserts.
__global__ __launch_bounds__(HD_BUILD_NT) void csr_panel_build_kernel(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const double *__restrict__ val, int64_t m, int64_t nnz, const int32_t *__restrict__ S,
    int32_t nj, int64_t n, void *base)
{
    constexpr int NWB = HD_BUILD_NT / 64;
    const PanelPtrs q = panel_ptrs(base, n);
    __shared__ int32_t hkey[HD_HS];
    __shared__ uint32_t hmask[HD_HS];
    __shared__ int32_t hcode[HD_HS];       // first entry of the column, then its code
    __shared__ int32_t rowoff[HD_NJ + 1];
    __shared__ int64_t rowbeg[HD_NJ];
    __shared__ int32_t wsum[2][HD_EPT][NWB];
    __shared__ int32_t hist[HD_NJ + 2];
    __shared__ int32_t info[1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    auto rp = [&](int64_t r) { return clampi(row_ptr[clampi(r, 0, m)], 0, nnz); };

    // 1. the new epoch (after the last one every record is reset first); empty
    //    hash; entry ranges of the sampled rows
    uint32_t epoch = q.meta->epoch + 1u;
    if (epoch >= HD_EPOCH_END) {
        for (int64_t c = tid; c < n; c += HD_BUILD_NT) q.code[c] = 0u;
        epoch = 1u;
    }
    for (int x = tid; x < HD_HEAD * HD_NJ; x += HD_BUILD_NT) q.Bh[x] = 0.0;
    for (int x = tid; x < HD_HS; x += HD_BUILD_NT) {
        hkey[x] = -1;
        hmask[x] = 0u;
        hcode[x] = INT32_MAX;
    }
    if (tid < HD_NJ + 2) hist[tid] = 0;
    if (wid == 0) {
        int len = 0;
        int64_t b0 = 0;
        if (lane < nj) {
            const int64_t r = clampi(S[lane], 0, m - 1);
            b0 = rp(r);
            len = (int)(rp(r + 1) - b0);
        }
        int incl = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int up = __shfl_up(incl, o, 64);
            if (lane >= o) incl += up;
        }
        if (lane < nj) {
            rowoff[lane + 1] = incl;
            rowbeg[lane] = b0;
        }
        if (lane == 0) rowoff[0] = 0;
    }
    __syncthreads();
    const int total = rowoff[nj];
    if (total > HD_CAP) {
        if (tid == 0) *q.meta = PanelMeta{epoch, 0, 1, 0};
        return;
    }

    // 2. this thread's entries and their sampled rows
    int32_t cc[HD_EPT], jv[HD_EPT], hh[HD_EPT];
    double vv[HD_EPT];
#pragma unroll
    for (int u = 0; u < HD_EPT; ++u) {
        const int f = tid + HD_BUILD_NT * u;
        int jj = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1)
            if (jj + step < nj && rowoff[jj + step] <= f) jj += step;
        const int64_t e = clampi(rowbeg[jj] + (f - rowoff[jj]), 0, nnz - 1);
        jv[u] = jj;
        cc[u] = f < total ? col_idx[e] : -1;
        vv[u] = f < total ? val[e] : 0.0;
    }
    // 3. hash the columns: slot, sampled-row mask, first entry
#pragma unroll
    for (int u = 0; u < HD_EPT; ++u) {
        hh[u] = -1;
        const int32_t c = cc[u];
        if (c < 0 || c >= n) continue;    // also a malformed matrix (its check reports it)
        uint32_t h = hd_hash(c);
        for (;;) {                         // at most HD_CAP keys in HD_HS slots: ends
            const int32_t old = atomicCAS(&hkey[h], -1, c);
            if (old == -1 || old == c) break;
            h = (h + 1) & (HD_HS - 1);
        }
        hh[u] = (int)h;
        atomicMin(&hcode[h], tid + HD_BUILD_NT * u);
        atomicOr(&hmask[h], 1u << jv[u]);
    }
    __syncthreads();
    // 4. owners (first entries) and the histogram of their sampled-row counts
    bool own[HD_EPT];
    uint32_t mk[HD_EPT];
#pragma unroll
    for (int u = 0; u < HD_EPT; ++u) {
        own[u] = hh[u] >= 0 && hcode[hh[u]] == tid + HD_BUILD_NT * u;
        mk[u] = hh[u] >= 0 ? hmask[hh[u]] : 0u;
        if (own[u]) atomicAdd(&hist[__popc(mk[u])], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int t = HD_NJ + 1, acc = 0;
        while (t > 1 && acc + hist[t - 1] <= HD_HEAD) acc += hist[--t];
        info[0] = t;          // columns stored by >= t sampled rows form the head
    }
    __syncthreads();
    const int tstar = info[0];
    // 5. head positions and tail offsets in chunk order: scans over the waves
    int hx[HD_EPT], tx[HD_EPT];
    bool head[HD_EPT];
#pragma unroll
    for (int u = 0; u < HD_EPT; ++u) {
        head[u] = own[u] && __popc(mk[u]) >= tstar;
        const int a0 = head[u] ? 1 : 0, b0 = (own[u] && !head[u]) ? __popc(mk[u]) : 0;
        int a = a0, b = b0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int ua = __shfl_up(a, o, 64), ub = __shfl_up(b, o, 64);
            if (lane >= o) {
                a += ua;
                b += ub;
            }
        }
        if (lane == 63) {
            wsum[0][u][wid] = a;
            wsum[1][u][wid] = b;
        }
        hx[u] = a - a0;
        tx[u] = b - b0;
    }
    __syncthreads();
    const uint32_t ep = epoch << HD_EPOCH_SHIFT;
    int oa = 0, ob = 0;
#pragma unroll
    for (int u = 0; u < HD_EPT; ++u) {
        int pa = oa, pb = ob;
        for (int w = 0; w < NWB; ++w) {
            if (w < wid) {
                pa += wsum[0][u][w];
                pb += wsum[1][u][w];
            }
            oa += wsum[0][u][w];
            ob += wsum[1][u][w];
        }
        if (own[u]) hcode[hh[u]] = (int32_t)(ep | (head[u] ? (HD_HEADBIT | (uint32_t)(pa + hx[u]))
                                                              : (uint32_t)(pb + tx[u])));
    }
    const int nh = oa;
    __syncthreads();
    // 6. values into the head block or tval; the owners write the records
#pragma unroll
    for (int u = 0; u < HD_EPT; ++u) {
        if (hh[u] < 0) continue;
        const uint32_t code = (uint32_t)hcode[hh[u]];
        const int jj = jv[u];
        if (code & HD_HEADBIT)
            q.Bh[(code & HD_VALMASK) * HD_NJ + jj] = vv[u];
        else
            q.tval[(code & HD_VALMASK) + __popc(mk[u] & ((1u << jj) - 1u))] = vv[u];
        if (own[u]) {
            q.code[cc[u]] = code;
            if (!(code & HD_HEADBIT)) q.tail[cc[u]] = TailRec{mk[u], 0u, vv[u]};
        }
    }
    if (tid == 0) *q.meta = PanelMeta{epoch, nh, 0, 0};
}

// One workgroup = two waves on blocks of 16 data rows.  Wave w walks the
// entries of rows 8 w .. 8 w + 7 of a block (eight lanes a row, entry k of a
// row at lane k % 8) into X and Pt, and forms output columns 16 w .. 16 w + 15
// (a 16 x 16 MFMA block) of all 16 rows.  Each wave writes only its own rows
// of X and Pt, so Pt's atomics stay in one wave (fixed order).
template <int KIND>
__global__ __launch_bounds__(HD_NT) __attribute__((amdgpu_waves_per_eu(KIND == KDCD_KERNEL_RBF ? 3 : 4))) void kblock_csr_head_kernel(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const double *__restrict__ val, int64_t m, int64_t nnz, int64_t n,
    const int32_t *__restrict__ S, int32_t sb, int32_t j0, int32_t nj,
    const double *__restrict__ norms, KParams kp, const double *__restrict__ beta,
    const double *__restrict__ bscale, double *__restrict__ partial, double *__restrict__ W,
    int32_t n_row_groups, const void *__restrict__ pbase, double *__restrict__ U)
{
    const PanelPtrs q = panel_ptrs(const_cast<void *>(pbase), n);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool is_w = (int)blockIdx.x >= n_row_groups;
    if (q.meta->fallback) {
        // the broadcast kernel runs this chunk on its first HD_FBGROUPS row
        // groups; the other groups' sums for it are zero
        if (!is_w && (int)blockIdx.x >= HD_FBGROUPS && tid < nj)
            partial[(int64_t)blockIdx.x * sb + j0 + tid] = 0.0;
        return;
    }
    if (is_w && W == nullptr) return;
    __shared__ double X[HD_RB][HD_XLD];
    __shared__ double Pt[HD_RB][HD_PLD];
    __shared__ double bsh[HD_RB], nsh[HD_RB];   // the block's rows: beta (scaled), norms
    __shared__ int64_t rsh[HD_RB];              // and their row indices

    auto rp = [&](int64_t r) { return clampi(row_ptr[clampi(r, 0, m)], 0, nnz); };
    const int li = lane & 15, lk = lane >> 4;          // MFMA operand row / k slot
    const int tr = 8 * wid + (lane >> 3), sub = lane & 7;   // entry walk: row tr, every 8th entry
    const int jj = 16 * wid + li;                      // this lane's output column
    const uint32_t epoch = q.meta->epoch;

    // this lane's part of Bh (B operand of every k-step), in registers
    double bh[HD_HEAD / 4];
#pragma unroll
    for (int ks = 0; ks < HD_HEAD / 4; ++ks) bh[ks] = q.Bh[(4 * ks + lk) * HD_NJ + jj];
    const int64_t Sj = clampi(S[j0 + (jj < nj ? jj : 0)], 0, m - 1);
    const double nb = (KIND == KDCD_KERNEL_RBF) ? norms[Sj] : 0.0;
    double colsum = 0.0;

    const int64_t nblk = is_w ? (sb + HD_RB - 1) / HD_RB : (m + HD_RB - 1) / HD_RB;
    const int64_t b_first = is_w ? (int64_t)((int)blockIdx.x - n_row_groups) : (int64_t)blockIdx.x;
    const int64_t b_end = is_w ? min(nblk, b_first + 1) : nblk;
    const int64_t b_step = is_w ? 1 : (int64_t)n_row_groups;
    // entry range of this lane's row tr of block blk
    auto rowinfo = [&](int64_t blk, int64_t &b0, int32_t &len) {
        b0 = 0;
        len = 0;
        if (blk < b_end) {
            const int64_t rix = blk * HD_RB + tr;
            const bool rok = is_w ? rix < sb : rix < m;
            const int64_t row = is_w ? clampi(S[clampi(rix, 0, sb - 1)], 0, m - 1) : rix;
            if (rok) {
                b0 = rp(row);
                len = (int32_t)(rp(row + 1) - b0);
            }
        }
    };
    // Every lane loads an entry of its row (index clamped into the row) and
    // then a record (column clamped into [0, n)); entries past the row's end
    // are dropped afterwards.
    constexpr int HD_EPL = KIND == KDCD_KERNEL_RBF ? 5 : 7;
    constexpr int BATCH = 8 * HD_EPL;                  // entries of a row per batch
    const uint32_t nlast = (uint32_t)(n - 1);
    double *xrow = &X[tr][0];
    double *prow = &Pt[tr][0];
    int64_t nb0;
    int32_t nlen;
    rowinfo(b_first, nb0, nlen);
    for (int64_t blk = b_first; blk < b_end; blk += b_step) {
        // this lane's row's entries (the next block's range is loaded now, in
        // flight while this one is processed); this wave's rows of the tiles
        // zeroed
        const int32_t len = nnz > 0 ? nlen : 0;
        // a row with no entries reads entry 0 of its range, moved into the array
        const int64_t b0 = len > 0 ? nb0 : min(nb0, nnz - 1);
        const int32_t *cp = col_idx + b0;
        const double *vp = val + b0;
        rowinfo(blk + b_step, nb0, nlen);
        constexpr int XW = (HD_RB / 2) * HD_XLD, PW = (HD_RB / 2) * HD_PLD;
#pragma unroll
        for (int i = 0; i < (XW + 63) / 64; ++i) {
            const int x = lane + 64 * i;
            if (i + 1 < (XW + 63) / 64 || x < XW) (&X[8 * wid][0])[x] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < (PW + 63) / 64; ++i) {
            const int x = lane + 64 * i;
            if (i + 1 < (PW + 63) / 64 || x < PW) (&Pt[8 * wid][0])[x] = 0.0;
        }
        // wave 0, lanes < 16: row blk * 16 + lane's beta, scale and norm
        double b0v = 0.0, b0s = 1.0, n0v = 0.0;
        int64_t r0 = 0;
        bool rok0 = false;
        if (wid == 0 && lane < HD_RB) {
            const int64_t rix = blk * HD_RB + lane;
            rok0 = is_w ? rix < sb : rix < m;
            r0 = is_w ? clampi(S[clampi(rix, 0, sb - 1)], 0, m - 1) : clampi(rix, 0, m - 1);
            if (!is_w) {
                b0v = beta[r0];
                if (bscale) b0s = bscale[r0];
            }
            if (KIND == KDCD_KERNEL_RBF) n0v = norms[r0];
        }
        wave_lds_sync();
        const int32_t klast = max(len - 1, 0);
        for (int k0 = 0; __ballot(k0 < len) != 0; k0 += BATCH) {    // uniform
            int32_t cu[HD_EPL];
            double vu[HD_EPL];
#pragma unroll
            for (int u = 0; u < HD_EPL; ++u) {
                const int k = min(k0 + sub + 8 * u, klast);
                cu[u] = cp[k];
                vu[u] = vp[k];
            }
            // code words: head entries go to X now; tail entries fetch their
            // column's tail record (all fetches in flight together)
            uint32_t cd[HD_EPL];
#pragma unroll
            for (int u = 0; u < HD_EPL; ++u) cd[u] = q.code[min((uint32_t)cu[u], nlast)];
            bool tl[HD_EPL];
#pragma unroll
            for (int u = 0; u < HD_EPL; ++u) {
                const bool in = k0 + sub + 8 * u < len && (cd[u] >> HD_EPOCH_SHIFT) == epoch &&
                                (uint32_t)cu[u] <= nlast;
                tl[u] = in && !(cd[u] & HD_HEADBIT);
                if (in && (cd[u] & HD_HEADBIT)) xrow[cd[u] & (HD_HEAD - 1)] = vu[u];
            }
            TailRec ru[HD_EPL];
#pragma unroll
            for (int u = 0; u < HD_EPL; ++u) ru[u] = tl[u] ? q.tail[cu[u]] : TailRec{0u, 0u, 0.0};
            uint32_t rem[HD_EPL];
            bool more = false;
#pragma unroll
            for (int u = 0; u < HD_EPL; ++u) {
                rem[u] = 0u;
                if (tl[u]) {
                    const uint32_t msk = ru[u].mask;
                    atomicAdd(&prow[__builtin_ctz(msk)], vu[u] * ru[u].v0);
                    rem[u] = msk & (msk - 1u);
                }
                more |= rem[u] != 0u;
            }
            // further sampled rows of tail entries, in rounds: one tval load per
            // entry and round
            for (int kk = 1; __ballot(more) != 0; ++kk) {    // uniform
                double tv[HD_EPL];
#pragma unroll
                for (int u = 0; u < HD_EPL; ++u)
                    tv[u] = q.tval[rem[u] ? (cd[u] & HD_VALMASK) + kk : 0];
                more = false;
#pragma unroll
                for (int u = 0; u < HD_EPL; ++u) {
                    if (rem[u]) {
                        atomicAdd(&prow[__builtin_ctz(rem[u])], vu[u] * tv[u]);
                        rem[u] &= rem[u] - 1u;
                    }
                    more |= rem[u] != 0u;
                }
            }
        }
        // the block's rows, staged for the epilogue by wave 0 (loaded before
        // the entry walk, so their latency hides behind it)
        if (wid == 0 && lane < HD_RB) {
            bsh[lane] = rok0 ? b0v * b0s : 0.0;
            nsh[lane] = n0v;
            rsh[lane] = r0;
        }
        lds_barrier();            // both waves' rows of X / Pt, and the staged rows, are in
        double bvv[4], nav[4];
        int64_t rowv[4];
        bool rokv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = lk + 4 * v;
            const int64_t rix = blk * HD_RB + t;
            rokv[v] = is_w ? rix < sb : rix < m;
            rowv[v] = rsh[t];
            bvv[v] = bsh[t];
            nav[v] = nsh[t];
        }
        // head product on MFMA: this wave's 16 x 16 block of P = X Bh^T (X
        // columns and Bh rows past the head are zero)
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < HD_HEAD / 4; ++ks)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[li][4 * ks + lk], bh[ks], acc, 0, 0, 0);
        // item v of lane l: row l/16 + 4 v of the block.  U-part: rows past the
        // end have beta 0, and the sums of sampled rows past nj are never
        // written.  (The exponential map is not unrolled: its copies would spill.)
#pragma unroll(KIND == KDCD_KERNEL_RBF ? 1 : 4)
        for (int v = 0; v < 4; ++v) {
            const int t = lk + 4 * v;
            const double pv = acc[v] + Pt[t][jj];
            const double kv = kernel_map<KIND>(pv, nav[v], nb, rowv[v] == Sj, kp);
            if (is_w) {
                if (rokv[v] && jj < nj) W[(blk * HD_RB + t) * sb + j0 + jj] = kv;
            } else {
                colsum += bvv[v] * kv;
                if (U && rokv[v] && jj < nj) U[(int64_t)(j0 + jj) * m + rowv[v]] = kv;
            }
        }
        lds_barrier();            // the block's X / Pt reads are done
    }
    if (!is_w) {
        // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same column
        double v = colsum;
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lane < 16 && jj < nj) partial[(int64_t)blockIdx.x * sb + j0 + jj] = v;
    }
}

int64_t groups_for(int64_t m)
{
    const int64_t steps = (m + 15) / 16;
    return steps < CSR_MAXGROUPS ? steps : CSR_MAXGROUPS;
}

}  // namespace

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

// Kernel choice: long rows (average >= kCsrWaveMinAvg at <= 8 sampled rows per
// chunk) -> one wave per row; more than 16 sampled rows -> the dense-head
// kernel; otherwise the broadcast / scatter kernel.
enum CsrPath { CSR_BROADCAST, CSR_WAVE, CSR_HEAD };
CsrPath csr_path(const kdcd_matrix *A, int32_t sb)
{
    const int rpw = csr_rows_per_wave(A, sb);
    if (rpw == 8 && (double)A->nnz >= kCsrWaveMinAvg * (double)A->m) return CSR_WAVE;
    return sb > 16 ? CSR_HEAD : CSR_BROADCAST;
}

int64_t kblock_csr_row_groups(const kdcd_matrix *A, int32_t sb)
{
    if (csr_path(A, sb) == CSR_HEAD) {
        const int64_t steps = (A->m + HD_RB - 1) / HD_RB;   // 16 rows per step
        return steps < HD_MAXGROUPS ? steps : HD_MAXGROUPS;
    }
    return groups_for(A->m);
}

int64_t kblock_csr_max_row_groups(int64_t m)
{
    const int64_t head = std::min<int64_t>((m + HD_RB - 1) / HD_RB, HD_MAXGROUPS);
    return std::max<int64_t>(head, groups_for(m));
}

size_t kblock_csr_panel_bytes(int64_t n) { return panel_bytes(n); }

hipError_t launch_csr_panel_init(const kdcd_matrix *A, void *panel, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>((A->n + 255) / 256, 4096);
    hipLaunchKernelGGL(csr_panel_init_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256),
                       0, st, panel, A->n);
    return hipGetLastError();
}

hipError_t launch_kblock_csr(const KBlockArgs &a, hipStream_t st)
{
    const kdcd_matrix *A = a.A;
    const int rpw = csr_rows_per_wave(A, a.sb);
    const CsrPath path = csr_path(A, a.sb);
    if (path == CSR_HEAD && a.csr_panel) {
        // per chunk of HD_NJ sampled rows: panel build, dense-head pass, and the
        // broadcast kernel gated on the build's fallback flag (left out when the
        // longest row of A says that the chunk fits the panel)
        const int64_t groups = kblock_csr_row_groups(A, a.sb);
        const int64_t n_w = a.W ? (a.sb + HD_RB - 1) / HD_RB : 0;
        const PanelPtrs q = panel_ptrs(a.csr_panel, A->n);
        const int64_t rows_per_wg_b = (CSR_NT / 64) * rpw;
        const int64_t n_w_b = a.W ? (a.sb + rows_per_wg_b - 1) / rows_per_wg_b : 0;
        const int64_t groups_b = std::min<int64_t>(groups, HD_FBGROUPS);
        // the stage timer covers the dense-head passes (from the first chunk's to
        // the last chunk's; the builds and gated passes between them included)
        ArmedEvents armed = armed_events();
        armed_events() = ArmedEvents{nullptr, nullptr};
        for (int32_t j0 = 0; j0 < a.sb; j0 += HD_NJ) {
            const int32_t nj = std::min<int32_t>(HD_NJ, a.sb - j0);
            const bool first = j0 == 0, lastc = j0 + HD_NJ >= a.sb;
            hipLaunchKernelGGL(csr_panel_build_kernel, dim3(1), dim3(HD_BUILD_NT), 0, st, A->row_ptr,
                               A->col_idx, A->values, A->m, A->nnz, a.S + j0, nj, A->n, a.csr_panel);
            if (first && armed.start) (void)hipEventRecord(armed.start, st);
            dim3 grid((unsigned)(groups + n_w)), block(HD_NT);
#define KDCD_CSR_HEAD(KIND)                                                                    \
    hipLaunchKernelGGL((kblock_csr_head_kernel<KIND>), grid, block, 0, st, A->row_ptr,          \
                       A->col_idx, A->values, A->m, A->nnz, A->n, a.S, a.sb, j0, nj, a.norms,  \
                       a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.csr_panel, a.U)
            switch (a.kp.kind) {
            case KDCD_KERNEL_LINEAR: KDCD_CSR_HEAD(KDCD_KERNEL_LINEAR); break;
            case KDCD_KERNEL_POLY: KDCD_CSR_HEAD(KDCD_KERNEL_POLY); break;
            default: KDCD_CSR_HEAD(KDCD_KERNEL_RBF); break;
            }
#undef KDCD_CSR_HEAD
            if (lastc && armed.stop) (void)hipEventRecord(armed.stop, st);
            // no chunk of nj rows of at most csr_max_row entries overflows the panel
            if (a.csr_max_row >= 0 && a.csr_max_row * (int64_t)nj <= HD_CAP) continue;
            dim3 gridb((unsigned)(groups_b + n_w_b)), blockb(CSR_NT);
#define KDCD_CSR_FB(RPW, KIND)                                                                  \
    hipLaunchKernelGGL((kblock_csr_kernel<RPW, KIND>), gridb, blockb, 0, st, A->row_ptr,          \
                       A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms, a.kp, a.beta,    \
                       a.beta_scale, a.partial, a.W, (int32_t)groups_b, a.carry, a.status, j0,   \
                       j0 + nj, &q.meta->fallback, a.U)
#define KDCD_CSR_FB_KIND(RPW)                                                                   \
    switch (a.kp.kind) {                                                                        \
    case KDCD_KERNEL_LINEAR: KDCD_CSR_FB(RPW, KDCD_KERNEL_LINEAR); break;                       \
    case KDCD_KERNEL_POLY: KDCD_CSR_FB(RPW, KDCD_KERNEL_POLY); break;                           \
    default: KDCD_CSR_FB(RPW, KDCD_KERNEL_RBF); break;                                          \
    }
            switch (rpw) {
            case 1: KDCD_CSR_FB_KIND(1) break;
            case 2: KDCD_CSR_FB_KIND(2) break;
            case 4: KDCD_CSR_FB_KIND(4) break;
            default: KDCD_CSR_FB_KIND(8) break;
            }
#undef KDCD_CSR_FB_KIND
#undef KDCD_CSR_FB
        }
        return hipGetLastError();
    }
    // long rows: one wave per data row and per-lane sums (chunks of <= 8 rows)
    const bool wave = path == CSR_WAVE;
    const int64_t groups = kblock_csr_row_groups(A, a.sb);
    const int rows_per_wg = (CSR_NT / 64) * (wave ? 1 : rpw);
    const int64_t n_w = a.W ? (a.sb + rows_per_wg - 1) / rows_per_wg : 0;
    dim3 grid((unsigned)(groups + n_w)), block(CSR_NT);
#define KDCD_CSR(RPW, KIND)                                                                   \
    KDCD_TIMED_LAUNCH((kblock_csr_kernel<RPW, KIND>), grid, block, 0, st, A->row_ptr,          \
                       A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms, a.kp, a.beta,  \
                       a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status, 0, a.sb, \
                       nullptr, a.U)
#define KDCD_CSR_KIND(RPW)                                                                    \
    switch (a.kp.kind) {                                                                      \
    case KDCD_KERNEL_LINEAR: KDCD_CSR(RPW, KDCD_KERNEL_LINEAR); break;                        \
    case KDCD_KERNEL_POLY: KDCD_CSR(RPW, KDCD_KERNEL_POLY); break;                            \
    default: KDCD_CSR(RPW, KDCD_KERNEL_RBF); break;                                           \
    }
    if (wave) {
        switch (a.kp.kind) {
        case KDCD_KERNEL_LINEAR:
            KDCD_TIMED_LAUNCH((kblock_csr_wave_kernel<KDCD_KERNEL_LINEAR>), grid, block, 0, st,
                               A->row_ptr, A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms,
                               a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status,
                               0, a.sb, nullptr, a.U);
            break;
        case KDCD_KERNEL_POLY:
            KDCD_TIMED_LAUNCH((kblock_csr_wave_kernel<KDCD_KERNEL_POLY>), grid, block, 0, st,
                               A->row_ptr, A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms,
                               a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status,
                               0, a.sb, nullptr, a.U);
            break;
        default:
            KDCD_TIMED_LAUNCH((kblock_csr_wave_kernel<KDCD_KERNEL_RBF>), grid, block, 0, st,
                               A->row_ptr, A->col_idx, A->values, A->m, A->nnz, a.S, a.sb, a.norms,
                               a.kp, a.beta, a.beta_scale, a.partial, a.W, (int32_t)groups, a.carry, a.status,
                               0, a.sb, nullptr, a.U);
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
