// The recurrence of one K-RR index block run inside a lookahead launch (see
// LookaheadArgs): workgroup 0 of the dense FP64, the FP32 and the
// low-precision kernel-block products calls it.
#pragma once

#include "common.hpp"

namespace kdcd {

__device__ __forceinline__ int64_t la_clamp(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double la_readlane(double v, int l)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The recurrence of one K-RR index block (Algorithm 4's inner loop, Eq. (3)),
// run by workgroup 0 of a lookahead launch while the other workgroups compute
// the next block's product.  With c_e = y_{S_e} - m alpha_{S_e} - r_e / lambda
// and G[t][u] = W[t][u] / lambda + m [S_t = S_u], the blocks are taken in
// order: block j's c (final once every earlier block is folded in) is
// published in LDS, lanes l < b of every wave form Delta_l = (D_j^{-1} c_j)_l
// and hand Delta_l / lambda to all lanes, and every element u of a later block
// subtracts sum_l W'[jb+l][u] Delta_l / lambda -- one barrier per block.  W' is
// the Gram with lambda m already added where a row's coordinate comes again
// later (the finish pass adds it while it copies such rows), so W' / lambda = G
// on every entry the recurrence reads.  Thread tid owns elements tid and
// tid + NT.  Nothing is written to alpha: the updates go to trace, and the
// summed update of each coordinate (in element order) to Dc on the element
// that the row -> position table names for it.  BX > 0 fixes b = BX at compile
// time.  LDS (inside the product's A buffers): S of the block, the updates, c
// of the current and next block, a ring of four D_j^{-1}, one bit per element.
template <int NT, int BX>
__device__ void la_recur(const LookaheadArgs &a, char *smem)
{
    constexpr int LB = BX > 0 ? BX : kLaMaxB;
    int32_t *S_l = reinterpret_cast<int32_t *>(smem);                  // [2 NT]
    double *d_l = reinterpret_cast<double *>(smem + 8 * NT);           // [2 NT]
    double *c_l = reinterpret_cast<double *>(smem + 24 * NT);          // [2][kLaMaxB]
    double *D_l = c_l + 2 * kLaMaxB;                                   // [4][64]
    uint32_t *mark = reinterpret_cast<uint32_t *>(D_l + 4 * 64);       // [2 NT / 32]
    const int tid = threadIdx.x, lane = tid & 63;
    const int sb = a.sb, sk = a.sk;
    const int b = BX > 0 ? BX : a.b;
    const int64_t m = a.m;
    const double inv_lambda = 1.0 / a.lambda, mdbl = a.mdbl;

    int32_t Se[kLaEPT];
    int blk[kLaEPT], ecl[kLaEPT];
    double c[kLaEPT];
#pragma unroll
    for (int i = 0; i < kLaEPT; ++i) {
        const int e = tid + i * NT;
        const bool act = e < sb;
        Se[i] = act ? (int32_t)la_clamp(a.S[e], 0, m - 1) : -1;
        blk[i] = act ? e / b : sk;              // sk: never folded, never published
        ecl[i] = act ? e : sb - 1;              // a valid column for the loads
        c[i] = act ? a.y[Se[i]] - mdbl * a.alpha[Se[i]] - a.r[e] / a.lambda : 0.0;
        if (act) S_l[e] = Se[i];
        if (blk[i] == 0) c_l[e] = c[i];
    }
    for (int x = tid; x < (2 * NT) / 32; x += NT) mark[x] = 0u;
    // Every load of the loop is unconditional, from an index clamped into the
    // array (values nobody uses are loaded and ignored): with a fixed number
    // of loads per block the compiler waits for exactly the stage it needs,
    // where a load behind a branch made it wait for all of them.
    // D_j^{-1} (b*b <= 64 values): one value per lane, stored by wave 0
    auto dinv_load = [&](int j) -> double {
        const int jj = j < sk ? j : sk - 1;
        const int ll = lane < b * b ? lane : b * b - 1;
        return a.Dinv[(int64_t)jj * b * b + ll];
    };
    // W' values of block j for this thread's elements (used for later blocks);
    // the row pointer is uniform, so each load is a scalar base plus a lane
    // offset (rows jj*b + l < sb when l < b)
    auto w_load = [&](int j, double (&w)[kLaEPT][LB]) {
        const int jj = j < sk ? j : sk - 1;
        const double *r0 = a.W + (int64_t)jj * b * sb;
#pragma unroll
        for (int l = 0; l < LB; ++l) {
            const double *rp = r0 + (int64_t)(BX > 0 || l < b ? l : b - 1) * sb;
#pragma unroll
            for (int i = 0; i < kLaEPT; ++i) w[i][l] = rp[ecl[i]];
        }
    };
    // Three register stages of W' values: block j is folded out of one while
    // the loads of blocks j + 1 and j + 2 are in flight in the other two (the
    // loop is unrolled by three so that no stage is ever copied: a copy would
    // wait for the loads).  D_j^{-1} goes through a ring of four LDS slots; its
    // load is issued before the block's W' loads, so storing it two blocks
    // later does not wait for them.
    double w0[kLaEPT][LB], w1[kLaEPT][LB], w2[kLaEPT][LB];
    if (tid < 64) {
        D_l[0 * 64 + lane] = dinv_load(0);
        D_l[1 * 64 + lane] = dinv_load(1);
    }
    double dreg = dinv_load(2);
    w_load(0, w0);
    w_load(1, w1);
    __syncthreads();
    // an index block holds distinct coordinates (Algorithm 4 samples without
    // replacement inside a block)
#pragma unroll
    for (int i = 0; i < kLaEPT; ++i) {
        const int e = tid + i * NT;
        if (blk[i] < sk)
            for (int q = blk[i] * b; q < blk[i] * b + b; ++q)
                if (q != e && S_l[q] == Se[i]) set_status(a.status, KDCD_ERR_INDEX_DUPLICATE);
    }

    auto step = [&](int j, const double (&wc)[kLaEPT][LB], double (&wf)[kLaEPT][LB]) {
        const int cb = j & 1;
        if (tid < 64) D_l[((j + 2) & 3) * 64 + lane] = dreg;
        dreg = dinv_load(j + 3);
        w_load(j + 2, wf);
        double dl = 0.0;
        if (lane < b) {
#pragma unroll
            for (int t = 0; t < LB; ++t)
                if (BX > 0 || t < b) dl += D_l[(j & 3) * 64 + lane * b + t] * c_l[cb * kLaMaxB + t];
            if (tid < 64) d_l[j * b + lane] = dl;
        }
        // Delta / lambda of the block on every lane (lane reads: scalar registers)
        const double dls = dl * inv_lambda;
        double dvs[LB];
#pragma unroll
        for (int l = 0; l < LB; ++l) dvs[l] = la_readlane(dls, l);   // lanes >= b hold 0
#pragma unroll
        for (int i = 0; i < kLaEPT; ++i) {
            const int e = tid + i * NT;
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < LB; ++l) acc += wc[i][l] * dvs[l];
            const bool later = blk[i] > j && blk[i] < sk;
            c[i] = later ? c[i] - acc : c[i];
            // the next block's c (an element past the end has blk = sk: never)
            if (later && blk[i] == j + 1) c_l[(cb ^ 1) * kLaMaxB + (e - (j + 1) * b)] = c[i];
        }
        lds_barrier();
    };
    for (int j = 0; j < sk; j += 3) {
        step(j, w0, w2);
        if (j + 1 < sk) step(j + 1, w1, w0);
        if (j + 2 < sk) step(j + 2, w2, w1);
    }

    // Canonical element of a coordinate: the one the row table names (its
    // last).  Every earlier element of the coordinate marks the canonical one,
    // and only a marked canonical element sums the coordinate's updates.
    int canon[kLaEPT];   // 1 canonical, 0 not, -1 no element
#pragma unroll
    for (int i = 0; i < kLaEPT; ++i) {
        const int e = tid + i * NT;
        canon[i] = -1;
        if (e < sb) {
            const int32_t q = a.pos[Se[i]];
            canon[i] = q == e ? 1 : 0;
            if (q != e && q >= 0 && q < sb) atomicOr(&mark[q >> 5], 1u << (q & 31));
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kLaEPT; ++i) {
        const int e = tid + i * NT;
        if (canon[i] < 0) continue;
        const double de = d_l[e];
        double v = 0.0;
        if (canon[i] == 1) {
            v = de;
            if (mark[e >> 5] & (1u << (e & 31))) {
                // earlier elements of this coordinate, in element order (eight
                // coordinates per step, read ahead of the compares)
                double sacc = 0.0;
                int t = 0;
                for (; t + 8 <= e; t += 8) {
                    int32_t s8[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) s8[q] = S_l[t + q];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (s8[q] == Se[i]) sacc += d_l[t + q];
                }
                for (; t < e; ++t)
                    if (S_l[t] == Se[i]) sacc += d_l[t];
                v = sacc + de;
            }
        }
        a.Dc[e] = v;
        a.Sc[e] = canon[i] == 1 ? Se[i] : -1;
        if (a.trace) a.trace[e] = de;
    }
}

}  // namespace kdcd
