// Learned coordinate sampler: a 4 -> 64 -> 64 -> 1 tanh MLP in FP32 that
// scores every coordinate of a K-SVM from its state, Gumbel-top-k selection
// of the s coordinates of an outer iteration (radix select over order-
// preserving 32-bit keys, then one bitonic sort of the candidates), the
// maintained dual gradient g = Q alpha - 1 + omega alpha, and the training
// kernels (per-sample forward/backward with a deterministic reduction, Adam).
//
// The paper draws coordinates uniformly (Algorithms 1-4 take the sequence as
// an input); this replaces only that draw.  Random numbers: Philox4x32-10
// (Salmon et al., SC 2011), counters (i, k, 0, 0) for coordinate noise,
// (j, k, 1, 0) for slot j, (p, 0, 2, 0) for initial weight p.
#include "common.hpp"
#include "sampler.hpp"

namespace kdcd {

// ------------------------------------------------------------------ Philox

__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c[0];
        const uint64_t p1 = (uint64_t)M1 * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__host__ __device__ inline double unit_of(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

// Glorot-uniform weights, zero biases (host side, once per model).
void sampler_init_params(float *p, uint64_t seed)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int q = 0; q < SMP_NP; ++q) {
        double a = 0.0;
        if (q < SMP_B1) a = std::sqrt(6.0 / (SMP_NIN + SMP_NH));
        else if (q >= SMP_W2 && q < SMP_B2) a = std::sqrt(6.0 / (SMP_NH + SMP_NH));
        else if (q >= SMP_W3 && q < SMP_B3) a = std::sqrt(6.0 / (SMP_NH + 1));
        if (a == 0.0) {
            p[q] = 0.0f;
            continue;
        }
        uint32_t c[4] = {(uint32_t)q, 0u, 2u, 0u};
        philox4x32_10(c, k0, k1);
        p[q] = (float)(a * (2.0 * unit_of(c[0]) - 1.0));
    }
}

namespace {

// ---------------------------------------------------------------- the MLP

// Parameters as staged in LDS: W2 rows padded to 65 floats so that the four
// lanes of a quad (rows o = q + 4j) read distinct banks.
constexpr int LW2 = SMP_NH + 1;
constexpr int LP_W1 = 0, LP_B1 = LP_W1 + SMP_NH * SMP_NIN, LP_W2 = LP_B1 + SMP_NH,
              LP_B2 = LP_W2 + SMP_NH * LW2, LP_W3 = LP_B2 + SMP_NH, LP_B3 = LP_W3 + SMP_NH,
              LP_N = LP_B3 + 1;

__device__ __forceinline__ void load_params_padded(float *sp, const float *__restrict__ params)
{
    for (int q = threadIdx.x; q < SMP_NP; q += blockDim.x) {
        int d;
        if (q < SMP_W2) d = q;                                   // W1, b1
        else if (q < SMP_B2) d = LP_W2 + ((q - SMP_W2) / SMP_NH) * LW2 + (q - SMP_W2) % SMP_NH;
        else d = LP_B2 + (q - SMP_B2);                           // b2, w3, b3
        sp[d] = params[q];
    }
    __syncthreads();
}

__device__ __forceinline__ void load_params(float *sp, const float *__restrict__ params)
{
    for (int q = threadIdx.x; q < SMP_NP; q += blockDim.x) sp[q] = params[q];
    __syncthreads();
}

// The scoring MLP f(x), evaluated by a quad of lanes (q = lane & 3) that
// holds the same x.  Lane q owns hidden units o = q + 4j, j = 0..15:
//   h1_o = tanh(b1_o + sum_i W1[o][i] x_i)            (fma chain, i ascending)
//   h2_o = tanh(b2_o + sum_i W2[o][i] h1_i)           (fma chain, i ascending)
//   C_q  = sum_j w3_o h2_o                             (fma chain from 0, j ascending)
//   f    = ((C_0 + C_1) + (C_2 + C_3)) + b3
// Every inference path uses this routine, so a coordinate's score has the
// same bits wherever it is computed.  h1row: this quad's 64-float LDS row.
__device__ __forceinline__ float quad_mlp_eval(const float *sp, const float x[4], float *h1row)
{
    const int q = threadIdx.x & 3;
#pragma unroll
    for (int j = 0; j < SMP_NH / 4; ++j) {
        const int o = q + 4 * j;
        float z = sp[LP_B1 + o];
#pragma unroll
        for (int i = 0; i < SMP_NIN; ++i) z = fmaf(sp[LP_W1 + o * SMP_NIN + i], x[i], z);
        h1row[o] = tanhf(z);
    }
    wave_lds_sync();
    float c = 0.0f;
    for (int j = 0; j < SMP_NH / 4; ++j) {
        const int o = q + 4 * j;
        const float *w2 = sp + LP_W2 + o * LW2;
        float z = sp[LP_B2 + o];
#pragma unroll
        for (int i = 0; i < SMP_NH; ++i) z = fmaf(w2[i], h1row[i], z);
        c = fmaf(sp[LP_W3 + o], tanhf(z), c);
    }
    wave_lds_sync();   // h1row may be reused by the next candidate
    const float s01 = c + __shfl_xor(c, 1);
    const float s = s01 + __shfl_xor(s01, 2);
    return s + sp[LP_B3];
}

// Gumbel key of coordinate i in outer iteration k: float(score / tau + G).
__device__ __forceinline__ float gumbel_key(float score, double tau, uint32_t i, uint32_t k,
                                            uint32_t k0, uint32_t k1)
{
    uint32_t c[4] = {i, k, 0u, 0u};
    philox4x32_10(c, k0, k1);
    const double u = unit_of(c[0]);
    return (float)((double)score / tau - log(-log(u)));
}

// Order-preserving map float -> uint32 (larger float, larger code).
__device__ __forceinline__ uint32_t order_code(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float kdiag_of(double nrm, const KParams &kp)
{
    if (kp.kind == KDCD_KERNEL_RBF) return 1.0f;
    if (kp.kind == KDCD_KERNEL_LINEAR) return (float)nrm;
    double base = kp.c + nrm, r = base;
    for (int t = 1; t < kp.degree; ++t) r *= base;
    return (float)r;
}

// Signed pseudo-logarithm of the gradient: v = float(|g| 2^20); v below 1
// is kept, above it the exponent plus the mantissa's fraction (a piecewise-
// linear log2) is used, 1 + e + (m - 1) for v = m 2^e, m in [1, 2); the sign
// of g is restored and the result scaled by 1/8.  Every step is an exact or
// correctly rounded float operation, so the host reproduces it bit for bit.
__device__ __forceinline__ float slog_feature(double g)
{
    const float v = (float)(fabs(g) * 1048576.0);
    float L = v;
    if (v >= 1.0f) {
        int e = 0;
        const float mant = frexpf(v, &e);    // v = mant 2^e, mant in [0.5, 1)
        const float frac = 2.0f * mant - 1.0f;
        L = 1.0f + ((float)(e - 1) + frac);
    }
    return copysignf(L, (float)g) * 0.125f;
}

__device__ __forceinline__ void state_features(int64_t i, const double *alpha, const double *g,
                                               const double *norms, const double *y,
                                               const KParams &kp, double invC, float x[4])
{
    x[0] = (float)(alpha[i] * invC);
    x[1] = slog_feature(g[i]);
    x[2] = kdiag_of(norms[i], kp);
    x[3] = (float)y[i];
}

// 256 threads = 64 quads = 64 coordinates per workgroup.
constexpr int QB = 64;
constexpr int QB_LD = SMP_NH + 1;   // padded h1 rows: the 16 quads of a wave hit distinct banks

__global__ __launch_bounds__(256) void forward_kernel(const float *__restrict__ params,
                                                      const float *__restrict__ x, int64_t n,
                                                      float *__restrict__ out)
{
    __shared__ float sp[LP_N];
    __shared__ float h1s[QB * QB_LD];
    load_params_padded(sp, params);
    const int cq = threadIdx.x >> 2;
    const int64_t i = (int64_t)blockIdx.x * QB + cq;
    float xi[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < n)
        for (int e = 0; e < 4; ++e) xi[e] = x[4 * i + e];
    const float f = quad_mlp_eval(sp, xi, h1s + cq * QB_LD);
    if (i < n && (threadIdx.x & 3) == 0) out[i] = f;
}

__global__ __launch_bounds__(256) void keys_kernel(const float *__restrict__ params,
                                                   const float *__restrict__ x, int64_t n,
                                                   double tau, uint32_t k, uint32_t k0,
                                                   uint32_t k1, float *__restrict__ keys)
{
    __shared__ float sp[LP_N];
    __shared__ float h1s[QB * QB_LD];
    load_params_padded(sp, params);
    const int cq = threadIdx.x >> 2;
    const int64_t i = (int64_t)blockIdx.x * QB + cq;
    float xi[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < n)
        for (int e = 0; e < 4; ++e) xi[e] = x[4 * i + e];
    const float f = quad_mlp_eval(sp, xi, h1s + cq * QB_LD);
    if (i < n && (threadIdx.x & 3) == 0) keys[i] = gumbel_key(f, tau, (uint32_t)i, k, k0, k1);
}

// ----------------------------------------------------- radix top-k select
// Three digit passes (bits 31..21, 20..10, 9..0) find the code T of the k-th
// largest key and how many keys equal to T are needed; a collect pass gathers
// every key > T and the keys == T; one workgroup sorts them by (code desc,
// index asc) and fills the slots.

constexpr int SEL_BINS = 2048;
constexpr int SEL_CEQ = 2048;      // capacity for keys tied with T
constexpr int SEL_CAND = 4096;     // power of two >= kMaxSB + SEL_CEQ
constexpr int TK_CH = 2048;        // the one-chunk path ranks up to this many coordinates
constexpr int POOL_MAX = 2048;     // candidate-pool size limit

__device__ __forceinline__ int pass_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }
__device__ __forceinline__ uint32_t pass_dmask(int pass) { return pass == 2 ? 0x3FFu : 0x7FFu; }
__device__ __forceinline__ uint32_t pass_hmask(int pass)   // bits fixed before this pass
{
    return pass == 0 ? 0u : (pass == 1 ? 0xFFE00000u : 0xFFFFFC00u);
}

__device__ __forceinline__ void hist_flush(uint32_t *lh, uint32_t *hist)
{
    __syncthreads();
    for (int b = threadIdx.x; b < SEL_BINS; b += blockDim.x)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

__device__ __forceinline__ void hist_clear(uint32_t *lh)
{
    for (int b = threadIdx.x; b < SEL_BINS; b += blockDim.x) lh[b] = 0u;
    __syncthreads();
}

__device__ __forceinline__ uint64_t composite(uint32_t code, uint32_t i)
{
    return ((uint64_t)code << 32) | (uint64_t)(0xFFFFFFFFu - i);   // value desc, index asc
}

// Bitonic sort of key[0, N) (N a power of two) into descending order.
__device__ __forceinline__ void bitonic_desc(uint64_t *key, int N)
{
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = threadIdx.x; e < N; e += blockDim.x) {
                const int p = e ^ stride;
                if (p > e) {
                    const bool desc = (e & size) == 0;
                    const uint64_t a = key[e], b = key[p];
                    if (desc ? (a < b) : (a > b)) {
                        key[e] = b;
                        key[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Pass 0 fused with the keys of the solve's state (hist may be null: codes only).
__global__ __launch_bounds__(256) void state_keys_kernel(
    const float *__restrict__ params, const double *__restrict__ alpha,
    const double *__restrict__ g, const double *__restrict__ norms, const double *__restrict__ y,
    KParams kp, double invC, int64_t m, double tau, uint32_t k, uint32_t k0, uint32_t k1,
    uint32_t *__restrict__ codes, uint32_t *__restrict__ hist, int32_t *status)
{
    __shared__ float sp[LP_N];
    __shared__ float h1s[QB * QB_LD];
    __shared__ uint32_t lh[SEL_BINS];
    if (hist) hist_clear(lh);
    load_params_padded(sp, params);
    const int cq = threadIdx.x >> 2;
    const int64_t i = (int64_t)blockIdx.x * QB + cq;
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < m) state_features(i, alpha, g, norms, y, kp, invC, x);
    const float f = quad_mlp_eval(sp, x, h1s + cq * QB_LD);
    if (i < m && (threadIdx.x & 3) == 0) {
        const float key = gumbel_key(f, tau, (uint32_t)i, k, k0, k1);
        if (!isfinite(key)) set_status(status, KDCD_ERR_NONFINITE);
        const uint32_t c = order_code(key);
        codes[i] = c;
        if (hist) atomicAdd(&lh[c >> 21], 1u);
    }
    if (hist) hist_flush(lh, hist);
}

// Pass 0 over caller-given float keys.
__global__ __launch_bounds__(256) void codes_kernel(const float *__restrict__ keys, int64_t m,
                                                    uint32_t *__restrict__ codes,
                                                    uint32_t *__restrict__ hist, int32_t *status)
{
    __shared__ uint32_t lh[SEL_BINS];
    hist_clear(lh);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float key = keys[i];
        if (!isfinite(key)) set_status(status, KDCD_ERR_NONFINITE);
        const uint32_t c = order_code(key);
        codes[i] = c;
        if (hist) atomicAdd(&lh[c >> 21], 1u);
    }
    if (hist) hist_flush(lh, hist);
}



// Passes 1 and 2: histogram of the next digit among codes matching the prefix.
__global__ __launch_bounds__(256) void hist_kernel(const uint32_t *__restrict__ codes, int64_t m,
                                                   const SelState *__restrict__ st, int pass,
                                                   uint32_t *__restrict__ hist)
{
    __shared__ uint32_t lh[SEL_BINS];
    hist_clear(lh);
    const uint32_t prefix = st->prefix, hm = pass_hmask(pass), dm = pass_dmask(pass);
    const int sh = pass_shift(pass);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = codes[i];
        if ((c & hm) == prefix) atomicAdd(&lh[(c >> sh) & dm], 1u);
    }
    hist_flush(lh, hist);
}

// One workgroup of 1024: the digit holding the k-th largest remaining code.
// Pass 0 starts the state from k; the histogram is cleared for the next pass.
__global__ __launch_bounds__(1024) void pick_kernel(uint32_t *__restrict__ hist,
                                                    SelState *__restrict__ st, int pass,
                                                    int32_t k)
{
    __shared__ uint32_t sc[1024];
    const int t = threadIdx.x;
    const uint32_t krem = pass == 0 ? (uint32_t)k : st->krem;
    const uint32_t prefix = pass == 0 ? 0u : st->prefix;
    // thread t owns bins 2047-2t and 2046-2t (descending digit order)
    const int b0 = SEL_BINS - 1 - 2 * t, b1 = b0 - 1;
    const uint32_t h0 = hist[b0], h1 = hist[b1];
    uint32_t v = h0 + h1;
    sc[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan
        const uint32_t add = t >= off ? sc[t - off] : 0u;
        __syncthreads();
        v += add;
        sc[t] = v;
        __syncthreads();
    }
    const uint32_t incl = v, excl = incl - h0 - h1;
    if (excl < krem && krem <= incl) {
        uint32_t d, above;
        if (excl + h0 >= krem) { d = (uint32_t)b0; above = excl; }
        else { d = (uint32_t)b1; above = excl + h0; }
        st->prefix = prefix | (d << pass_shift(pass));
        st->krem = krem - above;
    }
    hist[b0] = 0u;
    hist[b1] = 0u;
}

__global__ __launch_bounds__(256) void collect_kernel(const uint32_t *__restrict__ codes,
                                                      int64_t m, SelState *__restrict__ st,
                                                      int32_t *__restrict__ cand_gt,
                                                      int32_t *__restrict__ cand_eq)
{
    const uint32_t T = st->prefix;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = codes[i];
        if (c > T) {
            const uint32_t pos = atomicAdd(&st->n_gt, 1u);
            if (pos < (uint32_t)kMaxSB) cand_gt[pos] = (int32_t)i;
        } else if (c == T) {
            const uint32_t pos = atomicAdd(&st->n_eq, 1u);
            if (pos < (uint32_t)SEL_CEQ) cand_eq[pos] = (int32_t)i;
        }
    }
}

// Sort the candidates, fill the slots.  Slot j: uniform when u(x0) < epsilon
// (coordinate floor(x1 * m / 2^32)), else the next best key.  With topk == 0
// every slot is uniform and no candidates are read.
// Candidate pool: P candidates c_j = floor(x0 m / 2^32) from counters
// (j, k, 3, 0), scored from the state and keyed with the noise of their
// coordinate, (i, k, 0, 0); pkey[j] = composite(code, j), pcid[j] = c_j.
__global__ __launch_bounds__(256) void pool_score_kernel(
    const float *__restrict__ params, const double *__restrict__ alpha,
    const double *__restrict__ g, const double *__restrict__ norms, const double *__restrict__ y,
    KParams kp, double invC, int64_t m, int32_t P, double tau, uint32_t k, uint32_t k0,
    uint32_t k1, uint64_t *__restrict__ pkey, int32_t *__restrict__ pcid, int32_t *status)
{
    __shared__ float sp[LP_N];
    __shared__ float h1s[QB * QB_LD];
    load_params_padded(sp, params);
    const int cq = threadIdx.x >> 2;
    const int j = blockIdx.x * QB + cq;
    int32_t i = 0;
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    if (j < P) {
        uint32_t c[4] = {(uint32_t)j, k, 3u, 0u};
        philox4x32_10(c, k0, k1);
        i = (int32_t)(((uint64_t)c[0] * (uint64_t)m) >> 32);
        state_features(i, alpha, g, norms, y, kp, invC, x);
    }
    const float f = quad_mlp_eval(sp, x, h1s + cq * QB_LD);
    if (j < P && (threadIdx.x & 3) == 0) {
        const float kv = gumbel_key(f, tau, (uint32_t)i, k, k0, k1);
        if (!isfinite(kv)) set_status(status, KDCD_ERR_NONFINITE);
        pkey[j] = composite(order_code(kv), (uint32_t)j);
        pcid[j] = i;
    }
}

// mode 0: every slot uniform; mode 1: candidates of the radix select
// (cand_gt / cand_eq with their codes); mode 2: all ncand = m <= TK_CH codes;
// mode 3: the ncand pool keys pkey, coordinates pcid.
__global__ __launch_bounds__(1024) void slots_kernel(const uint32_t *__restrict__ codes,
                                                     int64_t m, SelState *__restrict__ st,
                                                     const int32_t *__restrict__ cand_gt,
                                                     const int32_t *__restrict__ cand_eq,
                                                     const uint64_t *__restrict__ pkey,
                                                     const int32_t *__restrict__ pcid,
                                                     int32_t ncand, int32_t ns, double epsilon,
                                                     uint32_t k, uint32_t k0, uint32_t k1,
                                                     int mode, int32_t *__restrict__ S,
                                                     int32_t *status)
{
    __shared__ uint64_t key[SEL_CAND];
    __shared__ int32_t rank[1024];
    const int t = threadIdx.x;
    const bool topk = mode != 0;
    if (mode == 1) {
        const uint32_t ngt = st->n_gt, neq = st->n_eq, krem = st->krem;
        if (neq > (uint32_t)SEL_CEQ && krem < neq) {
            if (t == 0) set_status(status, KDCD_ERR_UNSUPPORTED);
        }
        const int cg = (int)min(ngt, (uint32_t)kMaxSB), ce = (int)min(neq, (uint32_t)SEL_CEQ);
        const int cnt = cg + ce;
        int N = 1;
        while (N < cnt) N <<= 1;
        for (int e = t; e < N; e += 1024) {
            uint64_t v = 0;
            if (e < cnt) {
                const int32_t i = e < cg ? cand_gt[e] : cand_eq[e - cg];
                v = composite(codes[i], (uint32_t)i);
            }
            key[e] = v;
        }
        __syncthreads();
        bitonic_desc(key, N);
    } else if (mode == 3) {
        int N = 1;
        while (N < ncand) N <<= 1;
        for (int e = t; e < N; e += 1024) key[e] = e < ncand ? pkey[e] : 0ull;
        __syncthreads();
        bitonic_desc(key, N);
    } else if (mode == 2) {     // ncand = m <= TK_CH: rank every coordinate
        int N = 1;
        while (N < ncand) N <<= 1;
        for (int e = t; e < N; e += 1024) key[e] = e < ncand ? composite(codes[e], (uint32_t)e) : 0ull;
        __syncthreads();
        bitonic_desc(key, N);
    }
    // slot kinds and the rank of every top-k slot
    bool uni = true;
    uint32_t x1 = 0;
    if (t < ns) {
        uint32_t c[4] = {(uint32_t)t, k, 1u, 0u};
        philox4x32_10(c, k0, k1);
        uni = !topk || unit_of(c[0]) < epsilon;
        x1 = c[1];
    }
    int v = (t < ns && !uni) ? 1 : 0;
    rank[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int add = t >= off ? rank[t - off] : 0;
        __syncthreads();
        v += add;
        rank[t] = v;
        __syncthreads();
    }
    if (t < ns) {
        int32_t idx;
        if (uni) {
            idx = (int32_t)(((uint64_t)x1 * (uint64_t)m) >> 32);
        } else {
            const int r = v - 1;   // exclusive rank among top-k slots
            idx = (int32_t)(0xFFFFFFFFu - (uint32_t)(key[r] & 0xFFFFFFFFu));
            if (mode == 3) idx = pcid[idx];
        }
        S[t] = idx;
    }
    if (t == 0 && mode == 1) {
        st->n_gt = 0u;
        st->n_eq = 0u;
        st->prefix = 0u;
    }
}

// ------------------------------------------------------ gradient upkeep

// g = y o (K (y o alpha)) - 1 + omega alpha from Kb = K (y o alpha).
__global__ __launch_bounds__(256) void grad_init_kernel(const double *__restrict__ Kb,
                                                        const double *__restrict__ y,
                                                        const double *__restrict__ alpha,
                                                        double omega, int64_t m,
                                                        double *__restrict__ g)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        g[i] = (Kb ? y[i] * Kb[i] : 0.0) - 1.0 + omega * alpha[i];
}

__global__ __launch_bounds__(256) void product_kernel(const double *__restrict__ a,
                                                      const double *__restrict__ b, int64_t m,
                                                      double *__restrict__ out,
                                                      int32_t *__restrict__ any_nonzero)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = a[i] * b[i];
        out[i] = v;
        if (v != 0.0) *any_nonzero = 1;
    }
}

__global__ __launch_bounds__(256) void features_kernel(const int32_t *__restrict__ S, int32_t ns,
                                                       const double *__restrict__ alpha,
                                                       const double *__restrict__ g,
                                                       const double *__restrict__ norms,
                                                       const double *__restrict__ y, KParams kp,
                                                       double invC, float *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns) return;
    float x[4];
    state_features(S[t], alpha, g, norms, y, kp, invC, x);
    for (int e = 0; e < 4; ++e) out[4 * t + e] = x[e];
}

// ------------------------------------------------------------ training
// One block of 256 threads takes TR_NS samples; the two threads of a sample
// split the 64 hidden units of layer 2.  Per-block parameter gradients are
// written to gpart[block][*] and summed in block order by the update kernel.

constexpr int TR_NS = 128;
constexpr int TR_LD = SMP_NH + 1;   // padded rows: per-sample rows spread over banks

__global__ __launch_bounds__(256) void grad_kernel(const float *__restrict__ params,
                                                   const float *__restrict__ x,
                                                   const float *__restrict__ tgt, int64_t n,
                                                   float inv_n, float *__restrict__ gpart,
                                                   float *__restrict__ lpart)
{
    __shared__ float sp[SMP_NP];
    __shared__ float h1s[TR_NS * TR_LD], dz2s[TR_NS * TR_LD], e3s[TR_NS * TR_LD],
        dz1s[TR_NS * TR_LD];
    __shared__ float xs[TR_NS * 4], ds[TR_NS], fpart[2 * TR_NS], ls[TR_NS];
    load_params(sp, params);
    const int tid = threadIdx.x;
    const int s = tid >> 1, half = tid & 1;
    const int64_t gi = (int64_t)blockIdx.x * TR_NS + s;
    const bool valid = gi < n;
    float xi[4] = {0.f, 0.f, 0.f, 0.f};
    if (valid)
        for (int e = 0; e < 4; ++e) xi[e] = x[4 * gi + e];
    if (half == 0)
        for (int e = 0; e < 4; ++e) xs[4 * s + e] = xi[e];
    float h1[SMP_NH];
#pragma unroll
    for (int o = 0; o < SMP_NH; ++o) {
        float z = sp[SMP_B1 + o];
#pragma unroll
        for (int i = 0; i < SMP_NIN; ++i) z = fmaf(sp[SMP_W1 + o * SMP_NIN + i], xi[i], z);
        h1[o] = tanhf(z);
    }
    constexpr int HH = SMP_NH / 2;
    float h2[HH];
    float fp = 0.f;
#pragma unroll
    for (int q = 0; q < HH; ++q) {
        const int o = half * HH + q;
        float z = sp[SMP_B2 + o];
#pragma unroll
        for (int i = 0; i < SMP_NH; ++i) z = fmaf(sp[SMP_W2 + o * SMP_NH + i], h1[i], z);
        h2[q] = tanhf(z);
        fp = fmaf(sp[SMP_W3 + o], h2[q], fp);
    }
    fpart[2 * s + half] = fp;
    if (half == 0) {
#pragma unroll
        for (int o = 0; o < SMP_NH; ++o) h1s[s * TR_LD + o] = h1[o];
    }
    __syncthreads();
    const float f = fpart[2 * s] + fpart[2 * s + 1] + sp[SMP_B3];
    const float e = valid ? f - tgt[gi] : 0.f;
    const float d = e * inv_n;
    if (half == 0) {
        ds[s] = d;
        ls[s] = 0.5f * e * e * inv_n;
    }
#pragma unroll
    for (int q = 0; q < HH; ++q) {
        const int o = half * HH + q;
        dz2s[s * TR_LD + o] = d * sp[SMP_W3 + o] * (1.f - h2[q] * h2[q]);
        e3s[s * TR_LD + o] = d * h2[q];
    }
    __syncthreads();
    for (int q = 0; q < HH; ++q) {
        const int i = half * HH + q;
        float acc = 0.f;
        for (int o = 0; o < SMP_NH; ++o) acc = fmaf(sp[SMP_W2 + o * SMP_NH + i], dz2s[s * TR_LD + o], acc);
        const float hv = h1s[s * TR_LD + i];
        dz1s[s * TR_LD + i] = acc * (1.f - hv * hv);
    }
    __syncthreads();
    // parameter gradients of this block, samples summed in order
    float *gp = gpart + (int64_t)blockIdx.x * SMP_NP;
    for (int q = tid; q < SMP_NP; q += blockDim.x) {
        float acc = 0.f;
        if (q < SMP_B1) {
            const int o = q / SMP_NIN, i = q % SMP_NIN;
            for (int r = 0; r < TR_NS; ++r) acc = fmaf(dz1s[r * TR_LD + o], xs[4 * r + i], acc);
        } else if (q < SMP_W2) {
            const int o = q - SMP_B1;
            for (int r = 0; r < TR_NS; ++r) acc += dz1s[r * TR_LD + o];
        } else if (q < SMP_B2) {
            const int o = (q - SMP_W2) / SMP_NH, i = (q - SMP_W2) % SMP_NH;
            for (int r = 0; r < TR_NS; ++r) acc = fmaf(dz2s[r * TR_LD + o], h1s[r * TR_LD + i], acc);
        } else if (q < SMP_W3) {
            const int o = q - SMP_B2;
            for (int r = 0; r < TR_NS; ++r) acc += dz2s[r * TR_LD + o];
        } else if (q < SMP_B3) {
            const int o = q - SMP_W3;
            for (int r = 0; r < TR_NS; ++r) acc += e3s[r * TR_LD + o];
        } else {
            for (int r = 0; r < TR_NS; ++r) acc += ds[r];
        }
        gp[q] = acc;
    }
    if (tid == 0) {
        float l = 0.f;
        for (int r = 0; r < TR_NS; ++r) l += ls[r];
        lpart[blockIdx.x] = l;
    }
}

// Sum the block gradients in order; optionally one Adam step.
__global__ __launch_bounds__(256) void update_kernel(const float *__restrict__ gpart,
                                                     const float *__restrict__ lpart, int nblk,
                                                     float *__restrict__ params,
                                                     float *__restrict__ mom,
                                                     float *__restrict__ vel, int adam, float lr,
                                                     float bc1, float bc2, float *__restrict__ grad,
                                                     float *__restrict__ loss, double *lacc,
                                                     double lweight)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        float l = 0.f;
        for (int b = 0; b < nblk; ++b) l += lpart[b];
        if (loss) *loss = l;
        if (lacc) *lacc += (double)l * lweight;
    }
    if (q >= SMP_NP) return;
    float gq = 0.f;
    for (int b = 0; b < nblk; ++b) gq += gpart[(int64_t)b * SMP_NP + q];
    if (grad) grad[q] = gq;
    if (!adam) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mq = b1 * mom[q] + (1.f - b1) * gq;
    const float vq = b2 * vel[q] + (1.f - b2) * gq * gq;
    mom[q] = mq;
    vel[q] = vq;
    const float mh = mq / bc1, vh = vq / bc2;
    params[q] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void lacc_to_float_kernel(const double *__restrict__ lacc, float *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = (float)*lacc;
}

__global__ void zero_f64_kernel(double *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

unsigned grid_for(int64_t n, int64_t cap = 2048)
{
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    return (unsigned)(b < cap ? b : cap);
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, float *out,
                              hipStream_t st)
{
    hipLaunchKernelGGL(forward_kernel, dim3((unsigned)((n + QB - 1) / QB)), dim3(256), 0, st, params,
                       x, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_keys(const float *params, const float *x, int64_t n, double tau,
                           uint32_t k, uint64_t seed, float *keys, hipStream_t st)
{
    hipLaunchKernelGGL(keys_kernel, dim3((unsigned)((n + QB - 1) / QB)), dim3(256), 0, st, params,
                       x, n, tau, k,
                       (uint32_t)seed, (uint32_t)(seed >> 32), keys);
    return hipGetLastError();
}


hipError_t launch_select(const SelectArgs &a, hipStream_t st)
{
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const unsigned grid = grid_for(a.m, 1024);
    const unsigned qgrid = (unsigned)((a.m + QB - 1) / QB);
    int mode = 0;
    int32_t ncand = 0;
    if (a.topk && a.pool > 0) {
        mode = 3;
        ncand = a.pool;
        hipLaunchKernelGGL(pool_score_kernel, dim3((unsigned)((a.pool + QB - 1) / QB)), dim3(256), 0,
                           st, a.params, a.alpha, a.g, a.norms, a.y, a.kp, a.invC, a.m, a.pool,
                           a.tau, a.outer, k0, k1, a.ws.pkey, a.ws.pcid, a.status);
    } else if (a.topk) {
        // small problems: every coordinate is a candidate of one sort
        const int64_t nc = a.m <= TK_CH ? a.m : 0;
        uint32_t *hist = nc ? nullptr : a.ws.hist;
        if (a.params)
            hipLaunchKernelGGL(state_keys_kernel, dim3(qgrid), dim3(256), 0, st, a.params, a.alpha,
                               a.g, a.norms, a.y, a.kp, a.invC, a.m, a.tau, a.outer, k0, k1,
                               a.ws.codes, hist, a.status);
        else
            hipLaunchKernelGGL(codes_kernel, dim3(grid), dim3(256), 0, st, a.keys, a.m, a.ws.codes,
                               hist, a.status);
        if (nc) {
            mode = 2;
            ncand = (int32_t)nc;
        } else {
            mode = 1;
            for (int pass = 0; pass < 3; ++pass) {
                if (pass > 0)
                    hipLaunchKernelGGL(hist_kernel, dim3(grid), dim3(256), 0, st, a.ws.codes, a.m,
                                       a.ws.state, pass, a.ws.hist);
                hipLaunchKernelGGL(pick_kernel, dim3(1), dim3(1024), 0, st, a.ws.hist, a.ws.state,
                                   pass, a.ns);
            }
            hipLaunchKernelGGL(collect_kernel, dim3(grid), dim3(256), 0, st, a.ws.codes, a.m,
                               a.ws.state, a.ws.cand_gt, a.ws.cand_eq);
        }
    }
    hipLaunchKernelGGL(slots_kernel, dim3(1), dim3(1024), 0, st, a.ws.codes, a.m, a.ws.state,
                       a.ws.cand_gt, a.ws.cand_eq, a.ws.pkey, a.ws.pcid, ncand, a.ns, a.epsilon,
                       a.outer,
                       k0, k1, mode, a.S, a.status);
    return hipGetLastError();
}

size_t select_workspace_bytes(int64_t m)
{
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    return al(sizeof(uint32_t) * (size_t)m) + al(sizeof(uint32_t) * SEL_BINS) + al(sizeof(SelState)) +
           al(sizeof(int32_t) * kMaxSB) + al(sizeof(int32_t) * SEL_CEQ) +
           al(sizeof(uint64_t) * POOL_MAX) + al(sizeof(int32_t) * POOL_MAX);
}

SelectWs select_workspace(void *base, int64_t m)
{
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    char *p = static_cast<char *>(base);
    SelectWs w;
    w.codes = reinterpret_cast<uint32_t *>(p);
    p += al(sizeof(uint32_t) * (size_t)m);
    w.hist = reinterpret_cast<uint32_t *>(p);
    p += al(sizeof(uint32_t) * SEL_BINS);
    w.state = reinterpret_cast<SelState *>(p);
    p += al(sizeof(SelState));
    w.cand_gt = reinterpret_cast<int32_t *>(p);
    p += al(sizeof(int32_t) * kMaxSB);
    w.cand_eq = reinterpret_cast<int32_t *>(p);
    p += al(sizeof(int32_t) * SEL_CEQ);
    w.pkey = reinterpret_cast<uint64_t *>(p);
    p += al(sizeof(uint64_t) * POOL_MAX);
    w.pcid = reinterpret_cast<int32_t *>(p);
    return w;
}

hipError_t launch_select_reset(const SelectWs &w, hipStream_t st)
{
    // histogram and state words are cleared by a kernel (no memset nodes)
    hipLaunchKernelGGL(zero_f64_kernel, dim3((SEL_BINS / 2 + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<double *>(w.hist), (int64_t)(SEL_BINS / 2));
    hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(256), 0, st,
                       reinterpret_cast<double *>(w.state), (int64_t)(sizeof(SelState) / 8));
    return hipGetLastError();
}

hipError_t launch_grad_update(const double *U, int64_t m, int32_t sb, const int32_t *S,
                              const double *theta, const double *y, double omega, double *g,
                              hipStream_t st)
{
    return launch_dual_update(U, m, sb, S, theta, y, 1.0, y, omega, g, nullptr, st);
}

hipError_t launch_grad_init(const double *Kb, const double *y, const double *alpha, double omega,
                            int64_t m, double *g, hipStream_t st)
{
    hipLaunchKernelGGL(grad_init_kernel, dim3(grid_for(m)), dim3(256), 0, st, Kb, y, alpha, omega,
                       m, g);
    return hipGetLastError();
}

hipError_t launch_features(const int32_t *S, int32_t ns, const double *alpha, const double *g,
                           const double *norms, const double *y, KParams kp, double invC,
                           float *out, hipStream_t st)
{
    hipLaunchKernelGGL(features_kernel, dim3((ns + 255) / 256), dim3(256), 0, st, S, ns, alpha, g,
                       norms, y, kp, invC, out);
    return hipGetLastError();
}

hipError_t launch_product(const double *a, const double *b, int64_t m, double *out,
                          int32_t *any_nonzero, hipStream_t st)
{
    hipLaunchKernelGGL(product_kernel, dim3(grid_for(m)), dim3(256), 0, st, a, b, m, out,
                       any_nonzero);
    return hipGetLastError();
}

int train_blocks(int64_t n) { return (int)((n + TR_NS - 1) / TR_NS); }

hipError_t launch_train_step(const TrainArgs &a, hipStream_t st)
{
    const int nblk = train_blocks(a.n);
    hipLaunchKernelGGL(grad_kernel, dim3(nblk), dim3(256), 0, st, a.params, a.x, a.t, a.n,
                       1.0f / (float)a.n, a.gpart, a.lpart);
    hipLaunchKernelGGL(update_kernel, dim3((SMP_NP + 255) / 256), dim3(256), 0, st, a.gpart,
                       a.lpart, nblk, a.params, a.mom, a.vel, a.adam, a.lr, a.bc1, a.bc2, a.grad,
                       a.loss, a.lacc, a.lweight);
    return hipGetLastError();
}

hipError_t launch_lacc(double *lacc, float *out, bool to_float, hipStream_t st)
{
    if (to_float) hipLaunchKernelGGL(lacc_to_float_kernel, dim3(1), dim3(64), 0, st, lacc, out);
    else hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(64), 0, st, lacc, (int64_t)1);
    return hipGetLastError();
}

}  // namespace kdcd
