// Internal interface of the learned sampler (sampler.hip).
#pragma once

#include "common.hpp"

namespace kdcd {

// MLP 4 -> 64 -> 64 -> 1; flat FP32 parameters W1[64][4], b1[64], W2[64][64],
// b2[64], w3[64], b3.
constexpr int SMP_NIN = 4;
constexpr int SMP_NH = 64;
constexpr int SMP_W1 = 0;
constexpr int SMP_B1 = SMP_W1 + SMP_NH * SMP_NIN;
constexpr int SMP_W2 = SMP_B1 + SMP_NH;
constexpr int SMP_B2 = SMP_W2 + SMP_NH * SMP_NH;
constexpr int SMP_W3 = SMP_B2 + SMP_NH;
constexpr int SMP_B3 = SMP_W3 + SMP_NH;
constexpr int SMP_NP = SMP_B3 + 1;
static_assert(SMP_NP == KDCD_SAMPLER_NPARAMS, "parameter count");

constexpr int SMP_MAX_BATCH = 65536;   // training minibatch limit
constexpr int SMP_MAX_POOL = 2048;     // candidate-pool size limit

// Radix-select state (device).
struct SelState {
    uint32_t prefix, krem, n_gt, n_eq;
};

struct SelectWs {
    uint32_t *codes;    // m order-preserving key codes
    uint32_t *hist;     // 2048 digit counts
    SelState *state;
    int32_t *cand_gt;   // kMaxSB candidates above the threshold
    int32_t *cand_eq;   // candidates tied with it
    uint64_t *pkey;     // pool keys (composite with the pool position)
    int32_t *pcid;      // pool coordinates
};

struct SelectArgs {
    SelectWs ws;
    int64_t m;
    int32_t ns;            // slots to fill (<= kMaxSB, <= m when topk)
    bool topk;             // false: every slot uniform
    int32_t pool;          // > 0: score only this many random candidates (<= 2048)
    double epsilon, tau;
    uint64_t seed;
    uint32_t outer;        // outer-iteration counter k
    // keys from the solve's state (params != nullptr) ...
    const float *params;
    const double *alpha, *g, *norms, *y;
    KParams kp;
    double invC;
    // ... or from caller-given float keys
    const float *keys;
    int32_t *S;            // ns outputs
    int32_t *status;
};

struct TrainArgs {
    float *params, *mom, *vel;
    const float *x, *t;
    int64_t n;
    float *gpart, *lpart;
    int adam;
    float lr, bc1, bc2;
    float *grad, *loss;
    double *lacc;
    double lweight;
};

void sampler_init_params(float *p, uint64_t seed);
hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, float *out,
                              hipStream_t st);
hipError_t launch_mlp_keys(const float *params, const float *x, int64_t n, double tau, uint32_t k,
                           uint64_t seed, float *keys, hipStream_t st);
size_t select_workspace_bytes(int64_t m);
SelectWs select_workspace(void *base, int64_t m);
hipError_t launch_select_reset(const SelectWs &w, hipStream_t st);
hipError_t launch_select(const SelectArgs &a, hipStream_t st);
hipError_t launch_grad_update(const double *U, int64_t m, int32_t sb, const int32_t *S,
                              const double *theta, const double *y, double omega, double *g,
                              hipStream_t st);
hipError_t launch_grad_init(const double *Kb, const double *y, const double *alpha, double omega,
                            int64_t m, double *g, hipStream_t st);
hipError_t launch_features(const int32_t *S, int32_t ns, const double *alpha, const double *g,
                           const double *norms, const double *y, KParams kp, double invC,
                           float *out, hipStream_t st);
// out = a o b; any_nonzero is set to 1 when some product is nonzero.
hipError_t launch_product(const double *a, const double *b, int64_t m, double *out,
                          int32_t *any_nonzero, hipStream_t st);
int train_blocks(int64_t n);
hipError_t launch_train_step(const TrainArgs &a, hipStream_t st);
hipError_t launch_lacc(double *lacc, float *out, bool to_float, hipStream_t st);

}  // namespace kdcd

// The opaque model of the C-ABI.
struct kdcd_sampler {
    int device = 0;
    float *params = nullptr, *mom = nullptr, *vel = nullptr;
    float *gpart = nullptr, *lpart = nullptr;
    double *lacc = nullptr;
    int64_t step = 0;
};
