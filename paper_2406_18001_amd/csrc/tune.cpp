// Process-wide tuning table of the kernel-block products: the tile
// configuration chosen per (compute, n, sb) -- the FP64 product's, or the
// single-problem bf16 / fp16 / bf16x3 product's -- filled by kdcd_autotune or
// kdcd_tune_set, saved to and loaded from a plain text file ("compute n sb id"
// per line).
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"

namespace kdcd {
namespace {

using Key = std::tuple<int32_t, int64_t, int32_t>;

std::mutex &table_mutex()
{
    static std::mutex mu;
    return mu;
}

std::map<Key, int> &table()
{
    static std::map<Key, int> t;
    return t;
}

}  // namespace

int tune_lookup(int32_t compute, int64_t n, int32_t sb)
{
    std::lock_guard<std::mutex> lk(table_mutex());
    const auto it = table().find(Key(compute, n, sb));
    return it == table().end() ? -1 : it->second;
}

void tune_store(int32_t compute, int64_t n, int32_t sb, int id)
{
    std::lock_guard<std::mutex> lk(table_mutex());
    if (id < 0) table().erase(Key(compute, n, sb));
    else table()[Key(compute, n, sb)] = id;
}

}  // namespace kdcd

using namespace kdcd;

namespace {

// Number of tile configurations of the product computed in `compute` (0: not
// tunable); compute + KDCD_TUNE_BATCH names the batched product.
int config_count(int32_t compute)
{
    switch (compute) {
    case KDCD_F64: return f64_config_count();
    case KDCD_BF16: case KDCD_F16: case KDCD_BF16X3: return lowp_config_count();
    case KDCD_F64 + KDCD_TUNE_BATCH: return f64_batch_config_count();
    case KDCD_F32 + KDCD_TUNE_BATCH: case KDCD_BF16 + KDCD_TUNE_BATCH:
    case KDCD_F16 + KDCD_TUNE_BATCH: case KDCD_BF16X3 + KDCD_TUNE_BATCH:
        return mixed_batch_config_count();
    default: return 0;
    }
}

void config_shape(int32_t compute, int id, int *bm, int *bn, int *w)
{
    if (compute == KDCD_F64) f64_config_shape(id, bm, bn, w);
    else if (compute == KDCD_F64 + KDCD_TUNE_BATCH) f64_batch_config_shape(id, bm, bn, w);
    else if (compute >= KDCD_TUNE_BATCH) mixed_batch_config_shape(id, bm, bn, w);
    else lowp_config_shape(id, bm, bn, w);
}

}  // namespace

extern "C" {

int32_t kdcd_tune_configs(int32_t compute, int32_t *bm, int32_t *bn, int32_t *waves, int32_t max)
{
    const int n = config_count(compute);
    for (int i = 0; i < n && i < max; ++i) {
        int a, b, w;
        config_shape(compute, i, &a, &b, &w);
        if (bm) bm[i] = a;
        if (bn) bn[i] = b;
        if (waves) waves[i] = w;
    }
    return n;
}

kdcd_status kdcd_tune_set(int32_t compute, int64_t n, int32_t sb, int32_t id)
{
    const int nc = config_count(compute);
    if (nc == 0) return KDCD_ERR_UNSUPPORTED;
    if (n < 1 || sb < 1 || sb > kMaxSB || id >= nc) return KDCD_ERR_INVALID_ARG;
    tune_store(compute, n, sb, id < 0 ? -1 : id);
    return KDCD_OK;
}

int32_t kdcd_tune_get(int32_t compute, int64_t n, int32_t sb)
{
    if (config_count(compute) == 0 || n < 1 || sb < 1 || sb > kMaxSB) return -1;
    if (compute == KDCD_F64) return f64_config_id(n, sb);
    if (compute == KDCD_F64 + KDCD_TUNE_BATCH) return f64_batch_config_id(n, sb);
    if (compute >= KDCD_TUNE_BATCH) return mixed_batch_config_id(compute - KDCD_TUNE_BATCH, n, sb);
    return lowp_config_id(compute, n, sb);
}

kdcd_status kdcd_tune_save(const char *path)
{
    if (!path) return KDCD_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "w");
    if (!f) return KDCD_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(table_mutex());
        for (const auto &e : table())
            std::fprintf(f, "%d %lld %d %d\n", (int)std::get<0>(e.first),
                         (long long)std::get<1>(e.first), (int)std::get<2>(e.first), e.second);
    }
    return std::fclose(f) == 0 ? KDCD_OK : KDCD_ERR_INVALID_ARG;
}

kdcd_status kdcd_tune_load(const char *path)
{
    if (!path) return KDCD_ERR_INVALID_ARG;
    FILE *f = std::fopen(path, "r");
    if (!f) return KDCD_ERR_INVALID_ARG;
    int c, sb, id;
    long long n;
    kdcd_status rc = KDCD_OK;
    while (true) {
        const int got = std::fscanf(f, "%d %lld %d %d", &c, &n, &sb, &id);
        if (got == EOF) break;
        if (got != 4 || config_count(c) == 0 || n < 1 || sb < 1 || sb > kMaxSB || id < 0 ||
            id >= config_count(c)) {
            rc = KDCD_ERR_INVALID_ARG;
            break;
        }
        tune_store(c, n, sb, id);
    }
    std::fclose(f);
    return rc;
}

}  // extern "C"
