// Work-item shape search: times the batched solve of one model for candidate shapes of the
// decoder, residual and constraint work items and keeps the fastest.
//
// The shapes change only how the evaluation kernels split their work (rows per decoder work
// item, sampled nodes per residual work item, interface rows per constraint work item), so every
// candidate computes the same solves up to the grouping of partial sums.  The search is a
// coordinate descent from the library defaults: each dimension in turn takes the candidate
// value with the lowest median solve time, the others held at the best so far.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "ddrom.h"
#include "internal.h"

namespace {

const int kDecRows[] = {16, 24, 32, 48, 64};
const int kResNodes[] = {8, 12, 16, 24, 32, 48};
const int kConRows[] = {32, 64, 128, 256};

struct Bufs {
    double *x = nullptr, *lam = nullptr, *fn = nullptr;
    int *it = nullptr, *st = nullptr;
    ~Bufs() {
        if (x) (void)hipFree(x);
        if (lam) (void)hipFree(lam);
        if (fn) (void)hipFree(fn);
        if (it) (void)hipFree(it);
        if (st) (void)hipFree(st);
    }
};

// Median device time (ms) of `reps` solves with shape `tile`, after one untimed solve;
// a negative value is an error code.
float time_shape(const ddrom_model_desc* desc, const int tile[3], const double* mu_d, int B, const ddrom_opts* o,
                 int reps, hipStream_t s, int* rc_out) {
    ddrom_model_desc d = *desc;
    for (int k = 0; k < 3; ++k) d.tile[k] = tile[k];
    ddrom_model* m = nullptr;
    ddrom_workspace* ws = nullptr;
    int rc = ddrom_model_create(&d, &m);
    if (!rc) rc = ddrom_workspace_create(m, B, &ws);
    Bufs b;
    std::vector<float> t;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) {
        const long long nD = ddrom_model_size(m, 1, -1), nC = std::max(1LL, ddrom_model_size(m, 2, -1));
        if (hipMalloc(&b.x, sizeof(double) * B * nD) != hipSuccess || hipMalloc(&b.lam, sizeof(double) * B * nC) != hipSuccess ||
            hipMalloc(&b.fn, sizeof(double) * B) != hipSuccess || hipMalloc(&b.it, sizeof(int) * B) != hipSuccess ||
            hipMalloc(&b.st, sizeof(int) * B) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess)
            rc = DDROM_ENOMEM;
        if (rc) ddrom::set_error("autotune buffer allocation failed");
    }
    for (int r = -1; r < reps && !rc; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = DDROM_EHIP;
        if (!rc)
            rc = rom_solve_batch(m, ws, mu_d, B, nullptr, nullptr, o, b.x, b.lam, b.it, b.st, b.fn, nullptr, s);
        if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)) rc = DDROM_EHIP;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DDROM_EHIP;
        if (!rc && r >= 0) t.push_back(ms);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ws) ddrom_workspace_destroy(ws);
    if (m) ddrom_model_destroy(m);
    *rc_out = rc;
    if (rc) return -1.f;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

extern "C" int ddrom_autotune(const ddrom_model_desc* desc, const double* mu_d, int B, const ddrom_opts* o, int reps,
                              int* tile_out, float* table_h, int max_table, int* n_tried) {
    if (!desc || !mu_d || B <= 0 || !o || reps <= 0 || !tile_out || (table_h && max_table < 0)) {
        ddrom::set_error("bad arguments to ddrom_autotune");
        return DDROM_EINVAL;
    }
    // defaults of the library, read back from a model built with shape 0
    int cur[3];
    {
        ddrom_model_desc d = *desc;
        d.tile[0] = d.tile[1] = d.tile[2] = 0;
        ddrom_model* m = nullptr;
        int rc = ddrom_model_create(&d, &m);
        if (rc) return rc;
        for (int k = 0; k < 3; ++k) cur[k] = (int)ddrom_model_size(m, 7 + k, -1);
        ddrom_model_destroy(m);
    }
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        ddrom::set_error("stream creation failed");
        return DDROM_EHIP;
    }
    std::map<std::tuple<int, int, int>, float> seen;
    int count = 0, rc = 0;
    auto measure = [&](const int t[3]) -> float {
        const auto key = std::make_tuple(t[0], t[1], t[2]);
        auto it = seen.find(key);
        if (it != seen.end()) return it->second;
        const float ms = time_shape(desc, t, mu_d, B, o, reps, s, &rc);
        if (rc) return -1.f;
        seen[key] = ms;
        if (table_h && count < max_table) {
            for (int k = 0; k < 3; ++k) table_h[4 * count + k] = (float)t[k];
            table_h[4 * count + 3] = ms;
        }
        ++count;
        return ms;
    };
    float best = measure(cur);
    const int* cand[3] = {kDecRows, kResNodes, kConRows};
    const int ncand[3] = {(int)(sizeof(kDecRows) / sizeof(int)), (int)(sizeof(kResNodes) / sizeof(int)),
                          (int)(sizeof(kConRows) / sizeof(int))};
    for (int dim = 0; dim < 3 && !rc; ++dim)
        for (int c = 0; c < ncand[dim] && !rc; ++c) {
            int t[3] = {cur[0], cur[1], cur[2]};
            t[dim] = cand[dim][c];
            const float ms = measure(t);
            if (!rc && ms < best) {
                best = ms;
                cur[dim] = t[dim];
            }
        }
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    for (int k = 0; k < 3; ++k) tile_out[k] = cur[k];
    if (n_tried) *n_tried = count;
    return 0;
}
