// Autotuner for the step executors: picks the executor (level-grouped
// launches or one persistent launch, and its workgroup count), the plot
// strip length, the streaming-contraction tile size, the MFMA K-split
// target and the MFMA operand path for a workload by
// timing candidates on the device.  Coordinate descent from the defaults;
// results are cached per structural signature of the workload and GPU
// architecture for the life of the process.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pa_plan.h"

namespace pa {

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t _e = (expr);                                                                         \
        if (_e != hipSuccess) return fail(PA_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

static void fnv(uint64_t &h, uint64_t v) {
    for (int i = 0; i < 8; ++i) {
        h ^= (v >> (8 * i)) & 0xff;
        h *= 0x100000001b3ull;
    }
}

// Resolutions, relation scopes and degrees, exposed lists and the options
// that change the plan.  The coefficients decide the densities of the plots
// and intermediates; every candidate but the sparse pass alone costs the
// same at any density, so they enter the key only when the tuner is free to
// pick the pass alone (opts->sparse_pass == 0): such a choice is reused only
// for the same instance, whose operands it was timed on.
static std::string signature(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                             const int32_t *n_exposed, const pa_opts &o) {
    uint64_t h = 0xcbf29ce484222325ull;
    fnv(h, (uint64_t)n_sys);
    for (int32_t i = 0; i < n_sys; ++i) {
        const pa_system &s = systems[i];
        fnv(h, (uint64_t)s.n_vars);
        for (int v = 0; v < s.n_vars; ++v) fnv(h, (uint64_t)s.axes[v].res);
        fnv(h, (uint64_t)s.n_rel);
        for (int r = 0; r < s.n_rel; ++r) {
            fnv(h, (uint64_t)s.rel[r].arity * 16 + (uint64_t)s.rel[r].degree);
            for (int j = 0; j < s.rel[r].arity; ++j) fnv(h, (uint64_t)s.rel[r].vars[j]);
            if (o.sparse_pass == 0 && s.rel[r].coef && s.rel[r].arity >= 1 && s.rel[r].arity <= PA_MAX_ARITY &&
                s.rel[r].degree >= 0 && s.rel[r].degree <= PA_MAX_DEGREE) {
                const int64_t nc = n_monomials(s.rel[r].arity, s.rel[r].degree);
                for (int64_t c = 0; c < nc; ++c) {
                    uint64_t bits;
                    std::memcpy(&bits, &s.rel[r].coef[c], sizeof(bits));
                    fnv(h, bits);
                }
            }
        }
        if (o.sparse_pass == 0) {
            for (int v = 0; v < s.n_vars; ++v) {
                uint64_t lo, hi;
                std::memcpy(&lo, &s.axes[v].lo, sizeof(lo));
                std::memcpy(&hi, &s.axes[v].hi, sizeof(hi));
                fnv(h, lo);
                fnv(h, hi);
            }
        }
        fnv(h, (uint64_t)n_exposed[i]);
        for (int j = 0; j < n_exposed[i]; ++j) fnv(h, (uint64_t)exposed[i][j]);
    }
    fnv(h, (uint64_t)o.order_policy * 97 + (uint64_t)o.precision * 7 + (uint64_t)o.graph);
    {
        uint64_t tol;
        std::memcpy(&tol, &o.tolerance, sizeof(tol));
        fnv(h, (uint64_t)o.plot_rule);
        fnv(h, (uint64_t)o.measure_density);
        fnv(h, tol);
        for (int32_t i = 0; i < n_sys; ++i)
            for (int r = 0; r < systems[i].n_rel; ++r) fnv(h, (uint64_t)systems[i].rel[r].target);
    }
    fnv(h, (uint64_t)(o.sparse_pass + 1));
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "?";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    return arch + ":" + std::to_string(h);
}

static std::mutex g_tune_mu;
static std::map<std::string, pa_tuning> g_tune_cache;

static void apply(pa_opts &o, const pa_tuning &t) {
    o.single_launch = t.single_launch;
    o.persist_wg = t.persist_wg;
    o.plot_strip = t.plot_strip;
    o.contract_units = t.contract_units;
    o.gemm_split = t.gemm_split;
    o.gemm_path = t.gemm_path;
    o.sparse_pass = t.sparse_pass;
}

// Milliseconds per execution of a batch built with `o`, after one untimed
// execution (which also captures the graph when o.graph is set).
static int time_candidate(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                          const int32_t *n_exposed, const pa_opts &o, int reps, hipStream_t s,
                          std::vector<pa_bitarray> &outs, double *ms) {
    pa_batch *B = nullptr;
    int rc = pa_batch_create(systems, n_sys, exposed, n_exposed, &o, &B);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = pa_batch_execute(B, outs.data(), nullptr, nullptr, s);
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(PA_EHIP, "autotune: event creation failed");
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fail(PA_EHIP, "autotune: event record failed");
    for (int i = 0; i < reps && !rc; ++i) rc = pa_batch_execute(B, outs.data(), nullptr, nullptr, s);
    float t = 0.f;
    if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = fail(PA_EHIP, "autotune: event timing failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    pa_batch_destroy(B);
    if (!rc) *ms = (double)t / reps;
    return rc;
}

int autotune(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed, const int32_t *n_exposed,
             const pa_opts &base, int reps, hipStream_t s, pa_tuning *best_out, pa_tuning *tried, int32_t cap,
             int32_t *n_tried) {
    if (reps < 1) reps = 3;
    pa_opts o = base;
    o.autotune = 0;
    o.timing = 0;
    o.audit = 0;
    o.plain = 0;
    o.per_op = 0;
    // outputs, allocated once for all candidates
    std::vector<pa_bitarray> outs(n_sys);
    std::vector<void *> bufs;
    int rc = PA_OK;
    for (int32_t i = 0; i < n_sys && !rc; ++i) {
        pa_bitarray &b = outs[i];
        std::memset(&b, 0, sizeof(b));
        b.ndim = n_exposed[i];
        int32_t dims[PA_MAX_DIMS];
        for (int j = 0; j < n_exposed[i]; ++j) {
            const int v = exposed[i][j];
            if (v < 0 || v >= systems[i].n_vars) rc = fail(PA_EINVAL, "autotune: exposed variable out of range");
            else dims[j] = b.dims[j] = systems[i].axes[v].res;
        }
        if (rc) break;
        b.row_words = n_exposed[i] ? pa_row_words(dims[n_exposed[i] - 1]) : 1;
        void *p = nullptr;
        const int64_t words = pa_array_words(n_exposed[i], dims);
        if (words < 1 || hipMalloc(&p, sizeof(uint32_t) * (size_t)words) != hipSuccess)
            rc = fail(PA_ENOMEM, "autotune: output allocation failed");
        b.data = p;
        bufs.push_back(p);
    }
    int32_t k = 0;
    pa_tuning best{};
    best.ms = -1.0;
    auto trial = [&](pa_tuning t) -> int {
        pa_opts c = o;
        apply(c, t);
        double ms = 0.0;
        const int r = time_candidate(systems, n_sys, exposed, n_exposed, c, reps, s, outs, &ms);
        if (r == PA_ENOMEM) return PA_OK;       // candidate does not fit: skip it
        if (r) return r;
        t.ms = ms;
        if (tried && k < cap) tried[k] = t;
        ++k;
        if (best.ms < 0.0 || ms < best.ms) best = t;
        return PA_OK;
    };
    // 1) executor
    const int cus_wg[] = {256, 512, 1024, 2048};
    pa_tuning cur{};
    cur.plot_strip = base.plot_strip > 0 ? base.plot_strip : 4;
    cur.contract_units = base.contract_units > 0 ? base.contract_units : 2048;
    cur.gemm_split = base.gemm_split > 0 ? base.gemm_split : 512;
    cur.gemm_path = base.gemm_path > 0 ? base.gemm_path : 1;
    cur.sparse_pass = base.sparse_pass;
    if (!rc) rc = trial(cur);
    for (int wg : cus_wg) {
        if (rc) break;
        pa_tuning t = cur;
        t.single_launch = 1;
        t.persist_wg = wg;
        rc = trial(t);
    }
    // 2) plot strip, 3) streaming tile, each with the best so far
    const int strips[] = {1, 2, 4, 8};
    for (int st : strips) {
        if (rc || best.ms < 0.0 || st == best.plot_strip) continue;
        pa_tuning t = best;
        t.plot_strip = st;
        rc = trial(t);
    }
    const int units[] = {512, 2048, 8192, 32768};
    for (int u : units) {
        if (rc || best.ms < 0.0 || u == best.contract_units) continue;
        pa_tuning t = best;
        t.contract_units = u;
        rc = trial(t);
    }
    const int splits[] = {1, 64, 128, 256, 512, 1024, 2048};
    for (int sp : splits) {
        if (rc || best.ms < 0.0 || sp == best.gemm_split) continue;
        pa_tuning t = best;
        t.gemm_split = sp;
        rc = trial(t);
    }
    for (int path : {1, 2, 3, 4}) {
        if (rc || best.ms < 0.0 || path == best.gemm_path) continue;
        pa_tuning t = best;
        t.gemm_path = path;
        rc = trial(t);
    }
    // 4) the sparse pass alone (exact whatever the density; faster when the
    // plotted operands are sparse and the contractions large), then with
    // pairs of passes fused into the streamed contraction that reads them
    for (int sp : {2, 3}) {
        if (rc || best.ms < 0.0 || base.sparse_pass != 0) break;
        pa_tuning t = best;
        t.sparse_pass = sp;
        rc = trial(t);
    }
    for (void *p : bufs) (void)hipFree(p);
    if (rc) return rc;
    if (best.ms < 0.0) return fail(PA_ENOMEM, "autotune: no candidate fits the workspace");
    if (n_tried) *n_tried = k;
    *best_out = best;
    return PA_OK;
}

// Tuned settings for a workload, from the cache or by tuning on stream 0.
int autotuned_opts(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                   const int32_t *n_exposed, pa_opts &o) {
    const std::string key = signature(systems, n_sys, exposed, n_exposed, o);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            apply(o, it->second);
            o.autotune = 0;
            return PA_OK;
        }
    }
    pa_tuning t{};
    int rc = autotune(systems, n_sys, exposed, n_exposed, o, 3, nullptr, &t, nullptr, 0, nullptr);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = t;
    }
    apply(o, t);
    o.autotune = 0;
    return PA_OK;
}

}  // namespace pa

using namespace pa;

extern "C" int pa_autotune(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                           const int32_t *n_exposed, const pa_opts *opts, int32_t reps, pa_tuning *best,
                           pa_tuning *tried, int32_t cap, int32_t *n_tried, void *stream) {
    if (!systems || n_sys < 1 || !exposed || !n_exposed || !best) return fail(PA_EINVAL, "autotune: bad arguments");
    pa_opts o{};
    if (opts) o = *opts;
    int rc = autotune(systems, n_sys, exposed, n_exposed, o, reps, static_cast<hipStream_t>(stream), best, tried,
                      cap, n_tried);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[signature(systems, n_sys, exposed, n_exposed, o)] = *best;
    return PA_OK;
}
