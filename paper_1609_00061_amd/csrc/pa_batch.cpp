// Batched solving: many independent systems, each planned on its own (cluster
// tree, layouts), share one workspace and one merged step table.  Steps of
// every system are sorted together by (tree level, kind, mode), so each
// grouped launch -- or the single persistent launch -- runs tiles of many
// systems at once, and the whole batch is one hipGraph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "pa_plan.h"

struct pa_batch {
    std::vector<std::unique_ptr<pa_plan>> subs;
    pa_plan master;                 // merged step table and executor state; owns the workspace
    std::vector<size_t> sub_off;
};

namespace pa {

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t _e = (expr);                                                                         \
        if (_e != hipSuccess) return fail(PA_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

static int merge_steps(pa_batch *B) {
    pa_plan &M = B->master;
    struct Ref {
        int level, kind, mode, sys, local;
    };
    std::vector<Ref> refs;
    std::vector<int> first(B->subs.size());
    for (size_t i = 0; i < B->subs.size(); ++i) {
        first[i] = (int)refs.size();
        const pa_plan &P = *B->subs[i];
        for (size_t j = 0; j < P.steps_host.size(); ++j)
            refs.push_back({P.step_level[j], P.steps_host[j].kind, P.steps_host[j].mode, (int)i, (int)j});
    }
    std::vector<int> order(refs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto key = [&](int i) { return std::make_tuple(refs[i].level, refs[i].kind, refs[i].mode); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<int> pos(refs.size());
    for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;
    M.steps_host.clear();
    M.step_level.clear();
    M.step_macs.clear();
    int64_t tbase = 0;
    for (int g : order) {
        const Ref &r = refs[g];
        const pa_plan &P = *B->subs[r.sys];
        PStep s = P.steps_host[r.local];
        for (int j = 0; j < s.ndep; ++j) s.dep[j] = pos[first[r.sys] + s.dep[j]];
        s.tile_base = tbase;
        tbase += s.n_tiles;
        M.steps_host.push_back(s);
        M.step_level.push_back(r.level);
        M.step_macs.push_back(P.step_macs[r.local]);
    }
    M.step_out_refs.clear();
    for (size_t i = 0; i < B->subs.size(); ++i)
        for (const auto &ref : B->subs[i]->step_out_refs) M.step_out_refs.push_back({pos[first[i] + ref.first], (int)i});
    M.n_items = tbase;
    make_groups(&M);
    return PA_OK;
}

int measure_leaf_densities(const pa_system *systems, int32_t n_sys, const pa_opts &o,
                           std::vector<std::vector<double>> &ld) {
    ld.assign(n_sys, {});
    struct One {
        std::vector<int32_t> vars;
        std::vector<pa_axis> axes;
        pa_relation rel;
        std::vector<int64_t> dims;
        int sys, r;
    };
    std::vector<One> ones;
    for (int32_t i = 0; i < n_sys; ++i) {
        const pa_system &S = systems[i];
        if (!S.rel || !S.axes || S.n_rel < 1 || S.n_rel > PA_MAX_RELATIONS || S.n_vars < 1) continue;
        bool ok = true;
        for (int r = 0; r < S.n_rel && ok; ++r) {
            const pa_relation &R = S.rel[r];
            if (R.arity < 1 || R.arity > PA_MAX_ARITY || !R.vars) { ok = false; break; }
            std::vector<pa_axis> ax;
            for (int j = 0; j < R.arity; ++j) {
                if (R.vars[j] < 0 || R.vars[j] >= S.n_vars) { ok = false; break; }
                ax.push_back(S.axes[R.vars[j]]);
            }
            ok = ok && validate_relation(R, ax.data(), -1, "density probe") == PA_OK;
        }
        if (!ok) {
            g_err.clear();
            continue;
        }
        ld[i].assign(S.n_rel, 0.0);
        for (int r = 0; r < S.n_rel; ++r) {
            One one;
            const pa_relation &R = S.rel[r];
            one.sys = i;
            one.r = r;
            for (int j = 0; j < R.arity; ++j) {
                one.vars.push_back(j);
                one.axes.push_back(S.axes[R.vars[j]]);
                one.dims.push_back(S.axes[R.vars[j]].res);
            }
            one.rel = R;
            ones.push_back(std::move(one));
        }
    }
    if (ones.empty()) return PA_OK;
    // one single-relation system per plot, every variable exposed: the plot itself
    const size_t n = ones.size();
    std::vector<pa_system> subs(n);
    std::vector<const int32_t *> exp(n);
    std::vector<int32_t> n_exp(n);
    std::vector<int64_t> off(n);
    int64_t words = 0;
    for (size_t k = 0; k < n; ++k) {
        One &one = ones[k];
        one.rel.vars = one.vars.data();
        subs[k] = {one.rel.arity, one.axes.data(), 1, &one.rel};
        exp[k] = one.vars.data();
        n_exp[k] = one.rel.arity;
        off[k] = words;
        std::vector<int32_t> d32(one.dims.begin(), one.dims.end());
        words += pa_array_words(one.rel.arity, d32.data());
    }
    pa_opts po{};
    po.precision = o.precision;
    po.plot_rule = o.plot_rule;
    po.tolerance = o.tolerance;
    pa_batch *B = nullptr;
    int rc = pa_batch_create(subs.data(), (int32_t)n, exp.data(), n_exp.data(), &po, &B);
    if (rc) return rc;
    void *buf = nullptr;
    if (hipMalloc(&buf, sizeof(uint32_t) * (size_t)std::max<int64_t>(1, words)) != hipSuccess) {
        pa_batch_destroy(B);
        return fail(PA_ENOMEM, "density probe: output allocation failed");
    }
    std::vector<pa_bitarray> outs(n);
    for (size_t k = 0; k < n; ++k) {
        std::memset(&outs[k], 0, sizeof(pa_bitarray));
        outs[k].data = static_cast<uint32_t *>(buf) + off[k];
        outs[k].ndim = ones[k].rel.arity;
        for (int j = 0; j < outs[k].ndim; ++j) outs[k].dims[j] = (int32_t)ones[k].dims[j];
        outs[k].row_words = pa_row_words(outs[k].dims[outs[k].ndim - 1]);
    }
    std::vector<pa_report> reps(n);
    rc = pa_batch_execute(B, outs.data(), nullptr, reps.data(), nullptr);
    pa_batch_destroy(B);
    (void)hipFree(buf);
    if (rc) return rc;
    for (size_t k = 0; k < n; ++k) {
        double cells = 1.0;
        for (int64_t d : ones[k].dims) cells *= (double)d;
        const double nnz = (double)reps[k].nnz_out;
        ld[ones[k].sys][ones[k].r] = nnz > 0.0 ? std::log2(nnz / cells) : -std::numeric_limits<double>::infinity();
    }
    return PA_OK;
}

}  // namespace pa

using namespace pa;

extern "C" int pa_batch_create(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                               const int32_t *n_exposed, const pa_opts *opts, pa_batch **out) {
    if (!out) return fail(PA_EINVAL, "batch_create: null batch pointer");
    *out = nullptr;
    if (!systems || n_sys < 1 || !exposed || !n_exposed) return fail(PA_EINVAL, "batch_create: bad arguments");
    pa_opts o{};
    if (opts) o = *opts;
    if (o.plain || o.per_op) return fail(PA_EINVAL, "batch_create: batches run on the step executors (no plain/per_op)");
    if (o.autotune) {
        int rc = autotuned_opts(systems, n_sys, exposed, n_exposed, o);
        if (rc) return rc;
    }
    if (o.timing == 2) o.timing = 0;       // op events live on the merged plan, below
    std::vector<std::vector<double>> dens;
    if (o.measure_density) {
        int rc = measure_leaf_densities(systems, n_sys, o, dens);
        if (rc) return rc;
    }
    std::unique_ptr<pa_batch> B(new pa_batch());
    size_t off = 0;
    for (int32_t i = 0; i < n_sys; ++i) {
        std::unique_ptr<pa_plan> P(new pa_plan());
        if (o.measure_density) P->leaf_log2d = dens[i];
        int rc = build_plan(&systems[i], exposed[i], n_exposed[i], &o, P.get());
        if (rc) {
            g_err = "system " + std::to_string(i) + ": " + g_err;
            return rc;
        }
        B->sub_off.push_back(off);
        off += (P->ws_bytes + 255) / 256 * 256;
        B->subs.push_back(std::move(P));
    }
    pa_plan &M = B->master;
    M.per_op = 0;
    M.graph = o.graph;
    M.single_launch = o.single_launch && o.plot_rule != PA_RULE_CENTER;   // corner plots only (as for plans)
    M.persist_wg = o.persist_wg;
    M.timing = o.timing;
    size_t nsteps = 0;
    for (auto &P : B->subs) nsteps += P->plots.size() + P->ops.size();
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    M.steps_off = take(sizeof(PStep) * std::max<size_t>(1, nsteps));
    M.pgroups_off = take(sizeof(PGroup) * std::max<size_t>(1, nsteps));
    M.levels_off = take(2 * sizeof(int64_t) * std::max<size_t>(1, nsteps));
    M.state_off = take(sizeof(PersistState));
    M.counters_off = take(sizeof(PlotCounters) * (size_t)n_sys);   // one block per system
    M.popcnt_off = take(sizeof(unsigned long long) * (size_t)n_sys);
    M.ws_bytes = off;
    int rc;
    if (o.workspace) {
        if (o.workspace_bytes < M.ws_bytes)
            return fail(PA_ENOMEM, "workspace too small: need " + std::to_string(M.ws_bytes) + " bytes");
        M.ws.ptr = o.workspace;
        M.ws.cap = o.workspace_bytes;
        M.ws.external = true;
    } else {
        size_t cap = 0;
        rc = plan_workspace_cap(&cap);
        if (rc) return rc;
        if (M.ws_bytes > cap)
            return fail(PA_ENOMEM, "batch needs " + std::to_string(M.ws_bytes) + " bytes of workspace, " +
                                       std::to_string(cap) + " available");
        rc = M.ws.ensure(std::max<size_t>(M.ws_bytes, 256));
        if (rc) return rc;
    }
    char *base = static_cast<char *>(M.ws.ptr);
    M.total_macs = 0.0;
    M.corners = 0;
    for (size_t i = 0; i < B->subs.size(); ++i) {
        pa_plan &P = *B->subs[i];
        P.ws.ptr = base + B->sub_off[i];
        P.ws.cap = P.ws_bytes;
        P.ws.external = true;
        P.counters_dev = reinterpret_cast<PlotCounters *>(base + M.counters_off) + i;
        rc = upload_plan(&P);
        if (rc) return rc;
        M.total_macs += P.total_macs;
        M.corners += P.corners;
    }
    rc = merge_steps(B.get());
    if (rc) return rc;
    HIP_TRY(hipMemset(base + M.counters_off, 0, sizeof(PlotCounters) * (size_t)n_sys));
    HIP_TRY(hipMemset(base + M.state_off, 0, sizeof(PersistState)));
    HIP_TRY(hipMemcpy(base + M.state_off + offsetof(PersistState, wait_limit), &kDefaultWaitLimit,
                      sizeof(kDefaultWaitLimit), hipMemcpyHostToDevice));
    rc = upload_pgroups(&M);
    if (rc) return rc;
    if (opts && opts->timing == 2) {
        M.op_events.resize(M.single_launch ? 2 : std::max<size_t>(2, 2 * M.groups.size()));
        for (auto &e : M.op_events) HIP_TRY(hipEventCreate(&e));
    }
    *out = B.release();
    return PA_OK;
}

// Steps of a plan counted in a report: the pairwise contractions (not
// projections of one operand, fills, count steps, or a sparse pass whose MFMA
// contraction is counted).
static int counted_steps(const pa_plan &P) {
    int steps = 0;
    for (const auto &op : P.ops) steps += counted_steps_of(op);
    return steps;
}

extern "C" int pa_batch_execute(pa_batch *B, pa_bitarray *outs, pa_report *rep, pa_report *reports, void *stream) {
    if (!B || !outs) return fail(PA_EINVAL, "batch_execute: null argument");
    const size_t n = B->subs.size();
    std::vector<void *> o(n);
    for (size_t i = 0; i < n; ++i) {
        int rc = check_bitarray(&outs[i], B->subs[i]->out_layout.dims, "batch_execute: out");
        if (rc) {
            g_err = "system " + std::to_string(i) + ": " + g_err;
            return rc;
        }
        o[i] = outs[i].data;
    }
    pa_plan &M = B->master;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int launches = 0;
    M.timing_active = false;
    char *base = static_cast<char *>(M.ws.ptr);
    auto *cdev = reinterpret_cast<PlotCounters *>(base + M.counters_off);
    std::vector<PlotCounters> cnt0(n), cnt(n);
    if (rep || reports) HIP_TRY(hipMemcpyAsync(cnt0.data(), cdev, n * sizeof(PlotCounters), hipMemcpyDeviceToHost, s));
    int rc = exec_steps(&M, o, s, &launches);
    if (rc) return rc;
    if (rep || reports) {
        auto *counts = reinterpret_cast<unsigned long long *>(base + M.popcnt_off);
        HIP_TRY(launch_fill(reinterpret_cast<uint32_t *>(counts), 2 * (int64_t)n, 0u, s));
        for (size_t i = 0; i < n; ++i)
            HIP_TRY(launch_popcount(static_cast<const uint32_t *>(o[i]), B->subs[i]->out_layout.words, counts + i, s));
        std::vector<unsigned long long> c(n);
        PersistState pst;
        HIP_TRY(hipMemcpyAsync(c.data(), counts, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(cnt.data(), cdev, n * sizeof(PlotCounters), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&pst, base + M.state_off, sizeof(pst), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (pst.abort) return fail(PA_EHIP, "persistent executor gave up a dependency wait");
        pa_report tot;
        std::memset(&tot, 0, sizeof(tot));
        for (size_t i = 0; i < n; ++i) {
            const pa_plan &P = *B->subs[i];
            pa_report r;
            std::memset(&r, 0, sizeof(r));
            r.corners = P.corners;
            r.corners_flagged = (int64_t)(cnt[i].flagged - cnt0[i].flagged);
            r.corners_disagree = (int64_t)(cnt[i].disagree - cnt0[i].disagree);
            r.corners_disagree_unflagged = (int64_t)(cnt[i].disagree_unflagged - cnt0[i].disagree_unflagged);
            r.nnz_out = (int64_t)c[i];
            r.n_steps = counted_steps(P);
            r.n_launches = launches;
            for (size_t k = 0; k < P.tree.merges.size() && k < 2 * PA_MAX_RELATIONS; ++k) r.merges[k] = P.tree.merges[k];
            r.cost_macs = P.tree.cost;
            r.t_plan_ms = P.t_plan_ms;
            if (reports) reports[i] = r;
            tot.corners += r.corners;
            tot.corners_flagged += r.corners_flagged;
            tot.corners_disagree += r.corners_disagree;
            tot.corners_disagree_unflagged += r.corners_disagree_unflagged;
            tot.nnz_out += r.nnz_out;
            tot.n_steps += r.n_steps;
            tot.cost_macs += r.cost_macs;
            tot.t_plan_ms += r.t_plan_ms;
        }
        tot.n_launches = launches;
        if (rep) *rep = tot;
    }
    return PA_OK;
}

extern "C" size_t pa_batch_workspace_bytes(const pa_batch *B) { return B ? B->master.ws_bytes : 0; }

extern "C" int32_t pa_batch_op_times(pa_batch *B, double *ms, int32_t *kind, double *macs, int32_t cap) {
    if (!B) return fail(PA_EINVAL, "batch_op_times: null batch"), -1;
    return pa_plan_op_times(&B->master, ms, kind, macs, cap);
}

extern "C" int32_t pa_batch_time_groups(pa_batch *B, int32_t reps, double *ms, int32_t *kind, double *macs,
                                        int32_t cap, void *stream) {
    if (!B) return fail(PA_EINVAL, "time_groups: null batch"), -1;
    return time_groups(&B->master, reps, ms, kind, macs, cap, static_cast<hipStream_t>(stream));
}

extern "C" int pa_batch_set_wait_limit(pa_batch *B, int64_t polls) {
    if (!B) return fail(PA_EINVAL, "set_wait_limit: null batch");
    return set_wait_limit(&B->master, polls);
}

extern "C" void pa_batch_destroy(pa_batch *B) { delete B; }

extern "C" int pa_solve_batch(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                              const int32_t *n_exposed, const pa_opts *opts, pa_bitarray *outs, pa_report *reports,
                              void *stream) {
    pa_batch *B = nullptr;
    int rc = pa_batch_create(systems, n_sys, exposed, n_exposed, opts, &B);
    if (rc) return rc;
    rc = pa_batch_execute(B, outs, nullptr, reports, stream);
    if (rc == PA_OK && hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        rc = fail(PA_EHIP, "sync failed");
    pa_batch_destroy(B);
    return rc;
}
