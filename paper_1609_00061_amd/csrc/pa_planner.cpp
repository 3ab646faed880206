// Choice of the cluster tree (Sec. 3.5): which pairs of packs are multiplied
// in which order.  Every tree gives the same array (Thm "associative"); the
// tree only decides the work.  Node cost is the naive cost r^L of the node's
// generalized array multiplication (eqn naive_cost), L = the union of the
// children's packs; a tree's cost is the sum over its nodes.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "pa_plan.h"

namespace pa {

int build_sysinfo(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, SysInfo &si) {
    if (!sys || !sys->axes || !sys->rel) return fail(PA_EINVAL, "system: null pointer");
    if (sys->n_vars < 1 || sys->n_vars > PA_MAX_VARS) return fail(PA_EINVAL, "system: n_vars must be 1..64");
    if (sys->n_rel < 1 || sys->n_rel > PA_MAX_RELATIONS) return fail(PA_EINVAL, "system: n_rel must be 1..32");
    if (n_exposed < 0 || n_exposed > PA_MAX_DIMS || (n_exposed > 0 && !exposed))
        return fail(PA_EINVAL, "system: bad exposed list");
    si = SysInfo();
    si.n_vars = sys->n_vars;
    si.n_rel = sys->n_rel;
    for (int v = 0; v < sys->n_vars; ++v) {
        const pa_axis &a = sys->axes[v];
        if (a.res < 2) return fail(PA_EINVAL, "system: resolution must be >= 2");
        if (!std::isfinite(a.lo) || !std::isfinite(a.hi) || !(a.lo <= a.hi))
            return fail(PA_EINVAL, "system: need finite lo <= hi");
        si.res.push_back(a.res);
    }
    uint64_t covered = 0;
    for (int r = 0; r < sys->n_rel; ++r) {
        const pa_relation &rel = sys->rel[r];
        int rc = validate_relation(rel, nullptr, sys->n_vars, "system");
        if (rc) return rc;
        uint64_t m = 0;
        std::vector<int> lst;
        for (int i = 0; i < rel.arity; ++i) {
            m |= 1ull << rel.vars[i];
            lst.push_back(rel.vars[i]);
        }
        for (int i = 0; i < n_monomials(rel.arity, rel.degree); ++i)
            if (!std::isfinite(rel.coef[i])) return fail(PA_EINVAL, "system: non-finite coefficient");
        si.rel_vars.push_back(m);
        si.rel_list.push_back(lst);
        covered |= m;
    }
    for (int v = 0; v < sys->n_vars; ++v)
        if (!((covered >> v) & 1)) return fail(PA_EINVAL, "system: variable " + std::to_string(v) + " is in no relation");
    for (int i = 0; i < n_exposed; ++i) {
        const int v = exposed[i];
        if (v < 0 || v >= sys->n_vars) return fail(PA_EINVAL, "system: exposed variable out of range");
        if ((si.exposed >> v) & 1) return fail(PA_EINVAL, "system: exposed variable repeated");
        si.exposed |= 1ull << v;
        si.exposed_list.push_back(v);
    }
    return PA_OK;
}

double mask_cost(uint64_t m, const SysInfo &si) {
    double c = 1.0;
    for (int v = 0; v < si.n_vars; ++v)
        if ((m >> v) & 1) c *= (double)si.res[v];
    return c;
}

uint64_t q_of(uint32_t cluster, const SysInfo &si) {
    uint64_t in = 0, out = si.exposed;
    for (int r = 0; r < si.n_rel; ++r) {
        if ((cluster >> r) & 1) in |= si.rel_vars[r];
        else out |= si.rel_vars[r];
    }
    return in & out;
}

static void add_leaves(const SysInfo &si, Tree &t) {
    t.nodes.clear();
    for (int r = 0; r < si.n_rel; ++r) {
        Node nd;
        nd.leaf = r;
        nd.leaves = 1u << r;
        nd.q = q_of(nd.leaves, si);
        t.nodes.push_back(nd);
    }
    t.merges.clear();
    t.cost = 0.0;
    t.root = si.n_rel == 1 ? 0 : -1;
}

int tree_from_merges(const SysInfo &si, const std::vector<int> &merges, Tree &t) {
    add_leaves(si, t);
    const int n = si.n_rel;
    if ((int)merges.size() != 2 * (n - 1)) return fail(PA_EINVAL, "given order: need n_rel - 1 merges");
    std::vector<char> used(2 * n, 0);
    for (int s = 0; s < n - 1; ++s) {
        const int a = merges[2 * s], b = merges[2 * s + 1];
        const int nid = n + s;
        if (a < 0 || b < 0 || a >= nid || b >= nid || a == b || used[a] || used[b])
            return fail(PA_EINVAL, "given order: merge " + std::to_string(s) + " names an unavailable factor");
        used[a] = used[b] = 1;
        Node nd;
        nd.c0 = a;
        nd.c1 = b;
        nd.leaves = t.nodes[a].leaves | t.nodes[b].leaves;
        nd.q = q_of(nd.leaves, si);
        t.cost += mask_cost(t.nodes[a].q | t.nodes[b].q, si);
        t.nodes.push_back(nd);
        t.merges.push_back(a);
        t.merges.push_back(b);
    }
    t.root = n == 1 ? 0 : 2 * n - 2;
    // a relation with latent variables of its own is first projected by a
    // one-pack cluster node (cost r^vars of the relation)
    for (int r = 0; r < n; ++r)
        if (si.rel_vars[r] & ~t.nodes[r].q) t.cost += mask_cost(si.rel_vars[r], si);
    return PA_OK;
}

// Greedy: repeatedly multiply the pair of current factors whose node is the
// cheapest among pairs sharing a variable (a pair without one is a Kronecker
// product and is taken only when no factors share anything); ties: smaller
// output pack, then lowest factor ids.
int plan_greedy(const SysInfo &si, Tree &t) {
    const int n = si.n_rel;
    std::vector<int> alive(n);
    for (int i = 0; i < n; ++i) alive[i] = i;
    std::vector<uint32_t> leaves(n);
    std::vector<uint64_t> q(n);
    for (int i = 0; i < n; ++i) {
        leaves[i] = 1u << i;
        q[i] = q_of(leaves[i], si);
    }
    std::vector<int> merges;
    int next = n;
    std::vector<int> ids(alive);
    while (ids.size() > 1) {
        double best = std::numeric_limits<double>::infinity(), best_out = 0.0;
        int bi = -1, bj = -1;
        bool best_shares = false;
        for (size_t i = 0; i < ids.size(); ++i)
            for (size_t j = i + 1; j < ids.size(); ++j) {
                const bool shares = (q[i] & q[j]) != 0;
                const double c = mask_cost(q[i] | q[j], si);
                const double out = mask_cost(q_of(leaves[i] | leaves[j], si), si);
                const bool better = (shares && !best_shares) ||
                                    (shares == best_shares && (c < best || (c == best && out < best_out)));
                if (bi < 0 || better) {
                    best = c;
                    best_out = out;
                    best_shares = shares;
                    bi = (int)i;
                    bj = (int)j;
                }
            }
        merges.push_back(ids[bi]);
        merges.push_back(ids[bj]);
        const uint32_t lv = leaves[bi] | leaves[bj];
        ids[bi] = next++;
        leaves[bi] = lv;
        q[bi] = q_of(lv, si);
        ids.erase(ids.begin() + bj);
        leaves.erase(leaves.begin() + bj);
        q.erase(q.begin() + bj);
    }
    return tree_from_merges(si, merges, t);
}

// Exhaustive: the cheapest binary cluster tree, by dynamic programming over
// subsets of relations (a cluster's intermediate pack depends only on its set
// of relations).  Among trees of equal cost the one with the lowest parallel
// cost (a node's cost plus the max of its children's, Sec. 3.5.1) wins: its
// independent subtrees run side by side.
int plan_exhaustive(const SysInfo &si, Tree &t) {
    const int n = si.n_rel;
    if (n > 16) return plan_greedy(si, t);
    const uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    std::vector<double> best((size_t)full + 1, std::numeric_limits<double>::infinity());
    std::vector<double> pbest((size_t)full + 1, std::numeric_limits<double>::infinity());
    std::vector<uint32_t> split((size_t)full + 1, 0);
    std::vector<uint64_t> q((size_t)full + 1, 0);
    for (uint32_t S = 1; S <= full; ++S) q[S] = q_of(S, si);
    for (int i = 0; i < n; ++i) best[1u << i] = pbest[1u << i] = 0.0;
    for (uint32_t S = 1; S <= full; ++S) {
        if ((S & (S - 1)) == 0) continue;
        const uint32_t low = S & (~S + 1);
        // enumerate S1 subset of S containing the lowest bit, S2 = S \ S1 nonempty
        const uint32_t rest = S ^ low;
        for (uint32_t sub = rest;; sub = (sub - 1) & rest) {
            const uint32_t S1 = sub | low, S2 = S ^ S1;
            if (S2) {
                const double node = mask_cost(q[S1] | q[S2], si);
                const double c = best[S1] + best[S2] + node;
                const double pc = node + std::max(pbest[S1], pbest[S2]);
                const double tol = 1e-12 * best[S];
                if (c < best[S] - tol || (c <= best[S] + tol && pc < pbest[S])) {
                    best[S] = c;
                    pbest[S] = pc;
                    split[S] = S1;
                }
            }
            if (sub == 0) break;
        }
    }
    // rebuild merges in post-order
    std::vector<int> merges;
    int next = n;
    std::vector<std::pair<uint32_t, int>> stack;
    // iterative post-order via recursion on a small depth (<= n)
    struct Rec {
        static int go(uint32_t S, const std::vector<uint32_t> &split, std::vector<int> &merges, int &next) {
            if ((S & (S - 1)) == 0) {
                int i = 0;
                while (!((S >> i) & 1)) ++i;
                return i;
            }
            const int a = go(split[S], split, merges, next);
            const int b = go(S ^ split[S], split, merges, next);
            merges.push_back(a);
            merges.push_back(b);
            return next++;
        }
    };
    if (n > 1) Rec::go(full, split, merges, next);
    return tree_from_merges(si, merges, t);
}

}  // namespace pa
