// Plan construction (layouts of every intermediate and the op list) and
// execution, plus the C ABI entry points that use them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "pa_plan.h"

namespace pa {

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t _e = (expr);                                                                         \
        if (_e != hipSuccess) return fail(PA_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

static std::vector<int> mask_list(uint64_t m) {
    std::vector<int> out;
    for (int v = 0; v < 64; ++v)
        if ((m >> v) & 1) out.push_back(v);
    return out;
}

static uint64_t list_mask(const std::vector<int> &l) {
    uint64_t m = 0;
    for (int v : l) m |= 1ull << v;
    return m;
}


// The latent variable to pack (bit axis) among `cands`: least row padding,
// then larger resolution, then lower id.
static int pick_packed(uint64_t cands, const std::vector<int64_t> &res) {
    int best = -1;
    int64_t bw = 0, br = 0;
    for (int v : mask_list(cands)) {
        const int64_t waste = row_words_of(res[v]) * 32 - res[v];
        if (best < 0 || waste < bw || (waste == bw && res[v] > br)) {
            best = v;
            bw = waste;
            br = res[v];
        }
    }
    return best;
}

static std::vector<int> move_last(std::vector<int> l, int v) {
    auto it = std::find(l.begin(), l.end(), v);
    if (it != l.end()) {
        l.erase(it);
        l.push_back(v);
    }
    return l;
}

// A layout requirement on a node's output array.
struct Constraint {
    int kind = 0;             // 0 free, 1 full order, 2 packed variable (+ hint for the axis before it)
    std::vector<int> order;
    int packed = -1, hint = -1;
    static Constraint full(const std::vector<int> &o) {
        Constraint c;
        c.kind = 1;
        c.order = o;
        return c;
    }
    static Constraint pk(int v, int hint) {
        Constraint c;
        c.kind = 2;
        c.packed = v;
        c.hint = hint;
        return c;
    }
    std::string key() const {
        std::string s = std::to_string(kind) + ":" + std::to_string(packed) + ":" + std::to_string(hint) + ":";
        for (int v : order) s += std::to_string(v) + ",";
        return s;
    }
};

// Output order under a constraint, from a preferred order.
static std::vector<int> order_under(const Constraint &cons, const std::vector<int> &pref) {
    if (cons.kind == 1) return cons.order;
    if (cons.kind == 2) {
        std::vector<int> o = pref;
        if (cons.hint >= 0 && std::find(o.begin(), o.end(), cons.hint) != o.end()) o = move_last(o, cons.hint);
        return move_last(o, cons.packed);
    }
    return pref;
}

static bool fits_gemm(const std::vector<int> &L, uint64_t b, uint64_t ea, uint64_t eb) {
    const int nb = __builtin_popcountll(b), na = __builtin_popcountll(ea), nn = __builtin_popcountll(eb);
    if ((int)L.size() != nb + na + nn || nn == 0) return false;
    std::vector<int> p0(L.begin(), L.begin() + nb), p1(L.begin() + nb, L.begin() + nb + na),
        p2(L.begin() + nb + na, L.end());
    return list_mask(p0) == b && list_mask(p1) == ea && list_mask(p2) == eb;
}

static std::vector<std::vector<int>> orders_of(uint64_t m, int packed_last, size_t cap) {
    std::vector<int> l = mask_list(m);
    std::vector<std::vector<int>> out;
    std::sort(l.begin(), l.end());
    do {
        if (packed_last < 0 || l.back() == packed_last) out.push_back(l);
        if (out.size() >= cap) break;
    } while (std::next_permutation(l.begin(), l.end()));
    return out;
}

// Rough time model (microseconds) used to rank layout choices: MFMA GEMM,
// word-streaming and bit-level contraction throughputs, HBM traffic and a
// launch overhead.  Only the ranking matters.
static double est_op_us(int kind, double macs, double bytes) {
    const double launch = 4.0;
    double rate;   // MAC per microsecond
    switch (kind) {
        case 0: rate = 1.0e9; break;      // MFMA
        case 1: rate = 4.0e7; break;      // word streaming
        default: rate = 5.0e5; break;     // bit level
    }
    return launch + macs / rate + bytes / 4.0e6;
}

struct Choice {
    int kind = -1;            // 0 gemm, 1 stream (mode chosen from layouts), 2 leaf
    int roleB = -1;           // gemm: 0 -> c0 is the B operand, 1 -> c1 is
    std::vector<int> oc;      // output order
    Constraint cx, cy;        // child constraints (c0, c1)
    int nb = 0, nm = 0;       // gemm group sizes
    double cost = 0.0;
};

static void set_ksplit(GemmArgs &g, int64_t want);

// Default operand path of one MFMA contraction: 256 x 128 tiles (fewer
// operand spreads and tile set-ups per MFMA) once the output has at least
// 8192 tiles of 128 x 128, where the extra tiles in flight cost nothing --
// with the A operands kept in registers across tiles when K is one chunk
// (at most 256 bits) and output rows are at least 1024 bits --; 128 x 128
// tiles below that, where parallelism matters more.
static int auto_gemm_path(const GemmArgs &g) {
    const int64_t tiles = g.nbatch * ((g.M + 127) / 128) * ((g.No * g.rwc * 32 + 127) / 128);
    if (tiles < 8192) return 0;
    // the resident path writes output rows in groups of 8 column tiles
    // (1024 bits): narrower outputs would flush (and reload A) every tile or two
    return g.Kw <= 8 && g.No * g.rwc * 32 >= 1024 ? 3 : 2;
}

struct Builder {
    pa_plan *P;
    const pa_system *sys;
    std::map<std::string, Choice> memo;

    int new_buf(const Layout &L) {
        P->buf_layout.push_back(L);
        P->buf_words.push_back(L.words);
        P->buf_off.push_back(-1);
        return (int)P->buf_layout.size() - 1;
    }
    Layout lay(const std::vector<int> &o) { return make_layout(o, P->si.res); }
    double bytes_of(uint64_t m) { return mask_cost(m, P->si) / 8.0; }

    // ------------------------------------------------------------ search
    const Choice &best(int id, const Constraint &cons) {
        const std::string key = std::to_string(id) + "|" + cons.key();
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        Choice ch = decide(id, cons);
        return memo.emplace(key, ch).first->second;
    }

    Choice decide(int id, const Constraint &cons) {
        const Node &nd = P->tree.nodes[id];
        const auto &si = P->si;
        Choice bestc;
        bestc.cost = 1e300;
        if (nd.leaf >= 0) {
            const int r = nd.leaf;
            const uint64_t priv = si.rel_vars[r] & ~nd.q;
            std::vector<int> qdecl;
            for (int v : si.rel_list[r])
                if ((nd.q >> v) & 1) qdecl.push_back(v);
            bestc.kind = 2;
            bestc.oc = order_under(cons, qdecl);
            const double full = mask_cost(si.rel_vars[r], si);
            bestc.cost = est_op_us(1, full / 64.0, full / 8.0);      // plotting ~ one pass
            if (priv) bestc.cost += est_op_us(1, full, full / 8.0);
            return bestc;
        }
        const Node &X = P->tree.nodes[nd.c0], &Y = P->tree.nodes[nd.c1];
        const uint64_t qx = X.q, qy = Y.q, q = nd.q;
        const uint64_t b = q & qx & qy, k = qx & qy & ~q, ex = qx & ~qy, ey = qy & ~qx;
        const double macs = mask_cost(qx | qy, si);
        const double io = bytes_of(qx) + bytes_of(qy) + bytes_of(q);
        // ---- dense Boolean GEMM on MFMA
        if (k && ex && ey && mask_cost(k, si) >= 32 && mask_cost(ex, si) >= 32 && mask_cost(ey, si) >= 32) {
            for (int roleB = 0; roleB < 2; ++roleB) {
                const uint64_t ea = roleB ? ex : ey, eb = roleB ? ey : ex;
                std::vector<int> bo, mo, no;
                if (cons.kind == 1) {
                    if (!fits_gemm(cons.order, b, ea, eb)) continue;
                    const int nb = __builtin_popcountll(b), na = __builtin_popcountll(ea);
                    bo.assign(cons.order.begin(), cons.order.begin() + nb);
                    mo.assign(cons.order.begin() + nb, cons.order.begin() + nb + na);
                    no.assign(cons.order.begin() + nb + na, cons.order.end());
                } else {
                    if (cons.kind == 2 && !((eb >> cons.packed) & 1)) continue;
                    bo = mask_list(b);
                    mo = mask_list(ea);
                    no = mask_list(eb);
                    no = move_last(no, cons.kind == 2 ? cons.packed : pick_packed(eb, si.res));
                }
                for (const auto &ko : orders_of(k, -1, 24)) {
                    std::vector<int> oa = bo, ob = bo, oc = bo;
                    oa.insert(oa.end(), mo.begin(), mo.end());
                    oa.insert(oa.end(), ko.begin(), ko.end());
                    ob.insert(ob.end(), no.begin(), no.end());
                    ob.insert(ob.end(), ko.begin(), ko.end());
                    oc.insert(oc.end(), mo.begin(), mo.end());
                    oc.insert(oc.end(), no.begin(), no.end());
                    const Constraint ca = Constraint::full(oa), cb = Constraint::full(ob);
                    const int ida = roleB ? nd.c0 : nd.c1, idb = roleB ? nd.c1 : nd.c0;
                    // padding of the packed k axis wastes MFMA work
                    const int kl = ko.back();
                    const double kpad = (double)(row_words_of(si.res[kl]) * 32) / (double)si.res[kl];
                    const double c = est_op_us(0, macs * kpad, io) + best(ida, ca).cost + best(idb, cb).cost;
                    if (c < bestc.cost) {
                        bestc = Choice();
                        bestc.kind = 0;
                        bestc.roleB = roleB;
                        bestc.oc = oc;
                        bestc.cx = roleB ? ca : cb;
                        bestc.cy = roleB ? cb : ca;
                        bestc.nb = (int)bo.size();
                        bestc.nm = (int)mo.size();
                        bestc.cost = c;
                    }
                }
            }
        }
        // ---- bitwise streaming contractions
        std::vector<int> pref = mask_list(b);
        for (int v : mask_list(ex)) pref.push_back(v);
        for (int v : mask_list(ey)) pref.push_back(v);
        const std::vector<int> oc = order_under(cons, pref);
        const int cp = oc.empty() ? -1 : oc.back();
        if (k) {
            for (int kp : mask_list(k)) {
                const Constraint c0 = Constraint::pk(kp, cp), c1 = Constraint::pk(kp, cp);
                const double c = est_op_us(1, macs, io) + best(nd.c0, c0).cost + best(nd.c1, c1).cost;
                if (c < bestc.cost) {
                    bestc = Choice();
                    bestc.kind = 1;
                    bestc.oc = oc;
                    bestc.cx = c0;
                    bestc.cy = c1;
                    bestc.cost = c;
                }
            }
        }
        if (bestc.kind < 0) {
            // no latent variable: every child variable is an output variable.
            // Word streaming with the children holding the output's packed
            // axis packed along it (a child without it contributes a bit)
            Constraint c0, c1;
            int kind = 2;
            if (cp >= 0 && ((qx >> cp) & 1)) c0 = Constraint::pk(cp, -1);
            if (cp >= 0 && ((qy >> cp) & 1)) c1 = Constraint::pk(cp, -1);
            if (cp >= 0 && (((qx | qy) >> cp) & 1)) kind = 1;
            bestc.kind = 1;
            bestc.oc = oc;
            bestc.cx = c0;
            bestc.cy = c1;
            bestc.cost = est_op_us(kind, macs, io) + best(nd.c0, c0).cost + best(nd.c1, c1).cost;
        }
        return bestc;
    }

    // ------------------------------------------------------------ emission
    void emit_contract(int a, const Layout &la, int b, const Layout *lb, int c, const Layout &lc, int node) {
        Op op;
        op.kind = OP_CONTRACT;
        op.a = a;
        op.b = b;
        op.c = c;
        op.la = la;
        if (lb) op.lb = *lb;
        op.lc = lc;
        op.node = node;
        uint64_t ins = list_mask(la.vars) | (lb ? list_mask(lb->vars) : 0);
        op.kvars = mask_list(ins & ~list_mask(lc.vars));
        op.macs = mask_cost(ins, P->si);
        P->ops.push_back(op);
    }

    void emit_gemm(int a, const Layout &la, int b, const Layout &lb, int c, const Layout &lc, int nb_vars, int m_vars,
                   int node) {
        Op op;
        op.kind = OP_GEMM;
        op.a = a;
        op.b = b;
        op.c = c;
        op.la = la;
        op.lb = lb;
        op.lc = lc;
        op.node = node;
        op.macs = mask_cost(list_mask(la.vars) | list_mask(lb.vars), P->si);
        GemmArgs &g = op.ga;
        const int nk = (int)la.vars.size() - nb_vars - m_vars;
        const int nn = (int)lb.vars.size() - nb_vars - nk;
        g.nbatch = 1;
        for (int i = 0; i < nb_vars; ++i) g.nbatch *= la.dims[i];
        g.M = 1;
        for (int i = nb_vars; i < nb_vars + m_vars; ++i) g.M *= la.dims[i];
        g.No = 1;
        for (int i = nb_vars; i < nb_vars + nn - 1; ++i) g.No *= lb.dims[i];
        g.rn = lb.dims[nb_vars + nn - 1];
        g.Kw = la.rw;
        for (int i = nb_vars + m_vars; i < (int)la.vars.size() - 1; ++i) g.Kw *= la.dims[i];
        g.rwc = lc.rw;
        g.sA_b = g.M * g.Kw;
        g.sB_b = g.No * g.rn * g.Kw;
        g.sC_b = g.M * g.No * g.rwc;
        g.path = P->gemm_path >= 0 ? P->gemm_path : auto_gemm_path(g);
        if (g.path == 3 && g.Kw > 8) g.path = 2;      // the resident path takes one K chunk
        const int64_t tm = g.path >= 2 ? 256 : 128;   // tile rows of the operand path
        g.tiles_m = (g.M + tm - 1) / tm;
        g.tiles_n = (g.No * g.rwc * 32 + 127) / 128;
        // the K split (and the fill it needs) is set by split_gemms once
        // every step of the tree is known
        set_ksplit(g, 1);
        g.fd_tiles_n = make_fastdiv((uint64_t)std::max<int64_t>(1, g.tiles_n));
        g.fd_tiles_m = make_fastdiv((uint64_t)std::max<int64_t>(1, g.tiles_m));
        g.fd_wc = make_fastdiv((uint64_t)(g.rwc * 32));
        P->ops.push_back(op);
    }

    // An MFMA contraction with a sparse pass, when B is a plotted relation: the
    // relation is plotted a second time as Bt = [batch vars, latent vars in
    // A's order, output n vars in C's order] (rows of Bt have C's row layout).
    // With a fallback (at least 2^32 MACs, or sparse_pass = 1) a count step
    // adds up the set bits of A and then either the pass (at most
    // sparse_max_density set bits per 1024 bits of A) or the MFMA kernel
    // computes the output; the other exits at once.  With sparse_pass = 2
    // the pass alone computes it (no count, and B's first plot is dropped
    // when nothing else reads it): for callers who know A is sparse.
    void emit_gemm_with_pass(int a, const Layout &la, int b, const Layout &lb, int bnode, int c, const Layout &lc,
                             int nb, int nm, int node) {
        const Node &bn = P->tree.nodes[bnode];
        const bool b_plot = bn.leaf >= 0 && !(P->si.rel_vars[bn.leaf] & ~bn.q);
        const double macs = mask_cost(list_mask(la.vars) | list_mask(lb.vars), P->si);
        int mode = 0;         // 0: MFMA only, 1: pass with MFMA fallback, 2: pass only
        if (b_plot && P->sparse_pass >= 0) {
            if (P->sparse_pass >= 1) mode = std::min(P->sparse_pass, 2);
            else if (macs >= 4294967296.0) mode = 1;
        }
        if (mode == 0) {
            emit_gemm(a, la, b, lb, c, lc, nb, nm, node);
            return;
        }
        std::vector<int> order(lc.vars.begin(), lc.vars.begin() + nb);
        order.insert(order.end(), la.vars.begin() + nb + nm, la.vars.end());
        order.insert(order.end(), lc.vars.begin() + nb + nm, lc.vars.end());
        const int bt = plot_leaf(bn.leaf, order);
        GatherArgs ga{};
        int64_t nbatch = 1, M = 1, kout = 1, kall = 1, nout = 1;
        for (int i = 0; i < nb; ++i) nbatch *= lc.dims[i];
        for (int i = nb; i < nb + nm; ++i) M *= lc.dims[i];
        for (size_t i = nb + nm; i < la.vars.size(); ++i) {
            kall *= la.dims[i];
            if (i + 1 < la.vars.size()) kout *= la.dims[i];
        }
        for (size_t i = nb + nm; i + 1 < lc.vars.size(); ++i) nout *= lc.dims[i];
        ga.rows = nbatch * M;
        ga.M = M;
        ga.rwk = la.rw;
        ga.Kw = kout * la.rw;
        ga.rkp = la.dims.back();
        ga.Nw = nout * lc.rw;
        ga.sBt_b = kall * ga.Nw;
        ga.chunks = (ga.Nw + 2047) / 2048;
        // bits of A (rows x latent entries) times the density threshold
        ga.max_total = (int64_t)std::floor((double)ga.rows * (double)kall * P->sparse_max_density / 1024.0);
        ga.fd_chunks = make_fastdiv((uint64_t)std::max<int64_t>(1, ga.chunks));
        ga.fd_M = make_fastdiv((uint64_t)std::max<int64_t>(1, M));
        if (mode == 2) {
            Op g;
            g.kind = OP_GATHER;
            g.a = a;
            g.b = bt;
            g.c = c;
            g.la = la;
            g.lb = P->buf_layout[bt];
            g.lc = lc;
            g.node = node;
            g.macs = macs;
            g.dense_macs = macs;
            g.gg = ga;
            g.gg.max_total = -1;      // no decision: the pass always runs
            P->ops.push_back(g);
            return;
        }
        // the count's partial sums: four per tile of kCountTileWords words of A
        ga.nparts = 4 * ((ga.rows * ga.Kw + kCountTileWords - 1) / kCountTileWords);
        Layout cl;            // the partial sums, then the decision word
        cl.rw = (ga.nparts + 2) / 2 * 2;
        cl.words = cl.rw;
        const int flag = new_buf(cl);
        Op k;
        k.kind = OP_COUNT;
        k.a = a;
        k.flag = flag;
        k.la = la;
        k.node = node;
        k.gg = ga;
        P->ops.push_back(k);
        Op g;
        g.kind = OP_GATHER;
        g.a = a;
        g.b = bt;
        g.c = c;
        g.flag = flag;
        g.la = la;
        g.lb = P->buf_layout[bt];
        g.lc = lc;
        g.node = node;
        g.dense_macs = macs;
        g.gg = ga;
        P->ops.push_back(g);
        emit_gemm(a, la, b, lb, c, lc, nb, nm, node);
        P->ops.back().flag = flag;

    }

    int plot_leaf(int r, const std::vector<int> &order) {
        const auto &decl = P->si.rel_list[r];
        PlotItem it;
        it.rel = r;
        for (int v : order) it.storage.push_back((int)(std::find(decl.begin(), decl.end(), v) - decl.begin()));
        it.layout = lay(order);
        it.buf = new_buf(it.layout);
        P->plots.push_back(it);
        return it.buf;
    }

    // Emits the ops producing node `id` under `cons` (following the searched
    // choices); out_buf = -1 allocates, kBufOutput writes the caller's array.
    int build(int id, const Constraint &cons, int out_buf, Layout *got) {
        const Choice ch = best(id, cons);
        const Node &nd = P->tree.nodes[id];
        const auto &si = P->si;
        if (nd.leaf >= 0) {
            const int r = nd.leaf;
            const uint64_t priv = si.rel_vars[r] & ~nd.q;
            const std::vector<int> &qo = ch.oc;
            if (!priv) {
                const int buf = plot_leaf(r, qo);
                if (out_buf == -1) {
                    *got = P->buf_layout[buf];
                    return buf;
                }
                Layout lc = lay(qo);
                emit_contract(buf, P->buf_layout[buf], -1, nullptr, out_buf, lc, id);
                *got = lc;
                return out_buf;
            }
            // project out the private latent variables (they occur in this
            // relation only): plot with one of them packed, then reduce
            const int kp = pick_packed(priv, si.res);
            std::vector<int> po;
            const int cp = qo.empty() ? -1 : qo.back();
            for (int v : qo)
                if (v != cp) po.push_back(v);
            for (int v : mask_list(priv))
                if (v != kp) po.push_back(v);
            if (cp >= 0) po.push_back(cp);
            po.push_back(kp);
            const int pb = plot_leaf(r, po);
            Layout lc = lay(qo);
            const int dst = (out_buf == -1) ? new_buf(lc) : out_buf;
            emit_contract(pb, P->buf_layout[pb], -1, nullptr, dst, lc, id);
            *got = lc;
            return dst;
        }
        Layout lx, ly;
        const int bx = build(nd.c0, ch.cx, -1, &lx);
        const int by = build(nd.c1, ch.cy, -1, &ly);
        Layout lc = lay(ch.oc);
        const int dst = (out_buf == -1) ? new_buf(lc) : out_buf;
        if (ch.kind == 0) {
            if (ch.roleB) emit_gemm_with_pass(bx, lx, by, ly, nd.c1, dst, lc, ch.nb, ch.nm, id);
            else emit_gemm_with_pass(by, ly, bx, lx, nd.c0, dst, lc, ch.nb, ch.nm, id);
        } else {
            emit_contract(bx, lx, by, &ly, dst, lc, id);
        }
        *got = lc;
        return dst;
    }
};

// Fill ContractArgs strides and pick the streaming mode from the layouts.
static void finish_contract(Op &op, bool has_b) {
    ContractArgs &a = op.ca;
    std::memset(&a, 0, sizeof(a));
    const Layout &la = op.la, &lb = op.lb, &lc = op.lc;
    a.nout = (int)lc.vars.size();
    a.c_row_words = lc.rw;
    a.n_out_rows = 1;
    for (int i = 0; i < a.nout; ++i) {
        a.out_dim[i] = lc.dims[i];
        if (i + 1 < a.nout) a.n_out_rows *= lc.dims[i];
    }
    a.a_pk_out = a.b_pk_out = a.a_pk_k = a.b_pk_k = -1;
    for (int i = 0; i < a.nout; ++i) {
        const int v = lc.vars[i];
        a.a_str[i] = la.stride(v);
        a.b_str[i] = has_b ? lb.stride(v) : 0;
        if (la.packed() == v) a.a_pk_out = i;
        if (has_b && lb.packed() == v) a.b_pk_out = i;
    }
    a.nk = (int)op.kvars.size();
    for (int j = 0; j < a.nk; ++j) {
        const int v = op.kvars[j];
        a.k_dim[j] = la.has(v) ? la.dims[std::find(la.vars.begin(), la.vars.end(), v) - la.vars.begin()]
                               : lb.dims[std::find(lb.vars.begin(), lb.vars.end(), v) - lb.vars.begin()];
        a.ka_str[j] = la.stride(v);
        a.kb_str[j] = has_b ? lb.stride(v) : 0;
        if (la.packed() == v) a.a_pk_k = j;
        if (has_b && lb.packed() == v) a.b_pk_k = j;
    }
    a.a_row_words = la.rw;
    a.b_row_words = has_b ? lb.rw : 0;
    // A 0-dim operand has no packed axis: its bit is bit 0 of word 0.
    const bool k_ok = a.a_pk_k >= 0 && (!has_b || a.b_pk_k == a.a_pk_k) && a.a_pk_out < 0 && (!has_b || a.b_pk_out < 0);
    // mode W: every operand holding the output's packed variable is packed
    // along it; an operand without it must be packed along an output variable
    // (it then contributes one bit per output row)
    bool w_ok = a.nout >= 1 && !la.vars.empty();
    if (w_ok) {
        const int last = a.nout - 1, cvar = lc.vars[last];
        if (la.has(cvar)) w_ok = a.a_pk_out == last;
        else w_ok = (a.a_bcast = a.a_pk_out >= 0);
        if (w_ok && has_b) {
            if (lb.has(cvar)) w_ok = a.b_pk_out == last;
            else w_ok = (a.b_bcast = a.b_pk_out >= 0);
        }
    }
    if (!w_ok) a.a_bcast = a.b_bcast = 0;
    if (k_ok) op.mode = kModeStreamK;
    else if (w_ok) op.mode = kModeStreamW;
    else op.mode = kModeBits;
    // latent-entry offset table for the streaming modes (mode K leaves out the
    // shared packed latent axis, which the kernel walks word by word)
    op.ktab.clear();
    if (op.mode != kModeBits) {
        int64_t n = 1;
        for (int j = 0; j < a.nk; ++j)
            if (!(op.mode == kModeStreamK && j == a.a_pk_k)) n *= a.k_dim[j];
        if (n > ((int64_t)1 << 22)) {
            op.mode = kModeBits;       // table too large: visit bit by bit
        } else {
            op.ktab.reserve(2 * n);
            std::vector<int64_t> idx(a.nk, 0);
            for (int64_t e = 0; e < n; ++e) {
                int64_t oa = 0, ob = 0;
                for (int j = 0; j < a.nk; ++j) {
                    oa += idx[j] * a.ka_str[j];
                    ob += idx[j] * a.kb_str[j];
                }
                op.ktab.push_back(oa);
                op.ktab.push_back(ob);
                for (int j = a.nk - 1; j >= 0; --j) {
                    if (op.mode == kModeStreamK && j == a.a_pk_k) continue;
                    if (++idx[j] < a.k_dim[j]) break;
                    idx[j] = 0;
                }
            }
        }
    }
    a.nktab = (int64_t)op.ktab.size() / 2;
    for (int i = 0; i < a.nout; ++i) a.fd_dim[i] = make_fastdiv((uint64_t)std::max<int64_t>(1, a.out_dim[i]));
    a.fd_rowbits = make_fastdiv((uint64_t)std::max<int64_t>(1, a.c_row_words * 32));
    a.fd_rowwords = make_fastdiv((uint64_t)std::max<int64_t>(1, a.c_row_words));
    // stream mode K: the row x bit shape of a wave's 64 outputs that touches
    // the fewest 128-byte lines with its first 16-byte loads of A and B; on a
    // tie, the fewest 256-byte segments (longer runs: the ternary system's
    // final step reads 8 runs of 256 bytes from each operand with 8 x 8 tiles
    // instead of 16 x 128 and 4 x 512 with 4 x 16, 13% faster measured)
    a.tq = 1;
    if (op.mode == kModeStreamK && a.nout >= 2) {
        auto lines = [&](int tq, int64_t bytes) {
            const int tp = 64 / tq;
            std::vector<int64_t> la, lb;
            for (int i = 0; i < tq; ++i)
                for (int j = 0; j < tp; ++j) {
                    la.push_back(4 * (i * a.a_str[a.nout - 2] + j * a.a_str[a.nout - 1]) / bytes);
                    if (has_b) lb.push_back(4 * (i * a.b_str[a.nout - 2] + j * a.b_str[a.nout - 1]) / bytes);
                }
            std::sort(la.begin(), la.end());
            std::sort(lb.begin(), lb.end());
            return (int64_t)(std::unique(la.begin(), la.end()) - la.begin()) +
                   (int64_t)(std::unique(lb.begin(), lb.end()) - lb.begin());
        };
        const int64_t rowbits = a.c_row_words * 32;
        std::pair<int64_t, int64_t> best{lines(1, 128), lines(1, 256)};
        for (int tq : {2, 4, 8}) {
            const int64_t blocks = (a.n_out_rows + tq - 1) / tq * rowbits / (64 / tq);
            if (blocks >= ((int64_t)1 << 31)) continue;
            const std::pair<int64_t, int64_t> l{lines(tq, 128), lines(tq, 256)};
            if (l < best) {
                best = l;
                a.tq = tq;
            }
        }
    }
    a.fd_segs = make_fastdiv((uint64_t)std::max<int64_t>(1, a.c_row_words * 32 / (64 / a.tq)));
}

static std::string join(const std::vector<int> &v) {
    std::ostringstream s;
    s << "[";
    for (size_t i = 0; i < v.size(); ++i) s << (i ? "," : "") << v[i];
    s << "]";
    return s.str();
}

std::string Op::describe() const {
    std::ostringstream s;
    s.precision(17);
    const char *names[] = {"bits", "stream_k", "stream_w"};
    if (kind == OP_FILL) {
        s << "{\"op\":\"fill\",\"buf\":" << c << ",\"words\":" << fill_words << "}";
        return s.str();
    }
    if (kind == OP_COUNT) {
        s << "{\"op\":\"sparse_count\",\"a\":" << a << ",\"flag\":" << flag << ",\"words\":" << gg.rows * gg.Kw << "}";
        return s.str();
    }
    if (kind == OP_LIST) {
        s << "{\"op\":\"row_list\",\"a\":" << a << ",\"c\":" << c << ",\"a_vars\":" << join(la.vars)
          << ",\"n_o\":" << rl.n_o << ",\"n_s\":" << rl.n_s << ",\"rows\":" << rl.n_rows << ",\"lbase\":" << rl.lbase
          << ",\"zrow\":" << rl.zrow << ",\"cap\":" << rl.cap << "}";
        return s.str();
    }
    if (kind == OP_FUSED) {
        s << "{\"op\":\"fused_pass_pair\",\"lists\":" << a << ",\"btx\":" << b << ",\"bty\":" << flag
          << ",\"c\":" << c << ",\"c_vars\":" << join(lc.vars) << ",\"n_p\":" << fu.n_p << ",\"n_q\":" << fu.n_q
          << ",\"n_s\":" << fu.n_s << ",\"rwt\":" << fu.rwt << ",\"kx\":" << fu.kX << ",\"ky\":" << fu.kY
          << ",\"tiles\":" << fu.n_tiles << ",\"macs\":" << macs << ",\"dense_macs\":" << dense_macs << "}";
        return s.str();
    }
    if (kind == OP_GATHER) {
        s << "{\"op\":\"sparse_pass\",\"a\":" << a << ",\"bt\":" << b << ",\"c\":" << c << ",\"flag\":" << flag
          << ",\"a_vars\":" << join(la.vars) << ",\"bt_vars\":" << join(lb.vars) << ",\"c_vars\":" << join(lc.vars)
          << ",\"rows\":" << gg.rows << ",\"Kw\":" << gg.Kw << ",\"Nw\":" << gg.Nw
          << ",\"max_total\":" << gg.max_total << ",\"dense_macs\":" << dense_macs << "}";
        return s.str();
    }
    s << "{\"op\":\"" << (kind == OP_GEMM ? "gemm_mfma" : names[mode]) << "\",\"a\":" << a << ",\"b\":" << b
      << ",\"c\":" << c << ",\"a_vars\":" << join(la.vars) << ",\"b_vars\":" << join(lb.vars)
      << ",\"c_vars\":" << join(lc.vars) << ",\"macs\":" << macs;
    if (kind == OP_GEMM)
        s << ",\"batch\":" << ga.nbatch << ",\"M\":" << ga.M << ",\"No\":" << ga.No << ",\"rn\":" << ga.rn
          << ",\"Kw\":" << ga.Kw << ",\"ksplit\":" << ga.ksplit << ",\"path\":" << ga.path << ",\"flag\":" << flag;
    else if (mode == kModeStreamK)
        s << ",\"tq\":" << ca.tq;
    s << "}";
    return s.str();
}

// --------------------------------------------------------------- planning
// Plot tiles: tw words along the packed axis; the rest of the 256 threads
// spread over ta cells of the fixed axis (n == 3) x tb strips of s walk cells.
// Operand path of the MFMA kernels for the pa_opts value: 1 stages 128 x 128
// tiles in LDS, 2 loads straight into registers, 3 stages 256 x 128 tiles,
// 4 keeps A operands of 256 x 128 tiles in registers (K of at most 256
// bits, else 3); 0 (the default) is -1 here: chosen per contraction by
// auto_gemm_path.
static int gemm_path_of(int opt) { return opt == 0 ? -1 : opt == 2 ? 1 : opt == 3 ? 2 : opt == 4 ? 3 : 0; }

// K split of an MFMA contraction: about `want` parts of whole 256-bit
// chunks.  (The fp32 sums cannot overflow: each K bit adds at most 4.)
static void set_ksplit(GemmArgs &g, int64_t want) {
    int64_t ksplit = std::max<int64_t>(1, std::min<int64_t>(want, (g.Kw + 7) / 8));
    int64_t chunk = (g.Kw + ksplit - 1) / ksplit;
    chunk = (chunk + 7) / 8 * 8;
    ksplit = (g.Kw + chunk - 1) / chunk;
    g.kchunk = chunk;
    g.ksplit = (int)std::max<int64_t>(1, ksplit);
    g.fd_ksplit = make_fastdiv((uint64_t)g.ksplit);
}

// Level-aware K split: the MFMA contractions that run in one grouped launch
// (one level of the tree) split their K range until the launch holds about
// gemm_split work items (tiles x parts; 512: 256 CUs twice); partial
// products are OR-ed into a zeroed output (exact in the Boolean semiring),
// so every split contraction gets a fill step before it.
static void split_gemms(pa_plan *P) {
    std::map<int, int> level_of_buf;
    for (const auto &pl : P->plots) level_of_buf[pl.buf] = 0;
    std::vector<int> level(P->ops.size(), 0);
    std::map<int, int64_t> tiles_at;
    for (size_t i = 0; i < P->ops.size(); ++i) {
        const Op &op = P->ops[i];
        int lv = 0;
        // the steps of a sparse pass and its MFMA contraction read the counter
        for (int b : {op.a, op.b, op.kind == OP_FILL ? -1 : op.flag}) {
            if (b < 0 && b != kBufOutput) continue;
            auto it = level_of_buf.find(b);
            if (it != level_of_buf.end()) lv = std::max(lv, it->second + 1);
        }
        level[i] = lv;
        if (op.c >= 0 || op.c == kBufOutput) level_of_buf[op.c] = lv;
        if ((op.kind == OP_COUNT || op.kind == OP_GATHER) && op.flag >= 0) level_of_buf[op.flag] = lv;
        if (op.kind == OP_GEMM) tiles_at[lv] += op.ga.nbatch * op.ga.tiles_m * op.ga.tiles_n;
    }
    std::vector<Op> ops;
    for (size_t i = 0; i < P->ops.size(); ++i) {
        Op op = P->ops[i];
        if (op.kind == OP_GEMM) {
            const int64_t tiles = tiles_at[level[i]], target = P->gemm_split;
            set_ksplit(op.ga, (!P->plain && tiles < target) ? (target + tiles - 1) / tiles : 1);
            if (op.ga.ksplit > 1) {
                Op f;
                f.kind = OP_FILL;
                f.c = op.c;
                f.fill_words = op.lc.words;
                f.node = op.node;
                // the sparse pass writing the same output (just before) runs
                // after the zeroing
                if (op.flag >= 0 && !ops.empty() && ops.back().kind == OP_GATHER && ops.back().c == op.c)
                    ops.insert(ops.end() - 1, f);
                else
                    ops.push_back(f);
            }
        }
        ops.push_back(op);
    }
    P->ops.swap(ops);
}

static void plot_tiling(PlotRel &R, int strip) {
    const int n = R.n;
    if (n == 2) {
        // 4 words (one per wave) x 64 strips (one per lane) of s <= 2 rows
        R.tw = 4;
        R.ta = 1;
        R.tb = 64;
        R.s = strip <= 1 ? 1 : 2;
        R.tiles_w = (R.row_words + 3) / 4;
        R.tiles_walk = (R.res[0] + 64 * R.s - 1) / (64 * R.s);
        R.tiles_fixed = 1;
        R.n_tiles = R.tiles_w * R.tiles_walk;
        return;
    }
    R.tw = (int)std::min<int64_t>(32, R.row_words);
    const int ts = 256 / R.tw;
    R.s = std::max(1, strip);
    R.walk_fixed = 0;
    if (n == 3 && R.rule == kRuleCorner) {
        // a thread per word and strip, walking up to kMaxWalkFixed cells of
        // the fixed axis: each corner line it evaluates serves the cells on
        // both sides of it
        R.walk_fixed = 1;
        R.tb = ts;
        R.ta = kMaxWalkFixed;
        R.s = std::min(R.s, kMaxWalkStrip);
        auto wl = [&]() { return ((int64_t)R.tb * R.s + 1) * (R.ta + 1); };
        while (wl() > kMaxWalkLines) {
            if (R.s > 1) --R.s;
            else if (R.ta > 1) --R.ta;
            else --R.tb;
        }
        R.tiles_w = (R.row_words + R.tw - 1) / R.tw;
        R.tiles_walk = (R.res[1] + (int64_t)R.tb * R.s - 1) / ((int64_t)R.tb * R.s);
        R.tiles_fixed = (R.res[0] + R.ta - 1) / R.ta;
        R.n_tiles = R.tiles_w * R.tiles_walk * R.tiles_fixed;
        return;
    }
    if (n == 1) {
        R.ta = 1;
        R.tb = 1;
        R.s = 1;
    } else if (n == 2) {
        R.ta = 1;
        R.tb = ts;
    } else {
        R.ta = ts >= 8 ? 4 : std::max(1, ts / 2);
        R.tb = std::max(1, ts / R.ta);
    }
    auto lines = [&]() { return (n >= 2 ? R.tb * R.s + 1 : 1) * (n == 3 ? R.ta + 1 : 1); };
    while (lines() > kMaxTileLines) {
        if (R.s > 1) --R.s;
        else --R.tb;
    }
    R.tiles_w = (R.row_words + R.tw - 1) / R.tw;
    const int64_t rwalk = n >= 2 ? R.res[n - 2] : 1;
    R.tiles_walk = n >= 2 ? (rwalk + (int64_t)R.tb * R.s - 1) / ((int64_t)R.tb * R.s) : 1;
    R.tiles_fixed = n == 3 ? (R.res[0] + R.ta - 1) / R.ta : 1;
    R.n_tiles = R.tiles_w * R.tiles_walk * R.tiles_fixed;
}

static int64_t contract_units_of(const ContractArgs &a, int mode) { return contract_units(a, mode); }

static int check_contract_bounds(const ContractArgs &a, int64_t a_words, int64_t b_words, int64_t c_words, bool has_b);
static int check_gemm_bounds(const GemmArgs &g, int64_t a_words, int64_t b_words, int64_t c_words);
static int check_gather_bounds(const GatherArgs &g, int64_t a_words, int64_t bt_words, int64_t c_words);
static int check_list_bounds(const Op &op, int64_t a_words, int64_t list_words);
static int check_fused_bounds(const Op &op, int64_t list_words, int64_t btx_words, int64_t bty_words,
                              int64_t c_words);

// Every step's index ranges against its buffers, on the host at plan time
// (the same checks run again when the steps get their device pointers).
static int validate_ops(const pa_plan *P) {
    auto words = [&](int id, const Layout &l) { return id == kBufOutput ? l.words : P->buf_words[id]; };
    for (const Op &op : P->ops) {
        int rc = PA_OK;
        switch (op.kind) {
            case OP_FILL: break;
            case OP_GEMM: rc = check_gemm_bounds(op.ga, op.la.words, op.lb.words, op.lc.words); break;
            case OP_COUNT: rc = check_gather_bounds(op.gg, op.la.words, -1, -1); break;
            case OP_GATHER: rc = check_gather_bounds(op.gg, op.la.words, op.lb.words, op.lc.words); break;
            case OP_LIST: rc = check_list_bounds(op, op.la.words, words(op.c, op.lc)); break;
            case OP_FUSED:
                rc = check_fused_bounds(op, words(op.a, op.la), words(op.b, op.lb), words(op.flag, op.lb),
                                        words(op.c, op.lc));
                break;
            default:
                rc = check_contract_bounds(op.ca, op.la.words, op.lb.words, op.lc.words, op.b >= 0);
                break;
        }
        if (rc) return rc;
    }
    return PA_OK;
}

// One of the two passes of a fusable pair: its output C[r0][r1][o_col][t]
// (rows: the output variable o_row and the latent entry variable s of the
// streamed step, in either order; no batch variables), A rows in C's row
// order, kall latent bits (at most 256).
struct PassSide {
    int op = -1, o_row = -1, o_col = -1, s = -1;
    int64_t ro = 0, rs = 0, kall = 0;
};

static bool pass_side(const Op &G, int op, int p, int q, int t, PassSide &sd) {
    const Layout &lc = G.lc;
    if (G.kind != OP_GATHER || G.flag >= 0 || lc.vars.size() != 4 || lc.vars[3] != t) return false;
    if (G.gg.rows != G.gg.M || G.gg.rows != lc.dims[0] * lc.dims[1] || G.gg.Nw != lc.dims[2] * lc.rw) return false;
    if (G.la.vars.size() < 3 || G.la.vars[0] != lc.vars[0] || G.la.vars[1] != lc.vars[1]) return false;
    sd.op = op;
    sd.o_col = lc.vars[2];
    if (lc.vars[0] == p || lc.vars[0] == q) {
        sd.o_row = lc.vars[0];
        sd.s = lc.vars[1];
        sd.ro = lc.dims[1];
        sd.rs = 1;
    } else if (lc.vars[1] == p || lc.vars[1] == q) {
        sd.o_row = lc.vars[1];
        sd.s = lc.vars[0];
        sd.ro = 1;
        sd.rs = lc.dims[1];
    } else {
        return false;
    }
    if (sd.s == p || sd.s == q || sd.s == t || sd.o_col == sd.o_row || (sd.o_col != p && sd.o_col != q)) return false;
    if (G.gg.rwk < 1 || G.gg.Kw % G.gg.rwk) return false;
    sd.kall = G.gg.Kw / G.gg.rwk * G.gg.rkp;
    return sd.kall >= 1 && sd.kall <= 256;
}

// Fuses each streamed contraction (mode K) whose two operands are written
// by sparse passes alone and read by nothing else, in the pattern
// out[p][q] = OR_{s, t} X[q][s][p][t] AND Y[p][s][q][t] (t packed, at most
// 256 bits): the two passes and the contraction become two row-list steps
// and one fused step, and the pass outputs are never stored.
static void fuse_pass_pairs(pa_plan *P) {
    auto writer = [&](int buf) {
        for (size_t i = 0; i < P->ops.size(); ++i)
            if (P->ops[i].c == buf) return (int)i;
        return -1;
    };
    auto readers = [&](int buf) {
        int n = 0;
        for (const Op &op : P->ops)
            for (int id : {op.a, op.b, op.flag})
                if (id == buf) ++n;
        return n;
    };
    for (size_t si = 0; si < P->ops.size();) {
        const Op S = P->ops[si++];
        if (S.kind != OP_CONTRACT || S.mode != kModeStreamK || S.a < 0 || S.b < 0 || S.a == S.b) continue;
        if (S.lc.vars.size() != 2 || S.la.vars.size() != 4 || S.lb.vars.size() != 4) continue;
        const int p = S.lc.vars[0], q = S.lc.vars[1], t = S.la.vars[3];
        if (S.lb.vars[3] != t || t == p || t == q || S.la.rw > 8) continue;
        const int ia = writer(S.a), ib = writer(S.b);
        if (ia < 0 || ib < 0 || readers(S.a) != 1 || readers(S.b) != 1) continue;
        PassSide A, B;
        if (!pass_side(P->ops[ia], ia, p, q, t, A) || !pass_side(P->ops[ib], ib, p, q, t, B)) continue;
        PassSide X, Y;
        if (A.o_row == q && B.o_row == p) {
            X = A;
            Y = B;
        } else if (A.o_row == p && B.o_row == q) {
            X = B;
            Y = A;
        } else {
            continue;
        }
        if (X.s != Y.s) continue;
        const Op &GX = P->ops[X.op], &GY = P->ops[Y.op];
        const int64_t n_p = S.lc.dims[0], n_q = S.lc.dims[1], n_s = P->si.res[X.s];
        const int64_t rwt = GX.lc.rw;
        if (GY.lc.rw != rwt || rwt > 8 || X.kall + Y.kall + 1 > kFusedRows) continue;
        // list buffer: per operand the heads, the meta words and the tails
        const int64_t gX = (n_q + 7) / 8 * n_s, gY = (n_p + 7) / 8 * n_s;
        // 16-bit list entries per row: the latent bits, at least 8 (the fused
        // step always loads entries 0..7), rounded up to a multiple of 8
        const int64_t capX = (std::max<int64_t>(8, X.kall) + 7) / 8 * 8, capY = (std::max<int64_t>(8, Y.kall) + 7) / 8 * 8;
        if (gX * 8 >= ((int64_t)1 << 31) || gY * 8 >= ((int64_t)1 << 31)) continue;
        int64_t off = 0;
        auto region = [&](int64_t words) {
            const int64_t at = off;
            off += (words + 63) / 64 * 64;
            return at;
        };
        int64_t sub[6] = {0, 0, 0, 0, 0, 0};
        sub[0] = region(gX * 8 * capX / 2);
        sub[1] = region(gX);
        sub[2] = region(gY * 8 * capY / 2);
        sub[3] = region(gY);
        Layout ll;
        ll.rw = off;
        ll.words = off;
        P->buf_layout.push_back(ll);
        P->buf_words.push_back(off);
        P->buf_off.push_back(-1);
        const int lbuf = (int)P->buf_layout.size() - 1;
        const int zrow = (int)(X.kall + Y.kall);
        auto list_op = [&](const Op &G, const PassSide &sd, int64_t n_o, int lbase, int64_t cap, int k0) {
            Op L;
            L.kind = OP_LIST;
            L.a = G.a;
            L.c = lbuf;
            L.la = G.la;
            L.lc = ll;
            L.node = S.node;
            L.rl.n_o = n_o;
            L.rl.n_s = n_s;
            L.rl.ro = sd.ro;
            L.rl.rs = sd.rs;
            L.rl.Kw = G.gg.Kw;
            L.rl.rwk = G.gg.rwk;
            L.rl.rkp = G.gg.rkp;
            L.rl.lbase = lbase;
            L.rl.zrow = zrow;
            L.rl.cap = cap;
            L.rl.n_rows = (n_o + 7) / 8 * 8 * n_s;
            L.rl.fd_s = make_fastdiv((uint64_t)n_s);
            L.sub[0] = sub[k0];
            L.sub[1] = sub[k0 + 1];
            return L;
        };
        const Op LX = list_op(GX, X, n_q, 0, capX, 0), LY = list_op(GY, Y, n_p, (int)X.kall, capY, 2);
        Op F;
        F.kind = OP_FUSED;
        F.a = lbuf;
        F.b = GX.b;
        F.flag = GY.b;
        F.c = S.c;
        F.la = ll;
        F.lb = GX.lb;
        F.lc = S.lc;
        F.node = S.node;
        F.macs = GX.macs + GY.macs + S.macs;
        F.dense_macs = GX.dense_macs + GY.dense_macs + S.macs;
        FusedArgs &f = F.fu;
        f.n_p = n_p;
        f.n_q = n_q;
        f.n_s = n_s;
        f.btX_rw = GX.gg.Nw;
        f.btY_rw = GY.gg.Nw;
        f.rwt = (int)rwt;
        f.kX = (int)X.kall;
        f.kY = (int)Y.kall;
        f.capX = capX;
        f.capY = capY;
        f.c_rw = S.lc.rw;
        f.n_qb = (n_q + 7) / 8;
        f.n_tiles = (n_p + 7) / 8 * f.n_qb;
        for (int k = 0; k < 4; ++k) F.sub[k] = sub[k];
        std::vector<Op> ops;
        for (size_t k = 0; k < P->ops.size(); ++k) {
            if ((int)k == X.op || (int)k == Y.op) continue;
            if (k + 1 == si) {
                ops.push_back(LX);
                ops.push_back(LY);
                ops.push_back(F);
            } else {
                ops.push_back(P->ops[k]);
            }
        }
        P->ops.swap(ops);
        si = 0;              // indices moved: look again from the start
    }
}

int build_plan(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts, pa_plan *P) {
    auto t0 = std::chrono::steady_clock::now();
    int rc = build_sysinfo(sys, exposed, n_exposed, P->si);
    if (rc) return rc;
    if ((int)P->leaf_log2d.size() == P->si.n_rel) P->si.leaf_log2d = P->leaf_log2d;
    for (int r = 0; r < sys->n_rel; ++r) {
        std::vector<pa_axis> ax;
        for (int i = 0; i < sys->rel[r].arity; ++i) ax.push_back(sys->axes[sys->rel[r].vars[i]]);
        rc = validate_relation(sys->rel[r], ax.data(), sys->n_vars, "system");
        if (rc) return rc;
    }
    pa_opts dflt{};
    const pa_opts &o = opts ? *opts : dflt;
    P->precision = o.precision;
    P->plot_rule = o.plot_rule;
    P->tolerance = o.tolerance;
    if (o.plot_rule != PA_RULE_CORNER && o.plot_rule != PA_RULE_CENTER)
        return fail(PA_EINVAL, "opts: unknown plot rule");
    if (o.plot_rule == PA_RULE_CENTER && !(std::isfinite(o.tolerance) && o.tolerance >= 0.0))
        return fail(PA_EINVAL, "opts: the centre rule needs a finite tolerance >= 0");
    P->audit = o.audit;
    P->timing = o.timing;
    P->plain = o.plain;
    P->per_op = o.per_op || o.plain;
    P->graph = o.graph && !P->per_op;
    // the single persistent launch runs corner plots only: centre-rule plans
    // use the grouped executor
    P->single_launch = o.single_launch && !P->per_op && o.plot_rule != PA_RULE_CENTER;
    P->persist_wg = o.persist_wg;
    P->plot_strip = o.plot_strip > 0 ? o.plot_strip : 4;
    P->contract_units = o.contract_units > 0 ? o.contract_units : 2048;
    P->gemm_split = o.gemm_split > 0 ? o.gemm_split : 512;
    P->gemm_path = gemm_path_of(o.gemm_path);
    // the single persistent launch runs 128 x 128 tiles only
    if (P->single_launch && P->gemm_path != 1) P->gemm_path = 0;
    // the sparse pass: not in the plain path nor in a single persistent launch
    P->sparse_pass = (P->plain || P->single_launch) ? -1 : o.sparse_pass;
    P->fuse_passes = P->sparse_pass == 3;
    P->sparse_max_density = o.sparse_max_density > 0 ? o.sparse_max_density : 64;
    if (o.sparse_pass < -1 || o.sparse_pass > 3 || o.sparse_max_density < 0 || o.sparse_max_density > 1024)
        return fail(PA_EINVAL, "opts: sparse_pass must be -1..3 and sparse_max_density 0..1024");
    if (o.precision != PA_PLOT_FP32_ESCALATE && o.precision != PA_PLOT_FP64)
        return fail(PA_EINVAL, "opts: unknown precision");
    if (o.persist_wg < 0 || o.plot_strip < 0 || o.contract_units < 0 || o.gemm_split < 0 || o.gemm_path < 0 ||
        o.gemm_path > 4)
        return fail(PA_EINVAL, "opts: negative tuning parameter");
    switch (o.order_policy) {
        case PA_ORDER_GREEDY: rc = plan_greedy(P->si, P->tree); break;
        case PA_ORDER_EXHAUSTIVE: rc = plan_exhaustive(P->si, P->tree); break;
        case PA_ORDER_GIVEN: {
            if (o.n_given < 0 || (o.n_given > 0 && !o.given)) return fail(PA_EINVAL, "opts: bad given order");
            std::vector<int> m(o.given, o.given + 2 * o.n_given);
            rc = tree_from_merges(P->si, m, P->tree);
            break;
        }
        case PA_ORDER_LEARNED: rc = plan_learned(P->si, o.model, P->tree); break;
        default: return fail(PA_EINVAL, "opts: unknown order policy");
    }
    if (rc) return rc;
    Builder B{P, sys};
    P->out_layout = make_layout(P->si.exposed_list, P->si.res);
    Layout got;
    if (B.build(P->tree.root, Constraint::full(P->si.exposed_list), kBufOutput, &got) != kBufOutput)
        return g_err.empty() ? fail(PA_EINVAL, "internal: root not written to output") : PA_EINVAL;
    for (auto &op : P->ops)
        if (op.kind == OP_CONTRACT) finish_contract(op, op.b >= 0 || op.b == kBufOutput);
    if (P->fuse_passes) fuse_pass_pairs(P);
    split_gemms(P);
    // a buffer that no step reads or writes (the first plot of B in a
    // contraction left to the sparse pass alone, the outputs of fused passes)
    // takes no space, and a plot that no step reads is dropped
    {
        std::vector<char> read(P->buf_layout.size(), 0);
        for (const auto &op : P->ops)
            for (int id : {op.a, op.b, op.c, op.flag})
                if (id >= 0) read[id] = 1;
        for (size_t id = 0; id < read.size(); ++id)
            if (!read[id]) P->buf_words[id] = 0;
        std::vector<PlotItem> kept;
        for (const auto &it : P->plots)
            if (it.buf < 0 || read[it.buf]) kept.push_back(it);
        P->plots.swap(kept);
    }
    rc = validate_ops(P);
    if (rc) return rc;
    P->total_macs = 0.0;
    for (const auto &op : P->ops)
        if (op.kind != OP_FILL) P->total_macs += op.macs;
    // workspace layout: tables | plot records | counters | persistent state | buffers
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    std::vector<unsigned char> &T = P->tables_host;
    T.clear();
    auto put = [&](const void *p, size_t n) {
        const size_t at = T.size();
        T.resize((at + n + 255) / 256 * 256);
        std::memcpy(T.data() + at, p, n);
        return at;
    };
    (void)put;   // plot records carry their coefficients and axes by value
    const size_t nsteps = P->plots.size() + P->ops.size();
    P->tables_off = take(T.size());
    P->plotrel_off = take(sizeof(PlotRel) * std::max<size_t>(1, P->plots.size()));
    P->plotrel1_off = take(sizeof(PlotRel) * std::max<size_t>(1, P->plots.size()));
    P->counters_off = take(sizeof(PlotCounters));
    P->popcnt_off = take(64);
    P->steps_off = take(sizeof(PStep) * std::max<size_t>(1, nsteps));
    P->pgroups_off = take(sizeof(PGroup) * std::max<size_t>(1, nsteps));
    P->levels_off = take(2 * sizeof(int64_t) * std::max<size_t>(1, nsteps));
    P->state_off = take(sizeof(PersistState));
    int64_t corners = 0;     // points evaluated: corners, or centres under the centre rule
    for (const auto &it : P->plots) {
        int64_t cn = 1;
        for (int64_t dm : it.layout.dims) cn *= dm + (P->plot_rule == PA_RULE_CENTER ? 0 : 1);
        corners += cn;
    }
    P->corners = corners;
    for (auto &op : P->ops) {
        if (!op.ktab.empty()) op.ktab_off = (int64_t)take(op.ktab.size() * sizeof(int64_t));
        if (op.kind == OP_FUSED) op.fargs_off = (int64_t)take(sizeof(PStep));
    }
    for (size_t i = 0; i < P->buf_layout.size(); ++i) P->buf_off[i] = (int64_t)take(P->buf_words[i] * 4);
    P->ws_bytes = off;
    P->tables_bytes = T.size();
    // plot records with workspace offsets in the pointer fields (patched on upload)
    P->plotrel_host.clear();
    for (size_t i = 0; i < P->plots.size(); ++i) {
        const auto &it = P->plots[i];
        const pa_relation &rel = sys->rel[it.rel];
        PlotRel R;
        std::memset(&R, 0, sizeof(R));
        R.n = rel.arity;
        R.d = rel.degree;
        R.mode = P->precision;
        R.audit = P->audit;
        R.rule = P->plot_rule == PA_RULE_CENTER ? kRuleCenter : kRuleCorner;
        R.target = rel.target;
        R.eps = P->tolerance;
        R.row_words = it.layout.rw;
        {
            std::vector<double> c = dense_coef(rel);
            std::copy(c.begin(), c.end(), R.coef);
        }
        double vmax = 0.0;
        for (int s = 0; s < R.n; ++s) {
            const int dv = it.storage[s];
            const int var = rel.vars[dv];
            R.perm[s] = dv;
            R.res[s] = sys->axes[var].res;
            R.lo[s] = sys->axes[var].lo;
            R.step[s] = axis_step(sys->axes[var].lo, sys->axes[var].hi, sys->axes[var].res);
            if (s == R.n - 1) vmax = std::max(std::fabs(sys->axes[var].lo), std::fabs(sys->axes[var].hi));
        }
        // |x_k| <= max(|lo|, |hi|) up to the two roundings of x_k
        R.vmax = vmax * (1.0 + 0x1p-50) + 0x1p-1000;
        {
            const double u = 0x1p-24, K = 2.0 * R.d + 1.0;
            const double gam = K * u / (1.0 - K * u);
            R.ebound = (gam + 0x1p-40) * (1.0 + 0x1p-30);
            const double Vm = std::max(1.0, R.vmax);
            double p = 1.0;
            for (int t = 0; t <= R.d + 1; ++t) {
                R.vpow[t] = p;
                p *= Vm;
            }
        }
        R.out = reinterpret_cast<uint32_t *>((size_t)P->buf_off[it.buf]);
        plot_tiling(R, P->plot_strip);
        if (R.n_tiles >= ((int64_t)1 << 31)) return fail(PA_EUNSUPPORTED, "relation too large to plot in one array");
        P->plotrel_host.push_back(R);
    }
    int64_t tb = 0;
    for (auto &R : P->plotrel_host) {
        R.tile_base = tb;
        tb += R.n_tiles;
    }
    P->total_tiles = tb;
    auto t1 = std::chrono::steady_clock::now();
    P->t_plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return PA_OK;
}

// Host proof that a launch stays inside its buffers: the largest word index
// any thread can form from the strides, compared with the buffer sizes.
static int check_contract_bounds(const ContractArgs &a, int64_t a_words, int64_t b_words, int64_t c_words, bool has_b) {
    int64_t ma = a.a_row_words - 1, mb = has_b ? a.b_row_words - 1 : 0;
    for (int i = 0; i < a.nout; ++i) {
        ma += (a.out_dim[i] - 1) * a.a_str[i];
        mb += (a.out_dim[i] - 1) * a.b_str[i];
    }
    for (int j = 0; j < a.nk; ++j) {
        ma += (a.k_dim[j] - 1) * a.ka_str[j];
        mb += (a.k_dim[j] - 1) * a.kb_str[j];
    }
    const int64_t mc = (a.nout == 0) ? 0 : a.n_out_rows * a.c_row_words - 1;
    if (ma >= a_words || (has_b && mb >= b_words) || mc >= c_words || ma < 0 || mb < 0)
        return fail(PA_EINVAL, "internal: contraction would index outside its buffers");
    // the kernels divide output rows and row offsets in 32 bits
    const int64_t lim = (int64_t)1 << 31;
    if (a.n_out_rows >= lim || a.c_row_words * 32 + 1024 >= lim)
        return fail(PA_EUNSUPPORTED, "contraction output has too many rows for one array");
    for (int i = 0; i < a.nout; ++i)
        if (a.out_dim[i] >= lim) return fail(PA_EUNSUPPORTED, "contraction output dimension too large");
    return PA_OK;
}

static int check_gemm_bounds(const GemmArgs &g, int64_t a_words, int64_t b_words, int64_t c_words) {
    const int64_t ma = g.nbatch * g.sA_b, mb = g.nbatch * g.sB_b, mc = g.nbatch * g.sC_b;
    if (g.sA_b != g.M * g.Kw || g.sB_b != g.No * g.rn * g.Kw || g.sC_b != g.M * g.No * g.rwc || g.Kw % 2 ||
        g.rwc != row_words_of(g.rn) || ma > a_words || mb > b_words || mc > c_words || g.kchunk % 8 ||
        (int64_t)g.ksplit * g.kchunk < g.Kw)
        return fail(PA_EINVAL, "internal: GEMM would index outside its buffers");
    // the kernels decode tile indices and N coordinates in 32 bits
    const int64_t lim = (int64_t)1 << 31;
    if (g.nbatch * g.tiles_m * g.tiles_n * g.ksplit >= lim || g.tiles_n * 128 + 128 >= lim || g.M + 256 >= lim ||
        g.Kw >= lim)
        return fail(PA_EUNSUPPORTED, "GEMM too large for one launch");
    return PA_OK;
}

// Buffer sizes of a count step (bt_words, c_words < 0) or a sparse pass.
static int check_gather_bounds(const GatherArgs &g, int64_t a_words, int64_t bt_words, int64_t c_words) {
    const bool pass = bt_words >= 0;
    if (g.rows < 1 || g.M < 1 || g.rwk < 2 || g.Kw % g.rwk || g.rkp < 1 || g.rkp > 32 * g.rwk || g.Nw < 2 ||
        g.Nw % 2 || g.rows * g.Kw > a_words || (pass && g.rows * g.Nw > c_words) ||
        (pass && (g.rows / g.M) * g.sBt_b > bt_words) || g.sBt_b != (g.Kw / g.rwk) * g.rkp * g.Nw)
        return fail(PA_EINVAL, "internal: sparse pass would index outside its buffers");
    // wave-tile indices, rows, A word indices and Bt row indices are 32-bit
    if (g.rows * g.chunks >= ((int64_t)1 << 31) || g.Kw >= ((int64_t)1 << 31) ||
        (g.Kw / g.rwk) * g.rkp >= ((int64_t)1 << 31))
        return fail(PA_EUNSUPPORTED, "sparse pass too large for one launch");
    return PA_OK;
}

// Buffer sizes of a row-list step (its A and list buffer) and of a fused
// step (BtX, BtY, the list buffer, the output).
static int check_list_bounds(const Op &op, int64_t a_words, int64_t list_words) {
    const RowListArgs &l = op.rl;
    const int64_t groups = (l.n_o + 7) / 8 * l.n_s;
    if (l.n_o < 1 || l.n_s < 1 || l.Kw < 1 || l.rwk < 1 || l.Kw % l.rwk || l.rkp < 1 || l.rkp > 32 * l.rwk ||
        l.n_rows != groups * 8 || ((l.n_o - 1) * l.ro + (l.n_s - 1) * l.rs + 1) * l.Kw > a_words ||
        l.lbase < 0 || l.lbase + l.Kw / l.rwk * l.rkp > l.zrow || l.zrow >= kFusedRows || l.cap % 8 ||
        l.cap < l.Kw / l.rwk * l.rkp || op.sub[0] + l.n_rows * l.cap / 2 > list_words ||
        op.sub[1] + groups > list_words)
        return fail(PA_EINVAL, "internal: row-list step would index outside its buffers");
    // list rows are 32-bit
    if (l.n_rows >= ((int64_t)1 << 31))
        return fail(PA_EUNSUPPORTED, "row-list step too large for one launch");
    return PA_OK;
}

static int check_fused_bounds(const Op &op, int64_t list_words, int64_t btx_words, int64_t bty_words,
                              int64_t c_words) {
    const FusedArgs &f = op.fu;
    const int64_t gX = (f.n_q + 7) / 8 * f.n_s, gY = (f.n_p + 7) / 8 * f.n_s;
    if (f.n_p < 1 || f.n_q < 1 || f.n_s < 1 || f.rwt < 1 || f.rwt > 8 || f.kX < 1 || f.kY < 1 ||
        f.kX + f.kY + 1 > kFusedRows || f.btX_rw < f.n_p * f.rwt || f.btY_rw < f.n_q * f.rwt ||
        (int64_t)f.kX * f.btX_rw > btx_words || (int64_t)f.kY * f.btY_rw > bty_words ||
        f.n_qb != (f.n_q + 7) / 8 || 4 * f.c_rw < f.n_qb || f.n_p * f.c_rw > c_words ||
        f.n_tiles != (f.n_p + 7) / 8 * f.n_qb || f.capX % 8 || f.capY % 8 || f.capX < f.kX || f.capY < f.kY ||
        op.sub[0] + gX * 8 * f.capX / 2 > list_words || op.sub[1] + gX > list_words ||
        op.sub[2] + gY * 8 * f.capY / 2 > list_words || op.sub[3] + gY > list_words)
        return fail(PA_EINVAL, "internal: fused step would index outside its buffers");
    return PA_OK;
}

// Partial sums in the count buffer `buf` of a sparse pass (the decision word
// follows them).
static int64_t sparse_nparts_of(const pa_plan *P, int buf) {
    for (const Op &op : P->ops)
        if (op.kind == OP_COUNT && op.flag == buf) return op.gg.nparts;
    return 0;
}

static uint32_t *buf_ptr(pa_plan *P, int id, void *out) {
    if (id == kBufOutput) return static_cast<uint32_t *>(out);
    if (id < 0) return nullptr;
    return reinterpret_cast<uint32_t *>(static_cast<char *>(P->ws.ptr) + P->buf_off[id]);
}

static int64_t buf_words_of(const pa_plan *P, int id, const Layout &l) {
    return id == kBufOutput ? l.words : P->buf_words[id];
}

// Arguments of a row-list or fused step with its buffer pointers (bounds
// checked); out is the caller's output.
static int list_args(pa_plan *P, const Op &op, void *out, RowListArgs &l) {
    int rc = check_list_bounds(op, op.la.words, P->buf_words[op.c]);
    if (rc) return rc;
    l = op.rl;
    l.A = buf_ptr(P, op.a, out);
    uint32_t *lb = buf_ptr(P, op.c, out);
    l.ent = reinterpret_cast<uint16_t *>(lb + op.sub[0]);
    l.meta = lb + op.sub[1];
    return PA_OK;
}

static int fused_args(pa_plan *P, const Op &op, void *out, FusedArgs &f) {
    int rc = check_fused_bounds(op, P->buf_words[op.a], P->buf_words[op.b], P->buf_words[op.flag],
                                buf_words_of(P, op.c, op.lc));
    if (rc) return rc;
    f = op.fu;
    f.BtX = buf_ptr(P, op.b, out);
    f.BtY = buf_ptr(P, op.flag, out);
    const uint32_t *lb = buf_ptr(P, op.a, out);
    f.entX = reinterpret_cast<const uint16_t *>(lb + op.sub[0]);
    f.metaX = lb + op.sub[1];
    f.entY = reinterpret_cast<const uint16_t *>(lb + op.sub[2]);
    f.metaY = lb + op.sub[3];
    f.C = buf_ptr(P, op.c, out);
    return PA_OK;
}

// Persistent step list: plots, then ops, sorted by level (a step's level is
// one more than its producers'), each with its producer steps as dependencies.
static int build_steps(pa_plan *P) {
    char *base = static_cast<char *>(P->ws.ptr);
    std::vector<PStep> st;
    std::vector<int> level;
    std::map<int, int> producer;     // buffer id -> step
    for (size_t i = 0; i < P->plots.size(); ++i) {
        PStep s;
        std::memset(&s, 0, sizeof(s));
        s.kind = kStepPlot;
        // one kernel per kind of plot tile: corner, centre rule, or the
        // fixed-axis-walking trivariate corner tiles
        s.mode = P->plotrel1_dev[i].rule == kRuleCenter ? 1 : (P->plotrel1_dev[i].walk_fixed ? 2 : 0);
        s.plot = P->plotrel1_dev[i];
        s.n_tiles = s.plot.n_tiles;
        producer[P->plots[i].buf] = (int)st.size();
        st.push_back(s);
        level.push_back(0);
    }
    std::vector<int> out_refs;
    std::map<int, std::vector<int>> list_steps;     // list buffer -> its row-list steps
    int fill_for_next = -1;
    for (size_t oi = 0; oi < P->ops.size(); ++oi) {
        const Op &op = P->ops[oi];
        PStep s;
        std::memset(&s, 0, sizeof(s));
        int lv = 0;
        auto dep = [&](int buf) {
            if (buf < 0 && buf != kBufOutput) return;
            auto it = producer.find(buf);
            if (it == producer.end()) return;
            s.dep[s.ndep++] = it->second;
            lv = std::max(lv, level[it->second] + 1);
        };
        if (op.kind == OP_FILL) {
            s.kind = kStepFill;
            s.fill_ptr = buf_ptr(P, op.c, nullptr);
            s.units = op.fill_words;
            s.per_tile = 4096;
            s.n_tiles = (s.units + s.per_tile - 1) / s.per_tile;
            fill_for_next = (int)st.size();
            if (op.c == kBufOutput) out_refs.push_back((int)st.size());
        } else if (op.kind == OP_COUNT || op.kind == OP_GATHER) {
            const bool pass = op.kind == OP_GATHER;
            int rc = check_gather_bounds(op.gg, op.la.words, pass ? op.lb.words : -1, pass ? op.lc.words : -1);
            if (rc) return rc;
            s.kind = pass ? kStepGather : kStepCount;
            s.gather = op.gg;
            s.gather.A = buf_ptr(P, op.a, nullptr);
            s.gather.Bt = pass ? buf_ptr(P, op.b, nullptr) : nullptr;
            s.gather.C = pass ? buf_ptr(P, op.c, nullptr) : nullptr;
            s.gather.parts = op.flag >= 0 ? buf_ptr(P, op.flag, nullptr) : nullptr;
            s.gather.dense = op.flag >= 0 ? s.gather.parts + op.gg.nparts : nullptr;
            s.n_tiles = pass ? (gather_wave_tiles(op.gg) + 3) / 4
                             : (op.gg.rows * op.gg.Kw + kCountTileWords - 1) / kCountTileWords;
            dep(op.a);
            if (pass) {
                dep(op.flag);       // the count
                dep(op.b);
                dep(op.c);          // the zeroing of a split contraction's output
                if (op.c == kBufOutput) out_refs.push_back((int)st.size());
            }
            if (op.flag >= 0) producer[op.flag] = (int)st.size();
        } else if (op.kind == OP_LIST) {
            int rc = list_args(P, op, nullptr, s.list);
            if (rc) return rc;
            s.kind = kStepList;
            s.n_tiles = (op.rl.n_rows + kListRowsPerTile - 1) / kListRowsPerTile;
            dep(op.a);
            list_steps[op.c].push_back((int)st.size());
        } else if (op.kind == OP_FUSED) {
            int rc = fused_args(P, op, nullptr, s.fused);
            if (rc) return rc;
            s.kind = kStepFused;
            s.n_tiles = op.fu.n_tiles;
            for (int ls : list_steps[op.a]) {
                s.dep[s.ndep++] = ls;
                lv = std::max(lv, level[ls] + 1);
            }
            dep(op.b);
            dep(op.flag);
            if (op.c == kBufOutput) out_refs.push_back((int)st.size());
        } else if (op.kind == OP_GEMM) {
            int rc = check_gemm_bounds(op.ga, op.la.words, op.lb.words, op.lc.words);
            if (rc) return rc;
            s.kind = kStepGemm;
            s.mode = op.ga.path;        // grouped launches: one instantiation per operand path
            s.gemm = op.ga;
            s.gemm.A = buf_ptr(P, op.a, nullptr);
            s.gemm.B = buf_ptr(P, op.b, nullptr);
            s.gemm.C = buf_ptr(P, op.c, nullptr);
            s.gemm.dense = op.flag >= 0 ? buf_ptr(P, op.flag, nullptr) + sparse_nparts_of(P, op.flag) : nullptr;
            s.n_tiles = op.ga.nbatch * op.ga.tiles_m * op.ga.tiles_n * op.ga.ksplit;
            dep(op.a);
            dep(op.b);
            if (op.flag >= 0) dep(op.flag);
            if (op.ga.ksplit > 1 && fill_for_next >= 0) {
                s.dep[s.ndep++] = fill_for_next;
                lv = std::max(lv, level[fill_for_next] + 1);
            }
            fill_for_next = -1;
            if (op.c == kBufOutput) out_refs.push_back((int)st.size());
        } else {
            int rc = check_contract_bounds(op.ca, op.la.words, op.lb.words, op.lc.words, op.b >= 0);
            if (rc) return rc;
            s.kind = kStepContract;
            s.mode = op.mode;
            s.ca = op.ca;
            s.ca.ktab = op.ktab_off >= 0 ? reinterpret_cast<const int64_t *>(base + op.ktab_off) : nullptr;
            s.ca.A = buf_ptr(P, op.a, nullptr);
            s.ca.B = buf_ptr(P, op.b, nullptr);
            s.ca.C = buf_ptr(P, op.c, nullptr);
            s.units = contract_units_of(op.ca, op.mode);
            {
                // units per tile: contract_units, fewer when each unit reads
                // many words (a tile then holds about contract_units * 64 reads)
                const int64_t cap = (op.mode == kModeStreamW) ? std::max<int64_t>(256, P->contract_units / 32)
                                                              : std::max<int64_t>(256, P->contract_units);
                int64_t work = 1;
                if (op.mode == kModeStreamK) work = std::max<int64_t>(1, op.ca.nktab * op.ca.a_row_words);
                else if (op.mode == kModeStreamW) work = std::max<int64_t>(1, op.ca.nktab);
                const int64_t want = std::max<int64_t>(1, (int64_t)P->contract_units * 64 / work);
                s.per_tile = std::max<int64_t>(256, std::min<int64_t>(cap, want) / 256 * 256);
            }
            s.n_tiles = (s.units + s.per_tile - 1) / s.per_tile;
            dep(op.a);
            dep(op.b);
            if (op.c == kBufOutput) out_refs.push_back((int)st.size());
        }
        if (op.c >= 0 || op.c == kBufOutput) producer[op.c] = (int)st.size();   // fills too: a sparse pass waits for its zeroing
        st.push_back(s);
        level.push_back(lv);
    }
    // stable sort by (level, kind, mode), remap dependencies
    std::vector<int> order(st.size());
    for (size_t i = 0; i < st.size(); ++i) order[i] = (int)i;
    auto key = [&](int i) { return std::make_tuple(level[i], st[i].kind, st[i].mode); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<int> pos(st.size());
    for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;
    P->steps_host.clear();
    P->step_macs.clear();
    int64_t tbase = 0;
    for (int oi : order) {
        P->step_macs.push_back(oi >= (int)P->plots.size() ? (P->ops[oi - P->plots.size()].kind == OP_FILL
                                                                 ? 0.0
                                                                 : P->ops[oi - P->plots.size()].macs)
                                                           : 0.0);
        PStep s = st[oi];
        for (int j = 0; j < s.ndep; ++j) s.dep[j] = pos[s.dep[j]];
        s.tile_base = tbase;
        tbase += s.n_tiles;
        P->steps_host.push_back(s);
    }
    P->step_out_refs.clear();
    for (int r : out_refs) P->step_out_refs.push_back({pos[r], 0});
    P->step_level.clear();
    for (int oi : order) P->step_level.push_back(level[oi]);
    P->n_items = tbase;
    make_groups(P);
    return PA_OK;
}

// Groups: maximal runs of steps with the same (level, kind, mode), in the
// sorted step table; fills (which depend on nothing) join the plotting group
// of their level, so zeroing split-K outputs costs no launch of its own.
void make_groups(pa_plan *P) {
    P->groups.clear();
    for (size_t i = 0; i < P->steps_host.size(); ++i) {
        const PStep &x = P->steps_host[i];
        const bool same_level = i > 0 && P->step_level[i] == P->step_level[i - 1];
        const bool same = same_level && ((x.kind == P->steps_host[i - 1].kind && x.mode == P->steps_host[i - 1].mode) ||
                                         (x.kind == kStepFill && P->groups.back().kind == kStepPlot));
        const int flags = x.kind == kStepGemm && x.gemm.dense != nullptr;
        if (same) {
            P->groups.back().count += 1;
            P->groups.back().t1 = x.tile_base + x.n_tiles;
            P->groups.back().flags |= flags;
        } else {
            P->groups.push_back({x.kind, x.mode, (int)i, 1, x.tile_base, x.tile_base + x.n_tiles, flags});
        }
    }
}

int persist_default_workgroups();

int upload_pgroups(pa_plan *P) {
    const int64_t wg = std::max<int64_t>(1, P->persist_wg > 0 ? P->persist_wg : persist_default_workgroups());
    std::vector<PGroup> pg;
    std::vector<int64_t> lv;          // items per level, then (zeroed) done counters
    int64_t cbase = 0;
    int nlev = 0;
    for (const auto &g : P->groups) {
        PGroup x;
        std::memset(&x, 0, sizeof(x));
        x.kind = g.kind;
        x.mode = g.mode;
        x.first = g.first;
        x.count = g.count;
        x.level = P->step_level[g.first];
        x.t0 = g.t0;
        x.t1 = g.t1;
        const int64_t n = g.t1 - g.t0;
        x.chunk = std::max<int64_t>(1, (n + wg - 1) / wg);
        x.cbase = cbase;
        cbase += (n + x.chunk - 1) / x.chunk;
        nlev = std::max(nlev, x.level + 1);
        if ((int)lv.size() < nlev) lv.resize(nlev, 0);
        lv[x.level] += n;
        pg.push_back(x);
    }
    P->n_pgroups = (int)pg.size();
    P->n_levels = nlev;
    P->n_chunks = cbase;
    lv.resize(2 * std::max(1, nlev), 0);
    char *base = static_cast<char *>(P->ws.ptr);
    if (!pg.empty()) HIP_TRY(hipMemcpy(base + P->pgroups_off, pg.data(), pg.size() * sizeof(PGroup), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + P->levels_off, lv.data(), lv.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    return PA_OK;
}

static void patch_outputs(pa_plan *P, const std::vector<void *> &outs) {
    for (const auto &ref : P->step_out_refs) {
        PStep &s = P->steps_host[ref.first];
        uint32_t *o = static_cast<uint32_t *>(outs[ref.second]);
        if (s.kind == kStepGemm) s.gemm.C = o;
        else if (s.kind == kStepContract) s.ca.C = o;
        else if (s.kind == kStepGather) s.gather.C = o;
        else if (s.kind == kStepFused) s.fused.C = o;
        else if (s.kind == kStepFill) s.fill_ptr = o;
    }
}

int upload_plan(pa_plan *P) {
    char *base = static_cast<char *>(P->ws.ptr);
    std::vector<PlotRel> rels = P->plotrel_host;
    auto fix = [&](const void *off) { return (void *)(base + P->tables_off + (size_t)off); };
    (void)fix;
    PlotCounters *cdev = P->counters_dev ? P->counters_dev : reinterpret_cast<PlotCounters *>(base + P->counters_off);
    for (auto &R : rels) {
        R.out = (uint32_t *)(base + (size_t)R.out);
        R.counters = cdev;
    }
    if (!P->tables_host.empty())
        HIP_TRY(hipMemcpy(base + P->tables_off, P->tables_host.data(), P->tables_host.size(), hipMemcpyHostToDevice));
    P->plotrel1_dev = rels;
    for (auto &R : P->plotrel1_dev) R.tile_base = 0;
    if (!rels.empty()) {
        HIP_TRY(hipMemcpy(base + P->plotrel_off, rels.data(), rels.size() * sizeof(PlotRel), hipMemcpyHostToDevice));
        // copies with zero tile bases, for one-relation-per-launch plotting
        HIP_TRY(hipMemcpy(base + P->plotrel1_off, P->plotrel1_dev.data(), rels.size() * sizeof(PlotRel),
                          hipMemcpyHostToDevice));
    }
    for (const auto &op : P->ops)
        if (op.ktab_off >= 0)
            HIP_TRY(hipMemcpy(base + op.ktab_off, op.ktab.data(), op.ktab.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice));
    for (const auto &op : P->ops)
        if (op.kind == OP_FUSED) {
            // the per-op launch's one-step table (its output pointer is passed apart)
            PStep st;
            std::memset(&st, 0, sizeof(st));
            st.kind = kStepFused;
            st.n_tiles = op.fu.n_tiles;
            int rc = fused_args(P, op, nullptr, st.fused);
            if (rc) return rc;
            HIP_TRY(hipMemcpy(base + op.fargs_off, &st, sizeof(st), hipMemcpyHostToDevice));
        }
    int rc = build_steps(P);
    if (rc) return rc;
    // counters and executor state start at zero (plot counters only grow)
    HIP_TRY(hipMemset(base + P->counters_off, 0, sizeof(PlotCounters)));
    HIP_TRY(hipMemset(base + P->state_off, 0, sizeof(PersistState)));
    HIP_TRY(hipMemcpy(base + P->state_off + offsetof(PersistState, wait_limit), &kDefaultWaitLimit,
                      sizeof(kDefaultWaitLimit), hipMemcpyHostToDevice));
    rc = upload_pgroups(P);
    if (rc) return rc;
    P->uploaded = true;
    return PA_OK;
}

static int upload_steps(pa_plan *P, const std::vector<void *> &outs) {
    patch_outputs(P, outs);
    if (!P->steps_host.empty())
        HIP_TRY(hipMemcpy(static_cast<char *>(P->ws.ptr) + P->steps_off, P->steps_host.data(),
                          P->steps_host.size() * sizeof(PStep), hipMemcpyHostToDevice));
    P->last_outs = outs;
    return PA_OK;
}

static int run_ops(pa_plan *P, void *out, hipStream_t s, int *launches) {
    const bool per_op = P->op_events.size() == 2 + 2 * P->ops.size();
    for (size_t oi = 0; oi < P->ops.size(); ++oi) {
        const Op &op0 = P->ops[oi];
        if (per_op) HIP_TRY(hipEventRecord(P->op_events[2 + 2 * oi], s));
        if (op0.kind == OP_FILL) {
            HIP_TRY(launch_fill(buf_ptr(P, op0.c, out), op0.fill_words, 0u, s));
            ++*launches;
        } else if (op0.kind == OP_GEMM) {
            GemmArgs g = op0.ga;
            int rc = check_gemm_bounds(g, op0.la.words, op0.lb.words, op0.lc.words);
            if (rc) return rc;
            g.A = buf_ptr(P, op0.a, out);
            g.B = buf_ptr(P, op0.b, out);
            g.C = buf_ptr(P, op0.c, out);
            g.dense = op0.flag >= 0 ? buf_ptr(P, op0.flag, out) + sparse_nparts_of(P, op0.flag) : nullptr;
            HIP_TRY(launch_gemm(g, s));
            ++*launches;
        } else if (op0.kind == OP_LIST) {
            RowListArgs l;
            int rc = list_args(P, op0, out, l);
            if (rc) return rc;
            HIP_TRY(launch_row_list(l, s));
            ++*launches;
        } else if (op0.kind == OP_FUSED) {
            FusedArgs f;
            int rc = fused_args(P, op0, out, f);
            if (rc) return rc;
            HIP_TRY(launch_fused(reinterpret_cast<const PStep *>(static_cast<char *>(P->ws.ptr) + op0.fargs_off),
                                 op0.fu.n_tiles, f.C, s));
            ++*launches;
        } else if (op0.kind == OP_COUNT || op0.kind == OP_GATHER) {
            const bool pass = op0.kind == OP_GATHER;
            GatherArgs g = op0.gg;
            int rc = check_gather_bounds(g, op0.la.words, pass ? op0.lb.words : -1, pass ? op0.lc.words : -1);
            if (rc) return rc;
            g.A = buf_ptr(P, op0.a, out);
            g.Bt = pass ? buf_ptr(P, op0.b, out) : nullptr;
            g.C = pass ? buf_ptr(P, op0.c, out) : nullptr;
            g.parts = op0.flag >= 0 ? buf_ptr(P, op0.flag, out) : nullptr;
            g.dense = op0.flag >= 0 ? g.parts + g.nparts : nullptr;
            HIP_TRY(pass ? launch_gather(g, s) : launch_count(g, s));
            ++*launches;
        } else {
            ContractArgs a = op0.ca;
            int rc = check_contract_bounds(a, op0.la.words, op0.lb.words, op0.lc.words, op0.b >= 0);
            if (rc) return rc;
            a.ktab = op0.ktab_off >= 0 ? reinterpret_cast<const int64_t *>(static_cast<char *>(P->ws.ptr) + op0.ktab_off)
                                       : nullptr;
            a.A = buf_ptr(P, op0.a, out);
            a.B = buf_ptr(P, op0.b, out);
            a.C = buf_ptr(P, op0.c, out);
            HIP_TRY(launch_contract(a, op0.mode, s));
            ++*launches;
        }
        if (per_op) HIP_TRY(hipEventRecord(P->op_events[3 + 2 * oi], s));
    }
    return PA_OK;
}

static int run_plots(pa_plan *P, hipStream_t s, int *launches) {
    char *base = static_cast<char *>(P->ws.ptr);
    const PlotRel *d_rels = reinterpret_cast<const PlotRel *>(base + P->plotrel_off);
    PlotCounters *cnt = reinterpret_cast<PlotCounters *>(base + P->counters_off);
    const int nrel = (int)P->plotrel_host.size();
    if (nrel == 0) return PA_OK;
    if (!P->plain) {
        HIP_TRY(launch_plot(d_rels, nrel, P->total_tiles, P->plot_rule == PA_RULE_CENTER, cnt, s));
        ++*launches;
    } else {
        const PlotRel *d_one = reinterpret_cast<const PlotRel *>(base + P->plotrel1_off);
        for (int i = 0; i < nrel; ++i) {
            HIP_TRY(launch_plot(d_one + i, 1, P->plotrel_host[i].n_tiles, P->plot_rule == PA_RULE_CENTER, cnt, s));
            ++*launches;
        }
    }
    return PA_OK;
}

static int run_persist(pa_plan *P, hipStream_t s, int *launches, hipEvent_t before = nullptr) {
    char *base = static_cast<char *>(P->ws.ptr);
    PersistState *state = reinterpret_cast<PersistState *>(base + P->state_off);
    const int64_t *level_items = reinterpret_cast<const int64_t *>(base + P->levels_off);
    unsigned long long *level_done =
        reinterpret_cast<unsigned long long *>(base + P->levels_off) + std::max(1, P->n_levels);
    PlotCounters *cnt = reinterpret_cast<PlotCounters *>(base + P->counters_off);
    int64_t wg = P->persist_wg > 0 ? P->persist_wg : persist_default_workgroups();
    wg = std::max<int64_t>(1, std::min<int64_t>(wg, P->n_chunks));
    // the plot counters only ever grow (a report takes the difference of
    // two reads), so the grouped executor needs no reset launch
    if (P->single_launch) HIP_TRY(launch_persist_reset(state, level_done, P->n_levels, s));
    if (before) HIP_TRY(hipEventRecord(before, s));
    const PStep *d_steps = reinterpret_cast<const PStep *>(base + P->steps_off);
    if (P->single_launch) {
        for (const PStep &st : P->steps_host)
            if ((st.kind == kStepGemm && (st.gemm.path >= 2 || st.gemm.dense)) || st.kind == kStepGather ||
                st.kind == kStepCount || st.kind == kStepList || st.kind == kStepFused ||
                (st.kind == kStepPlot && st.plot.rule != kRuleCorner))
                return fail(PA_EINVAL,
                            "internal: 256-row MFMA tiles, a sparse pass or a centre plot in a single persistent launch");
        HIP_TRY(launch_persist(d_steps, reinterpret_cast<const PGroup *>(base + P->pgroups_off), P->n_pgroups,
                               P->n_chunks, level_items, level_done, state, cnt, (int)wg, s));
        *launches += 2;
    } else {
        const bool ev = P->op_events.size() == 2 * P->groups.size() && before;
        for (size_t gi = 0; gi < P->groups.size(); ++gi) {
            const auto &g = P->groups[gi];
            if (ev && gi > 0) HIP_TRY(hipEventRecord(P->op_events[2 * gi], s));
            HIP_TRY(launch_group(g.kind, g.mode, d_steps, g.first, g.count, g.t0, g.t1, g.flags, cnt, s));
            if (ev) HIP_TRY(hipEventRecord(P->op_events[2 * gi + 1], s));
            ++*launches;
        }
        ++*launches;
    }
    return PA_OK;
}

// The step-table executors (grouped levels or one persistent launch), with
// the callers' output pointers patched in, directly or as a hipGraph replay.
int exec_steps(pa_plan *P, const std::vector<void *> &outs, hipStream_t s, int *launches) {
    int rc;
    const bool use_graph = P->graph && s != nullptr && P->op_events.empty() && !P->timing_active;
    const bool new_table = P->last_outs != outs;
    const bool new_graph = use_graph && (!P->graph_exec || P->graph_outs != outs || P->graph_stream != s);
    if ((new_table || new_graph) && P->has_run) {
        // the step table (a synchronous copy) and the graph are rewritten
        // below: earlier executions, on this stream or the one last used,
        // must have finished reading them
        HIP_TRY(hipStreamSynchronize(P->last_stream));
        if (s != P->last_stream) HIP_TRY(hipStreamSynchronize(s));
    }
    if (new_table) {
        rc = upload_steps(P, outs);
        if (rc) return rc;
    }
    P->has_run = true;
    P->last_stream = s;
    if (use_graph) {
        if (new_graph) {
            if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
            if (P->graph_h) (void)hipGraphDestroy(P->graph_h);
            P->graph_exec = nullptr;
            P->graph_h = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            int dummy = 0;
            rc = run_persist(P, s, &dummy);
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamEndCapture(s, &g));
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            HIP_TRY(hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0));
            P->graph_h = g;
            P->graph_outs = outs;
            P->graph_stream = s;
        }
        HIP_TRY(hipGraphLaunch(P->graph_exec, s));
        *launches += 1;
    } else {
        rc = run_persist(P, s, launches, P->op_events.empty() ? nullptr : P->op_events[0]);
        if (rc) return rc;
    }
    if (!P->op_events.empty()) {
        HIP_TRY(hipEventRecord(P->op_events.size() == 2 ? P->op_events[1] : P->op_events.back(), s));
        P->op_events_recorded = true;
    }
    return PA_OK;
}

int plan_workspace_cap(size_t *cap) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(PA_EHIP, "no usable HIP device");
    *cap = free_b > ((size_t)1 << 30) ? free_b - ((size_t)1 << 30) : 0;
    if (const char *env = std::getenv("PA_MAX_WORKSPACE_BYTES")) *cap = std::min<size_t>(*cap, std::strtoull(env, nullptr, 10));
    return PA_OK;
}

}  // namespace pa

// ====================================================================== ABI
using namespace pa;

// Milliseconds per execution of a plan built with `o` (one untimed and
// `reps` timed executions on stream 0 into a temporary output).
static int time_plan_once(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts &o,
                          int reps, double *ms, std::vector<int> *merges) {
    pa_plan *p = nullptr;
    int rc = pa_plan_create(sys, exposed, n_exposed, &o, &p);
    if (rc) return rc;
    std::unique_ptr<pa_plan> hold(p);
    if (merges) *merges = p->tree.merges;
    pa_bitarray out;
    std::memset(&out, 0, sizeof(out));
    out.ndim = (int32_t)p->out_layout.dims.size();
    for (int i = 0; i < out.ndim; ++i) out.dims[i] = (int32_t)p->out_layout.dims[i];
    out.row_words = p->out_layout.rw;
    void *buf = nullptr;
    if (hipMalloc(&buf, sizeof(uint32_t) * (size_t)std::max<int64_t>(1, p->out_layout.words)) != hipSuccess)
        return fail(PA_ENOMEM, "verify_order: output allocation failed");
    out.data = buf;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = pa_plan_execute(p, &out, nullptr, nullptr);
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(PA_EHIP, "verify_order: event creation failed");
    if (!rc && hipEventRecord(e0, nullptr) != hipSuccess) rc = fail(PA_EHIP, "verify_order: event record failed");
    for (int i = 0; i < reps && !rc; ++i) rc = pa_plan_execute(p, &out, nullptr, nullptr);
    float t = 0.f;
    if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = fail(PA_EHIP, "verify_order: event timing failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (!rc) *ms = (double)t / reps;
    return rc;
}

// The exhaustive search judges a learned tree by measurement: both trees are
// planned and timed, the faster order is returned in *choice.
static int verify_learned_order(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts &o,
                                int *choice) {
    pa_opts lo = o, eo = o;
    lo.verify_order = 0;
    lo.timing = 0;
    lo.autotune = 0;
    lo.workspace = nullptr;
    lo.workspace_bytes = 0;
    eo = lo;
    eo.order_policy = PA_ORDER_EXHAUSTIVE;
    double tl = 0.0, te = 0.0;
    std::vector<int> ml, me;
    int rc = time_plan_once(sys, exposed, n_exposed, eo, 2, &te, &me);
    if (rc) return rc;
    rc = time_plan_once(sys, exposed, n_exposed, lo, 2, &tl, &ml);
    if (rc == PA_ENOMEM) {               // the learned tree does not fit: the exhaustive one does
        *choice = PA_ORDER_EXHAUSTIVE;
        return PA_OK;
    }
    if (rc) return rc;
    *choice = (ml == me || tl <= te) ? PA_ORDER_LEARNED : PA_ORDER_EXHAUSTIVE;
    return PA_OK;
}

extern "C" int pa_plan_create(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts,
                              pa_plan **plan) {
    if (!plan) return fail(PA_EINVAL, "plan_create: null plan pointer");
    *plan = nullptr;
    std::unique_ptr<pa_plan> P(new pa_plan());
    pa_opts tuned{};
    if (opts && opts->autotune && !opts->plain && !opts->per_op && sys) {
        tuned = *opts;
        int rc = autotuned_opts(sys, 1, &exposed, &n_exposed, tuned);
        if (rc) return rc;
        opts = &tuned;
    }
    bool verified_fallback = false;
    if (opts && opts->order_policy == PA_ORDER_LEARNED && opts->verify_order && !opts->plain && !opts->per_op && sys) {
        int choice = PA_ORDER_LEARNED;
        int rc = verify_learned_order(sys, exposed, n_exposed, *opts, &choice);
        if (rc) return rc;
        if (choice != PA_ORDER_LEARNED) {
            if (opts != &tuned) tuned = *opts;
            tuned.order_policy = choice;
            opts = &tuned;
            verified_fallback = true;
        }
    }
    if (opts && opts->measure_density && sys) {
        std::vector<std::vector<double>> dens;
        int rc = measure_leaf_densities(sys, 1, *opts, dens);
        if (rc) return rc;
        P->leaf_log2d = dens[0];
    }
    int rc = build_plan(sys, exposed, n_exposed, opts, P.get());
    if (rc) return rc;
    if (verified_fallback) P->tree.learned_fallback = true;
    if (opts && opts->workspace) {
        if (opts->workspace_bytes < P->ws_bytes)
            return fail(PA_ENOMEM, "workspace too small: need " + std::to_string(P->ws_bytes) + " bytes");
        P->ws.ptr = opts->workspace;
        P->ws.cap = opts->workspace_bytes;
        P->ws.external = true;
    } else {
        // refuse plans whose intermediates cannot fit instead of attempting
        // an allocation the device cannot satisfy
        size_t cap = 0;
        rc = plan_workspace_cap(&cap);
        if (rc) return rc;
        if (P->ws_bytes > cap)
            return fail(PA_ENOMEM, "plan needs " + std::to_string(P->ws_bytes) + " bytes of workspace, " +
                                       std::to_string(cap) + " available (choose another order)");
        rc = P->ws.ensure(std::max<size_t>(P->ws_bytes, 256));
        if (rc) return rc;
    }
    rc = upload_plan(P.get());
    if (rc) return rc;
    if (opts && opts->timing == 2) {
        P->op_events.resize(P->per_op ? 2 + 2 * P->ops.size()
                                      : (P->single_launch ? 2 : std::max<size_t>(2, 2 * P->groups.size())));
        for (auto &e : P->op_events) HIP_TRY(hipEventCreate(&e));
    }
    *plan = P.release();
    return PA_OK;
}

pa_plan::~pa_plan() {
    for (auto &e : op_events)
        if (e) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph_h) (void)hipGraphDestroy(graph_h);
}

// PA_OPKIND_* of an op, and of a group of steps (kind, mode).
static int op_kind_code(const Op &op) {
    switch (op.kind) {
        case OP_GEMM: return PA_OPKIND_GEMM;
        case OP_FILL: return PA_OPKIND_FILL;
        case OP_GATHER: return PA_OPKIND_GATHER;
        case OP_COUNT: return PA_OPKIND_COUNT;
        case OP_LIST: return PA_OPKIND_ROWLIST;
        case OP_FUSED: return PA_OPKIND_FUSED;
        default: return op.mode;
    }
}

static int step_kind_code(int kind, int mode) {
    switch (kind) {
        case kStepPlot: return PA_OPKIND_PLOT;
        case kStepGemm: return PA_OPKIND_GEMM;
        case kStepFill: return PA_OPKIND_FILL;
        case kStepGather: return PA_OPKIND_GATHER;
        case kStepCount: return PA_OPKIND_COUNT;
        case kStepList: return PA_OPKIND_ROWLIST;
        case kStepFused: return PA_OPKIND_FUSED;
        default: return mode;
    }
}

extern "C" int32_t pa_plan_op_times(pa_plan *P, double *ms, int32_t *kind, double *macs, int32_t cap) {
    if (!P || P->op_events.empty() || !P->op_events_recorded) return fail(PA_EINVAL, "op_times: no op timings"), -1;
    const bool per_op = P->per_op;
    const bool groups = !per_op && !P->single_launch && !P->groups.empty();
    const int32_t n = per_op ? 1 + (int32_t)P->ops.size() : (groups ? (int32_t)P->groups.size() : 1);
    if (hipEventSynchronize(P->op_events.back()) != hipSuccess) return fail(PA_EHIP, "op_times: sync"), -1;
    for (int32_t i = 0; i < n && i < cap; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, P->op_events[2 * i], P->op_events[2 * i + 1]) != hipSuccess) t = -1.f;
        if (ms) ms[i] = t;
        int k = PA_OPKIND_PERSIST;
        double mc = P->total_macs;
        if (per_op) {
            k = PA_OPKIND_PLOT;
            mc = 0.0;
            if (i > 0) {
                const Op &op = P->ops[i - 1];
                k = op_kind_code(op);
                mc = (op.kind == OP_FILL || op.kind == OP_COUNT || op.kind == OP_LIST) ? 0.0 : op.macs;
            }
        } else if (groups) {
            const auto &g = P->groups[i];
            k = step_kind_code(g.kind, g.mode);
            mc = 0.0;
            for (int j = g.first; j < g.first + g.count; ++j) mc += P->step_macs[j];
        }
        if (kind) kind[i] = k;
        if (macs) macs[i] = mc;
    }
    return n;
}

namespace pa {
int time_groups(pa_plan *P, int32_t reps, double *ms, int32_t *kind, double *macs, int32_t cap, hipStream_t s) {
    if (P->per_op || P->single_launch || P->groups.empty() || P->last_outs.empty())
        return fail(PA_EINVAL, "time_groups: need an executed plan on the grouped executor"), -1;
    if (reps < 1) return fail(PA_EINVAL, "time_groups: reps must be >= 1"), -1;
    char *base = static_cast<char *>(P->ws.ptr);
    const PStep *d_steps = reinterpret_cast<const PStep *>(base + P->steps_off);
    PlotCounters *cnt = reinterpret_cast<PlotCounters *>(base + P->counters_off);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(PA_EHIP, "time_groups: event creation failed"), -1;
    int rc = PA_OK;
    const int32_t n = (int32_t)P->groups.size();
    for (int32_t gi = 0; gi < n && !rc; ++gi) {
        const auto &g = P->groups[gi];
        if (hipEventRecord(e0, s) != hipSuccess) rc = fail(PA_EHIP, "time_groups: event record failed");
        for (int r = 0; r < reps && !rc; ++r)
            if (launch_group(g.kind, g.mode, d_steps, g.first, g.count, g.t0, g.t1, g.flags, cnt, s) != hipSuccess)
                rc = fail(PA_EHIP, "time_groups: launch failed");
        float t = 0.f;
        if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            rc = fail(PA_EHIP, "time_groups: event timing failed");
        if (!rc && gi < cap) {
            if (ms) ms[gi] = (double)t / reps;
            if (kind) kind[gi] = step_kind_code(g.kind, g.mode);
            double mc = 0.0;
            for (int j = g.first; j < g.first + g.count; ++j) mc += P->step_macs[j];
            if (macs) macs[gi] = mc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc ? -1 : n;
}
}  // namespace pa

extern "C" int32_t pa_plan_time_groups(pa_plan *P, int32_t reps, double *ms, int32_t *kind, double *macs, int32_t cap,
                                       void *stream) {
    if (!P) return fail(PA_EINVAL, "time_groups: null plan"), -1;
    return time_groups(P, reps, ms, kind, macs, cap, static_cast<hipStream_t>(stream));
}

extern "C" size_t pa_plan_workspace_bytes(const pa_plan *plan) { return plan ? plan->ws_bytes : 0; }

namespace pa {
// Writes the persistent executor's wait bound into the plan's device state,
// after every call in flight on the device has finished.
int set_wait_limit(pa_plan *P, int64_t polls) {
    if (!P->ws.ptr) return fail(PA_EINVAL, "set_wait_limit: the plan has no device state");
    const long long v = (long long)polls;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(static_cast<char *>(P->ws.ptr) + P->state_off + offsetof(PersistState, wait_limit), &v,
                      sizeof(v), hipMemcpyHostToDevice));
    return PA_OK;
}
}  // namespace pa

extern "C" int pa_plan_set_wait_limit(pa_plan *P, int64_t polls) {
    if (!P) return fail(PA_EINVAL, "set_wait_limit: null plan");
    return set_wait_limit(P, polls);
}

extern "C" void pa_plan_destroy(pa_plan *plan) { delete plan; }

extern "C" int pa_plan_execute(pa_plan *P, pa_bitarray *out, pa_report *rep, void *stream) {
    if (!P) return fail(PA_EINVAL, "plan_execute: null plan");
    int rc = check_bitarray(out, P->out_layout.dims, "plan_execute: out");
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(P->ws.ptr);
    int launches = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    const bool timing = P->timing && rep;
    if (timing)
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    PlotCounters cnt0;
    std::memset(&cnt0, 0, sizeof(cnt0));
    if (rep) HIP_TRY(hipMemcpyAsync(&cnt0, base + P->counters_off, sizeof(cnt0), hipMemcpyDeviceToHost, s));
    if (timing) HIP_TRY(hipEventRecord(ev[0], s));
    if (!P->op_events.empty() && P->per_op) HIP_TRY(hipEventRecord(P->op_events[0], s));
    if (P->per_op) {
        rc = run_plots(P, s, &launches);
        if (rc) return rc;
        if (!P->op_events.empty()) HIP_TRY(hipEventRecord(P->op_events[1], s));
        if (timing) HIP_TRY(hipEventRecord(ev[1], s));
        rc = run_ops(P, out->data, s, &launches);
        if (rc) return rc;
    } else {
        P->timing_active = timing;
        rc = exec_steps(P, {out->data}, s, &launches);
        if (rc) return rc;
        if (timing) HIP_TRY(hipEventRecord(ev[1], s));
    }
    if (!P->op_events.empty()) P->op_events_recorded = true;
    if (timing) HIP_TRY(hipEventRecord(ev[2], s));
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        HIP_TRY(launch_fill(reinterpret_cast<uint32_t *>(base + P->popcnt_off), 2, 0u, s));
        HIP_TRY(launch_popcount(static_cast<const uint32_t *>(out->data), P->out_layout.words,
                                reinterpret_cast<unsigned long long *>(base + P->popcnt_off), s));
        PlotCounters cnt;
        PersistState pst;
        unsigned long long nnz = 0;
        HIP_TRY(hipMemcpyAsync(&cnt, base + P->counters_off, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&nnz, base + P->popcnt_off, sizeof(nnz), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&pst, base + P->state_off, sizeof(pst), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!P->per_op && pst.abort) return fail(PA_EHIP, "persistent executor gave up a dependency wait");
        rep->corners = P->corners;
        rep->corners_flagged = (int64_t)(cnt.flagged - cnt0.flagged);
        rep->corners_disagree = (int64_t)(cnt.disagree - cnt0.disagree);
        rep->corners_disagree_unflagged = (int64_t)(cnt.disagree_unflagged - cnt0.disagree_unflagged);
        rep->nnz_out = (int64_t)nnz;
        rep->n_launches = launches;
        int steps = 0;
        for (const auto &op : P->ops) steps += counted_steps_of(op);
        rep->n_steps = steps;
        rep->cost_macs = P->tree.cost;
        for (size_t i = 0; i < P->tree.merges.size() && i < 2 * PA_MAX_RELATIONS; ++i) rep->merges[i] = P->tree.merges[i];
        rep->t_plan_ms = P->t_plan_ms;
        if (timing) {
            float a = 0.f, b = 0.f;
            HIP_TRY(hipEventElapsedTime(&a, ev[0], ev[1]));
            HIP_TRY(hipEventElapsedTime(&b, ev[1], ev[2]));
            rep->t_plot_ms = a;
            rep->t_contract_ms = b;
        }
    }
    if (timing)
        for (auto &e : ev) (void)hipEventDestroy(e);
    return PA_OK;
}

extern "C" int pa_solve_system(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts,
                               pa_bitarray *out, pa_report *report, void *stream) {
    pa_plan *P = nullptr;
    int rc = pa_plan_create(sys, exposed, n_exposed, opts, &P);
    if (rc) return rc;
    rc = pa_plan_execute(P, out, report, stream);
    if (rc == PA_OK && !report) {
        // the plan's workspace is freed below: wait for the work to finish
        if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) rc = fail(PA_EHIP, "sync failed");
    }
    pa_plan_destroy(P);
    return rc;
}

extern "C" size_t pa_workspace_bytes(const pa_system *sys, const int32_t *exposed, int32_t n_exposed,
                                     const pa_opts *opts) {
    std::unique_ptr<pa_plan> P(new pa_plan());
    if (build_plan(sys, exposed, n_exposed, opts, P.get()) != PA_OK) return 0;
    return std::max<size_t>(P->ws_bytes, 256);
}

extern "C" int64_t pa_plan_describe(const pa_system *sys, const int32_t *exposed, int32_t n_exposed,
                                    const pa_opts *opts, char *buf, int64_t buf_len) {
    std::unique_ptr<pa_plan> P(new pa_plan());
    int rc = PA_OK;
    if (opts && opts->measure_density && sys) {
        std::vector<std::vector<double>> dens;
        rc = measure_leaf_densities(sys, 1, *opts, dens);
        if (rc == PA_OK) P->leaf_log2d = dens[0];
    }
    if (rc == PA_OK) rc = build_plan(sys, exposed, n_exposed, opts, P.get());
    std::ostringstream s;
    s.precision(17);
    if (rc) {
        s << "{\"error\":" << rc << "}";
    } else {
        s << "{\"merges\":" << join(std::vector<int>(P->tree.merges.begin(), P->tree.merges.end()))
          << ",\"cost\":" << P->tree.cost << ",\"workspace_bytes\":" << P->ws_bytes << ",\"corners\":" << P->corners
          << ",\"total_macs\":" << P->total_macs << ",\"predicted_us\":" << P->tree.predicted_us
          << ",\"learned_fallback\":" << (P->tree.learned_fallback ? "true" : "false")
          << ",\"leaf_log2_density\":[";
        for (size_t i = 0; i < P->si.leaf_log2d.size(); ++i) {
            const double v = P->si.leaf_log2d[i];
            s << (i ? "," : "");
            if (std::isfinite(v)) s << v;
            else s << "null";
        }
        s << "]"
          << ",\"plots\":[";
        for (size_t i = 0; i < P->plots.size(); ++i) {
            s << (i ? "," : "") << "{\"rel\":" << P->plots[i].rel << ",\"buf\":" << P->plots[i].buf
              << ",\"vars\":" << join(P->plots[i].layout.vars);
            if (i < P->plotrel_host.size()) {
                // the plotting tiles: words x strips x fixed-axis cells, rows per strip
                const PlotRel &R = P->plotrel_host[i];
                s << ",\"tiles\":" << R.n_tiles << ",\"tile\":[" << R.tw << "," << R.tb << "," << R.ta << "," << R.s
                  << "],\"walk_fixed\":" << R.walk_fixed;
            }
            s << "}";
        }
        s << "],\"ops\":[";
        for (size_t i = 0; i < P->ops.size(); ++i) s << (i ? "," : "") << P->ops[i].describe();
        s << "],\"buffers\":[";
        for (size_t i = 0; i < P->buf_layout.size(); ++i)
            s << (i ? "," : "") << "{\"vars\":" << join(P->buf_layout[i].vars) << ",\"words\":" << P->buf_words[i] << "}";
        s << "]}";
    }
    const std::string str = s.str();
    if (buf && buf_len > 0) {
        const int64_t n = std::min<int64_t>(buf_len - 1, (int64_t)str.size());
        std::memcpy(buf, str.data(), (size_t)n);
        buf[n] = 0;
    }
    return (int64_t)str.size();
}

// ------------------------------------------------------ one-relation plot
namespace {
struct SmallScratch {
    std::mutex mu;
    pa::Workspace ws;
};
SmallScratch &scratch() {
    static SmallScratch s;
    return s;
}
}  // namespace

extern "C" int pa_plot_relation(const pa_relation *rel, const pa_axis *axes_of_vars, const pa_opts *opts,
                                pa_bitarray *out, pa_report *report, void *stream) {
    if (!rel || !axes_of_vars) return fail(PA_EINVAL, "plot_relation: null argument");
    // a one-relation system over its own variables 0..arity-1
    std::vector<int32_t> vars(rel->arity);
    for (int i = 0; i < rel->arity; ++i) vars[i] = i;
    int rc = validate_relation(*rel, axes_of_vars, -1, "plot_relation");
    if (rc) return rc;
    std::vector<int64_t> dims;
    for (int i = 0; i < rel->arity; ++i) dims.push_back(axes_of_vars[i].res);
    rc = check_bitarray(out, dims, "plot_relation: out");
    if (rc) return rc;
    pa_relation r2 = *rel;
    r2.vars = vars.data();
    pa_system sys{rel->arity, axes_of_vars, 1, &r2};
    // plan: the single leaf, plotted in declared order, copied to out
    pa_plan *P = nullptr;
    rc = pa_plan_create(&sys, vars.data(), rel->arity, opts, &P);
    if (rc) return rc;
    rc = pa_plan_execute(P, out, report, stream);
    if (rc == PA_OK && !report && hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
        rc = fail(PA_EHIP, "sync failed");
    pa_plan_destroy(P);
    return rc;
}

extern "C" int pa_popcount(const pa_bitarray *a, int64_t *count, void *stream) {
    if (!a || !count || !a->data || a->ndim < 0 || a->ndim > PA_MAX_DIMS) return fail(PA_EINVAL, "popcount: bad args");
    auto &S = scratch();
    std::lock_guard<std::mutex> lk(S.mu);
    int rc = S.ws.ensure(256);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_fill(static_cast<uint32_t *>(S.ws.ptr), 2, 0u, s));
    HIP_TRY(launch_popcount(static_cast<const uint32_t *>(a->data), pa_array_words(a->ndim, a->dims),
                            static_cast<unsigned long long *>(S.ws.ptr), s));
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, S.ws.ptr, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *count = (int64_t)c;
    return PA_OK;
}

extern "C" int pa_lds_read_rate(double *bytes_per_second, void *stream) {
    if (!bytes_per_second) return fail(PA_EINVAL, "lds_read_rate: null output");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus < 1) return fail(PA_EINVAL, "lds_read_rate: no compute units");
    constexpr int kIters = 4096;
    auto &S = scratch();
    std::lock_guard<std::mutex> lk(S.mu);
    int rc = S.ws.ensure((size_t)cus * 1024 * 4);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *out = static_cast<uint32_t *>(S.ws.ptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PA_EHIP, "lds_read_rate: hipEventCreate failed");
    }
    float ms = 0.f;
    hipError_t e = launch_lds_rate(out, cus, kIters, s);     // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_lds_rate(out, cus, kIters, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(PA_EHIP, std::string("lds_read_rate: ") + hipGetErrorString(e));
    if (!(ms > 0.f)) return fail(PA_EHIP, "lds_read_rate: no elapsed time");
    *bytes_per_second = (double)cus * 1024.0 * kIters * 8.0 * 16.0 / (ms * 1e-3);
    return PA_OK;
}

extern "C" int pa_tile_popcount(const pa_bitarray *a, int32_t tile_rows, int32_t tile_words, uint32_t *counts,
                                void *stream) {
    if (!a || !counts || !a->data || a->ndim < 0 || a->ndim > PA_MAX_DIMS) return fail(PA_EINVAL, "tile_popcount: bad args");
    if (tile_rows < 1 || tile_words < 1 || (double)tile_rows * tile_words * 32.0 >= 4294967296.0)
        return fail(PA_EINVAL, "tile_popcount: tile sizes must be >= 1 with fewer than 2^32 bits per tile");
    int64_t rows = 1;
    for (int i = 0; i + 1 < a->ndim; ++i) {
        if (a->dims[i] < 1) return fail(PA_EINVAL, "tile_popcount: dims must be >= 1");
        rows *= a->dims[i];
    }
    const int64_t rw = a->ndim == 0 ? 1 : pa_row_words(a->dims[a->ndim - 1]);
    if (a->ndim > 0 && a->row_words != rw) return fail(PA_EINVAL, "tile_popcount: row_words must be 2*ceil(d/64)");
    HIP_TRY(launch_tile_popcount(static_cast<const uint32_t *>(a->data), rows, rw, tile_rows, tile_words, counts,
                                 static_cast<hipStream_t>(stream)));
    return PA_OK;
}

// ---------------------------------------------------------- pa_contract
// pa_contract, and (with `tab` a device buffer of tab_cap int64 entries)
// its variant that allocates nothing: the latent-entry table of a streamed
// contraction is then written into `tab` by a kernel on the stream instead of
// being copied from the host into a stream-ordered allocation.
// Is a two-pack contraction in the MFMA kernel's canonical layout, A =
// [batch][m][k], B = [batch][n][k], C = [batch][m][n] (k the shared latent
// variables, contiguous, with the packed one last in both; batch variables
// shared and kept)?  nb and nm: the counts of batch and m variables.
static bool canonical_gemm(const ContractLayouts &cl, int &nb, int &nm) {
    const std::vector<int> &av = cl.av, &bv = cl.bv, &ov = cl.ov;
    const uint64_t outm = cl.outm;
    const uint64_t ma = list_mask(av), mb = list_mask(bv);
    const uint64_t bm = ma & mb & outm, km = ma & mb & ~outm, em = ma & ~mb, en = mb & ~ma;
    nb = __builtin_popcountll(bm);
    nm = __builtin_popcountll(em);
    const int nn = __builtin_popcountll(en), nk = __builtin_popcountll(km);
    bool canon = km && em && en && ((em | en) & ~outm) == 0 && (int)av.size() == nb + nm + nk &&
                 (int)bv.size() == nb + nn + nk && (int)ov.size() == nb + nm + nn;
    if (canon) {
        auto seg = [](const std::vector<int> &l, int a, int n) { return std::vector<int>(l.begin() + a, l.begin() + a + n); };
        canon = list_mask(seg(av, 0, nb)) == bm && seg(av, 0, nb) == seg(bv, 0, nb) && seg(av, 0, nb) == seg(ov, 0, nb) &&
                list_mask(seg(av, nb, nm)) == em && seg(av, nb, nm) == seg(ov, nb, nm) &&
                list_mask(seg(bv, nb, nn)) == en && seg(bv, nb, nn) == seg(ov, nb + nm, nn) &&
                list_mask(seg(av, nb + nm, nk)) == km && seg(av, nb + nm, nk) == seg(bv, nb + nn, nk);
    }
    return canon;
}

// Validation and layouts of a two-pack contraction's arguments (shared by
// the Boolean and the count entry points): variable lengths from A and B,
// A's and B's layouts checked against their arrays, C's layout from out_vars.
int pa::contract_layouts(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                         const int32_t *out_vars, int32_t n_out, bool has_c, ContractLayouts &cl) {
    std::vector<int64_t> &res = cl.res;
    std::vector<int> &av = cl.av, &bv = cl.bv, &ov = cl.ov;
    uint64_t &outm = cl.outm;
    Layout &la = cl.la, &lb = cl.lb, &lc = cl.lc;
    if (!A || !has_c || (!a_vars && A->ndim > 0) || (n_out > 0 && !out_vars)) return fail(PA_EINVAL, "contract: null argument");
    if (A->ndim < 0 || A->ndim > PA_MAX_DIMS || n_out < 0 || n_out > PA_MAX_DIMS || (B && (B->ndim < 0 || B->ndim > PA_MAX_DIMS)))
        return fail(PA_EINVAL, "contract: rank out of range");
    res.assign(PA_MAX_VARS, -1);
    auto note = [&](const pa_bitarray *X, const int32_t *vs) -> int {
        uint64_t seen = 0;
        for (int i = 0; i < X->ndim; ++i) {
            const int v = vs[i];
            if (v < 0 || v >= PA_MAX_VARS) return fail(PA_EINVAL, "contract: variable label out of range");
            if ((seen >> v) & 1) return fail(PA_EINVAL, "contract: repeated variable in one array");
            seen |= 1ull << v;
            if (X->dims[i] < 1) return fail(PA_EINVAL, "contract: dims must be >= 1");
            if (res[v] >= 0 && res[v] != X->dims[i]) return fail(PA_EINVAL, "contract: shared variable with different lengths");
            res[v] = X->dims[i];
        }
        return PA_OK;
    };
    int rc = note(A, a_vars);
    if (rc) return rc;
    if (B) {
        rc = note(B, b_vars);
        if (rc) return rc;
    }
    outm = 0;
    ov.clear();
    for (int i = 0; i < n_out; ++i) {
        const int v = out_vars[i];
        if (v < 0 || v >= PA_MAX_VARS || res[v] < 0) return fail(PA_EINVAL, "contract: output variable not in A or B");
        if ((outm >> v) & 1) return fail(PA_EINVAL, "contract: repeated output variable");
        outm |= 1ull << v;
        ov.push_back(v);
    }
    av.assign(a_vars, a_vars + A->ndim);
    bv.clear();
    if (B) bv.assign(b_vars, b_vars + B->ndim);
    la = make_layout(av, res);
    lb = B ? make_layout(bv, res) : Layout();
    lc = make_layout(ov, res);
    rc = check_bitarray(A, la.dims, "contract: A");
    if (rc) return rc;
    if (B) {
        rc = check_bitarray(B, lb.dims, "contract: B");
        if (rc) return rc;
    }
    return PA_OK;
}

int pa::contract_impl(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                      const int32_t *out_vars, int32_t n_out, pa_bitarray *C, const pa_opts *opts, void *stream,
                      int64_t *tab_dev, int64_t tab_cap) {
    ContractLayouts cl;
    int rc = contract_layouts(A, a_vars, B, b_vars, out_vars, n_out, C != nullptr, cl);
    if (rc) return rc;
    std::vector<int64_t> &res = cl.res;
    std::vector<int> &av = cl.av, &bv = cl.bv, &ov = cl.ov;
    const uint64_t outm = cl.outm;
    const Layout &la = cl.la, &lb = cl.lb, &lc = cl.lc;
    rc = check_bitarray(C, lc.dims, "contract: C");
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // canonical GEMM layout: A = [b][m][k], B = [b][n][k], C = [b][m][n]
    if (B) {
        int nb = 0, nm = 0;
        const bool canon = canonical_gemm(cl, nb, nm);
        if (canon) {
            pa_plan tmp;
            tmp.plain = opts ? opts->plain : 0;
            tmp.si.res = res;
            tmp.si.n_vars = PA_MAX_VARS;
            Builder Bd{&tmp, nullptr};
            tmp.gemm_path = gemm_path_of(opts ? opts->gemm_path : 0);
            Bd.emit_gemm(0, la, 1, lb, kBufOutput, lc, nb, nm, -1);
            tmp.gemm_split = opts && opts->gemm_split > 0 ? opts->gemm_split : 512;
            split_gemms(&tmp);
            for (auto &op : tmp.ops) {
                if (op.kind == OP_FILL) {
                    HIP_TRY(launch_fill(static_cast<uint32_t *>(C->data), op.fill_words, 0u, s));
                } else {
                    GemmArgs g = op.ga;
                    rc = check_gemm_bounds(g, la.words, lb.words, lc.words);
                    if (rc) return rc;
                    g.A = static_cast<const uint32_t *>(A->data);
                    g.B = static_cast<const uint32_t *>(B->data);
                    g.C = static_cast<uint32_t *>(C->data);
                    HIP_TRY(launch_gemm(g, s));
                }
            }
            return PA_OK;
        }
    }
    Op op;
    op.la = la;
    op.lb = lb;
    op.lc = lc;
    op.kvars = mask_list((list_mask(av) | (B ? list_mask(bv) : 0)) & ~outm);
    finish_contract(op, B != nullptr);
    rc = check_contract_bounds(op.ca, la.words, B ? lb.words : 0, lc.words, B != nullptr);
    if (rc) return rc;
    op.ca.A = static_cast<const uint32_t *>(A->data);
    op.ca.B = B ? static_cast<const uint32_t *>(B->data) : nullptr;
    op.ca.C = static_cast<uint32_t *>(C->data);
    if (tab_dev) {
        if ((int64_t)op.ktab.size() > tab_cap)
            return fail(PA_ENOMEM, "contract: latent-entry table of " + std::to_string(op.ktab.size() / 2) +
                                       " entries exceeds the static buffer (" + std::to_string(tab_cap / 2) + ")");
        if (!op.ktab.empty()) {
            HIP_TRY(launch_ktab(op.ca, op.mode, tab_dev, op.ca.nktab, s));
            op.ca.ktab = tab_dev;
        }
        HIP_TRY(launch_contract(op.ca, op.mode, s));
        return PA_OK;
    }
    void *tab = nullptr;
    if (!op.ktab.empty()) {
        // stream-ordered table: allocated, filled, used and freed on `s`
        const size_t bytes = op.ktab.size() * sizeof(int64_t);
        if (hipMallocAsync(&tab, bytes, s) != hipSuccess) return fail(PA_ENOMEM, "contract: table allocation failed");
        HIP_TRY(hipMemcpyAsync(tab, op.ktab.data(), bytes, hipMemcpyHostToDevice, s));
        op.ca.ktab = static_cast<const int64_t *>(tab);
    }
    const hipError_t le = launch_contract(op.ca, op.mode, s);
    if (tab) {
        // the host table must outlive the asynchronous copy
        (void)hipStreamSynchronize(s);
        (void)hipFreeAsync(tab, s);
    }
    if (le != hipSuccess) return fail(PA_EHIP, std::string("contract launch: ") + hipGetErrorString(le));
    return PA_OK;
}

extern "C" int pa_contract(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                           const int32_t *out_vars, int32_t n_out, pa_bitarray *C, const pa_opts *opts, void *stream) {
    return contract_impl(A, a_vars, B, b_vars, out_vars, n_out, C, opts, stream, nullptr, 0);
}

// ------------------------------------------------------ count semiring
extern "C" int pa_contract_count(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B,
                                 const int32_t *b_vars, const int32_t *out_vars, int32_t n_out, uint32_t *C,
                                 const pa_opts *opts, void *stream) {
    ContractLayouts cl;
    int rc = contract_layouts(A, a_vars, B, b_vars, out_vars, n_out, C != nullptr, cl);
    if (rc) return rc;
    const Layout &la = cl.la, &lb = cl.lb, &lc = cl.lc;
    // latent entries: the largest count (int32 accumulation in the kernels)
    double nlat = 1.0;
    const uint64_t all = list_mask(cl.av) | (B ? list_mask(cl.bv) : 0);
    for (int v : mask_list(all & ~cl.outm)) nlat *= (double)cl.res[v];
    if (nlat >= 2147483648.0) return fail(PA_EUNSUPPORTED, "contract_count: more than 2^31 - 1 latent entries");
    int64_t n_elems = 1;
    for (int64_t d : lc.dims) n_elems *= d;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int nb = 0, nm = 0;
    if (B && canonical_gemm(cl, nb, nm)) {
        pa_plan tmp;
        tmp.si.res = cl.res;
        tmp.si.n_vars = PA_MAX_VARS;
        tmp.gemm_path = 0;
        Builder Bd{&tmp, nullptr};
        Bd.emit_gemm(0, la, 1, lb, kBufOutput, lc, nb, nm, -1);
        GemmArgs g = tmp.ops.back().ga;
        rc = check_gemm_bounds(g, la.words, lb.words, lc.words);
        if (rc) return rc;
        // counts: C[b][m][n] dense, n = (no, j) with j < rn
        g.sC_b = g.M * g.No * g.rn;
        g.path = 0;
        g.tiles_m = (g.M + 127) / 128;
        g.fd_tiles_m = make_fastdiv((uint64_t)std::max<int64_t>(1, g.tiles_m));
        // split K until the launch has about 512 work items (parts add into a
        // zeroed output)
        const int64_t tiles = g.nbatch * g.tiles_m * g.tiles_n;
        set_ksplit(g, std::max<int64_t>(1, 512 / std::max<int64_t>(1, tiles)));
        if (tiles * g.ksplit >= ((int64_t)1 << 31) || g.M * g.No * g.rn >= ((int64_t)1 << 40))
            return fail(PA_EUNSUPPORTED, "contract_count: too many tiles");
        g.A = static_cast<const uint32_t *>(A->data);
        g.B = static_cast<const uint32_t *>(B->data);
        g.C = C;
        if (g.ksplit > 1) HIP_TRY(launch_fill(C, n_elems, 0u, s));
        HIP_TRY(launch_gemm_count(g, s));
        return PA_OK;
    }
    Op op;
    op.la = la;
    op.lb = lb;
    op.lc = lc;
    op.kvars = mask_list(all & ~cl.outm);
    finish_contract(op, B != nullptr);
    rc = check_contract_bounds(op.ca, la.words, B ? lb.words : 0, lc.words, B != nullptr);
    if (rc) return rc;
    op.ca.A = static_cast<const uint32_t *>(A->data);
    op.ca.B = B ? static_cast<const uint32_t *>(B->data) : nullptr;
    op.ca.C = C;
    HIP_TRY(launch_count_bits(op.ca, n_elems, s));
    (void)opts;
    return PA_OK;
}
