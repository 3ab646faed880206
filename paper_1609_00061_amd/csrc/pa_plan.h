// Plans: cluster tree, per-node layouts, the op list and the workspace.
#pragma once
#include <array>
#include <utility>
#include <stdint.h>
#include <string>
#include <vector>

#include "pa.h"
#include "pa_internal.h"

namespace pa {

extern thread_local std::string g_err;
int fail(int code, const std::string &msg);

// Axis order of a bit-packed array; the last variable is the packed axis.
struct Layout {
    std::vector<int> vars;
    std::vector<int64_t> dims;
    int64_t rw = 1;
    int64_t words = 1;
    int packed() const;
    int64_t stride(int v) const;
    bool has(int v) const;
};

int64_t row_words_of(int64_t d);
Layout make_layout(const std::vector<int> &vars, const std::vector<int64_t> &res_of_var);
std::vector<std::array<int, 3>> graded_lex(int n, int d);
int64_t n_monomials(int n, int d);
std::vector<double> dense_coef(const pa_relation &r);
double axis_step(double lo, double hi, int r);   // corner k: lo + k * step (two roundings)
int validate_relation(const pa_relation &r, const pa_axis *axes_of_vars, int n_vars_total, const char *who);
int check_bitarray(const pa_bitarray *a, const std::vector<int64_t> &dims, const char *who);

struct Workspace {
    void *ptr = nullptr;
    size_t cap = 0;
    bool external = false;
    int ensure(size_t bytes);
    ~Workspace();
};

// ---------------------------------------------------------------- planning
// Cluster tree node.  Leaves are relations; internal nodes are pairwise
// generalized array multiplications whose output pack is Q (Def.
// "efficient_factorization": the cluster's links also used outside it).
struct Node {
    int leaf = -1;                // relation index, or -1
    int c0 = -1, c1 = -1;         // children (internal)
    uint64_t q = 0;               // output variables
    uint32_t leaves = 0;          // relations under this node
};

struct Tree {
    std::vector<Node> nodes;      // leaves first (node i = relation i), then merges
    int root = -1;
    std::vector<int> merges;      // PA_ORDER_GIVEN format
    double cost = 0.0;            // sum of node costs (eqn naive_cost)
    double predicted_us = 0.0;    // learned order: the model's predicted total step time
    bool learned_fallback = false;  // learned order: the exhaustive optimum replaced the model's tree
};

struct SysInfo {
    int n_vars = 0, n_rel = 0;
    std::vector<int64_t> res;                 // per variable
    std::vector<uint64_t> rel_vars;           // bitmask per relation
    std::vector<std::vector<int>> rel_list;   // declared order per relation
    uint64_t exposed = 0;
    std::vector<int> exposed_list;
    // measured log2 density of each relation's plot (set cells / cells;
    // empty: not measured, the features then use an analytic estimate)
    std::vector<double> leaf_log2d;
};

int build_sysinfo(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, SysInfo &si);
double mask_cost(uint64_t m, const SysInfo &si);      // product of resolutions
uint64_t q_of(uint32_t cluster, const SysInfo &si);   // intermediate pack of a set of relations
int tree_from_merges(const SysInfo &si, const std::vector<int> &merges, Tree &t);
int plan_greedy(const SysInfo &si, Tree &t);
int plan_exhaustive(const SysInfo &si, Tree &t);
int plan_learned(const SysInfo &si, const pa_model *model, Tree &t);

// ---------------------------------------------------------------- op list
enum OpKind { OP_CONTRACT = 0, OP_GEMM = 1, OP_FILL = 2, OP_GATHER = 3, OP_COUNT = 4, OP_LIST = 5, OP_FUSED = 6 };

constexpr int kBufOutput = -2;

struct Op {
    OpKind kind = OP_CONTRACT;
    int mode = kModeBits;         // contract mode
    int a = -1, b = -1, c = -1;   // buffer ids (kBufOutput = caller's output)
    int flag = -1;                // sparse pass (OP_COUNT, OP_GATHER: b is the Bt plot) and its
                                  // MFMA contraction: the two-word buffer of A's set-bit count
    GatherArgs gg{};              // OP_COUNT, OP_GATHER (pointers patched at execution)
    // OP_LIST (a: the pass's A, c: the list buffer) and OP_FUSED (a: the list
    // buffer, b: BtX, flag: BtY); pointers patched at execution from word
    // offsets into the list buffer: OP_LIST entries and meta words in
    // sub[0..1], OP_FUSED X's in sub[0..1] and Y's in sub[2..3]
    RowListArgs rl{};
    FusedArgs fu{};
    int64_t sub[6] = {0, 0, 0, 0, 0, 0};
    int64_t fargs_off = -1;       // OP_FUSED: byte offset of a one-step table in the workspace (per-op launches)
    Layout la, lb, lc;
    std::vector<int> kvars;
    ContractArgs ca{};            // pointers patched at execution
    std::vector<int64_t> ktab;    // streaming modes: (A, B) word offsets of latent entries
    int64_t ktab_off = -1;        // byte offset of ktab in the workspace
    GemmArgs ga{};
    int64_t fill_words = 0;
    double macs = 0.0;            // product of the step's link resolutions
    double dense_macs = 0.0;      // sparse pass: the MACs of the contraction it computes (its
                                  // dense equivalent; counted in macs only without a fallback)
    int node = -1;
    std::string describe() const;
};

// Pairwise contractions an op computes, as counted in reports: a fused
// pass pair computes three (its two passes and their streamed contraction);
// projections of one operand, fills, count and row-list steps, and a sparse
// pass whose MFMA contraction is counted, none.
inline int counted_steps_of(const Op &op) {
    if (op.kind == OP_FUSED) return 3;
    if (op.kind == OP_FILL || op.kind == OP_COUNT || op.kind == OP_LIST || (op.kind == OP_GATHER && op.flag >= 0) ||
        op.b == -1)
        return 0;
    return 1;
}

struct PlotItem {
    int rel = -1;
    int buf = -1;
    std::vector<int> storage;     // storage axis s holds declared variable storage[s]
    Layout layout;
};

struct pa_plan_impl;

}  // namespace pa

struct pa_plan;
namespace pa {
int build_plan(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts, pa_plan *P);
int upload_plan(pa_plan *P);
int exec_steps(pa_plan *P, const std::vector<void *> &outs, hipStream_t s, int *launches);
int plan_workspace_cap(size_t *cap);
// The log2 density of every relation's plot, per system, measured on the
// current device (all relations of all systems plotted in one batch, their
// set cells counted; synchronizes).  A system with an invalid relation gets
// an empty list (planning reports the error).
int measure_leaf_densities(const pa_system *systems, int32_t n_sys, const pa_opts &o,
                           std::vector<std::vector<double>> &ld);
int time_groups(pa_plan *P, int32_t reps, double *ms, int32_t *kind, double *macs, int32_t cap, hipStream_t s);
int set_wait_limit(pa_plan *P, int64_t polls);
int autotuned_opts(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed, const int32_t *n_exposed,
                   pa_opts &o);
void make_groups(pa_plan *P);
// The single persistent launch's tables from the groups: chunk sizes (about
// one chunk per workgroup and group), chunk bases, items per level; written
// to the workspace.
int upload_pgroups(pa_plan *P);
struct ContractLayouts {
    std::vector<int64_t> res;          // length per variable label (-1: unused)
    std::vector<int> av, bv, ov;       // variables of A, B and the output
    uint64_t outm = 0;                 // output variables as a mask
    Layout la, lb, lc;
};
int contract_layouts(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                     const int32_t *out_vars, int32_t n_out, bool has_c, ContractLayouts &cl);
int contract_impl(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                  const int32_t *out_vars, int32_t n_out, pa_bitarray *C, const pa_opts *opts, void *stream,
                  int64_t *tab_dev, int64_t tab_cap);
}  // namespace pa

struct pa_plan {
    pa::SysInfo si;
    pa::Tree tree;
    std::vector<pa::PlotItem> plots;
    std::vector<pa::Op> ops;
    std::vector<int64_t> buf_off;     // byte offsets into the workspace
    std::vector<int64_t> buf_words;
    std::vector<pa::Layout> buf_layout;
    size_t tables_off = 0, tables_bytes = 0, ws_bytes = 0;
    size_t plotrel_off = 0, plotrel1_off = 0, counters_off = 0, popcnt_off = 0;
    size_t steps_off = 0, pgroups_off = 0, levels_off = 0, state_off = 0;
    std::vector<pa::PlotRel> plotrel_host;    // records with prefix tile bases (fused launch)
    std::vector<pa::PlotRel> plotrel1_dev;    // device-pointer records with zero tile bases
    std::vector<pa::PStep> steps_host;        // persistent executor (device pointers, output patched)
    std::vector<std::pair<int, int>> step_out_refs;   // (step, output index): steps writing a caller's output
    std::vector<int> step_level;              // per sorted step
    int64_t n_items = 0;
    int per_op = 0, graph = 0, single_launch = 0, persist_wg = 0, plot_strip = 0, contract_units = 0, gemm_split = 512, gemm_path = 0;
    int sparse_pass = 0, sparse_max_density = 64;
    bool fuse_passes = false;          // sparse_pass 3: pairs of passes fused into their streamed step
    struct Group {
        int kind, mode, first, count;
        int64_t t0, t1;
        int flags;         // MFMA steps of the group that follow a sparse pass
    };
    std::vector<Group> groups;                // level-synchronous executor
    // the single persistent launch's group table (device, at pgroups_off),
    // and per level its item count then its done counter (at levels_off)
    int n_pgroups = 0, n_levels = 0;
    int64_t n_chunks = 0;
    std::vector<double> step_macs;            // per sorted step (0 for plots and fills)
    std::vector<void *> last_outs;
    hipGraph_t graph_h = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<void *> graph_outs;
    hipStream_t graph_stream = nullptr;
    hipStream_t last_stream = nullptr;        // stream of the last execution (has_run)
    bool has_run = false;
    double total_macs = 0.0;
    std::vector<unsigned char> tables_host;   // uploaded once
    pa::Workspace ws;
    std::vector<double> leaf_log2d;            // measured plot densities to plan with (opts->measure_density)
    pa::PlotCounters *counters_dev = nullptr;   // set by a batch: the system's counters in the batch's
                                                // table (else the plan's own, at counters_off)
    int precision = PA_PLOT_FP32_ESCALATE;
    int plot_rule = PA_RULE_CORNER;
    double tolerance = 0.0;
    int audit = 0, timing = 0, plain = 0;
    int device = 0;
    int64_t corners = 0, total_tiles = 0;
    int n_rel_plots = 0;
    bool uploaded = false;
    double t_plan_ms = 0.0;
    pa::Layout out_layout;
    std::vector<hipEvent_t> op_events;     // timing == 2: 2 per op + 2 for plotting
    bool op_events_recorded = false;
    bool timing_active = false;
    ~pa_plan();
};
