// Internal definitions shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa.h"

namespace pa {

constexpr int kMaxD = PA_MAX_DEGREE;
constexpr int kMaxA = PA_MAX_ARITY;
constexpr int kDense = (kMaxD + 1) * (kMaxD + 1) * (kMaxD + 1);
constexpr int kMaxDim = PA_MAX_DIMS;
constexpr int kLineFloats = kMaxD + 2;          // a_0..a_d, E per corner line
constexpr int kMaxTileLines = 160;              // corner lines of a plot tile with one line per thread
// corner lines of a trivariate corner tile whose threads walk the fixed axis
// (lines built in rounds; their FP64 coordinates are not kept in LDS)
constexpr int kMaxWalkLines = 648;
constexpr int kMaxWalkFixed = 4;                // fixed-axis cells a thread of such a tile walks
constexpr int kMaxWalkStrip = 8;                // walk-axis cells of its strip
// LDS of a plot tile: the line table (floats), then as doubles the
// declared-order coefficient table and the FP64 coordinates (two per line)
// of the tile's corner lines
// (for the fixed-axis-walking tiles also each thread's cell masks of its
// previous fixed-axis line: 2 (kMaxWalkStrip + 1) words per thread)
constexpr int kPlotLineWords = (kMaxWalkLines * kLineFloats + 2 * (kMaxWalkStrip + 1) * 256 + 1) / 2 * 2;
constexpr int kPlotLdsWords = kPlotLineWords + 2 * (kDense + 2 * kMaxTileLines);
static_assert(kMaxTileLines <= 256, "one corner line per thread of a 256-thread plot tile");

// One relation to plot.  The relation's declared variables x_0..x_{n-1} are
// stored on storage axes in the order perm: storage axis s holds declared
// variable perm[s]; the last storage axis is the bit-packed one.
//
// Plot tiles (one 256-thread workgroup each): tw words along the packed axis
// x (ta cells of storage axis 0 when n == 3) x (tb strips of s cells along the
// walk axis, storage axis n-2).  A thread walks its strip, so each corner
// line of the strip is evaluated once; the tile's line coefficients are built
// cooperatively in LDS.
struct PlotCounters {
    unsigned long long flagged;
    unsigned long long disagree;
    unsigned long long disagree_unflagged;
    unsigned long long pad;
};

enum PlotRule { kRuleCorner = 0, kRuleCenter = 1 };

struct PlotRel {
    int n, d, mode, audit;
    int rule;                  // kRuleCorner: corner sampling; kRuleCenter: sample in the pixel centre
    int target;                // f = 0 (0), f <= 0 (1), f < 0 (2)
    double eps;                // kRuleCenter: the tolerance
    int perm[kMaxA];
    int res[kMaxA];            // resolution per storage axis
    int64_t row_words;
    // corner k of storage axis s is lo[s] + k * step[s] in FP64 (a product
    // and a sum, each rounded), its FP32 copy the nearest float to that
    double lo[kMaxA], step[kMaxA];
    double vmax;               // upper bound of |x| on the packed storage axis
    double ebound;             // (gamma_{2d+1} + 2^-40)(1 + 2^-30): the FP32 line bound's factor of S
    double vpow[kMaxD + 2];    // max(1, vmax)^t, t = 0..d+1
    double coef[kDense];       // dense table c[e0 + (d+1)*(e1 + (d+1)*e2)], declared exponents
    uint32_t *out;
    PlotCounters *counters;    // escalation counters of the relation's system (null: the launch's)
    int tw, ta, tb, s;
    int walk_fixed;            // trivariate corner tiles: a thread walks ta fixed-axis cells (tw x tb threads)
    int64_t tiles_w, tiles_walk, tiles_fixed, n_tiles;
    int64_t tile_base;         // prefix over relations of n_tiles (multi-relation launches)
};



// Division by a value fixed at plan time, for 0 <= n < 2^31 and
// 1 <= d < 2^31: q = floor(n * m / 2^(31 + s)) with s = ceil(log2 d) and
// m = ceil(2^(31+s) / d) < 2^32 (Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994).  The error term
// n (m d - 2^(31+s)) / (d 2^(31+s)) is below 2^-s <= 1/d, so the floor is
// exact.
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint64_t d) {
    FastDiv f;
    f.d = (uint32_t)d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)(((1ull << (31 + s)) + d - 1) / d);
    return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv &f) {
    return (uint32_t)(((uint64_t)n * f.m) >> (31 + f.s));
}

// General strided bitwise contraction C(out) = OR_k A AND B.  Each variable of
// the output or of the latent set has, per operand, either a word stride
// (non-packed axis of that operand, 0 if absent) or is that operand's packed
// axis (then it indexes bits).  B == nullptr means B is all ones.
enum ContractMode { kModeBits = 0, kModeStreamK = 1, kModeStreamW = 2 };

struct ContractArgs {
    const uint32_t *A, *B;
    uint32_t *C;
    int nout;                       // output rank (0: one-bit output)
    int64_t out_dim[kMaxDim];       // output dims in layout order, last packed
    int64_t c_row_words;
    int64_t a_str[kMaxDim], b_str[kMaxDim];   // word strides of output vars
    int a_pk_out, b_pk_out;         // output index that is A's / B's packed axis, or -1
    int nk;                         // latent variables
    int64_t k_dim[kMaxDim];
    int64_t ka_str[kMaxDim], kb_str[kMaxDim];
    int a_pk_k, b_pk_k;             // latent index that is A's / B's packed axis, or -1
    int64_t a_row_words, b_row_words;
    int64_t n_out_rows;             // product of out_dim except the last
    // streaming modes: word offsets (A, B) of every latent entry except the
    // packed latent axis (mode K), precomputed on the host
    const int64_t *ktab;
    int64_t nktab;
    // stream mode W: an operand without the output's packed variable
    // contributes one bit per output row (its packed variable is an output
    // variable), broadcast over the word
    int a_bcast, b_bcast;
    // divisions by out_dim[i], by the output row length in bits and in
    // words (output rows and row offsets are below 2^31, checked on the host)
    FastDiv fd_dim[kMaxDim];
    FastDiv fd_rowbits, fd_rowwords;
    // stream mode K: a wave's 64 output bits are tq consecutive output rows
    // x 64/tq consecutive bits (tq = 1, 2, 4, 8), so that both operands are
    // read in long runs when one is contiguous along the packed output
    // variable and the other along the last row variable; fd_segs divides a
    // block index by the row's 64/tq-bit segments
    int tq;
    FastDiv fd_segs;
};

// Work units of a contraction: output bits (rows padded to whole groups of
// tq in stream mode K), or output words in stream mode W.
inline int64_t contract_units(const ContractArgs &a, int mode) {
    if (mode == kModeStreamW) return a.n_out_rows * a.c_row_words;
    if (a.nout == 0) return 64;
    const int64_t tq = a.tq > 1 ? a.tq : 1;
    return (a.n_out_rows + tq - 1) / tq * tq * a.c_row_words * 32;
}

// Dense Boolean GEMM in canonical layout:
//   A[b][m][k], B[b][n][k] with the k vector contiguous (Kw words, bits),
//   C[b][m][n] where n = (no, j): no in [0, No) outer, j in [0, rn) packed.
struct GemmArgs {
    const uint32_t *A, *B;
    uint32_t *C;
    int64_t nbatch, M, No, rn, Kw;
    int64_t rwc;              // C row words (2*ceil(rn/64))
    int64_t sA_b, sB_b, sC_b; // batch strides (words)
    int64_t tiles_m, tiles_n; // 128-row and 128-column tiles (N in padded coordinates)
    int64_t kchunk;           // words per K split (multiple of 8)
    int ksplit;               // >1: partial results OR-ed with atomics into zeroed C
    const uint32_t *dense;    // non-null: the tiles run only if *dense != 0, written by the
                              // contraction's sparse pass when A is too dense for it
    int path;                 // operand path: 0 = K chunks staged in LDS, 128 x 128 tiles;
                              // 1 = waves load K chunks straight into registers (no LDS);
                              // 2 = staged in LDS, 256 x 128 tiles (tiles_m counts 256 rows);
                              // 3 = 256 x 128 tiles with A operands kept in registers across
                              //     a workgroup's tiles (K <= 256 bits, no split)
    // divisions of the tile index (below 2^31) and of N coordinates by the
    // padded C row length in bits (below 2^31), checked on the host
    FastDiv fd_ksplit, fd_tiles_n, fd_tiles_m, fd_wc;
};


// Sparse pass of a canonical Boolean GEMM (a row gather): output row r =
// (b, m) is the OR, over the set bits k of A row r, of row k of Bt[b], which
// holds B with the n variables packed (the layout of an output row).  Bit
// `bit` of A word w = ko * rwk + wp is k = ko * rkp + 32 wp + bit (ko indexes
// the latent variables before the packed one, rkp is the packed one's
// resolution, rwk its row words).  A count step first writes the set bits
// of A as nparts partial sums (one per wave of its tiles: re-running it
// changes nothing); the pass runs iff their total is at most max_total (A
// sparse enough that reading one Bt row per set bit costs less than the
// MFMA kernel, which runs in the other case: every wave of the pass writes
// the decision to *dense).  A wave handles 2048 words of one output row.
struct GatherArgs {
    const uint32_t *A, *Bt;
    uint32_t *C;
    uint32_t *parts, *dense;
    int64_t nparts;
    int64_t rows;             // nbatch * M
    int64_t M, Kw, rwk, rkp, Nw;
    int64_t sBt_b;            // Bt words per batch entry
    int64_t chunks;           // 2048-word chunks per output row
    int64_t max_total;        // the pass runs iff the set bits of A are at most this
    FastDiv fd_chunks, fd_M;  // divisions of wave-tile indices (below 2^31, host check)
};

constexpr int64_t kCountTileWords = 8192;    // A words per tile of a count step (4 partial sums)

// Two sparse passes read only by one streamed contraction (mode K), fused
// so that their outputs are never stored.  With output out[p][q] (q packed),
// latent entries s and the packed latent variable t (words w):
//   out[p][q] = OR_{s, w} X[q][s][p][w] AND Y[p][s][q][w]
//   X[q][s][p][.] = OR over set bits k of AX row (q, s) of BtX[k][p][.]
//   Y[p][s][q][.] = OR over set bits k of AY row (p, s) of BtY[k][q][.]
// (eqn GAM for the contraction, the two passes its operands).  A row-list
// step turns every A row into the list of its set bits; a fused tile
// stages the rows of BtX for 8 p and of BtY for 8 q in LDS and gathers.
//
// Row lists: rows are taken in groups of 8 consecutive values of the row's
// output variable o (o-block ob) for one s: group g = ob * n_s + s, list
// row 8 g + i for o = 8 ob + i.  List row r holds its set bits k as the
// 16-bit LDS row indices lbase + k, in any order, in entries r cap .. r cap +
// m - 1, m the largest count of the group's rows (the group's meta word),
// padded with the all-zero row zrow up to m (cap is
// a multiple of 8: every list row starts 16-byte aligned and its entries
// 0..7 are one 16-byte load; those from m on are never read).  Rows with
// o >= n_o have no set bits.
struct RowListArgs {
    const uint32_t *A;        // the pass's A operand: row (o, s) at (o ro + s rs) Kw words
    uint16_t *ent;            // cap entries per list row
    uint32_t *meta;           // one word per group
    int64_t n_o, n_s, ro, rs;
    int64_t Kw, rwk, rkp;     // A row words; bit b of word w = ko rwk + wp is k = ko rkp + 32 wp + b
    int lbase, zrow;
    int64_t cap;              // entries per list row: the latent bits rounded up to a multiple of 4
    int64_t n_rows;           // 8 ceil(n_o / 8) n_s list rows
    FastDiv fd_s;             // division by n_s (of group indices below 2^31)
};

constexpr int kListRowsPerTile = 32;                  // a row-list tile: 256 threads, 8 to a row

constexpr int kFusedRows = 513;                        // LDS rows of a fused tile: BtX, BtY, the zero row
// LDS row pitch in words: 8 words of t x 8 values
constexpr int kFusedPitch = 64;
constexpr uint32_t kFusedRowBytes = 4u * kFusedPitch;
// a header row (the latent-entry counter at LDS address 0, where ds_append
// finds it with M0 = 0, then the tile's 8 output bytes, a word each), then
// the rows
constexpr int kFusedLdsWords = (kFusedRows + 1) * kFusedPitch;

// A fused tile: 8 p (block pb) x 8 q (block qb); tile = pb n_qb + qb.  Bt
// rows hold n_o x rwt words (rwt <= 8: the o-th 8-word slot of a staged LDS
// row is padded with zeros).
struct FusedArgs {
    const uint32_t *BtX, *BtY;
    const uint16_t *entX, *entY;
    const uint32_t *metaX, *metaY;
    uint32_t *C;
    int64_t n_p, n_q, n_s;
    int64_t btX_rw, btY_rw;   // Bt row words: n_p rwt, n_q rwt
    int rwt, kX, kY;          // words of t; LDS rows of BtX (0..kX-1) and BtY (kX..kX+kY-1)
    int64_t capX, capY;       // list entries per row of X, Y
    int64_t c_rw;             // output row words
    int64_t n_qb, n_tiles;    // ceil(n_q / 8); ceil(n_p / 8) n_qb
};

// Wave-tiles of a sparse pass (2048 words of one output row each).
__host__ __device__ inline int64_t gather_wave_tiles(const GatherArgs &g) { return g.rows * g.chunks; }

// One step of the persistent executor: a plot, a GEMM, a contraction, a
// fill or a sparse pass, cut into tiles.  Steps are listed so that every
// step's producers come earlier; a tile starts once all tiles of the step's
// producers are done.
enum StepKind {
    kStepPlot = 0, kStepGemm = 1, kStepContract = 2, kStepFill = 3, kStepGather = 4, kStepCount = 5,
    kStepList = 6, kStepFused = 7
};

struct PStep {
    int kind, mode;
    int ndep, dep[4];
    int64_t n_tiles, tile_base;
    int64_t units, per_tile;        // contract: output bits/words; fill: words
    PlotRel plot;
    GemmArgs gemm;
    ContractArgs ca;
    GatherArgs gather;              // sparse pass: tiles of 4 wave-tiles; count: of kCountTileWords words
    RowListArgs list;               // row lists: tiles of 256 list rows
    FusedArgs fused;                // fused pass pair: one tile per workgroup of 1024 threads
    uint32_t *fill_ptr;
};

struct PersistState {
    unsigned long long queue;       // next work item
    unsigned int abort;             // set when a dependency wait exceeds its bound
    unsigned int pad;
    long long wait_limit;           // polls per dependency wait (host-set; < 0: give up at once)
};

constexpr long long kDefaultWaitLimit = 1ll << 26;

// One group of the persistent launch: steps first .. first + count - 1 of
// one kind and mode at one dependency level, items [t0, t1), run in chunks
// of `chunk` items; its chunks are numbered from cbase in the launch.
struct PGroup {
    int kind, mode, first, count, level, pad;
    int64_t t0, t1, chunk, cbase;
};

// Kernel launchers (pa_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_plot(const PlotRel *d_rels, int nrel, int64_t total_tiles, bool center, PlotCounters *d_counters,
                       hipStream_t s);
hipError_t launch_contract(const ContractArgs &a, int mode, hipStream_t s);
// The latent-entry table of a streamed contraction (the host's ordering:
// entry e lists the A and B word offsets of the e-th latent index tuple, last
// latent variable fastest, the packed one left out in mode K), written by a
// kernel into tab (2 * n int64).
hipError_t launch_ktab(const ContractArgs &a, int mode, int64_t *tab, int64_t n, hipStream_t s);
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
// Count semiring: C[b][m][n] = number of k with A[b][m][k] and B[b][n][k]
// (canonical layout, 128 x 128 tiles; C dense uint32 with element
// ((b M + m) No + no) rn + j; with a K split the parts add into a zeroed C).
hipError_t launch_gemm_count(const GemmArgs &g, hipStream_t s);
// Count semiring, any layouts: C[e] (dense uint32, row-major over the output
// variables) = number of latent entries where A and B are both set.
hipError_t launch_count_bits(const ContractArgs &a, int64_t n_elems, hipStream_t s);
hipError_t launch_gather(const GatherArgs &g, hipStream_t s);
hipError_t launch_count(const GatherArgs &g, hipStream_t s);
hipError_t launch_row_list(const RowListArgs &l, hipStream_t s);
// One fused step (a one-step table in device memory, tile_base 0; C
// replaces its output pointer).
hipError_t launch_fused(const PStep *d_step, int64_t n_tiles, uint32_t *C, hipStream_t s);
hipError_t launch_fill(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_popcount(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t s);
// LDS read-rate reference: blocks workgroups of 1024 threads, each reading
// iters x 8 x 16 KiB of LDS; out holds blocks x 1024 words.
hipError_t launch_lds_rate(uint32_t *out, int blocks, int iters, hipStream_t s);
hipError_t launch_tile_popcount(const uint32_t *p, int64_t rows, int64_t rw, int tile_rows, int tile_words,
                                uint32_t *out, hipStream_t s);
// The single persistent launch: chunks of the groups (table of ngroups
// entries, nchunks chunks in all), level_items[L] items in level L,
// level_done[L] counts the done ones (reset by launch_persist_reset).
hipError_t launch_persist(const PStep *d_steps, const PGroup *d_groups, int ngroups, int64_t nchunks,
                          const int64_t *level_items, unsigned long long *level_done, PersistState *state,
                          PlotCounters *counters, int n_workgroups, hipStream_t s);
hipError_t launch_persist_reset(PersistState *state, unsigned long long *level_done, int nlevels, hipStream_t s);
// Steps first..first+count-1 (tiles t0..t1-1) of one kind and mode (plots:
// mode 1 = centre rule); flags: some of the MFMA contractions among them have
// a sparse pass (and may be skipped).
hipError_t launch_group(int kind, int mode, const PStep *d_steps, int first, int count, int64_t t0, int64_t t1,
                        int flags, PlotCounters *counters, hipStream_t s);
int persist_default_workgroups();

}  // namespace pa
