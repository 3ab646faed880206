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

// One relation to plot.  The relation's declared variables x_0..x_{n-1} are
// stored on storage axes in the order perm: storage axis s holds declared
// variable perm[s]; the last storage axis is the bit-packed one.
struct PlotRel {
    int n, d;                 // arity, degree
    int perm[kMaxA];
    int res[kMaxA];           // resolution per storage axis
    int mode;                 // PA_PLOT_FP32_ESCALATE or PA_PLOT_FP64
    int audit;
    int64_t row_words;
    const double *coef;       // dense table c[e0 + (d+1)*(e1 + (d+1)*e2)], declared exponents
    const double *ax[kMaxA];  // FP64 pixel boundaries per storage axis (res+1 entries)
    const float *axf[kMaxA];  // RN-to-FP32 copies
    double vmax;              // upper bound of |x| on the packed storage axis
    uint32_t *out;
    float *lines;             // FP32 line table: (d + 2) floats per corner line
    int64_t n_rows;           // product of res over non-packed storage axes
    int64_t n_lines;          // product of (res + 1) over non-packed storage axes
    int64_t word_base;        // prefix over relations of n_rows * row_words
    int64_t line_base;        // prefix over relations of n_lines
};

struct PlotCounters {
    unsigned long long flagged;
    unsigned long long disagree;
    unsigned long long disagree_unflagged;
    unsigned long long pad;
};

// General strided bitwise contraction C(out) = OR_k A AND B.  Each variable of
// the output or of the latent set has, per operand, either a word stride
// (non-packed axis of that operand, 0 if absent) or is that operand's packed
// axis (then it indexes bits).  B == nullptr means B is all ones.
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
};

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
};

// Kernel launchers (pa_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_plot(const PlotRel *d_rels, int nrel, int64_t total_lines, int64_t total_words,
                       int mode_any_fp32, PlotCounters *d_counters, hipStream_t s, int *n_launches);
hipError_t launch_contract(const ContractArgs &a, int mode, hipStream_t s);
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);
hipError_t launch_fill(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_popcount(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t s);

enum ContractMode { kModeBits = 0, kModeStreamK = 1, kModeStreamW = 2 };

}  // namespace pa
