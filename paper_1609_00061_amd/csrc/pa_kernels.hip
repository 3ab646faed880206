// gfx950 kernels of the pixel array method: corner plotting with FP32
// evaluation and FP64 escalation, bitwise OR-of-AND contractions, a dense
// Boolean contraction on fp4 MFMA with fp32 accumulation (the count semiring
// on int8 MFMA with int32 accumulation), and a persistent work-queue
// executor that runs all of them as tiles of one launch.
//
// Build flags (see build.py): -O3 --offload-arch=gfx950 -ffp-contract=off
// (no implicit FMA: every fused multiply-add below is an explicit fma/fmaf).
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "pa_internal.h"

namespace pa {

// ------------------------------------------------------------------ helpers
// Pointers read from step tables are generic to the compiler, which would
// access them with FLAT instructions (counted on both the vector-memory and
// the LDS counters, so an LDS wait also waits for every load in flight).
// Every array the kernels touch is in device global memory: accesses go
// through address-space-1 pointers (global_load / global_store).
#define PA_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ PA_G T *gp(T *p) {
    return (PA_G T *)p;
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Blocks for `total` threads, capped (the kernels loop over the rest).
static dim3 grid_for(int64_t total) {
    int64_t blocks = (total + 255) / 256;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    if (blocks < 1) blocks = 1;
    return dim3((unsigned)blocks);
}

// Canonical FP64 value of a relation at a point given in DECLARED variable
// order: nested Horner, last declared variable outermost, fma at every step.
// c is the dense table c[e0 + (d+1)*(e1 + (d+1)*e2)] (its LDS copy).
__device__ double canon_eval(const double *__restrict__ c, int n, int d, const double *x) {
    const int D1 = d + 1;
    if (n == 1) {
        double p = c[d];
        for (int i = d - 1; i >= 0; --i) p = fma(p, x[0], c[i]);
        return p;
    }
    if (n == 2) {
        double p = c[D1 * d];                          // A_d = coefficient of x1^d
        for (int i = d - 1; i >= 0; --i) {
            const int top = d - i;                     // A_i(x0) has degree d - i
            double a = c[top + D1 * i];
            for (int j = top - 1; j >= 0; --j) a = fma(a, x[0], c[j + D1 * i]);
            p = fma(p, x[1], a);
        }
        return p;
    }
    // n == 3: A_i(x0, x1) = sum_k B_ik(x0) x1^k, B_ik(x0) = sum_j c_jki x0^j
    auto Bik = [&](int i, int k) {
        const int top = d - i - k;
        const double *row = c + D1 * (k + D1 * i);
        double b = row[top];
        for (int j = top - 1; j >= 0; --j) b = fma(b, x[0], row[j]);
        return b;
    };
    auto Ai = [&](int i) {
        const int top = d - i;
        double a = Bik(i, top);
        for (int k = top - 1; k >= 0; --k) a = fma(a, x[1], Bik(i, k));
        return a;
    };
    double p = Ai(d);
    for (int i = d - 1; i >= 0; --i) p = fma(p, x[2], Ai(i));
    return p;
}

struct PlotCount {
    unsigned long long flagged = 0, dis = 0, dis_unf = 0;
};

// ------------------------------------------------------------ plot: tiles
// A tile (256 threads) covers tw words of the packed axis x tb strips of s
// cell rows along the walk axis (storage axis n-2) x ta cells of the fixed
// axis (n == 3).  A thread owns one 32-cell word of one strip: it evaluates
// the 33 corners of the word on every corner line bounding its strip (FP32,
// coordinates held in registers), so a corner line is evaluated once per
// strip.  (Bivariate relations use the lane-strip tiles of plot_tile2.)
// The tile first stages the coefficient table (carried by the plot record,
// declared order) in LDS with the FP64 coordinates of its corner lines, and
// builds the FP32 restriction and bound of each corner line there (FP64, one
// line per thread).  Corner coordinates are formed from the axis origin and
// step, not loaded: the record is the only memory a tile reads.

// Fields of a relation a tile uses, held in registers (the record itself is
// in global memory, which the tile's output stores could alias).
struct PlotView {
    int n, d, mode, audit;
    int target;                // f = 0 (0), f <= 0 (1), f < 0 (2)
    double eps;                // centre rule: the tolerance
    int perm0, perm1, perm2;   // declared variable of storage axis 0, 1, 2
    int res0, res1;            // resolutions of storage axes 0 and 1
    int rwalk, rp;             // walk axis (storage n-2; 1 if n == 1) and packed axis
    int64_t row_words;
    const PA_G double *coef;        // the record's dense coefficient table
    double lo0, st0, lo1, st1;      // corners of storage axes 0 and 1: lo + k * st
    double lop, stp;                // corners of the packed axis
    double ebound;                  // factor of S in the FP32 line bound
    const PA_G double *vpow;        // max(1, vmax)^t
    PA_G uint32_t *out;
};

// FP64 corner coordinate lo + k * st: the product, then the sum, each
// rounded (the build does not contract them into an fma), as on the host.
__device__ __forceinline__ double corner_coord(double lo, double st, int64_t k) {
    const double t = (double)k * st;
    return lo + t;
}

// FP64 centre of pixel k: lo + (k + 1/2) * st, the product and the sum each
// rounded, as on the host.
__device__ __forceinline__ double center_coord(double lo, double st, int64_t k) {
    const double t = ((double)k + 0.5) * st;
    return lo + t;
}

__device__ __forceinline__ PlotView plot_view(const PlotRel &R) {
    PlotView v;
    v.n = R.n;
    v.d = R.d;
    v.mode = R.mode;
    v.audit = R.audit;
    v.target = R.target;
    v.eps = R.eps;
    v.perm0 = R.perm[0];
    v.perm1 = R.perm[1];
    v.perm2 = R.perm[2];
    v.res0 = R.res[0];
    v.res1 = R.res[1];
    const int n = v.n;
    v.rp = n == 1 ? R.res[0] : (n == 2 ? R.res[1] : R.res[2]);
    v.rwalk = n == 1 ? 1 : (n == 2 ? R.res[0] : R.res[1]);
    v.row_words = R.row_words;
    v.coef = gp(&R.coef[0]);
    v.lo0 = R.lo[0];
    v.st0 = R.step[0];
    v.lo1 = R.lo[1];
    v.st1 = R.step[1];
    v.lop = n == 1 ? R.lo[0] : (n == 2 ? R.lo[1] : R.lo[2]);
    v.stp = n == 1 ? R.step[0] : (n == 2 ? R.step[1] : R.step[2]);
    v.ebound = R.ebound;
    v.vpow = gp(&R.vpow[0]);
    v.out = gp(R.out);
    return v;
}

// Declared-order coordinates from storage-axis coordinates (no dynamically
// indexed private arrays).
__device__ __forceinline__ void decl_point(const PlotView &V, double s0, double s1, double s2, double *xd) {
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double t = 0.0;
        if (V.perm0 == v) t = s0;
        if (V.n > 1 && V.perm1 == v) t = s1;
        if (V.n > 2 && V.perm2 == v) t = s2;
        xd[v] = t;
    }
}

// The dense coefficient table (declared order) for LDS: thread tid < kDense
// loads entry tid, with no dependence on the record's other fields, so the
// load is issued at once.  Loaded first, stored after other work.
__device__ __forceinline__ double load_coefs(const PlotView &V) {
    return (int)threadIdx.x < kDense ? V.coef[threadIdx.x] : 0.0;
}

__device__ __forceinline__ void store_coefs(double c, double *cdl) {
    if ((int)threadIdx.x < kDense) cdl[threadIdx.x] = c;
}

// Strides of the storage exponents in the declared-order table: exponent e
// on storage axis j moves the index by e * D1^perm[j].
struct CoefStrides {
    int m0, m1, m2;
};

__device__ __forceinline__ CoefStrides coef_strides(const PlotView &V) {
    const int D1 = V.d + 1;
    auto st = [&](int v) { return v == 0 ? 1 : (v == 1 ? D1 : D1 * D1); };
    return {st(V.perm0), st(V.perm1), st(V.perm2)};
}

// Coefficients of the relation restricted to one corner line (storage
// coordinates y0, y1 on the non-packed axes), as a polynomial in the packed
// variable, rounded to FP32, and the FP32 error bound E of evaluating them by
// Horner at any corner of the line.
//
// Bound.  Let v be a corner coordinate on the packed axis, v~ = RN32(v),
// a~_t = RN32(a^_t) with a^_t the FP64 sum below, and p^ the FP32 Horner
// value with fma.  Then p^ = sum_t a~_t v~^t (1 + theta_{k_t}), k_t <= d, so
// relative to the exact restriction every monomial carries at most
// d + 1 + t <= 2d + 1 factors (1 + delta), |delta| <= 2^-24 (Higham, Accuracy
// and Stability of Numerical Algorithms, Sec. 3.1 and 5.1):
//   |p^ - f(corner)| <= gamma_{2d+1} * S + (FP64 errors) + (underflow),
//   S = sum_t s_t * max(1, vmax)^t >= sum_m |c_m x^m| and >= every Horner
// partial sum, s_t = sum of |terms| feeding a_t.  All FP64 errors (of a^_t,
// of S, and of the canonical FP64 value) are below 2^-40 * S; underflow of
// FP32 intermediates or of flushed denormals is below 2^-100 (1 + S) V^d.
// A corner is escalated unless |p^| > E (E = +inf when S > 2^126, where
// FP32 could overflow); otherwise |f_exact| > E - gamma S >= |f64 - f_exact|,
// so sign(p^) = sign(f64) != 0.
__device__ void line_coefs(const PlotView &V, const double *cdl, double y0, double y1, float *dst) {
    const int n = V.n, d = V.d;
    const CoefStrides M = coef_strides(V);
    // storage-order entry (e0, e1, e2) of the declared-order table
    auto cst = [&](int e0, int e1, int e2) { return cdl[e0 * M.m0 + e1 * M.m1 + e2 * M.m2]; };
    const double ay0 = fabs(y0), ay1 = fabs(y1);
    // a_t and s_t as Horner polynomials in y0 (and y1): s_t uses |c| and
    // |y|, whose products are the |terms|; the d + 1 chains are independent
    double S = 0.0;
#pragma unroll
    for (int t = 0; t <= kMaxD; ++t) {
        double at = 0.0, st = 0.0;
        if (t <= d) {
            const int top = d - t;     // a_t has degree d - t in the other variables
            if (n == 1) {
                at = cst(t, 0, 0);
                st = fabs(at);
            } else if (n == 2) {
                at = cst(top, t, 0);
                st = fabs(at);
#pragma unroll
                for (int e0 = kMaxD - 1; e0 >= 0; --e0) {
                    if (e0 < top) {
                        const double c = cst(e0, t, 0);
                        at = fma(at, y0, c);
                        st = fma(st, ay0, fabs(c));
                    }
                }
            } else {
                // sum over e1 (Horner in y1) of B_e1(y0) (Horner in y0)
#pragma unroll
                for (int e1 = kMaxD; e1 >= 0; --e1) {
                    if (e1 <= top) {
                        const int tb = top - e1;
                        double b = cst(tb, e1, t), sb = fabs(b);
#pragma unroll
                        for (int e0 = kMaxD - 1; e0 >= 0; --e0) {
                            if (e0 < tb) {
                                const double c = cst(e0, e1, t);
                                b = fma(b, y0, c);
                                sb = fma(sb, ay0, fabs(c));
                            }
                        }
                        at = (e1 == top) ? b : fma(at, y1, b);
                        st = (e1 == top) ? sb : fma(st, ay1, sb);
                    }
                }
            }
            S = fma(st, V.vpow[t], S);
        }
        dst[t] = (t <= d) ? (float)at : 0.0f;
    }
    const double E = V.ebound * S + 0x1p-100 * (1.0 + S) * V.vpow[d + 1];
    float Ef = (float)E;
    if ((double)Ef < E) Ef = nextafterf(Ef, INFINITY);
    // every Horner partial sum is below 2S: with S <= 2^126 nothing overflows
    // FP32; otherwise no corner of the line is certain
    if (!(S <= 0x1p126)) Ef = INFINITY;
    dst[kLineFloats - 1] = Ef;
}

// FP32 pass over the corners k0..k0+kmax of one corner line (coordinates in
// registers), NF Horner steps (NF >= degree; coefficients above the degree
// are zero and fma(0, x, a) = a exactly).  E is +inf when the line's
// magnitude bound allows FP32 overflow: then FP64 decides every corner.
// Otherwise every f is finite (its partial sums stay below 2S <= 2^127) and
// a corner's FP32 sign is certain iff |f| > E (f then nonzero).  The sign
// bits are shifted into a word with one alignbit each (corners taken from 31
// down to 0); certainty is first tested for the whole line with the minimum
// of |f| (two corners per min3), and only a line with some |f| <= E repeats
// the pass to find its uncertain corners.  Out: LE/GE where the sign is
// certain, FL the corners FP64 decides.
// Bits of the 33 corners of a word (corner kk at bit kk of lo, corner 32 in
// hi): 32-bit operations on the common path.
struct Corners {
    uint32_t lo, hi;
};

template <int NF>
__device__ __forceinline__ void line_fp32(const float *ln, const float *xv, const Corners &valid, Corners &LE,
                                          Corners &GE, Corners &FL) {
    float ca[NF + 1];
#pragma unroll
    for (int t = 0; t <= NF; ++t) ca[t] = ln[t];
    const float E = ln[kLineFloats - 1];
    if (!(E < INFINITY)) {
        LE = {0u, 0u};
        GE = {0u, 0u};
        FL = valid;
        return;
    }
    auto value = [&](float x) {
        float f = ca[NF];
#pragma unroll
        for (int t = NF - 1; t >= 0; --t) f = fmaf(f, x, ca[t]);
        return f;
    };
    const float f32 = value(xv[32]);
    const uint32_t sg32 = __float_as_uint(f32) >> 31;
    uint32_t sg = 0;
    float amin = fabsf(f32);
    // four corners at a time, their Horner steps interleaved
#pragma unroll
    for (int kk = 31; kk >= 0; kk -= 4) {
        float f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = ca[NF];
#pragma unroll
        for (int t = NF - 1; t >= 0; --t)
#pragma unroll
            for (int i = 0; i < 4; ++i) f[i] = fmaf(f[i], xv[kk - i], ca[t]);
#pragma unroll
        for (int i = 0; i < 4; ++i) sg = __builtin_amdgcn_alignbit(sg, __float_as_uint(f[i]), 31);
        amin = fminf(fminf(amin, fabsf(f[0])), fabsf(f[1]));
        amin = fminf(fminf(amin, fabsf(f[2])), fabsf(f[3]));
    }
    uint32_t ok = ~0u, ok32 = 1u;
    if (!(amin > E)) {
        // some corner within the bound: the exact certainty bits
        ok = 0u;
#pragma unroll
        for (int kk = 31; kk >= 0; --kk) ok = __builtin_amdgcn_alignbit(ok, __float_as_uint(E - fabsf(value(xv[kk]))), 31);
        ok32 = __float_as_uint(E - fabsf(f32)) >> 31;
    }
    ok &= valid.lo;
    ok32 &= valid.hi;
    LE = {ok & sg, ok32 & sg32};
    GE = {ok & ~sg, ok32 & ~sg32};
    FL = {valid.lo & ~ok, valid.hi & ~ok32};
}

// Corner bits for the target of an inequality: a cell is set iff one of its
// corners satisfies it, so the "some corner f >= 0" half of the sign-change
// test becomes always true and the other half is f <= 0 (target 1) or f < 0
// (target 2: f <= 0 and not f >= 0; a corner with a certain FP32 sign is
// nonzero, an escalated one has its FP64 sign).
__device__ __forceinline__ void apply_target(int target, Corners &LE, Corners &GE) {
    if (target == 0) return;
    if (target == 2) LE = {LE.lo & ~GE.lo, LE.hi & ~GE.hi};
    GE = {~0u, ~0u};
}

// LE/GE bits of the corners k0..k0+kmax of one corner line: ln its FP32
// restriction and bound, ly its FP64 coordinates on the non-packed storage
// axes (walk axis first for n == 2; fixed, walk for n == 3), cdl the
// declared-order coefficient table (all three in LDS); `own` says whether
// this thread counts the line's corners (each corner is counted once).
__device__ __forceinline__ void eval_line(const PlotView &V, const float *ln, const float *xv, const double *ly,
                                          const double *cdl, int k0, int kmax, bool own, Corners &LE, Corners &GE,
                                          PlotCount &cnt) {
    const int n = V.n, rp = V.rp;
    // kmax <= 32 corners past k0 belong to this word
    const Corners valid = {kmax >= 31 ? ~0u : ((2u << kmax) - 1u), kmax >= 32 ? 1u : 0u};
    Corners FL = valid, todo;
    if (V.mode == PA_PLOT_FP32_ESCALATE) {
        if (V.d <= 3) line_fp32<3>(ln, xv, valid, LE, GE, FL);
        else line_fp32<kMaxD>(ln, xv, valid, LE, GE, FL);
        todo = V.audit ? valid : FL;
    } else {
        LE = {0u, 0u};
        GE = {0u, 0u};
        todo = valid;
    }
    if ((todo.lo | todo.hi) == 0u) return;       // the common case: every corner certain in FP32
    const bool last = k0 + kmax == rp;
    const Corners owned = {own ? (kmax >= 32 ? ~0u : ((1u << kmax) - 1u) | (last ? (1u << kmax) : 0u)) : 0u,
                           (own && last && kmax == 32) ? 1u : 0u};
    if (V.mode == PA_PLOT_FP32_ESCALATE) cnt.flagged += __popc(FL.lo & owned.lo) + (FL.hi & owned.hi);
    // FP64 decides the escalated corners (every corner in FP64 mode); in
    // audit mode every corner's FP32 sign is also compared with its FP64 sign
    const double y0 = ly[0], y1 = ly[1];
    uint64_t rest = (uint64_t)todo.lo | ((uint64_t)todo.hi << 32);
    while (rest) {
        const int kk = __ffsll((long long)rest) - 1;
        rest &= rest - 1;
        double xd[3];
        const double xk = corner_coord(V.lop, V.stp, k0 + kk);
        if (n == 1) decl_point(V, xk, 0.0, 0.0, xd);
        else if (n == 2) decl_point(V, y0, xk, 0.0, xd);
        else decl_point(V, y0, y1, xk, xd);
        const double f64 = canon_eval(cdl, n, V.d, xd);
        const bool hi = kk == 32;
        const uint32_t bit = hi ? 1u : (1u << kk);
        const bool flagged = ((hi ? FL.hi : FL.lo) & bit) != 0;
        if (flagged) {
            if (f64 <= 0.0) {
                if (hi) LE.hi |= 1u; else LE.lo |= bit;
            }
            if (f64 >= 0.0) {
                if (hi) GE.hi |= 1u; else GE.lo |= bit;
            }
        }
        if (V.mode == PA_PLOT_FP32_ESCALATE && V.audit) {
            // FP32 value of this corner, recomputed as in line_fp32 (same
            // RN32 coordinate)
            const float x = (float)xk;
            float f = ln[kMaxD];
#pragma unroll
            for (int t = kMaxD - 1; t >= 0; --t) f = fmaf(f, x, ln[t]);
            const int s32 = (f > 0.0f) - (f < 0.0f);
            const int s64 = (f64 > 0.0) - (f64 < 0.0);
            const bool is_owned = ((hi ? owned.hi : owned.lo) & bit) != 0;
            const bool dis = ((s32 != s64) || (f != f) || (f64 != f64)) && is_owned;
            cnt.dis += dis;
            cnt.dis_unf += dis && !flagged;
        }
    }
}

// Bivariate plot tile: 4 words x 64 s cell rows.  Wave v takes word
// 4 t_w + v of every row; lane l takes cell rows b0 + l s .. b0 + l s + s - 1
// and evaluates the corner lines on top of them (s lines).  The line below
// its last row is the next lane's first line (shuffled down); for lane 63 it
// is the tile's last line, which the wave evaluates one corner per lane and
// collects with ballots.  So every corner line is evaluated once per word
// (plus the tile's last line, also evaluated by the next tile).  The 33
// corner coordinates of the word are the same for the whole wave: lane k
// forms corner k and the wave reads them into scalar registers.
__device__ void plot_tile2(const PlotRel &R, int64_t tile, float *lines, double *tabs, PlotCount &cnt) {
    const PlotView V = plot_view(R);
    const double coefs = load_coefs(V);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = R.s, span = 64 * s;
    // tile counts are below 2^31 (checked on the host)
    const uint32_t tiles_w = (uint32_t)R.tiles_w, t = (uint32_t)tile;
    const int64_t t_w = t % tiles_w, t_walk = t / tiles_w;
    const int rwalk = V.rwalk, rp = V.rp;
    const int64_t b0 = t_walk * span;
    const int64_t w = t_w * 4 + wave;
    const bool wave_on = w < V.row_words, pad = w * 32 >= rp;
    const int k0 = (int)(w * 32);
    const int kmax = (pad || !wave_on) ? 0 : min(32, rp - k0);
    // lane k < 33: corner k0 + k of the word (FP64, then the nearest float)
    const int kk_lane = lane < 33 ? lane : 32;
    const double x64 = corner_coord(V.lop, V.stp, (int64_t)k0 + kk_lane);
    const float xk = (float)x64;
    // the tile's corner lines: thread i <= span takes line b0 + i
    double *cdl = tabs, *ly = tabs + kDense;
    const int nlines = span + 1;
    bool lvalid = false;
    double y0 = 0.0;
    if (tid < nlines) {
        lvalid = b0 + tid <= rwalk;
        if (lvalid) y0 = corner_coord(V.lo0, V.st0, b0 + tid);
    }
    store_coefs(coefs, cdl);
    if (tid < nlines) {
        ly[2 * tid] = y0;
        ly[2 * tid + 1] = 0.0;
    }
    __syncthreads();
    if (V.mode == PA_PLOT_FP32_ESCALATE && lvalid) line_coefs(V, cdl, y0, 0.0, lines + tid * kLineFloats);
    __syncthreads();
    if (!wave_on) return;
    float xv[33];
#pragma unroll
    for (int k = 0; k < 33; ++k) xv[k] = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(xk), k));
    // cell masks (cell i: corners i and i + 1) of this lane's own lines
    uint32_t lcq[2] = {0u, 0u}, gcq[2] = {0u, 0u};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int L = lane * s + q;
        if (q < s && !pad && b0 + L <= rwalk) {
            Corners LE, GE;
            eval_line(V, lines + L * kLineFloats, xv, ly + 2 * L, cdl, k0, kmax, true, LE, GE, cnt);
            apply_target(V.target, LE, GE);
            lcq[q] = LE.lo | __builtin_amdgcn_alignbit(LE.hi, LE.lo, 1);
            gcq[q] = GE.lo | __builtin_amdgcn_alignbit(GE.hi, GE.lo, 1);
        }
    }
    // the line below this lane's last row
    uint32_t lcb = (uint32_t)__shfl_down((int)lcq[0], 1), gcb = (uint32_t)__shfl_down((int)gcq[0], 1);
    if (!pad && b0 + span <= rwalk) {
        // the tile's last line, one corner per lane (lanes 0..kmax)
        const bool valid = lane <= kmax;
        const bool owned_line = b0 + span == rwalk;    // no later tile evaluates it
        const bool last_word = k0 + kmax == rp;
        const bool owned = owned_line && (lane < kmax || (lane == kmax && last_word));
        bool lb = false, gb = false, fl = valid;
        float f = 0.0f;
        if (V.mode == PA_PLOT_FP32_ESCALATE) {
            const float *le = lines + span * kLineFloats;
            const float E = le[kLineFloats - 1];
            f = le[kMaxD];
#pragma unroll
            for (int tt = kMaxD - 1; tt >= 0; --tt) f = fmaf(f, xk, le[tt]);
            if (E < INFINITY) {
                const bool ok = fabsf(f) > E;
                fl = valid && !ok;
                lb = valid && ok && f < 0.0f;
                gb = valid && ok && f > 0.0f;
            }
        }
        const bool todo = (V.mode != PA_PLOT_FP32_ESCALATE || V.audit) ? valid : fl;
        if (V.mode == PA_PLOT_FP32_ESCALATE && owned_line) {
            const uint64_t m = __ballot(fl && owned);
            if (lane == 0) cnt.flagged += __popcll(m);
        }
        if (__ballot(todo)) {
            if (todo) {
                double xd[3];
                decl_point(V, ly[2 * span], x64, 0.0, xd);
                const double f64 = canon_eval(cdl, 2, V.d, xd);
                if (fl) {
                    lb = f64 <= 0.0;
                    gb = f64 >= 0.0;
                }
                if (V.mode == PA_PLOT_FP32_ESCALATE && V.audit && owned) {
                    const int s32 = (f > 0.0f) - (f < 0.0f), s64 = (f64 > 0.0) - (f64 < 0.0);
                    const bool dis = (s32 != s64) || (f != f) || (f64 != f64);
                    cnt.dis += dis;
                    cnt.dis_unf += dis && !fl;
                }
            }
        }
        if (V.target == 2) lb = lb && !gb;
        if (V.target != 0) gb = true;
        const uint64_t lm = __ballot(lb), gm = __ballot(gb);
        if (lane == 63) {
            lcb = (uint32_t)(lm | (lm >> 1));
            gcb = (uint32_t)(gm | (gm >> 1));
        }
    }
    const uint32_t vmask = pad ? 0u : (kmax == 32 ? 0xffffffffu : ((1u << kmax) - 1u));
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int64_t row = b0 + lane * s + q;
        if (q < s && row < rwalk) {
            const uint32_t lbot = (q + 1 < s) ? lcq[1] : lcb, gbot = (q + 1 < s) ? gcq[1] : gcb;
            V.out[row * V.row_words + w] = (lcq[q] | lbot) & (gcq[q] | gbot) & vmask;
        }
    }
}

// epsilon-tolerance sample-in-center plot (Def. sample_in_center): a cell
// is set iff the distance from f at its centre to the target subset is at
// most eps -- |f| <= eps for f = 0, f <= eps for f <= 0, f < eps for f < 0 --
// with f the canonical FP64 value at the FP64 centre.  Tiles as plot_tile (tw
// words x tb strips of s rows x ta cells of the fixed axis); a thread owns a
// 32-cell word of a strip and evaluates the centre line of each of its rows
// at the word's 32 centres.  The FP32 value p of a centre differs from the
// FP64 one by at most E (the line bound of line_coefs), so with
// lo = RD32(eps - E) and hi = RU32(eps + E) (each pushed outward past the
// FP64 rounding of the difference) the decision is certain when the
// distance d (|p| or p) has d < lo (set: d64 <= d + E < eps) or d > hi
// (unset: d64 >= d - E > eps); the others, and every centre in FP64 mode,
// are decided by the canonical FP64 value.
__device__ __forceinline__ void center_thresholds(float E, double eps, float &lo, float &hi) {
    if (!(E < INFINITY)) {
        lo = -INFINITY;
        hi = INFINITY;
        return;
    }
    double t = eps - (double)E;
    t -= fabs(t) * 0x1p-50;
    lo = (float)t;
    if ((double)lo > t) lo = nextafterf(lo, -INFINITY);
    double u = eps + (double)E;
    u += fabs(u) * 0x1p-50;
    hi = (float)u;
    if ((double)hi < u) hi = nextafterf(hi, INFINITY);
}

__device__ __forceinline__ bool center_on(int target, double f, double eps) {
    return target == 0 ? fabs(f) <= eps : (target == 1 ? f <= eps : f < eps);
}

__device__ void center_tile(const PlotRel &R, int64_t tile, float *lines, double *tabs, PlotCount &cnt) {
    const PlotView V = plot_view(R);
    const double coefs = load_coefs(V);
    const int n = V.n;
    const int tid = threadIdx.x;
    const int tw_n = R.tw, ta = R.ta, tb = R.tb, s = R.s;
    const uint32_t tiles_w = (uint32_t)R.tiles_w, tiles_walk = (uint32_t)R.tiles_walk;
    uint32_t t = (uint32_t)tile;
    const int64_t t_w = t % tiles_w;
    t /= tiles_w;
    const int64_t t_walk = t % tiles_walk;
    const int64_t t_fixed = t / tiles_walk;
    const int rwalk = V.rwalk, rp = V.rp;
    const int span = tb * s;
    const int64_t b0 = t_walk * span;
    const int64_t a0 = t_fixed * ta;
    const int nwl = (n >= 2) ? span : 1;
    const int nfl = (n == 3) ? ta : 1;
    const int twi = tid % tw_n, slot = tid / tw_n;
    const int fa = (n == 3) ? slot % ta : 0;
    const int strip = (n == 3) ? slot / ta : slot;
    const int64_t w = t_w * tw_n + twi;
    const int64_t cs = b0 + (int64_t)strip * s;
    const int64_t cf = a0 + fa;
    bool active = strip < tb && !(n == 1 && slot != 0) && w < V.row_words;
    if (n >= 2) active = active && cs < rwalk;
    if (n == 3) active = active && cf < V.res0;
    const bool pad = w * 32 >= rp;
    const int k0 = (int)(w * 32);
    const int kmax = pad ? 0 : min(32, rp - k0);
    // the word's 32 centres (FP64, rounded to FP32)
    float xv[32];
    const int kb = (active && !pad) ? k0 : 0;
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) xv[kk] = (float)center_coord(V.lop, V.stp, kb + kk);
    // the tile's centre lines: thread i < nlines takes line (i / nwl, i % nwl)
    double *cdl = tabs, *ly = tabs + kDense;
    const int nlines = nwl * nfl;
    bool lvalid = false;
    double y0 = 0.0, y1 = 0.0;
    if (tid < nlines) {
        const int lf = tid / nwl, lw = tid % nwl;
        lvalid = true;
        if (n == 2) {
            const int64_t ib = b0 + lw;
            lvalid = ib < rwalk;
            if (lvalid) y0 = center_coord(V.lo0, V.st0, ib);
        } else if (n == 3) {
            const int64_t ia = a0 + lf, ib = b0 + lw;
            lvalid = ia < V.res0 && ib < rwalk;
            if (lvalid) {
                y0 = center_coord(V.lo0, V.st0, ia);
                y1 = center_coord(V.lo1, V.st1, ib);
            }
        }
    }
    store_coefs(coefs, cdl);
    if (tid < nlines) {
        ly[2 * tid] = y0;
        ly[2 * tid + 1] = y1;
    }
    __syncthreads();
    if (V.mode == PA_PLOT_FP32_ESCALATE && lvalid) line_coefs(V, cdl, y0, y1, lines + tid * kLineFloats);
    __syncthreads();
    if (!active) return;
    const uint32_t vmask = pad ? 0u : (kmax == 32 ? 0xffffffffu : ((1u << kmax) - 1u));
    const int64_t ce = (n >= 2) ? min((int64_t)rwalk, cs + s) : cs + 1;
    const int64_t row_base = (n == 3) ? cf * V.res1 : 0;
    const int target = V.target;
    const float eps32 = (float)V.eps;
    for (int64_t c = cs; c < ce; ++c) {
        if (pad) {                         // a row's padding word: zero
            V.out[(row_base + c) * V.row_words + w] = 0u;
            continue;
        }
        const int li = (n == 3 ? fa * nwl : 0) + (n >= 2 ? (int)(c - b0) : 0);
        const float *ln = lines + li * kLineFloats;
        uint32_t on = 0u, todo = vmask, fp32on = 0u;
        if (V.mode == PA_PLOT_FP32_ESCALATE) {
            float ca[kMaxD + 1];
#pragma unroll
            for (int tt = 0; tt <= kMaxD; ++tt) ca[tt] = ln[tt];
            float lo, hi;
            center_thresholds(ln[kLineFloats - 1], V.eps, lo, hi);
            uint32_t sure_on = 0u, sure_off = 0u;
#pragma unroll
            for (int kk = 0; kk < 32; ++kk) {
                float f = ca[kMaxD];
#pragma unroll
                for (int tt = kMaxD - 1; tt >= 0; --tt) f = fmaf(f, xv[kk], ca[tt]);
                const float dist = target == 0 ? fabsf(f) : f;
                sure_on |= (uint32_t)(dist < lo) << kk;
                sure_off |= (uint32_t)(dist > hi) << kk;
                if (V.audit) fp32on |= (uint32_t)(target == 2 ? dist < eps32 : dist <= eps32) << kk;
            }
            on = sure_on & vmask;
            todo = vmask & ~(sure_on | sure_off);
            cnt.flagged += __popc(todo);
        }
        const uint32_t flagged = todo;
        if (V.audit && V.mode == PA_PLOT_FP32_ESCALATE) todo = vmask;
        const double yy0 = ly[2 * li], yy1 = ly[2 * li + 1];
        uint32_t rest = todo;
        while (rest) {
            const int kk = __ffs(rest) - 1;
            rest &= rest - 1;
            double xd[3];
            const double xk = center_coord(V.lop, V.stp, k0 + kk);
            if (n == 1) decl_point(V, xk, 0.0, 0.0, xd);
            else if (n == 2) decl_point(V, yy0, xk, 0.0, xd);
            else decl_point(V, yy0, yy1, xk, xd);
            const double f64 = canon_eval(cdl, n, V.d, xd);
            const bool on64 = center_on(target, f64, V.eps);
            const uint32_t bit = 1u << kk;
            if (flagged & bit) on |= on64 ? bit : 0u;
            if (V.audit && V.mode == PA_PLOT_FP32_ESCALATE) {
                const bool dis = ((fp32on & bit) != 0) != on64;
                cnt.dis += dis;
                cnt.dis_unf += dis && !(flagged & bit);
            }
        }
        V.out[(row_base + c) * V.row_words + w] = on;
    }
}

// A trivariate corner tile whose threads walk the fixed axis (R.walk_fixed):
// tw words x tb strips of s cell rows along the walk axis x ta cells of the
// fixed axis.  A thread owns one 32-cell word of one strip and walks the
// tile's ta fixed-axis cells: it evaluates each of the (ta + 1) x (s + 1)
// corner lines bounding them once (a line between two fixed-axis cells
// serves both), keeping the previous fixed-axis line's cell masks in
// registers.  The tile stages the coefficient table and the FP32 restriction
// and bound of each of its corner lines in LDS (built in rounds of one line
// per thread); a line's FP64 coordinates, which only the escalated corners
// use, are formed again where needed.
__device__ void plot_tile3w(const PlotRel &R, int64_t tile, float *lines, double *tabs, PlotCount &cnt) {
    const PlotView V = plot_view(R);
    const double coefs = load_coefs(V);
    const int tid = threadIdx.x;
    const int tw_n = R.tw, ta = R.ta, tb = R.tb, s = R.s;
    const uint32_t tiles_w = (uint32_t)R.tiles_w, tiles_walk = (uint32_t)R.tiles_walk;
    uint32_t t = (uint32_t)tile;
    const int64_t t_w = t % tiles_w;
    t /= tiles_w;
    const int64_t t_walk = t % tiles_walk;
    const int64_t t_fixed = t / tiles_walk;
    const int rwalk = V.rwalk, rp = V.rp;
    const int span = tb * s;
    const int64_t b0 = t_walk * span, a0 = t_fixed * ta;
    const int nwl = span + 1, nlines = nwl * (ta + 1);
    const int twi = tid % tw_n, strip = tid / tw_n;
    const int64_t w = t_w * tw_n + twi;
    const int64_t cs = b0 + (int64_t)strip * s;
    const bool active = strip < tb && w < V.row_words && cs < rwalk;
    const bool pad = w * 32 >= rp;
    const int k0 = (int)(w * 32);
    const int kmax = pad ? 0 : min(32, rp - k0);
    float xv[33];
    const int kb = (active && !pad) ? k0 : 0;
#pragma unroll
    for (int kk = 0; kk < 33; ++kk) xv[kk] = (float)corner_coord(V.lop, V.stp, kb + kk);
    double *cdl = tabs;
    store_coefs(coefs, cdl);
    __syncthreads();
    if (V.mode == PA_PLOT_FP32_ESCALATE)
        for (int li = tid; li < nlines; li += (int)blockDim.x) {
            const int lf = li / nwl, lw = li - lf * nwl;
            const int64_t ia = a0 + lf, ib = b0 + lw;
            if (ia <= V.res0 && ib <= rwalk)
                line_coefs(V, cdl, corner_coord(V.lo0, V.st0, ia), corner_coord(V.lo1, V.st1, ib),
                           lines + li * kLineFloats);
        }
    __syncthreads();
    if (!active) return;
    const uint32_t vmask = pad ? 0u : (kmax == 32 ? 0xffffffffu : ((1u << kmax) - 1u));
    const int nc = (int)(min((int64_t)rwalk, cs + s) - cs);         // cell rows of the strip, 1..s
    const int na = (int)min((int64_t)ta, (int64_t)V.res0 - a0);     // fixed-axis cells of the tile, 1..ta
    // cell masks (some corner f <= 0 / f >= 0; corners i and i + 1 of cell
    // i) of this thread's walk lines cs + j on the previous fixed-axis line,
    // in LDS after the line table (2 (kMaxWalkStrip + 1) words per thread)
    uint32_t *prev = reinterpret_cast<uint32_t *>(lines + kMaxWalkLines * kLineFloats) + tid;
    constexpr int kPrevStride = 256;
    for (int lf = 0; lf <= na; ++lf) {
        // the last fixed-axis line of a tile belongs to the next tile, except
        // at the end of the axis; the first walk line of a strip to the
        // previous strip, except at 0
        const bool own_f = lf < na || a0 + lf == V.res0;
        const double y0 = corner_coord(V.lo0, V.st0, a0 + lf);
        const int64_t row_base = (a0 + lf - 1) * V.res1;
        uint32_t ql = 0u, qg = 0u;        // this fixed-axis line's masks at walk line j - 1
        for (int j = 0; j <= nc; ++j) {
            uint32_t l = 0u, g = 0u;
            if (!pad) {
                const int li = lf * nwl + (int)(cs - b0) + j;
                const double yl[2] = {y0, corner_coord(V.lo1, V.st1, cs + j)};
                Corners LE, GE;
                eval_line(V, lines + li * kLineFloats, xv, yl, cdl, k0, kmax, own_f && (j > 0 || cs == 0), LE, GE,
                          cnt);
                apply_target(V.target, LE, GE);
                l = LE.lo | __builtin_amdgcn_alignbit(LE.hi, LE.lo, 1);
                g = GE.lo | __builtin_amdgcn_alignbit(GE.hi, GE.lo, 1);
            }
            if (lf > 0 && j > 0) {
                // fixed-axis cell a0 + lf - 1, walk row cs + j - 1
                const uint32_t pl0 = prev[2 * (j - 1) * kPrevStride], pg0 = prev[(2 * (j - 1) + 1) * kPrevStride];
                const uint32_t pl1 = prev[2 * j * kPrevStride], pg1 = prev[(2 * j + 1) * kPrevStride];
                V.out[(row_base + cs + j - 1) * V.row_words + w] = (pl0 | pl1 | ql | l) & (pg0 | pg1 | qg | g) & vmask;
            }
            if (j > 0) {
                prev[2 * (j - 1) * kPrevStride] = ql;
                prev[(2 * (j - 1) + 1) * kPrevStride] = qg;
            }
            ql = l;
            qg = g;
        }
        prev[2 * nc * kPrevStride] = ql;
        prev[(2 * nc + 1) * kPrevStride] = qg;
    }
}

// One plot tile.  lines: kMaxTileLines * kLineFloats floats of LDS; tabs:
// the declared-order coefficient table (kDense doubles of LDS), then the FP64
// coordinates of the tile's corner lines (two per line).
__device__ void plot_tile(const PlotRel &R, int64_t tile, float *lines, double *tabs, PlotCount &cnt) {
    if (R.n == 2) {
        plot_tile2(R, tile, lines, tabs, cnt);
        return;
    }
    const PlotView V = plot_view(R);
    // the only loads of the tile (coefficients), issued first
    const double coefs = load_coefs(V);
    const int n = V.n;
    const int tid = threadIdx.x;
    const int tw_n = R.tw, ta = R.ta, tb = R.tb, s = R.s;
    // tile counts are below 2^31 (checked on the host): 32-bit decomposition
    const uint32_t tiles_w = (uint32_t)R.tiles_w, tiles_walk = (uint32_t)R.tiles_walk;
    uint32_t t = (uint32_t)tile;
    const int64_t t_w = t % tiles_w;
    t /= tiles_w;
    const int64_t t_walk = t % tiles_walk;
    const int64_t t_fixed = t / tiles_walk;
    const int rwalk = V.rwalk;
    const int rp = V.rp;
    const int span = tb * s;
    const int64_t b0 = t_walk * span;
    const int64_t a0 = t_fixed * ta;
    const int nwl = (n >= 2) ? span + 1 : 1;
    const int nfl = (n == 3) ? ta + 1 : 1;
    // this thread's word and strip
    const int twi = tid % tw_n, slot = tid / tw_n;
    const int fa = (n == 3) ? slot % ta : 0;
    const int strip = (n == 3) ? slot / ta : slot;
    const int64_t w = t_w * tw_n + twi;
    const int64_t cs = b0 + (int64_t)strip * s;
    const int64_t cf = a0 + fa;
    bool active = strip < tb && !(n == 1 && slot != 0) && w < V.row_words;
    if (n >= 2) active = active && cs < rwalk;
    if (n == 3) active = active && cf < V.res0;
    const bool pad = w * 32 >= rp;
    const int k0 = (int)(w * 32);
    const int kmax = pad ? 0 : min(32, rp - k0);
    // the 33 corner coordinates of this word (corners past kmax are masked
    // later), formed in FP64 and rounded to FP32
    float xv[33];
    const int kb = (active && !pad) ? k0 : 0;
#pragma unroll
    for (int kk = 0; kk < 33; ++kk) xv[kk] = (float)corner_coord(V.lop, V.stp, kb + kk);
    // this thread's corner line (one per thread: lines <= kMaxTileLines <=
    // 256) and its FP64 coordinates
    double *cdl = tabs, *ly = tabs + kDense;
    const int nlines = nwl * nfl;
    bool lvalid = false;
    double y0 = 0.0, y1 = 0.0;
    if (tid < nlines) {
        const int lf = tid / nwl, lw = tid % nwl;
        lvalid = true;
        if (n == 2) {
            const int64_t ib = b0 + lw;
            lvalid = ib <= rwalk;
            if (lvalid) y0 = corner_coord(V.lo0, V.st0, ib);
        } else if (n == 3) {
            const int64_t ia = a0 + lf, ib = b0 + lw;
            lvalid = ia <= V.res0 && ib <= rwalk;
            if (lvalid) {
                y0 = corner_coord(V.lo0, V.st0, ia);
                y1 = corner_coord(V.lo1, V.st1, ib);
            }
        }
    }
    store_coefs(coefs, cdl);
    if (tid < nlines) {
        ly[2 * tid] = y0;
        ly[2 * tid + 1] = y1;
    }
    __syncthreads();
    if (V.mode == PA_PLOT_FP32_ESCALATE && lvalid) line_coefs(V, cdl, y0, y1, lines + tid * kLineFloats);
    __syncthreads();
    if (!active) return;
    const uint32_t vmask = pad ? 0u : (kmax == 32 ? 0xffffffffu : ((1u << kmax) - 1u));
    const int64_t ce = (n >= 2) ? min((int64_t)rwalk, cs + s) : 0;
    const int64_t row_base = (n == 3) ? cf * V.res1 : 0;
    uint32_t prevL = 0, prevG = 0;
    for (int64_t c = cs; c <= ce; ++c) {
        uint32_t lc = 0, gc = 0;
        if (!pad) {
            for (int df = 0; df < (n == 3 ? 2 : 1); ++df) {
                bool own = true;
                int lf = 0;
                if (n == 2) {
                    own = (c > cs) || (cs == 0);
                } else if (n == 3) {
                    own = ((c > cs) || (cs == 0)) && ((df == 0) || (cf + 1 == V.res0));
                    lf = fa + df;
                }
                const int li = lf * nwl + (int)(c - b0);
                Corners LE, GE;
                eval_line(V, lines + li * kLineFloats, xv, ly + 2 * li, cdl, k0, kmax, own, LE, GE, cnt);
                apply_target(V.target, LE, GE);
                // cell i holds corners i and i + 1
                lc |= LE.lo | __builtin_amdgcn_alignbit(LE.hi, LE.lo, 1);
                gc |= GE.lo | __builtin_amdgcn_alignbit(GE.hi, GE.lo, 1);
            }
        }
        if (n == 1) {
            V.out[w] = lc & gc & vmask;
            break;
        }
        if (c > cs) V.out[(row_base + c - 1) * V.row_words + w] = (prevL | lc) & (prevG | gc) & vmask;
        prevL = lc;
        prevG = gc;
    }
}

// A plot tile of the kind MODE selects at compile time, so that each kernel
// holds the registers of its tiles only: 0 corner tiles other than the
// fixed-axis-walking trivariate ones, 1 the centre tiles of the
// sample-in-center plot, 2 the fixed-axis-walking trivariate corner tiles,
// -1 any corner tile (the one-relation plotting launch and the single
// persistent launch, which runs corner tiles only: centre-rule plans use the
// grouped executor).  The step of a relation carries its mode.
template <int MODE>
__device__ __forceinline__ void plot_tile_rule(const PlotRel &R, int64_t tile, float *lines, double *tabs,
                                               PlotCount &cnt) {
    if (MODE == 1) center_tile(R, tile, lines, tabs, cnt);
    else if (MODE == 2 || (MODE == -1 && R.walk_fixed)) plot_tile3w(R, tile, lines, tabs, cnt);
    else plot_tile(R, tile, lines, tabs, cnt);
}

__device__ __forceinline__ void flush_counts(const PlotCount &cnt, PlotCounters *counters) {
    if (!counters) return;
    if (cnt.flagged) atomicAdd(&counters->flagged, cnt.flagged);
    if (cnt.dis) atomicAdd(&counters->disagree, cnt.dis);
    if (cnt.dis_unf) atomicAdd(&counters->disagree_unflagged, cnt.dis_unf);
}

// A thread's escalation counts, kept until its tiles move to a relation with
// other counters (a batch gives every system its own), then added there.
struct CountSink {
    PlotCount cnt;
    PlotCounters *to = nullptr;
    __device__ __forceinline__ void use(const PlotRel &R, PlotCounters *launch_counters) {
        PlotCounters *p = R.counters ? R.counters : launch_counters;
        if (p != to) {
            flush_counts(cnt, to);
            cnt = PlotCount();
            to = p;
        }
    }
    __device__ __forceinline__ void finish() { flush_counts(cnt, to); }
};

__device__ __forceinline__ int find_rel(const PlotRel *rels, int nrel, int64_t tile) {
    int lo = 0, hi = nrel - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rels[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <bool CENTER>
__global__ __launch_bounds__(256) void k_plot(const PlotRel *__restrict__ rels, int nrel, int64_t total_tiles,
                                              PlotCounters *__restrict__ counters) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[kPlotLdsWords];
    CountSink sink;
    for (int64_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
        const PlotRel &R = rels[find_rel(rels, nrel, tile)];
        sink.use(R, counters);
        plot_tile_rule<CENTER ? 1 : -1>(R, tile - R.tile_base, reinterpret_cast<float *>(lds),
                  reinterpret_cast<double *>(lds + kPlotLineWords), sink.cnt);
        __syncthreads();
    }
    sink.finish();
}

hipError_t launch_plot(const PlotRel *d_rels, int nrel, int64_t total_tiles, bool center, PlotCounters *d_counters,
                       hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    const int64_t blocks = total_tiles < (1 << 20) ? total_tiles : (1 << 20);
    if (center)
        hipLaunchKernelGGL(k_plot<true>, dim3((unsigned)blocks), dim3(256), 0, s, d_rels, nrel, total_tiles,
                           d_counters);
    else
        hipLaunchKernelGGL(k_plot<false>, dim3((unsigned)blocks), dim3(256), 0, s, d_rels, nrel, total_tiles,
                           d_counters);
    return hipGetLastError();
}

// --------------------------------------------------- bitwise contractions
// Word offsets in A and B of one output entry (all axes but the packed one,
// plus the packed axis' bit index for each operand).
struct OutPos {
    int64_t baseA, baseB, pa, pb;
};

__device__ __forceinline__ OutPos out_pos(const ContractArgs &a, int64_t row, int64_t bit) {
    OutPos p{0, 0, 0, 0};
    if (a.nout > 0) {
        const int last = a.nout - 1;
        p.baseA = bit * a.a_str[last];
        p.baseB = bit * a.b_str[last];
        if (a.a_pk_out == last) p.pa = bit;
        if (a.b_pk_out == last) p.pb = bit;
    }
    // output rows are below 2^31 (checked on the host)
    uint32_t rem = (uint32_t)row;
    for (int i = a.nout - 2; i >= 0; --i) {
        const uint32_t q = fdiv(rem, a.fd_dim[i]);
        const int64_t ci = rem - q * (uint32_t)a.out_dim[i];
        rem = q;
        p.baseA += ci * a.a_str[i];
        p.baseB += ci * a.b_str[i];
        if (a.a_pk_out == i) p.pa = ci;
        if (a.b_pk_out == i) p.pb = ci;
    }
    return p;
}

// General mode: every latent entry visited bit by bit (any layouts).
__device__ unsigned bits_unit(const ContractArgs &a, int64_t row, int64_t bit) {
    const OutPos p = out_pos(a, row, bit);
    int kidx[kMaxDim];
    for (int j = 0; j < a.nk; ++j) kidx[j] = 0;
    int64_t offA = 0, offB = 0;
    for (;;) {
        const int64_t pa = (a.a_pk_k >= 0) ? kidx[a.a_pk_k] : p.pa;
        const int64_t pb = (a.b_pk_k >= 0) ? kidx[a.b_pk_k] : p.pb;
        const unsigned ba = (gp(a.A)[p.baseA + offA + (pa >> 5)] >> (pa & 31)) & 1u;
        const unsigned bb = a.B ? ((gp(a.B)[p.baseB + offB + (pb >> 5)] >> (pb & 31)) & 1u) : 1u;
        if (ba & bb) return 1u;
        int j = a.nk - 1;
        for (; j >= 0; --j) {
            ++kidx[j];
            offA += a.ka_str[j];
            offB += a.kb_str[j];
            if (kidx[j] < a.k_dim[j]) break;
            offA -= a.ka_str[j] * a.k_dim[j];
            offB -= a.kb_str[j] * a.k_dim[j];
            kidx[j] = 0;
        }
        if (j < 0) return 0u;
    }
}

// The latent-entry table is read-only while a kernel runs and indexed
// uniformly: read through the constant address space (scalar loads).
#define PA_K __attribute__((address_space(4)))

// Stream mode K with RW (4, 8 or 16) words per row of the shared packed
// latent axis and both operands: four latent entries at a time, all their
// loads issued before any is used.
template <int RW>
__device__ __forceinline__ uint32_t streamk_rows(const ContractArgs &a, const OutPos &p) {
    const PA_K int64_t *kt = (const PA_K int64_t *)a.ktab;
    const PA_G uint32_t *A = gp(a.A) + p.baseA, *B = gp(a.B) + p.baseB;
    constexpr int V = RW / 4;
    uint32_t acc = 0;
    int64_t j = 0;
    for (; j + 4 <= a.nktab; j += 4) {
        u32x4 x[4][V], y[4][V];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const PA_G uint32_t *pa = A + kt[2 * (j + e)], *pb = B + kt[2 * (j + e) + 1];
#pragma unroll
            for (int w = 0; w < V; ++w) {
                x[e][w] = *reinterpret_cast<const PA_G u32x4 *>(pa + 4 * w);
                y[e][w] = *reinterpret_cast<const PA_G u32x4 *>(pb + 4 * w);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int w = 0; w < V; ++w) {
                const u32x4 t = x[e][w] & y[e][w];
                acc |= t.x | t.y | t.z | t.w;
            }
    }
    for (; j < a.nktab; ++j) {
        const PA_G uint32_t *pa = A + kt[2 * j], *pb = B + kt[2 * j + 1];
#pragma unroll
        for (int w = 0; w < V; ++w) {
            const u32x4 t = *reinterpret_cast<const PA_G u32x4 *>(pa + 4 * w) &
                            *reinterpret_cast<const PA_G u32x4 *>(pb + 4 * w);
            acc |= t.x | t.y | t.z | t.w;
        }
    }
    return acc;
}

// Stream mode K: A and B are both bit-packed along the same latent variable;
// whole rows of it are ANDed (16 bytes at a time when rows allow) for every
// entry of the other latent variables (offsets from the host table).
template <bool VEC4>
__device__ __forceinline__ uint32_t streamk_unit(const ContractArgs &a, int64_t row, int64_t bit) {
    const OutPos p = out_pos(a, row, bit);
    const int64_t rw = a.a_row_words;
    if (VEC4 && a.B) {
        if (rw == 4) return streamk_rows<4>(a, p);
        if (rw == 8) return streamk_rows<8>(a, p);
        if (rw == 16) return streamk_rows<16>(a, p);
    }
    uint32_t acc = 0;
    for (int64_t j = 0; j < a.nktab; ++j) {
        const PA_G uint32_t *pa = gp(a.A) + p.baseA + gp(a.ktab)[2 * j];
        if (a.B) {
            const PA_G uint32_t *pb = gp(a.B) + p.baseB + gp(a.ktab)[2 * j + 1];
            if (VEC4) {
                for (int64_t w = 0; w < rw; w += 4) {
                    const u32x4 x = *reinterpret_cast<const PA_G u32x4 *>(pa + w);
                    const u32x4 y = *reinterpret_cast<const PA_G u32x4 *>(pb + w);
                    acc |= (x.x & y.x) | (x.y & y.y) | (x.z & y.z) | (x.w & y.w);
                }
            } else {
                for (int64_t w = 0; w < rw; ++w) acc |= pa[w] & pb[w];
            }
        } else {
            if (VEC4) {
                for (int64_t w = 0; w < rw; w += 4) {
                    const u32x4 x = *reinterpret_cast<const PA_G u32x4 *>(pa + w);
                    acc |= x.x | x.y | x.z | x.w;
                }
            } else {
                for (int64_t w = 0; w < rw; ++w) acc |= pa[w];
            }
        }
    }
    return acc;
}

// Stream mode W: C's packed variable is the packed variable of every operand
// that has it; whole words are ANDed and ORed over the latent entries (host
// table); an operand without it contributes its bit at this output row,
// broadcast over the word.
__device__ __forceinline__ uint32_t streamw_word(const ContractArgs &a, int64_t row, int64_t wc) {
    if (wc * 32 >= a.out_dim[a.nout - 1]) return 0u;
    const OutPos p = out_pos(a, row, 0);
    uint32_t acc = 0;
    for (int64_t j = 0; j < a.nktab; ++j) {
        uint32_t x;
        if (a.a_bcast) x = ((gp(a.A)[p.baseA + gp(a.ktab)[2 * j] + (p.pa >> 5)] >> (p.pa & 31)) & 1u) ? ~0u : 0u;
        else x = gp(a.A)[p.baseA + wc + gp(a.ktab)[2 * j]];
        if (a.B) {
            if (a.b_bcast) x &= ((gp(a.B)[p.baseB + gp(a.ktab)[2 * j + 1] + (p.pb >> 5)] >> (p.pb & 31)) & 1u) ? ~0u : 0u;
            else x &= gp(a.B)[p.baseB + wc + gp(a.ktab)[2 * j + 1]];
        }
        acc |= x;
    }
    return acc;
}

// Units [u0, u1) of a contraction by one 256-thread block: output bits for
// the bit-out modes (u0, u1 multiples of 64 or the end), words for mode W.
// Inlined, so that the step's fields (the latent-entry table above all)
// stay uniform: scalar loads, not a per-lane round trip per entry.
template <int MODE>
__device__ __forceinline__ void contract_range(const ContractArgs &a, int64_t u0, int64_t u1) {
    // the row of the block's first unit by one (uniform) division per step,
    // each thread's offset from it by a 32-bit fast division
    if (MODE == kModeStreamW) {
        const int64_t crw = a.c_row_words;
        for (int64_t g0 = u0; g0 < u1; g0 += blockDim.x) {
            const int64_t row0 = g0 / crw;
            const uint32_t off = (uint32_t)(g0 - row0 * crw) + threadIdx.x;
            const uint32_t q = fdiv(off, a.fd_rowwords);
            const int64_t row = row0 + q, wc = off - q * (uint32_t)crw;
            if (g0 + threadIdx.x < u1) gp(a.C)[row * crw + wc] = streamw_word(a, row, wc);
        }
        return;
    }
    const int64_t rowbits = a.c_row_words * 32;
    const int64_t total = (a.nout == 0) ? 64 : a.n_out_rows * rowbits;
    const bool vec4 = (a.a_row_words % 4) == 0;
    if (MODE == kModeStreamK && a.tq > 1) {
        // a wave's 64 units are tq rows x tp bits (blocks of 64 units; u0 is
        // a multiple of 64, block indices are below 2^31: host checks); the
        // first lane of each row stores its tp bits (tp >= 8: whole bytes,
        // disjoint from every other wave's)
        const int tq = a.tq, tp = 64 / tq;
        const int lane = threadIdx.x & 63;
        const int i = lane / tp, j = lane - i * tp;
        for (int64_t g0 = u0; g0 < u1; g0 += blockDim.x) {
            const int64_t gid = g0 + threadIdx.x;
            const uint32_t blk = (uint32_t)(gid >> 6);
            const uint32_t grp = fdiv(blk, a.fd_segs), seg = blk - grp * a.fd_segs.d;
            const int64_t row = (int64_t)grp * tq + i, bit = (int64_t)seg * tp + j;
            const bool in_row = gid < u1 && row < a.n_out_rows;
            uint32_t acc = 0;
            if (in_row && bit < a.out_dim[a.nout - 1])
                acc = vec4 ? streamk_unit<true>(a, row, bit) : streamk_unit<false>(a, row, bit);
            const unsigned long long bits = __ballot(acc != 0) >> (i * tp);
            if (j == 0 && in_row) {
                PA_G uint8_t *dst = reinterpret_cast<PA_G uint8_t *>(gp(a.C) + row * a.c_row_words) + bit / 8;
                if (tp == 32) *reinterpret_cast<PA_G uint32_t *>(dst) = (uint32_t)bits;
                else if (tp == 16) *reinterpret_cast<PA_G uint16_t *>(dst) = (uint16_t)bits;
                else *dst = (uint8_t)bits;
            }
        }
        return;
    }
    for (int64_t g0 = u0; g0 < u1; g0 += blockDim.x) {
        const int64_t gid = g0 + threadIdx.x;
        const int64_t row0 = g0 / rowbits;
        const uint32_t off = (uint32_t)(g0 - row0 * rowbits) + threadIdx.x;
        const uint32_t q = fdiv(off, a.fd_rowbits);
        const int64_t row = row0 + q, bit = off - q * (uint32_t)rowbits;
        bool valid;
        if (a.nout == 0) valid = (gid == 0);
        else valid = (gid < u1) && (row < a.n_out_rows) && (bit < a.out_dim[a.nout - 1]);
        uint32_t acc = 0;
        if (valid) {
            if (MODE == kModeStreamK) acc = vec4 ? streamk_unit<true>(a, row, bit) : streamk_unit<false>(a, row, bit);
            else acc = bits_unit(a, row, bit);
        }
        const unsigned long long bits = __ballot(acc != 0);
        if ((threadIdx.x & 63) == 0 && gid < total && gid < u1) {
            if (a.nout == 0) {
                gp(a.C)[0] = (uint32_t)(bits & 1ull);
            } else {
                PA_G uint32_t *dst = gp(a.C) + row * a.c_row_words + bit / 32;
                dst[0] = (uint32_t)bits;
                dst[1] = (uint32_t)(bits >> 32);
            }
        }
    }
}

__device__ __forceinline__ void contract_range_any(const ContractArgs &a, int mode, int64_t u0, int64_t u1) {
    if (mode == kModeStreamK) contract_range<kModeStreamK>(a, u0, u1);
    else if (mode == kModeStreamW) contract_range<kModeStreamW>(a, u0, u1);
    else contract_range<kModeBits>(a, u0, u1);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_contract(ContractArgs a, int64_t total) {
    for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < total; g0 += (int64_t)gridDim.x * blockDim.x)
        contract_range<MODE>(a, g0, min(total, g0 + (int64_t)blockDim.x));
}



hipError_t launch_contract(const ContractArgs &a, int mode, hipStream_t s) {
    const int64_t total = contract_units(a, mode);
    if (total == 0) return hipSuccess;
    if (mode == kModeStreamK) hipLaunchKernelGGL(k_contract<kModeStreamK>, grid_for(total), dim3(256), 0, s, a, total);
    else if (mode == kModeStreamW) hipLaunchKernelGGL(k_contract<kModeStreamW>, grid_for(total), dim3(256), 0, s, a, total);
    else hipLaunchKernelGGL(k_contract<kModeBits>, grid_for(total), dim3(256), 0, s, a, total);
    return hipGetLastError();
}

// Whether the sparse pass of a contraction runs: the count step's partial
// sums add up to at most max_total set bits of A (else the MFMA kernel
// computes the contraction).  Called by whole waves (a wave reduction).
__device__ __forceinline__ bool sparse_ran(const uint32_t *parts, int64_t nparts, int64_t max_total) {
    if (!parts) return true;      // a pass without a count always runs
    unsigned long long c = 0;
    for (int64_t i = __lane_id(); i < nparts; i += 64) c += gp(parts)[i];
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    return c <= (unsigned long long)max_total;
}

// Latent-entry table on the device: entry e is the mixed-radix tuple of the
// latent variables (last fastest; mode K skips the shared packed one, which
// the kernel walks word by word) and its word offsets in A and B.
__global__ void k_ktab(ContractArgs a, int mode, int64_t *tab, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = e, oa = 0, ob = 0;
        for (int j = a.nk - 1; j >= 0; --j) {
            if (mode == kModeStreamK && j == a.a_pk_k) continue;
            const int64_t idx = rem % a.k_dim[j];
            rem /= a.k_dim[j];
            oa += idx * a.ka_str[j];
            ob += idx * a.kb_str[j];
        }
        tab[2 * e] = oa;
        tab[2 * e + 1] = ob;
    }
}

hipError_t launch_ktab(const ContractArgs &a, int mode, int64_t *tab, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ktab, grid_for(n), dim3(256), 0, s, a, mode, tab, n);
    return hipGetLastError();
}

// ------------------------------------------------------- MFMA contraction
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;     // output tile columns (and rows of the 128 x 128 tile): 4 waves of 64 x 64
constexpr int kChunk = 8;      // K words staged per iteration (256 Boolean k)
constexpr int kPitch = 12;     // LDS row pitch in words: 16-byte reads of 8 rows hit distinct banks
// LDS words of the staged paths: A (64 WI rows) and B (128 rows), double-buffered;
// WI = 32-row blocks per wave (2: 128 x 128 tiles, 4: 256 x 128 tiles)
template <int WI>
constexpr int gemm_lds_words() { return 2 * (64 * WI + kTile) * kPitch; }
constexpr int kGemmLdsWords = gemm_lds_words<2>();
constexpr int kGemmLdsWordsWide = gemm_lds_words<4>();

__device__ __forceinline__ uint4 load_row4(const PA_G uint32_t *__restrict__ p, int64_t kw, int64_t kend, bool ok,
                                           bool vec4) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (!ok) return v;
    if (vec4) {
        if (kw + 3 < kend) {
            const u32x4 t = *reinterpret_cast<const PA_G u32x4 *>(p + kw);
            return make_uint4(t.x, t.y, t.z, t.w);
        }
    }
    // rows are an even number of words: pairs are 8-byte aligned
    if (kw + 1 < kend) { const u32x2 t = *reinterpret_cast<const PA_G u32x2 *>(p + kw); v.x = t.x; v.y = t.y; }
    if (kw + 3 < kend) { const u32x2 t = *reinterpret_cast<const PA_G u32x2 *>(p + kw + 2); v.z = t.x; v.w = t.y; }
    return v;
}

// The Boolean contraction runs on the fp4 (e2m1) MFMA 32 x 32 x 64 with fp32
// accumulation: lane half h supplies 32 of the 64 k of a step as one 32-bit
// word of Boolean k-entries, spread into 4 dwords of 8 nibbles.  Nibble i of
// dword j (j < 3) is bit 4i + j of x left in place (e2m1 codes 0001, 0010,
// 0100: 0.5, 1, 2); dword 3 takes bit 4i + 3 moved down one place (code
// 0100), the nibble's top bit being the sign.  A and B use the same map, so
// every product is 0 or a positive 0.25, 1 or 4, and an fp32 sum of them is
// > 0 iff some k has both bits (whatever the rounding: every term is >= 0).
// The instruction reads 4 of the 8 operand dwords for fp4; the rest are
// left undefined.
__device__ __forceinline__ v4i spread_fp4(uint32_t x) {
    v4i r;
    r[0] = (int)(x & 0x11111111u);
    r[1] = (int)(x & 0x22222222u);
    r[2] = (int)(x & 0x44444444u);
    r[3] = (int)((x >> 1) & 0x44444444u);
    return r;
}

// acc + A^T B over one 64-k step (both operands fp4, block scales 2^0); the
// operands are held as 4 dwords, widened to the builtin's 8 at the call
__device__ __forceinline__ v16f mfma_fp4(const v4i &b, const v4i &a, const v16f &acc) {
    const v8i b8 = __builtin_shufflevector(b, b, 0, 1, 2, 3, -1, -1, -1, -1);
    const v8i a8 = __builtin_shufflevector(a, a, 0, 1, 2, 3, -1, -1, -1, -1);
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b8, a8, acc, 4, 4, 0, 127, 0, 127);
}

// B rows are presented to the MFMA permuted within each 32-row block: MFMA
// row rho = 8a + 4h + b (accumulator register 4a + b of lane half h, in the
// 32 x 32 output layout) multiplies B row 16h + 4a + b.  Then register r of
// lane half h holds output column 16h + r, and each lane owns 16 consecutive
// output bits.
__device__ __forceinline__ int brow_of_mfma_row(int rho) { return ((rho >> 2) & 1) * 16 + (rho >> 3) * 4 + (rho & 3); }
__device__ __forceinline__ int mfma_row_of_brow(int n) { return ((n >> 2) & 3) * 8 + (n >> 4) * 4 + (n & 3); }

// The 16 output bits of one 32x32 accumulator block for this lane: bit r set
// iff sum r > 0.  The sums are fp32 >= 0, so as unsigned integers a positive
// one is >= 0x3e800000 (0.25) and saturates to 0xffff in a 16-bit pack:
// registers r and r + 8 are packed into dword d_r (0 or 0xffff in each
// half).  Bit-field inserts then merge them as a tree: d_0 and d_1 on
// alternate bits (d_0 on the even ones), likewise d_2, d_3 (bits 2 and 3
// are then d_2 and d_3), ...; those pairs on alternate bit pairs; the two
// quads on alternate nibbles.  Bits r and 16 + r end up as d_r, and byte 2
// moves next to byte 0: 16 instructions for 16 sums, with 3 masks.  The
// packs and the byte move are builtins, so that the compiler sees every
// read of an MFMA result (the hardware does not wait for one: the compiler
// inserts the wait states) and every write that a later cross-lane move
// reads; only the inserts, which the compiler would otherwise rewrite into
// ANDs and ORs, are written out.
__device__ __forceinline__ uint32_t pack_u16_sat(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pk_u16(__float_as_uint(lo), __float_as_uint(hi)));
}

__device__ __forceinline__ uint32_t block_bits16(const v16f &a) {
    uint32_t d[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) d[r] = pack_u16_sat(a[r], a[r + 8]);
    // VOP3 takes no literal: the masks come in SGPRs
    const uint32_t m1 = 0x55555555u, m2 = 0x33333333u, m4 = 0x0f0f0f0fu;
    uint32_t m, t, u;
    asm("v_bfi_b32 %0, %11, %3, %4\n"
        "v_bfi_b32 %1, %11, %5, %6\n"
        "v_bfi_b32 %0, %12, %0, %1\n"
        "v_bfi_b32 %1, %11, %7, %8\n"
        "v_bfi_b32 %2, %11, %9, %10\n"
        "v_bfi_b32 %1, %12, %1, %2\n"
        "v_bfi_b32 %0, %13, %0, %1\n"
        : "=&v"(m), "=&v"(t), "=&v"(u)
        : "v"(d[0]), "v"(d[1]), "v"(d[2]), "v"(d[3]), "v"(d[4]), "v"(d[5]), "v"(d[6]), "v"(d[7]), "s"(m1), "s"(m2),
          "s"(m4));
    return __builtin_amdgcn_perm(m, m, 0x0c0c0200u);
}

// One tile of a Boolean GEMM as the loaders and the epilogue see it.
// Loader thread tid stages row (tid >> 1), words (tid & 1) * 4 .. + 3 of each
// K chunk, for A and for B.
struct GemmTileRef {
    const PA_G uint32_t *a, *b;   // this thread's A and B rows
    PA_G uint32_t *c;             // C of the tile's batch
    const PA_G uint32_t *abase, *bbase;   // A and B of the tile's batch
    FastDiv fd_wc;                // division by the padded C row length in bits
    // 32-bit sizes and coordinates (below 2^31: host checks), which halves
    // the scalar registers three tiles in flight hold
    int32_t kw0, kw1, m0, n0, M, No, rwc, Kw, rn;
    bool a_ok, b_ok, vec4, atomic;
};

// B row of output column n0 + off (n0 a tile origin, off < 128) in the padded
// column space of C, where column n = no * Wc + j is B row no * rn + j if
// no < No and j < rn (else padding: ok = false, row 0).  q0 and r0 are the
// quotient and remainder of n0 by Wc (tile-uniform); Wc >= 64, so adding off
// wraps at most twice and no per-lane division is needed.
__device__ __forceinline__ uint32_t b_row_of(uint32_t q0, uint32_t r0, uint32_t off, uint32_t Wc, uint32_t rn,
                                             uint32_t No, bool &ok) {
    uint32_t x = r0 + off, q = q0;
    if (x >= Wc) { x -= Wc; ++q; }
    if (x >= Wc) { x -= Wc; ++q; }
    ok = q < No && x < rn;
    return ok ? q * rn + x : 0u;
}

template <int WI>
__device__ __forceinline__ GemmTileRef gemm_locate(const GemmArgs &g, int64_t t64) {
    GemmTileRef r;
    // tile index and N coordinates are below 2^31 (checked on the host)
    const uint32_t t = (uint32_t)t64;
    const uint32_t q1 = fdiv(t, g.fd_ksplit);
    const int ks = (int)(t - q1 * (uint32_t)g.ksplit);
    const uint32_t q2 = fdiv(q1, g.fd_tiles_n);
    const int64_t tn = q1 - q2 * (uint32_t)g.tiles_n;
    const uint32_t q3 = fdiv(q2, g.fd_tiles_m);
    const int64_t tm = q2 - q3 * (uint32_t)g.tiles_m;
    const int64_t b = q3;
    const int lrow = threadIdx.x >> 1;
    r.m0 = (int32_t)(tm * 64 * WI);
    r.n0 = (int32_t)(tn * kTile);
    r.kw0 = (int32_t)(ks * g.kchunk);
    r.kw1 = (int32_t)min(g.Kw, (int64_t)r.kw0 + g.kchunk);
    r.vec4 = (g.Kw % 4) == 0;
    const int64_t am = (int64_t)r.m0 + lrow;
    r.a_ok = am < g.M;
    r.a = gp(g.A) + b * g.sA_b + (r.a_ok ? am : 0) * g.Kw;
    const uint32_t Wc = (uint32_t)(g.rwc * 32);
    const uint32_t q0 = fdiv((uint32_t)r.n0, g.fd_wc);
    const uint32_t brow = b_row_of(q0, (uint32_t)r.n0 - q0 * Wc, (uint32_t)lrow, Wc, (uint32_t)g.rn, (uint32_t)g.No, r.b_ok);
    r.b = gp(g.B) + b * g.sB_b + (int64_t)brow * g.Kw;
    r.c = gp(g.C) + b * g.sC_b;
    r.abase = gp(g.A) + b * g.sA_b;
    r.bbase = gp(g.B) + b * g.sB_b;
    r.Kw = (int32_t)g.Kw;
    r.rn = (int32_t)g.rn;
    r.M = (int32_t)g.M;
    r.No = (int32_t)g.No;
    r.rwc = (int32_t)g.rwc;
    r.fd_wc = g.fd_wc;
    r.atomic = g.ksplit > 1;
    return r;
}

// Writes one tile's packed output (a wave's WI x 2 blocks of 32 x 32): lane
// (h, l32) of block (i, j) holds columns 16h .. 16h + 15 of the block's row
// l32.  Row addresses are formed once per tile; the block offsets are
// uniform.  Without a K split every lane stores its 16 bits; with one, the two
// halves of each word are merged and OR-ed into the (zeroed) output.
template <int WI>
__device__ __forceinline__ void gemm_epilogue(const GemmTileRef &T, v16f (&acc)[WI][2]) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wm = wave >> 1, wn = wave & 1;
    const uint32_t Wc = (uint32_t)(T.rwc * 32);
    const int64_t rs = (int64_t)T.No * T.rwc;                 // words per output row
    const int32_t mw = T.m0 + wm * (32 * WI);                 // the wave's first row
    PA_G uint32_t *crow = T.c + (int64_t)(mw + l32) * rs;     // this lane's row in block i = 0
    const int xor32 = (lane ^ 32) << 2;                       // ds_bpermute address of the other half
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const uint32_t n = (uint32_t)(T.n0 + wn * 64 + j * 32);
        const uint32_t no = fdiv(n, T.fd_wc);
        if (no >= (uint32_t)T.No) continue;
        const int64_t col = (int64_t)no * T.rwc + (n - no * Wc) / 32;
#pragma unroll
        for (int i = 0; i < WI; ++i) {
            const uint32_t v = block_bits16(acc[i][j]);
            const bool row_ok = mw + i * 32 + l32 < T.M;
            PA_G uint32_t *dst = crow + (int64_t)(i * 32) * rs + col;
            if (T.atomic) {
                const uint32_t w = v << (16 * h);
                const uint32_t word = w | (uint32_t)__builtin_amdgcn_ds_bpermute(xor32, (int)w);
                if (h == 0 && row_ok && word)
                    __hip_atomic_fetch_or(dst, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (row_ok) {
                reinterpret_cast<PA_G uint16_t *>(dst)[h] = (uint16_t)v;
            }
        }
    }
}

// MFMAs of one staged K chunk (kChunk words of A and B in LDS) for a wave's
// WI x 2 blocks; with `fresh` the first MFMA of each block starts from zero
// (a new tile).  Lane half h reads words 4h .. 4h + 3 of its rows; step q
// multiplies words q and 4 + q (halves 0 and 1).
template <int WI>
__device__ __forceinline__ void gemm_chunk(const uint32_t *sA, const uint32_t *sB, v16f (&acc)[WI][2], bool fresh) {
    const v16f zero = {};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1, l32 = lane & 31, h4 = (lane >> 5) * 4;
    uint4 a4[WI], b4[2];
#pragma unroll
    for (int i = 0; i < WI; ++i)
        a4[i] = *reinterpret_cast<const uint4 *>(&sA[(wm * (32 * WI) + i * 32 + l32) * kPitch + h4]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
        b4[j] = *reinterpret_cast<const uint4 *>(&sB[(wn * 64 + j * 32 + l32) * kPitch + h4]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v4i opa[WI], opb[2];
#pragma unroll
        for (int i = 0; i < WI; ++i)
            opa[i] = spread_fp4(q == 0 ? a4[i].x : q == 1 ? a4[i].y : q == 2 ? a4[i].z : a4[i].w);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            opb[j] = spread_fp4(q == 0 ? b4[j].x : q == 1 ? b4[j].y : q == 2 ? b4[j].z : b4[j].w);
        // MFMA rows index n (from B), columns index m (from A): each lane
        // then holds one column m, i.e. bits of one output row.
        if (q == 0 && fresh) {
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_fp4(opb[j], opa[i], zero);
        } else {
#pragma unroll
            for (int i = 0; i < WI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_fp4(opb[j], opa[i], acc[i][j]);
        }
        // keep the operands of one step live at a time (no hoisting of the
        // next steps' spreads above these MFMAs)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One K chunk of one tile in the workgroup's sequence.
struct GemmChunk {
    GemmTileRef T;
    int32_t kc;
    bool valid;
};

// (64 WI) x 128 output tiles of the canonical Boolean GEMM, one after another,
// as a sequence of K chunks software-pipelined two deep: while chunk i is
// multiplied from LDS, chunk i+1 is already in registers and chunk i+2 is
// being loaded, across tile boundaries.  next(T) yields the workgroup's next
// tile (false when done).  lds holds gemm_lds_words<WI>() words.  Loader
// thread tid stages A rows (tid >> 1) + 128 r (r < WI / 2) and B row
// (tid >> 1), words (tid & 1) * 4 .. + 3 of each chunk.
template <int WI>
struct GemmStage {
    uint4 a[WI / 2], b;
};

template <int WI, class Next>
__device__ void gemm_tiles(Next next, uint32_t *lds) {
    constexpr int TM = 64 * WI;
    uint32_t *sA[2] = {lds, lds + TM * kPitch};
    uint32_t *sB[2] = {lds + 2 * TM * kPitch, lds + 2 * TM * kPitch + kTile * kPitch};
    const int tid = threadIdx.x;
    const int lrow = tid >> 1, lw = (tid & 1) * 4;
    const int brow = (lrow & ~31) | mfma_row_of_brow(lrow & 31);   // LDS row of this thread's B row
    auto advance = [&](const GemmChunk &c) {
        GemmChunk n = c;
        if (!c.valid) return n;
        n.kc = c.kc + kChunk;
        if (n.kc >= c.T.kw1) {
            n.valid = next(n.T);
            n.kc = n.T.kw0;
        }
        return n;
    };
    auto load = [&](const GemmChunk &c, GemmStage<WI> &r) {
        if (c.valid) {
            r.a[0] = load_row4(c.T.a, c.kc + lw, c.T.kw1, c.T.a_ok, c.T.vec4);
#pragma unroll
            for (int q = 1; q < WI / 2; ++q) {
                // row lrow + 128 q exists only if row lrow does (T.a is then its row)
                const bool ok = c.T.m0 + lrow + 128 * q < c.T.M;
                r.a[q] = load_row4(c.T.a + (int64_t)(128 * q) * c.T.Kw, c.kc + lw, c.T.kw1, ok, c.T.vec4);
            }
            r.b = load_row4(c.T.b, c.kc + lw, c.T.kw1, c.T.b_ok, c.T.vec4);
        }
    };
    GemmChunk c0;
    c0.valid = next(c0.T);
    if (!c0.valid) return;
    c0.kc = c0.T.kw0;
    GemmStage<WI> r0, r1;
#pragma unroll
    for (int q = 0; q < WI / 2; ++q) r0.a[q] = r1.a[q] = make_uint4(0u, 0u, 0u, 0u);
    r0.b = r1.b = make_uint4(0u, 0u, 0u, 0u);
    load(c0, r0);
    GemmChunk c1 = advance(c0);
    load(c1, r1);
    v16f acc[WI][2];
    // one pipeline step: stage chunk c0 (in r) into LDS buffer `buf`, start
    // loading chunk c0+2 into r, multiply, finish a tile
    auto step = [&](GemmStage<WI> &r, int buf) {
#pragma unroll
        for (int q = 0; q < WI / 2; ++q)
            *reinterpret_cast<uint4 *>(&sA[buf][(lrow + 128 * q) * kPitch + lw]) = r.a[q];
        *reinterpret_cast<uint4 *>(&sB[buf][brow * kPitch + lw]) = r.b;
        __syncthreads();
        const GemmChunk c2 = advance(c1);
        load(c2, r);
        const bool fresh = c0.kc == c0.T.kw0;
        gemm_chunk<WI>(sA[buf], sB[buf], acc, fresh);
        if (c0.kc + kChunk >= c0.T.kw1) gemm_epilogue<WI>(c0.T, acc);
        c0 = c1;
        c1 = c2;
        return c0.valid;
    };
    for (;;) {
        if (!step(r0, 0)) break;
        if (!step(r1, 1)) break;
    }
}

// ---- direct path: no LDS, no barriers.  Each wave loads the two A rows
// and two B rows its lanes multiply (lane half h reads words 4h .. 4h + 3
// of each chunk) straight into registers, one K chunk ahead, and runs its 64 x 64
// quadrant of the tile on its own.
struct GemmRows {
    const PA_G uint32_t *a[2], *b[2];
    bool a_ok[2], b_ok[2];
};

__device__ __forceinline__ GemmRows gemm_rows(const GemmTileRef &T) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1, l32 = lane & 31;
    const uint32_t Wc = (uint32_t)(T.rwc * 32);
    const uint32_t q0 = fdiv((uint32_t)T.n0, T.fd_wc), r0 = (uint32_t)T.n0 - q0 * Wc;
    GemmRows R;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t am = T.m0 + wm * 64 + i * 32 + l32;
        R.a_ok[i] = am < T.M;
        R.a[i] = T.abase + (R.a_ok[i] ? am : 0) * T.Kw;
        const uint32_t off = (uint32_t)(wn * 64 + i * 32 + brow_of_mfma_row(l32));
        const uint32_t brow = b_row_of(q0, r0, off, Wc, (uint32_t)T.rn, (uint32_t)T.No, R.b_ok[i]);
        R.b[i] = T.bbase + (int64_t)brow * T.Kw;
    }
    return R;
}

struct GemmChunkD {
    GemmTileRef T;
    GemmRows R;
    int32_t kc;
    bool valid;
};

// MFMAs of one K chunk held in registers: a4[i] = words 4h .. 4h + 3 of this
// lane's A row i (h = lane half; b4 likewise for B); step q multiplies words
// q and 4 + q.
__device__ __forceinline__ void gemm_chunk_regs(const uint4 (&a4)[2], const uint4 (&b4)[2], v16f (&acc)[2][2],
                                                bool fresh) {
    const v16f zero = {};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v4i opa[2], opb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            opa[i] = spread_fp4(q == 0 ? a4[i].x : q == 1 ? a4[i].y : q == 2 ? a4[i].z : a4[i].w);
            opb[i] = spread_fp4(q == 0 ? b4[i].x : q == 1 ? b4[i].y : q == 2 ? b4[i].z : b4[i].w);
        }
        if (q == 0 && fresh) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_fp4(opb[j], opa[i], zero);
        } else {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_fp4(opb[j], opa[i], acc[i][j]);
        }
    }
}

template <class Next>
__device__ void gemm_tiles_direct(Next next) {
    const int h4 = ((threadIdx.x & 63) >> 5) * 4;
    auto advance = [&](const GemmChunkD &c) {
        GemmChunkD n = c;
        if (!c.valid) return n;
        n.kc = c.kc + kChunk;
        if (n.kc >= c.T.kw1) {
            n.valid = next(n.T);
            if (n.valid) {
                n.R = gemm_rows(n.T);
                n.kc = n.T.kw0;
            }
        }
        return n;
    };
    auto load = [&](const GemmChunkD &c, uint4 (&a4)[2], uint4 (&b4)[2]) {
        if (!c.valid) return;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a4[i] = load_row4(c.R.a[i], c.kc + h4, c.T.kw1, c.R.a_ok[i], c.T.vec4);
            b4[i] = load_row4(c.R.b[i], c.kc + h4, c.T.kw1, c.R.b_ok[i], c.T.vec4);
        }
    };
    GemmChunkD c0;
    c0.valid = next(c0.T);
    if (!c0.valid) return;
    c0.R = gemm_rows(c0.T);
    c0.kc = c0.T.kw0;
    uint4 A0[2], B0[2], A1[2], B1[2];
    load(c0, A0, B0);
    v16f acc[2][2];
    // chunk c0 is in (Ac, Bc); load the next chunk into (An, Bn), multiply
    auto step = [&](uint4 (&Ac)[2], uint4 (&Bc)[2], uint4 (&An)[2], uint4 (&Bn)[2]) {
        const GemmChunkD c1 = advance(c0);
        load(c1, An, Bn);
        gemm_chunk_regs(Ac, Bc, acc, c0.kc == c0.T.kw0);
        if (c0.kc + kChunk >= c0.T.kw1) gemm_epilogue<2>(c0.T, acc);
        c0 = c1;
        return c0.valid;
    };
    for (;;) {
        if (!step(A0, B0, A1, B1)) break;
        if (!step(A1, B1, A0, B0)) break;
    }
}

// Stores of output words that no later kernel of the launch reads:
// non-temporal, so the streamed output does not evict the operand rows that
// are re-read from L2 (the sparse pass's B rows, the resident MFMA path's B
// tiles).
__device__ __forceinline__ void store_words4(PA_G uint32_t *p, int64_t c, int64_t n, bool vec4, uint4 v) {
    if (c + 3 < n) {
        if (vec4) {
            __builtin_nontemporal_store(u32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<PA_G u32x4 *>(p + c));
        } else {
            __builtin_nontemporal_store(u32x2{v.x, v.y}, reinterpret_cast<PA_G u32x2 *>(p + c));
            __builtin_nontemporal_store(u32x2{v.z, v.w}, reinterpret_cast<PA_G u32x2 *>(p + c + 2));
        }
    } else if (c < n) {
        __builtin_nontemporal_store(u32x2{v.x, v.y}, reinterpret_cast<PA_G u32x2 *>(p + c));
    }
}

// ---- resident path: contractions with K <= 256 bits (one chunk, so no K
// split), 256 x 128 output tiles (4 waves of 128 x 64: 4 x 2 blocks).  Each
// workgroup runs a contiguous range of tiles (XCD-aware: each XCD owns a
// contiguous eighth of the tiles, split among its workgroups) in which
// consecutive tiles mostly share their A rows (tile columns vary fastest).
// Each wave keeps the fp4 operands of its 128 A rows (4 blocks x 4 steps) in
// registers for as long as the rows stay the same, loaded straight from
// global memory when they change; only the 128 B rows of a tile are staged
// in LDS (double-buffered, loaded one tile ahead) and spread per tile.
// The output bits of a group of 8 consecutive column tiles (128 bytes of
// each of the 256 rows) are gathered in LDS and written out as whole
// 128-byte lines with non-temporal stores: pieces of lines written from
// different places at different times cost several times their bytes in
// HBM writes.
constexpr int kResGroup = 8;                     // column tiles per output group
constexpr int kResPitch = 4 * kResGroup + 4;     // LDS words per staged output row (16-byte aligned rows)
constexpr int kResLdsWords = 2 * kTile * kPitch + 256 * kResPitch;

// Contiguous item range [lo, hi) of workgroup bid of nbid among n items:
// the XCD-aware split (workgroups go to the 8 XCDs round-robin; XCD x owns
// items [x per, (x + 1) per), shared evenly by its workgroups).
__device__ __forceinline__ void res_range(int64_t n, int64_t &lo, int64_t &hi, uint32_t bid, uint32_t nbid) {
    const int64_t per = (n + 7) >> 3;
    const int64_t nwg = ((int64_t)nbid + 7 - (bid & 7)) >> 3;   // workgroups on this XCD
    const int64_t k = bid >> 3, span = (per + nwg - 1) / nwg;
    lo = min(n, (int64_t)(bid & 7) * per + k * span);
    hi = min(min(n, (int64_t)((bid & 7) + 1) * per), lo + span);
}

// Epilogue into the LDS output group: for each row block i the lane halves
// trade block halves (v_permlane32_swap), so that lane half h holds the
// whole 32-bit word of block column h of its row, written to word
// 4 tt + 2 wn + h of the staged row (tt = the tile's place in its group).
__device__ __forceinline__ void gemm_epilogue_res(v16f (&acc)[4][2], uint32_t *sC, int tt) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wm = wave >> 1, wn = wave & 1;
    uint32_t *dst = sC + (wm * 128 + l32) * kResPitch + 4 * tt + 2 * wn + h;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t v0 = block_bits16(acc[i][0]), v1 = block_bits16(acc[i][1]);
        // lanes 32..63 of v0 trade places with lanes 0..31 of v1
        const auto sw = __builtin_amdgcn_permlane32_swap(v0, v1, false, false);
        dst[i * 32 * kResPitch] = sw[0] | (sw[1] << 16);
    }
}

// The output group being staged: output c, rows m0 .. m0 + 255 (those < M)
// of rs words each, words gw + w for w in [w0, w1) (the tiles of the group
// this workgroup computed; gw = the group's first word).
struct ResGroup {
    PA_G uint32_t *c;
    int64_t rs, gw;
    int32_t m0, M, w0, w1;
};

// Writes the staged output group, 4 words per thread and step, so that 8
// consecutive lanes write one 128-byte line.
__device__ __forceinline__ void res_flush(const ResGroup &G, const uint32_t *sC) {
    const bool vec4 = (G.rs % 4) == 0;
#pragma unroll 1
    for (int idx = threadIdx.x; idx < 256 * kResGroup; idx += 256) {
        const int r = idx / kResGroup, w = (idx % kResGroup) * 4;
        if (w < G.w0 || w >= G.w1 || G.m0 + r >= G.M) continue;
        const uint4 v = *reinterpret_cast<const uint4 *>(&sC[r * kResPitch + w]);
        store_words4(G.c + (int64_t)(G.m0 + r) * G.rs, G.gw + w, G.rs, vec4, v);
    }
}

template <class Next>
__device__ void gemm_tiles_res(Next next, uint32_t *lds) {
    // B buffer `buf` at lds + buf * kTile * kPitch (offsets from the LDS
    // array itself, so that every access stays an LDS access)
    uint32_t *sC = lds + 2 * kTile * kPitch;
    const int tid = threadIdx.x, lane = tid & 63, l32 = lane & 31, h4 = (lane >> 5) * 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = tid >> 1, lw = (tid & 1) * 4;
    const int brow = (lrow & ~31) | mfma_row_of_brow(lrow & 31);   // LDS row of this thread's B row
    const v16f zero = {};
    GemmTileRef T0, T1;
    if (!next(T0)) return;
    // B of the current tile, loaded one tile ahead (the B tiles are L2 hits)
    uint4 rb = load_row4(T0.b, T0.kw0 + lw, T0.kw1, T0.b_ok, T0.vec4);
    v4i opa[4][4];                            // A operands of block i, step q
    const PA_G uint32_t *a_base = nullptr;    // the rows they hold (uniform)
    int32_t a_m0 = -1;
    ResGroup G;                               // the staged output group (uniform)
    G.w0 = G.w1 = 0;                          // none yet
    v16f acc[4][2];
    int buf = 0;
    for (;;) {
        uint32_t *sB = lds + buf * (kTile * kPitch);
        *reinterpret_cast<uint4 *>(&sB[brow * kPitch + lw]) = rb;
        // the A operands, when the rows change
        if (T0.abase != a_base || T0.m0 != a_m0) {
            a_base = T0.abase;
            a_m0 = T0.m0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t row = T0.m0 + wm * 128 + i * 32 + l32;
                const bool ok = row < T0.M;
                const uint4 w = load_row4(T0.abase + (int64_t)(ok ? row : 0) * T0.Kw, h4, T0.kw1, ok, T0.vec4);
                opa[i][0] = spread_fp4(w.x);
                opa[i][1] = spread_fp4(w.y);
                opa[i][2] = spread_fp4(w.z);
                opa[i][3] = spread_fp4(w.w);
            }
        }
        __syncthreads();                      // B staged; the previous tile's output staged
        // the output group: flushed when this tile starts another one
        const int tt = (T0.n0 >> 7) & (kResGroup - 1);   // the tile's place in its group
        const int64_t gw = (T0.n0 >> 5) & ~(4 * kResGroup - 1);
        if (!(G.w1 > G.w0 && T0.c == G.c && T0.m0 == G.m0 && gw == G.gw)) {
            if (G.w1 > G.w0) {
                res_flush(G, sC);
                __syncthreads();              // the group is read before it is overwritten
            }
            G.c = T0.c;
            G.rs = (int64_t)T0.No * T0.rwc;
            G.gw = gw;
            G.m0 = T0.m0;
            G.M = T0.M;
            G.w0 = 4 * tt;
        }
        G.w1 = 4 * tt + 4;
        const bool more = next(T1);
        if (more) rb = load_row4(T1.b, T1.kw0 + lw, T1.kw1, T1.b_ok, T1.vec4);
        // B words are read from LDS one step at a time (fewer live registers)
        const uint32_t *sb = &sB[(wn * 64 + l32) * kPitch + h4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v4i opb[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) opb[j] = spread_fp4(sb[j * 32 * kPitch + q]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_fp4(opb[j], opa[i][q], q == 0 ? zero : acc[i][j]);
        }
        gemm_epilogue_res(acc, sC, tt);
        if (!more) break;
        T0 = T1;
        buf ^= 1;
    }
    __syncthreads();
    res_flush(G, sC);
}

// Operand paths of the MFMA contraction (GemmArgs::path): 0 stages 128 x 128
// tiles in LDS, 1 loads straight into registers, 2 stages 256 x 128 tiles
// (4 x 2 blocks per wave: fewer operand spreads per MFMA, two waves per SIMD),
// 3 keeps the A operands of 256 x 128 tiles in registers (K <= 256 bits).
constexpr int gemm_occupancy(int path) { return path == 0 ? 3 : 2; }
constexpr int gemm_lds_of(int path) {
    return path == 0 ? kGemmLdsWords : path == 2 ? kGemmLdsWordsWide : path == 3 ? kResLdsWords : 1;
}

// Tiles of the canonical GEMM on operand path PATH; next(T) yields the tiles.
template <int PATH, class Next>
__device__ __forceinline__ void gemm_run(Next next, uint32_t *lds) {
    if constexpr (PATH == 1) gemm_tiles_direct(next);
    else if constexpr (PATH == 3) gemm_tiles_res(next, lds);
    else gemm_tiles<PATH == 2 ? 4 : 2>(next, lds);
}

// XCD-aware order of a launch's n tiles.  Workgroups are dispatched to the
// 8 XCDs round-robin, so with a grid that is a multiple of 8, slot t of the
// persistent loop (workgroup t % grid) runs on XCD t % 8.  Slot t takes tile
// (t % 8) * per + t / 8 with per = ceil(n / 8): each XCD runs one contiguous
// eighth of the tiles, so tiles that write the same output lines (adjacent
// column tiles) and read the same operand rows meet in one L2 instead of
// being spread over all eight.  A bijection of [0, 8 per); tiles >= n are
// skipped.
__device__ __forceinline__ int64_t xcd_tile(int64_t t, int64_t per) { return (t & 7) * per + (t >> 3); }

template <int PATH>
__global__ __launch_bounds__(256, gemm_occupancy(PATH)) void k_gemm_mfma(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[gemm_lds_of(PATH)];
    // when the sparse pass ran (A sparse enough) there is nothing to do
    if (g.dense && __hip_atomic_load(gp(g.dense), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    const int64_t ntiles = g.nbatch * g.tiles_m * g.tiles_n * g.ksplit;
    if constexpr (PATH == 3) {
        int64_t t, tend;
        res_range(ntiles, t, tend, blockIdx.x, gridDim.x);
        auto next = [&](GemmTileRef &T) {
            if (t >= tend) return false;
            T = gemm_locate<4>(g, t++);
            return true;
        };
        gemm_run<PATH>(next, lds);
    } else {
        const int64_t per = (ntiles + 7) >> 3;
        int64_t t = blockIdx.x;
        auto next = [&](GemmTileRef &T) {
            for (; t < 8 * per; t += gridDim.x) {
                const int64_t tile = xcd_tile(t, per);
                if (tile < ntiles) {
                    T = gemm_locate<PATH == 2 ? 4 : 2>(g, tile);
                    t += gridDim.x;
                    return true;
                }
            }
            return false;
        };
        gemm_run<PATH>(next, lds);
    }
}

// Workgroups of a persistent tile loop: every CU's worth (a multiple of 8),
// capped by the tiles rounded up to a multiple of 8.
static int64_t gemm_grid(int64_t ntiles, int path) {
    static int cached[4] = {0, 0, 0, 0};
    if (!cached[path]) {
        int dev = 0, cus = 256, per_cu = 1;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const hipError_t e =
            path == 1   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm_mfma<1>, 256, 0)
            : path == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm_mfma<2>, 256, 0)
            : path == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm_mfma<3>, 256, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gemm_mfma<0>, 256, 0);
        if (e != hipSuccess || per_cu < 1) per_cu = 1;
        cached[path] = (cus * per_cu + 7) / 8 * 8;
    }
    const int64_t want = (ntiles + 7) / 8 * 8;
    return want < cached[path] ? want : cached[path];
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    if (g.nbatch == 0 || g.M == 0 || g.No == 0) return hipSuccess;
    if (g.path < 0 || g.path > 3) return hipErrorInvalidValue;
    if (g.path == 3 && (g.Kw > kChunk || g.ksplit != 1)) return hipErrorInvalidValue;
    const int64_t nt = g.nbatch * g.tiles_m * g.tiles_n * g.ksplit;
    const dim3 grid((unsigned)gemm_grid(nt, g.path));
    if (g.path == 1) hipLaunchKernelGGL(k_gemm_mfma<1>, grid, dim3(256), 0, s, g);
    else if (g.path == 2) hipLaunchKernelGGL(k_gemm_mfma<2>, grid, dim3(256), 0, s, g);
    else if (g.path == 3) hipLaunchKernelGGL(k_gemm_mfma<3>, grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(k_gemm_mfma<0>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ------------------------------------------------------- count semiring
// Spread one 32-bit word of Boolean k-entries into an int8 MFMA operand with
// every weight 1: byte p of dword j is bit (8p + 4h + j) of x as 0 or 1
// (h = lane half; the same positions as spread(), unscaled), so the int32
// sum over k is the number of k where both operands are set.
__device__ __forceinline__ v4i spread_count(uint32_t x, int h) {
    v4i r;
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = (int)((x >> (4 * h + j)) & 0x01010101u);
    return r;
}

// 128 x 128 output tiles of the canonical GEMM in the count semiring: each
// workgroup stages K chunks of its A and B rows in LDS (B rows permuted as in
// gemm_tiles, so a lane's 16 accumulators are 16 consecutive output
// columns) and each wave accumulates its 2 x 2 blocks of 32 x 32 counts;
// counts are stored as uint32 (added atomically with a K split).
__global__ __launch_bounds__(256) void k_gemm_count(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[2 * kTile * kPitch];
    uint32_t *sA = lds, *sB = lds + kTile * kPitch;
    const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5, l32 = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = tid >> 1, lw = (tid & 1) * 4;
    const int brow = (lrow & ~31) | mfma_row_of_brow(lrow & 31);
    const v16i zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t ntiles = g.nbatch * g.tiles_m * g.tiles_n * g.ksplit;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const GemmTileRef T = gemm_locate<2>(g, t);
        v16i acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = zero;
        for (int32_t kc = T.kw0; kc < T.kw1; kc += kChunk) {
            const uint4 a = load_row4(T.a, kc + lw, T.kw1, T.a_ok, T.vec4);
            const uint4 b = load_row4(T.b, kc + lw, T.kw1, T.b_ok, T.vec4);
            __syncthreads();                       // the previous chunk is consumed
            *reinterpret_cast<uint4 *>(&sA[lrow * kPitch + lw]) = a;
            *reinterpret_cast<uint4 *>(&sB[brow * kPitch + lw]) = b;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                v4i opa[2], opb[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    opa[i] = spread_count(sA[(wm * 64 + i * 32 + l32) * kPitch + q], h);
                    opb[i] = spread_count(sB[(wn * 64 + i * 32 + l32) * kPitch + q], h);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(opb[j], opa[i], acc[i][j], 0, 0, 0);
            }
        }
        // lane (h, l32) of block (i, j): row m0 + wm 64 + 32 i + l32, columns
        // n .. n + 15 with n = n0 + wn 64 + 32 j + 16 h (padded column space:
        // column n is output (no, jj) with n = no Wc + jj, valid if jj < rn)
        const uint32_t Wc = (uint32_t)(T.rwc * 32);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t nb = (uint32_t)(T.n0 + wn * 64 + j * 32);
            const uint32_t no = fdiv(nb, T.fd_wc);
            if (no >= (uint32_t)T.No) continue;
            const int32_t jj0 = (int32_t)(nb - no * Wc) + 16 * h;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int32_t m = T.m0 + wm * 64 + i * 32 + l32;
                if (m >= T.M) continue;
                PA_G uint32_t *dst = T.c + ((int64_t)m * T.No + no) * T.rn;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t jj = jj0 + r;
                    if (jj < T.rn) {
                        const uint32_t v = (uint32_t)acc[i][j][r];
                        if (T.atomic) {
                            if (v) __hip_atomic_fetch_add(dst + jj, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        } else {
                            dst[jj] = v;
                        }
                    }
                }
            }
        }
    }
}

hipError_t launch_gemm_count(const GemmArgs &g, hipStream_t s) {
    if (g.nbatch == 0 || g.M == 0 || g.No == 0) return hipSuccess;
    const int64_t nt = g.nbatch * g.tiles_m * g.tiles_n * g.ksplit;
    const int64_t blocks = nt < (1 << 20) ? nt : (1 << 20);
    hipLaunchKernelGGL(k_gemm_count, dim3((unsigned)blocks), dim3(256), 0, s, g);
    return hipGetLastError();
}

// Count semiring, any layouts: the number of latent entries where A and B
// are both set (every latent entry visited, as bits_unit does).
__device__ uint32_t count_unit(const ContractArgs &a, int64_t row, int64_t bit) {
    const OutPos p = out_pos(a, row, bit);
    int kidx[kMaxDim];
    for (int j = 0; j < a.nk; ++j) kidx[j] = 0;
    int64_t offA = 0, offB = 0;
    uint32_t count = 0;
    for (;;) {
        const int64_t pa = (a.a_pk_k >= 0) ? kidx[a.a_pk_k] : p.pa;
        const int64_t pb = (a.b_pk_k >= 0) ? kidx[a.b_pk_k] : p.pb;
        const unsigned ba = (gp(a.A)[p.baseA + offA + (pa >> 5)] >> (pa & 31)) & 1u;
        const unsigned bb = a.B ? ((gp(a.B)[p.baseB + offB + (pb >> 5)] >> (pb & 31)) & 1u) : 1u;
        count += ba & bb;
        int j = a.nk - 1;
        for (; j >= 0; --j) {
            ++kidx[j];
            offA += a.ka_str[j];
            offB += a.kb_str[j];
            if (kidx[j] < a.k_dim[j]) break;
            offA -= a.ka_str[j] * a.k_dim[j];
            offB -= a.kb_str[j] * a.k_dim[j];
            kidx[j] = 0;
        }
        if (j < 0) return count;
    }
}

// One thread per output element e = row * L + bit (L = the last output
// variable's length; one element for a 0-dim output).
__global__ __launch_bounds__(256) void k_count_bits(ContractArgs a, int64_t n_elems) {
    const int64_t L = a.nout > 0 ? a.out_dim[a.nout - 1] : 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / L, bit = e - row * L;
        gp(a.C)[e] = count_unit(a, row, bit);
    }
}

hipError_t launch_count_bits(const ContractArgs &a, int64_t n_elems, hipStream_t s) {
    if (n_elems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_bits, grid_for(n_elems), dim3(256), 0, s, a, n_elems);
    return hipGetLastError();
}

// ------------------------------------------------------- sparse pass
// Four words of a row of n words starting at word c (c and n even: pairs are
// 8-byte aligned; with vec4 the row and c are 16-byte aligned).
__device__ __forceinline__ uint4 load_words4(const PA_G uint32_t *p, int64_t c, int64_t n, bool vec4) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (c + 3 < n) {
        if (vec4) {
            const u32x4 t = *reinterpret_cast<const PA_G u32x4 *>(p + c);
            v = make_uint4(t.x, t.y, t.z, t.w);
        } else {
            const u32x2 t0 = *reinterpret_cast<const PA_G u32x2 *>(p + c);
            const u32x2 t1 = *reinterpret_cast<const PA_G u32x2 *>(p + c + 2);
            v = make_uint4(t0.x, t0.y, t1.x, t1.y);
        }
    } else if (c < n) {
        const u32x2 t0 = *reinterpret_cast<const PA_G u32x2 *>(p + c);
        v.x = t0.x;
        v.y = t0.y;
    }
    return v;
}

// Count step, tile t: the set bits of A words [t K, (t + 1) K) (K =
// kCountTileWords), one partial sum per wave stored at parts[4 t + wave].
// A full tile of 16-byte aligned words is read with eight independent
// 16-byte loads per lane.
__device__ void count_tile(const GatherArgs &g, int64_t t) {
    static_assert(kCountTileWords == 8 * 4 * 256, "count tile: eight 16-byte loads per lane of 256");
    const int64_t u0 = t * kCountTileWords, u1 = min(g.rows * g.Kw, u0 + kCountTileWords);
    uint32_t c = 0;
    const PA_G uint32_t *a = gp(g.A);
    if (u1 - u0 == kCountTileWords && ((uintptr_t)(a + u0) & 15u) == 0) {
        const PA_G u32x4 *a4 = reinterpret_cast<const PA_G u32x4 *>(a + u0);
        u32x4 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = a4[threadIdx.x + 256 * j];
#pragma unroll
        for (int j = 0; j < 8; ++j) c += __popc(v[j].x) + __popc(v[j].y) + __popc(v[j].z) + __popc(v[j].w);
    } else {
        for (int64_t i = u0 + threadIdx.x; i < u1; i += blockDim.x) c += __popc(a[i]);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if ((threadIdx.x & 63) == 0) gp(g.parts)[4 * t + (threadIdx.x >> 6)] = c;
}

// The set bits of one A row, in order, as row indices of Bt (latent entry
// ko * rkp + 32 wp + bit of A word w = ko * rwk + wp): the row's words are
// read 64 at a time, one per lane, so their loads overlap; a ballot finds
// the nonzero words and readlane hands each to the whole wave.  Padding
// bits are zero in every array; they are masked anyway, as they would
// index past Bt.  Every member but aw and base is uniform.
struct RowBits {
    const PA_G uint32_t *arow;
    uint32_t Kw, rwk, rkp;
    uint32_t aw, base;      // this lane's word and the Bt row of its bit 0
    uint64_t nz;            // lanes whose nonzero word is not taken yet
    uint32_t cur, cbase;    // the word being walked and its Bt row of bit 0

    // issue() starts the lane loads of words w0 .. w0 + 63; finish() waits
    // for them (the ballot is their first use)
    __device__ __forceinline__ void issue(uint32_t w0) {
        const uint32_t w = w0 + (threadIdx.x & 63);
        aw = 0u;
        base = 0u;
        if (w < Kw) {
            const uint32_t ko = w / rwk, wp = w - ko * rwk;
            const int32_t lim = (int32_t)rkp - 32 * (int32_t)wp;
            aw = arow[w] & (lim <= 0 ? 0u : lim >= 32 ? ~0u : ((1u << lim) - 1u));
            base = ko * rkp + 32u * wp;
        }
    }
    __device__ __forceinline__ void finish() {
        nz = __ballot(aw != 0u);
        cur = 0u;
    }
    __device__ __forceinline__ void load(uint32_t w0) {
        issue(w0);
        finish();
    }
    __device__ __forceinline__ bool more() const { return cur != 0u || nz != 0u; }
    // the next set bit's Bt row, or -1 when the 64 words hold no more
    __device__ __forceinline__ int64_t next() {
        if (cur == 0u) {
            if (nz == 0u) return -1;
            const int l = __builtin_ctzll(nz);
            nz &= nz - 1u;
            cur = (uint32_t)__builtin_amdgcn_readlane((int)aw, l);
            cbase = (uint32_t)__builtin_amdgcn_readlane((int)base, l);
        }
        const uint32_t bit = (uint32_t)__builtin_ctz(cur);
        cur &= cur - 1u;
        return (int64_t)(cbase + bit);
    }
};

// The A row of wave-tile wt with its first 64 words' loads issued, so that
// a wave can start them a tile ahead.
__device__ __forceinline__ RowBits gather_row_issue(const GatherArgs &g, int64_t wt) {
    const uint32_t row = fdiv((uint32_t)wt, g.fd_chunks);
    RowBits rb;
    rb.arow = gp(g.A) + (int64_t)row * g.Kw;
    rb.Kw = (uint32_t)g.Kw;
    rb.rwk = (uint32_t)g.rwk;
    rb.rkp = (uint32_t)g.rkp;
    rb.issue(0u);
    return rb;
}

// One wave-tile of the sparse pass: words ch * 2048 .. + 2047 of output row
// `row`; lane l holds words 4l + 256 j (j < 8), and for each set bit of the
// A row the matching 2048 words of Bt are OR-ed in (eight independent
// 16-byte loads per lane).  A row of at most 256 words is one wave-tile
// with one position per lane, and four set bits are taken at a time so that
// four Bt rows' loads are in flight together.  rb comes from
// gather_row_issue(g, wt).
__device__ void gather_wave(const GatherArgs &g, int64_t wt, RowBits rb) {
    const int lane = threadIdx.x & 63;
    const uint32_t row = fdiv((uint32_t)wt, g.fd_chunks);
    const uint32_t ch = (uint32_t)wt - row * (uint32_t)g.chunks;
    const uint32_t b = fdiv(row, g.fd_M);
    const int64_t n = g.Nw;
    const bool vec4 = (n & 3) == 0;
    const PA_G uint32_t *bt = gp(g.Bt) + (int64_t)b * g.sBt_b;
    PA_G uint32_t *crow = gp(g.C) + (int64_t)row * n;
    if (n <= 256) {
        const int64_t c = 4 * lane;
        uint4 acc = make_uint4(0u, 0u, 0u, 0u);
        for (uint32_t w0 = 0; w0 < rb.Kw; w0 += 64) {
            if (w0) rb.issue(w0);
            rb.finish();
            while (rb.more()) {
                int64_t k[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) k[q] = rb.next();
                uint4 v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    v[q] = k[q] >= 0 ? load_words4(bt + k[q] * n, c, n, vec4) : make_uint4(0u, 0u, 0u, 0u);
                acc.x |= (v[0].x | v[1].x) | (v[2].x | v[3].x);
                acc.y |= (v[0].y | v[1].y) | (v[2].y | v[3].y);
                acc.z |= (v[0].z | v[1].z) | (v[2].z | v[3].z);
                acc.w |= (v[0].w | v[1].w) | (v[2].w | v[3].w);
            }
        }
        store_words4(crow, c, n, vec4, acc);
        return;
    }
    const int64_t c0 = (int64_t)ch * 2048 + 4 * lane;
    uint4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t w0 = 0; w0 < rb.Kw; w0 += 64) {
        if (w0) rb.issue(w0);
        rb.finish();
        while (rb.more()) {
            const PA_G uint32_t *src = bt + rb.next() * n;
            uint4 v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = load_words4(src, c0 + 256 * j, n, vec4);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                acc[j].x |= v[j].x;
                acc[j].y |= v[j].y;
                acc[j].z |= v[j].z;
                acc[j].w |= v[j].w;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) store_words4(crow, c0 + 256 * j, n, vec4, acc[j]);
}

// Stand-alone sparse pass: workgroups of four wave-tiles, grid-stride.
// The decision of a wave of the sparse pass; the wave of wave-tile 0 also
// writes it for the MFMA kernel of the contraction (one store: thousands of
// stores to one word would serialize at the memory side).
__device__ __forceinline__ bool gather_decide(const GatherArgs &g, int64_t wt) {
    const bool run = sparse_ran(g.parts, g.nparts, g.max_total);
    if (g.dense && wt == 0 && __lane_id() == 0) gp(g.dense)[0] = run ? 0u : 1u;
    return run;
}

__global__ __launch_bounds__(256) void k_gather(GatherArgs g, int64_t ntiles) {
    const int wave0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (!gather_decide(g, blockIdx.x * 4 + wave0)) return;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t nw = gather_wave_tiles(g);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t wt = t * 4 + wave;
        if (wt < nw) gather_wave(g, wt, gather_row_issue(g, wt));
    }
}

__global__ __launch_bounds__(256) void k_count(GatherArgs g, int64_t ntiles) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) count_tile(g, t);
}

hipError_t launch_count(const GatherArgs &g, hipStream_t s) {
    const int64_t nt = (g.rows * g.Kw + kCountTileWords - 1) / kCountTileWords;
    if (nt <= 0) return hipSuccess;
    const int64_t blocks = nt < (1 << 20) ? nt : (1 << 20);
    hipLaunchKernelGGL(k_count, dim3((unsigned)blocks), dim3(256), 0, s, g, nt);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs &g, hipStream_t s) {
    const int64_t nt = (gather_wave_tiles(g) + 3) / 4;
    if (nt <= 0) return hipSuccess;
    const int64_t blocks = nt < (1 << 20) ? nt : (1 << 20);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, s, g, nt);
    return hipGetLastError();
}

// -------------------------------------------------------- fused pass pair
// Row lists: the set bits k of the A row as the 16-bit LDS row indices
// lbase + k, entries 0 .. m - 1 of the list row (m: the largest count of the
// row's group of 8), padded with the zero row; m is the group's meta word.
// One tile: kListRowsPerTile list rows, 8 lanes to a row (lane l takes the
// row's words l, l + 8, ..), so that a wave holds one group of 8 rows.  The
// lanes' counts give the row's count, the group's largest and each lane's
// first entry; every lane writes the entries of its own set bits, and the
// row's lanes together pad the row with the zero row up to m.
__device__ __forceinline__ void row_list_tile(const RowListArgs &L, int64_t tile) {
    const int lane = (int)(threadIdx.x & 63), l = lane & 7;
    const int64_t r = tile * kListRowsPerTile + (threadIdx.x >> 3);
    const bool valid = r < L.n_rows;   // whole waves: n_rows is a multiple of 8
    const int64_t g = r >> 3, ob = fdiv((uint32_t)g, L.fd_s), s = g - ob * L.n_s, o = ob * 8 + (r & 7);
    const bool has = valid && o < L.n_o;
    const PA_G uint32_t *row = gp(L.A) + (o * L.ro + s * L.rs) * L.Kw;
    const uint32_t Kw = (uint32_t)L.Kw, rwk = (uint32_t)L.rwk, rkp = (uint32_t)L.rkp;
    uint32_t cnt = 0;
    if (has)
        for (uint32_t w = (uint32_t)l; w < Kw; w += 8) cnt += __builtin_popcount(row[w]);
    uint32_t rc = cnt;
    rc += (uint32_t)__shfl_xor((int)rc, 1);
    rc += (uint32_t)__shfl_xor((int)rc, 2);
    rc += (uint32_t)__shfl_xor((int)rc, 4);
    uint32_t mx = rc;
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, 8));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, 16));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, 32));
    const uint32_t m = mx;
    uint32_t inc = cnt;
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, d, 8);
        if (l >= d) inc += t;
    }
    if (!valid) return;
    PA_G uint16_t *ent = gp(L.ent) + r * L.cap;
    uint32_t pos = inc - cnt;
    if (has)
        for (uint32_t w = (uint32_t)l; w < Kw; w += 8) {
            uint32_t x = row[w];
            const uint32_t ko = w / rwk;
            const uint32_t kb = (uint32_t)L.lbase + ko * rkp + (w - ko * rwk) * 32u;
            while (x) {
                ent[pos++] = (uint16_t)(kb + (uint32_t)__builtin_ctz(x));
                x &= x - 1;
            }
        }
    for (uint32_t e = rc + (uint32_t)l; e < m; e += 8) ent[e] = (uint16_t)L.zrow;
    if (lane == 0) gp(L.meta)[g] = m;
}

__global__ __launch_bounds__(256) void k_row_list(RowListArgs L, int64_t n_tiles) {
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) row_list_tile(L, t);
}

hipError_t launch_row_list(const RowListArgs &l, hipStream_t s) {
    const int64_t nt = (l.n_rows + kListRowsPerTile - 1) / kListRowsPerTile;
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_list, dim3((unsigned)(nt < (1 << 20) ? nt : (1 << 20))), dim3(256), 0, s, l, nt);
    return hipGetLastError();
}

// LDS rows row0 .. row0 + K - 1 of a fused tile (kFusedPitch words apart):
// word 32 (ol / 4) + 4 w + ol % 4 of row row0 + k is Bt[k][o0 + ol][w]
// (zero for o0 + ol >= n_o or w >= rwt): values 0..3 of word w are the 16
// bytes at 16 w, values 4..7 those at 128 + 16 w, so that 8 lanes reading
// one row's word w = 0..7 cover 128 contiguous bytes with each of their two
// 16-byte loads.  This stages t of fewer than 8 words (one word per lane, a
// wave writing one row: 64 distinct banks); fused_stage8_pair stages t of 8
// words.  1024 threads; the loads of four rounds are issued before their
// stores.
__device__ __forceinline__ void fused_stage(uint32_t *lds, const uint32_t *bt, int64_t bt_rw, int K, int64_t o0,
                                            int64_t n_o, int rwt, int row0) {
    const int tid = threadIdx.x;
    const int n = K * 64;
    for (int i0 = 0; i0 < n; i0 += 4096) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * 1024 + tid;
            const int k = i >> 6, ol = (i >> 3) & 7, w = i & 7;
            v[u] = 0u;
            if (i < n && w < rwt && o0 + ol < n_o) v[u] = gp(bt)[(int64_t)k * bt_rw + (o0 + ol) * rwt + w];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * 1024 + tid;
            if (i < n) {
                const int o = (i >> 3) & 7;
                lds[(row0 + (i >> 6)) * kFusedPitch + 32 * (o >> 2) + 4 * (i & 7) + (o & 3)] = v[u];
            }
        }
    }
}

// Both operands' rows when t has 8 words (BtX rows 0 .. kX - 1 for values
// o0x .., BtY rows kX .. kX + kY - 1 for values o0y ..), laid out as in
// fused_stage; each round issues the loads of both before any store, so
// that the two stagings share one wait.
__device__ __forceinline__ void fused_stage8_pair(uint32_t *lds, const uint32_t *btx, int64_t btx_rw, int KX,
                                                  int64_t o0x, int64_t n_ox, const uint32_t *bty, int64_t bty_rw,
                                                  int KY, int64_t o0y, int64_t n_oy) {
    const int tid = threadIdx.x;
    const int nx = KX * 16, ny = KY * 16, n = nx > ny ? nx : ny;
    auto load = [&](const uint32_t *bt, int64_t bt_rw, int64_t o0, int64_t n_o, int nn, int i) {
        const int k = i >> 4, c = i & 15;
        if (i < nn && o0 + (c >> 1) < n_o)
            return *reinterpret_cast<const PA_G u32x4 *>(gp(bt) + (int64_t)k * bt_rw + o0 * 8 + 4 * c);
        return u32x4{0u, 0u, 0u, 0u};
    };
    auto store = [&](int row0, int nn, int i, const u32x4 &v) {
        if (i < nn) {
            // words 4 (c & 1) .. + 3 of value o = c / 2
            const int c = i & 15, o = c >> 1;
            uint32_t *d = lds + (row0 + (i >> 4)) * kFusedPitch + 32 * (o >> 2) + 16 * (c & 1) + (o & 3);
            d[0] = v.x;
            d[4] = v.y;
            d[8] = v.z;
            d[12] = v.w;
        }
    };
    for (int i0 = 0; i0 < n; i0 += 4096) {
        u32x4 vx[4], vy[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            vx[u] = load(btx, btx_rw, o0x, n_ox, nx, i0 + u * 1024 + tid);
            vy[u] = load(bty, bty_rw, o0y, n_oy, ny, i0 + u * 1024 + tid);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            store(0, nx, i0 + u * 1024 + tid, vx[u]);
            store(KX, ny, i0 + u * 1024 + tid, vy[u]);
        }
    }
}

// The LDS byte addresses of the two list entries (16-bit row indices) in
// word e, each plus o0 (< 256, the lane's slot): (index << 8) | o0, built
// with one byte permutation each.
__device__ __forceinline__ uint32_t fused_addr_lo(uint32_t e, uint32_t o0) {
    return __builtin_amdgcn_perm(e, o0, 0x0c050400u);
}
__device__ __forceinline__ uint32_t fused_addr_hi(uint32_t e, uint32_t o0) {
    return __builtin_amdgcn_perm(e, o0, 0x0c070600u);
}

// N rows gathered into c with two 16-byte loads per row, at LDS byte
// addresses b and b ^ 128 (b = row start + o0).  Lane (a, w) (a = lane / 8,
// w = lane & 7) has o0 at the half of word w's values that holds values
// 4 (a & 1) .. + 3: c[v] |= value v ^ 4 (a & 1) of word w.  A 16-byte read
// is served in passes of 16 lanes, each pass taking 4 lanes from each of 4
// lane groups, two groups of each parity; with the halves alternating by
// group parity the 16 lanes of a pass read 16 distinct 16-byte slots of
// the 64 banks.  All loads are issued before any is used.
template <int N, bool First = false>
__device__ __forceinline__ void fused_gather(const uint32_t *lds, const uint32_t (&b)[N], uint32_t (&c)[8]) {
    const char *base = reinterpret_cast<const char *>(lds);
    u32x4 r[N][2];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        r[j][0] = *reinterpret_cast<const u32x4 *>(base + b[j]);
        r[j][1] = *reinterpret_cast<const u32x4 *>(base + (b[j] ^ 128u));
    }
    // First: c is set from these rows (no prior value to OR with)
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (First && j == 0) {
            c[0] = r[0][0].x;
            c[1] = r[0][0].y;
            c[2] = r[0][0].z;
            c[3] = r[0][0].w;
            c[4] = r[0][1].x;
            c[5] = r[0][1].y;
            c[6] = r[0][1].z;
            c[7] = r[0][1].w;
            continue;
        }
        c[0] |= r[j][0].x;
        c[1] |= r[j][0].y;
        c[2] |= r[j][0].z;
        c[3] |= r[j][0].w;
        c[4] |= r[j][1].x;
        c[5] |= r[j][1].y;
        c[6] |= r[j][1].z;
        c[7] |= r[j][1].w;
    }
}

// The list rows of one group, one per lane group (row a for lanes 8a ..
// 8a + 7): c[v] = OR over the entries of the lane group's row of value
// v ^ 4 (a & 1) of word w of its LDS row.  e holds the row's entries 0..7
// (loaded one latent entry ahead), m the group's entry count (uniform), ent
// the row's entries as words (two to a word), of which those beyond 8 are
// loaded here.  Whole pairs first, then an odd last entry alone.
__device__ __forceinline__ void fused_rows(const uint32_t *lds, uint32_t o0, const u32x4 &e, uint32_t m,
                                           const PA_G uint32_t *ent, uint32_t (&c)[8]) {
    const uint32_t mp = m >> 1;
    if (mp == 0u) {
        if (m == 0u) {
#pragma unroll
            for (int v = 0; v < 8; ++v) c[v] = 0u;
        } else {
            const uint32_t b[1] = {fused_addr_lo(e.x, o0)};
            fused_gather<1, true>(lds, b, c);
        }
        return;
    }
    if (mp == 1u) {
        const uint32_t b[2] = {fused_addr_lo(e.x, o0), fused_addr_hi(e.x, o0)};
        fused_gather<2, true>(lds, b, c);
    } else {
        {
            const uint32_t b[4] = {fused_addr_lo(e.x, o0), fused_addr_hi(e.x, o0), fused_addr_lo(e.y, o0),
                                   fused_addr_hi(e.y, o0)};
            fused_gather<4, true>(lds, b, c);
        }
        if (mp == 3u) {
            const uint32_t b[2] = {fused_addr_lo(e.z, o0), fused_addr_hi(e.z, o0)};
            fused_gather<2>(lds, b, c);
        } else if (mp >= 4u) {
            const uint32_t b[4] = {fused_addr_lo(e.z, o0), fused_addr_hi(e.z, o0), fused_addr_lo(e.w, o0),
                                   fused_addr_hi(e.w, o0)};
            fused_gather<4>(lds, b, c);
            for (uint32_t j = 4; j < mp; ++j) {
                const uint32_t t = ent[j];
                const uint32_t bb[2] = {fused_addr_lo(t, o0), fused_addr_hi(t, o0)};
                fused_gather<2>(lds, bb, c);
            }
        }
    }
    if (m & 1u) {
        const uint32_t t = mp == 1u ? e.y : mp == 2u ? e.z : mp == 3u ? e.w : ent[mp];
        const uint32_t b[1] = {fused_addr_lo(t, o0)};
        fused_gather<1>(lds, b, c);
    }
}

// Transpose of an 8 x 8 block held as c[j] in lane group a = lane / 8 (each
// of the group's 8 lanes holds its own word), whose odd groups hold their
// values with halves exchanged (c[j] of group a is value j ^ 4 (a & 1), as
// fused_gather leaves them): afterwards c[j] of group a is value a of group
// j.  Index bit 0 trades with lane bit 3 (DPP rotation by 8 within rows of
// 16 lanes, written to one half of each row), bit 1 with lane bit 4
// (v_permlane16_swap), bit 2 with lane bit 5 (v_permlane32_swap).  After the
// first two steps index bit 0 is the source group's parity, so the last
// step undoes the exchange by swapping the operands of the odd registers.
__device__ __forceinline__ void fused_transpose8(uint32_t (&c)[8]) {
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        const int a = (int)c[j], b = (int)c[j + 1];
        c[j] = (uint32_t)__builtin_amdgcn_update_dpp(a, b, 0x128, 0xf, 0xc, false);
        c[j + 1] = (uint32_t)__builtin_amdgcn_update_dpp(b, a, 0x128, 0xf, 0x3, false);
    }
#pragma unroll
    for (int j : {0, 1, 4, 5}) {
        const auto sw = __builtin_amdgcn_permlane16_swap(c[j], c[j + 2], false, false);
        c[j] = sw[0];
        c[j + 2] = sw[1];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const auto sw = (j & 1) ? __builtin_amdgcn_permlane32_swap(c[j + 4], c[j], false, false)
                                : __builtin_amdgcn_permlane32_swap(c[j], c[j + 4], false, false);
        c[j] = sw[0];
        c[j + 4] = sw[1];
    }
}

// One fused tile (1024 threads, 16 waves): 8 p x 8 q of the output (tile =
// pb n_qb + qb).  The rows of BtX for the tile's 8 p and of BtY for its 8 q
// are staged in LDS; the waves take latent entries s from a counter.  For
// one s, lane (a, w) gathers from the rows of its lane group's list rows:
// x[p] = X[q = a][s][p][w] from AX row (a, s) and y[q] = Y[p = a][s][q][w]
// from AY row (a, s) (two 16-byte loads per entry, free of bank conflicts,
// odd lane groups taking the halves of a word's values in the other order);
// x is transposed to lane (p, w), the halves of y put back in order, and the
// OR of x[q] AND y[q] kept.  The next s's list entries
// come with vector loads one s ahead.  The tile writes byte qb of its 8 output rows (the tile of the
// last q block also zeroes the row's padding bytes).
__device__ __forceinline__ void fused_tile(const FusedArgs &f, int64_t tile, uint32_t *lds) {
    const int64_t pb = tile / f.n_qb, qb = tile - pb * f.n_qb, p0 = pb * 8;
    const int tid = threadIdx.x, lane = tid & 63;
    // the 16-byte slot of word w in a row that holds values 4 (a & 1) .. + 3
    const uint32_t o0 = (uint32_t)(lane & 7) * 16u + (uint32_t)(lane & 8) * 16u;
    const bool odd = (lane & 8) != 0;
    // header: the latent-entry counter (word 0), 8 output bytes (a word each)
    uint32_t *cnt = lds, *out = lds + 8, *rows = lds + kFusedPitch;
    if (f.rwt == 8) {
        fused_stage8_pair(rows, f.BtX, f.btX_rw, f.kX, p0, f.n_p, f.BtY, f.btY_rw, f.kY, qb * 8, f.n_q);
    } else {
        fused_stage(rows, f.BtX, f.btX_rw, f.kX, p0, f.n_p, f.rwt, 0);
        fused_stage(rows, f.BtY, f.btY_rw, f.kY, qb * 8, f.n_q, f.rwt, f.kX);
    }
    if (tid < 64) rows[(f.kX + f.kY) * kFusedPitch + tid] = 0u;
    if (tid < 16) lds[tid] = 0u;
    __syncthreads();
    uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    // latent entries s come from the counter two ahead: the increment for
    // the s after next is issued as a step starts and its value read as the
    // step ends.  ds_append adds the number of active lanes (64: every wave
    // is whole here) and returns the former value.
    auto grab_issue = [&]() { return __builtin_amdgcn_ds_append((__attribute__((address_space(3))) int *)cnt); };
    auto grab_read = [&](int v) { return (int64_t)((uint32_t)__builtin_amdgcn_readfirstlane(v) >> 6); };
    // the list rows of lane group a: AX row (q = a, s) of group (qb, s) and
    // AY row (p = a, s) of group (pb, s) (entries 0..7 one 16-byte load);
    // the groups' entry counts
    const int a = lane >> 3;
    struct Lists {
        u32x4 x, y;
        uint32_t mx, my;
    };
    // a list row: its group's first row (uniform) plus the lane group's
    // byte offset
    const uint32_t offX = (uint32_t)a * (uint32_t)f.capX * 2u, offY = (uint32_t)a * (uint32_t)f.capY * 2u;
    auto list_row = [&](const uint16_t *ent, int64_t g, int64_t cap, uint32_t off) {
        return reinterpret_cast<const PA_G uint32_t *>(reinterpret_cast<const PA_G char *>(gp(ent) + g * 8 * cap) + off);
    };
    auto fetch = [&](int64_t s, Lists &l) {
        const int64_t gx = qb * f.n_s + s, gy = pb * f.n_s + s;
        l.x = *reinterpret_cast<const PA_G u32x4 *>(list_row(f.entX, gx, f.capX, offX));
        l.y = *reinterpret_cast<const PA_G u32x4 *>(list_row(f.entY, gy, f.capY, offY));
        l.mx = gp(f.metaX)[gx];
        l.my = gp(f.metaY)[gy];
    };
    // one step: s with lists c (in hand), the lists of sn into n (sn past
    // the end fetches the last s's, unused); returns the s after sn
    auto step = [&](int64_t s, int64_t sn, const Lists &c, Lists &n) {
        const int snn = grab_issue();
        fetch(sn < f.n_s ? sn : f.n_s - 1, n);
        const int64_t gx = qb * f.n_s + s, gy = pb * f.n_s + s;
        uint32_t x[8], y[8];
        fused_rows(rows, o0, c.y, __builtin_amdgcn_readfirstlane(c.my), list_row(f.entY, gy, f.capY, offY), y);
        fused_rows(rows, o0, c.x, __builtin_amdgcn_readfirstlane(c.mx), list_row(f.entX, gx, f.capX, offX), x);
        fused_transpose8(x);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t lo = y[i], hi = y[i + 4];
            y[i] = odd ? hi : lo;
            y[i + 4] = odd ? lo : hi;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] |= x[i] & y[i];
        return grab_read(snn);
    };
    int64_t s = grab_read(grab_issue());
    int64_t sn = grab_read(grab_issue());
    Lists cur;
    if (s < f.n_s) fetch(s, cur);
    // the first lists arrive before the loop (s_waitcnt vmcnt(0)), so that
    // within it only the lists of the next s are in flight while a step
    // works
    __builtin_amdgcn_s_waitcnt(0x0F70);
    while (s < f.n_s) {
        Lists nxt;
        const int64_t snn = step(s, sn, cur, nxt);
        s = sn;
        sn = snn;
        cur = nxt;
    }
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) bits |= (acc[i] != 0u ? 1u : 0u) << i;
    if (bits) atomicOr(out + (lane >> 3), bits);
    __syncthreads();
    if (tid < 8 && p0 + tid < f.n_p) {
        PA_G uint8_t *row = reinterpret_cast<PA_G uint8_t *>(gp(f.C) + (p0 + tid) * f.c_rw);
        row[qb] = (uint8_t)out[tid];
        if (qb == f.n_qb - 1)
            for (int64_t b = qb + 1; b < 4 * f.c_rw; ++b) row[b] = 0;
    }
}

// ------------------------------------------------- LDS read-rate reference
// One workgroup of 1024 threads per CU; every lane reads its own 16-byte slot
// of a 64 KiB LDS array (free of bank conflicts), 8 independent reads per
// iteration, folded into one word per lane that is written out (so that the
// reads stay).  The measured rate is the reference of the LDS-bound fused
// step's roofline.
__global__ __launch_bounds__(1024, 1) void k_lds_rate(uint32_t *out, int iters) {
    __shared__ __attribute__((aligned(16))) u32x4 lds[4096];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < 4096; i += 1024) lds[i] = u32x4{(uint32_t)i, (uint32_t)i + 1u, (uint32_t)i + 2u, (uint32_t)i + 3u};
    __syncthreads();
    const char *base = reinterpret_cast<const char *>(lds);
    const uint32_t w = (uint32_t)(tid >> 6);
    uint32_t acc0 = 0u, acc1 = 0u;
    for (int it = 0; it < iters; ++it) {
        const uint32_t blk = ((uint32_t)it * 8u + w) & 63u;
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // 1 KiB block (blk + 8 j) mod 64, slot lane
            const u32x4 a = *reinterpret_cast<const u32x4 *>(base + ((blk + 8u * (uint32_t)j) & 63u) * 1024u +
                                                             (uint32_t)lane * 16u);
            v[j] = a.x ^ a.y ^ a.z ^ a.w;
        }
        acc0 ^= v[0] ^ v[1] ^ v[2] ^ v[3];
        acc1 ^= v[4] ^ v[5] ^ v[6] ^ v[7];
    }
    gp(out)[(int64_t)blockIdx.x * 1024 + tid] = acc0 + acc1;
}

hipError_t launch_lds_rate(uint32_t *out, int blocks, int iters, hipStream_t s) {
    if (blocks <= 0 || iters <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lds_rate, dim3((unsigned)blocks), dim3(1024), 0, s, out, iters);
    return hipGetLastError();
}

// ------------------------------------------------------------ fill, count
__global__ void k_fill(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void k_popcount(const uint32_t *p, int64_t n, unsigned long long *out) {
    __shared__ unsigned long long part[4];
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += __popc(p[i]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

// Set bits per tile (tile_rows rows x tile_words words of a rows x rw word
// array): one workgroup per tile, grid-stride over tiles, a block reduction.
__global__ __launch_bounds__(256) void k_tile_popcount(const uint32_t *p, int64_t rows, int64_t rw, int tile_rows,
                                                       int tile_words, int64_t tiles_r, int64_t tiles_w,
                                                       uint32_t *out) {
    __shared__ uint32_t part[4];
    const int64_t ntiles = tiles_r * tiles_w;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t tr = t / tiles_w, tw = t - tr * tiles_w;
        const int64_t r0 = tr * tile_rows, w0 = tw * tile_words;
        const int64_t nr = min((int64_t)tile_rows, rows - r0), nw = min((int64_t)tile_words, rw - w0);
        uint32_t c = 0;
        for (int64_t i = threadIdx.x; i < nr * nw; i += blockDim.x) {
            const int64_t rr = i / nw, ww = i - rr * nw;
            c += __popc(p[(r0 + rr) * rw + w0 + ww]);
        }
        for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) out[t] = part[0] + part[1] + part[2] + part[3];
        __syncthreads();
    }
}

hipError_t launch_tile_popcount(const uint32_t *p, int64_t rows, int64_t rw, int tile_rows, int tile_words,
                                uint32_t *out, hipStream_t s) {
    const int64_t tiles_r = (rows + tile_rows - 1) / tile_rows, tiles_w = (rw + tile_words - 1) / tile_words;
    const int64_t nt = tiles_r * tiles_w;
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_popcount, dim3((unsigned)(nt < (1 << 20) ? nt : (1 << 20))), dim3(256), 0, s, p, rows,
                       rw, tile_rows, tile_words, tiles_r, tiles_w, out);
    return hipGetLastError();
}

hipError_t launch_popcount(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_popcount, dim3((unsigned)blocks), dim3(256), 0, s, p, n, out);
    return hipGetLastError();
}

// ------------------------------------------------- grouped executors
// Steps of one kind on one level of the cluster tree (possibly from many
// systems), contiguous in the step table, run by one launch; tiles are
// numbered by the steps' tile_base prefix.  A plotting launch also runs the
// fill steps of its level.
// The step holding tile `item`: the last of steps[first..first+count) whose
// tile_base is <= item.  With a full wave and at most 64 steps, every lane
// reads one tile_base at once and the answer is the population count of the
// ballot (tile bases ascend); otherwise a binary search.
__device__ __forceinline__ int find_step(const PStep *steps, int first, int count, int64_t item) {
    if (count <= 64 && __builtin_amdgcn_read_exec() == ~0ull) {
        const int lane = __lane_id();
        const int64_t tb = lane < count ? gp(steps)[first + lane].tile_base : INT64_MAX;
        return first + (int)__popcll(__ballot(tb <= item)) - 1;
    }
    int lo = first, hi = first + count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (steps[mid].tile_base <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// LDS words of a grouped kernel of kind KIND % 10, mode KIND / 10
template <int KIND>
constexpr int group_lds_words() {
    return KIND % 10 == kStepGemm ? gemm_lds_of(KIND / 10) : (KIND % 10 == kStepPlot ? kPlotLdsWords : 1);
}

// Items [t0, t1) of steps first .. first + count - 1 (one group: the same
// kind and mode), as workgroup bid of nbid runs its share of them.  KIND:
// a StepKind; for MFMA contractions and contractions the mode is fixed too
// (kind + 10 * mode).  lds holds group_lds_words<KIND>() words.
template <int KIND>
__device__ __forceinline__ void group_run(const PStep *__restrict__ steps, int first, int count, int64_t t0,
                                          int64_t t1, int flags, PlotCounters *counters, uint32_t *lds,
                                          uint32_t bid, uint32_t nbid) {
    constexpr int kind = KIND % 10, mode = KIND / 10;
    if (kind == kStepGemm) {
        // with `flags`, a contraction whose sparse pass handled every row is
        // skipped: lane i reads the flag of step first + i (at most 64 steps;
        // with more, every contraction runs: it writes the same bits)
        uint64_t active = ~0ull;
        if (flags && count <= 64) {
            const int lane = __lane_id();
            const uint32_t *dn = lane < count ? steps[first + lane].gemm.dense : nullptr;
            const bool on =
                lane < count && (!dn || __hip_atomic_load(gp(dn), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u);
            active = __ballot(on);
            if (active == 0) return;
        }
        if constexpr (mode == 3) {
            // a contiguous range of tiles per workgroup (the resident path
            // keeps A operands while consecutive tiles share their rows),
            // run one step at a time with a uniform copy of the step's
            // arguments (scalar registers, scalar tile decoding)
            int64_t lo, hi;
            res_range(t1 - t0, lo, hi, bid, nbid);
            int64_t item = t0 + lo;
            const int64_t iend = t0 + hi;
            while (item < iend) {
                // a scalar binary search (item is uniform)
                int si = first, sh = first + count - 1;
                while (si < sh) {
                    const int mid = (si + sh + 1) >> 1;
                    if (gp(steps)[mid].tile_base <= item) si = mid;
                    else sh = mid - 1;
                }
                si = __builtin_amdgcn_readfirstlane(si);
                const PStep &st = steps[si];
                const int64_t sb = st.tile_base, se = min(iend, sb + st.n_tiles);
                if ((active >> ((si - first) & 63)) & 1) {
                    const GemmArgs g = st.gemm;
                    int64_t t = item - sb;
                    const int64_t tend = se - sb;
                    auto next = [&](GemmTileRef &T) {
                        if (t >= tend) return false;
                        T = gemm_locate<4>(g, t++);
                        return true;
                    };
                    gemm_run<mode>(next, lds);
                    __syncthreads();          // the LDS is free for the next step
                }
                item = se;
            }
            return;
        }
        // persistent tile loop with cross-tile prefetch, tiles in XCD-aware order
        const int64_t per = (t1 - t0 + 7) >> 3;
        int64_t t = bid;
        auto next = [&](GemmTileRef &T) {
            for (; t < 8 * per; t += nbid) {
                const int64_t item = t0 + xcd_tile(t, per);
                if (item < t1) {
                    const int si = find_step(steps, first, count, item);
                    if (!((active >> ((si - first) & 63)) & 1)) continue;
                    const PStep &st = steps[si];
                    T = gemm_locate<mode == 2 ? 4 : 2>(st.gemm, item - st.tile_base);
                    t += nbid;
                    return true;
                }
            }
            return false;
        };
        gemm_run<mode>(next, lds);
        return;
    }
    if (kind == kStepGather) {
        // persistent waves over the launch's wave-tiles (no barriers); a
        // wave decides once per step (its first tile of a step is the one
        // with the lowest index, so the wave holding tile 0 writes the
        // decision word) and starts the loads of its next tile's A row
        // before working on the current one
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const int64_t slots = (t1 - t0) * 4, stride = (int64_t)nbid * 4;
        int si = -1;
        int64_t wt = 0;
        // the first slot at or after gi holding a wave-tile (slots if none)
        auto seek = [&](int64_t gi) {
            for (; gi < slots; gi += stride) {
                const int64_t item = t0 + (gi >> 2);
                si = find_step(steps, first, count, item);
                wt = (item - steps[si].tile_base) * 4 + (gi & 3);
                if (wt < gather_wave_tiles(steps[si].gather)) break;
            }
            return gi;
        };
        int64_t gi = seek((int64_t)bid * 4 + wave);
        RowBits rb;
        if (gi < slots) rb = gather_row_issue(steps[si].gather, wt);
        int decided = -1;
        bool run = false;
        while (gi < slots) {
            const int cs = si;
            const int64_t cwt = wt;
            const RowBits cur = rb;
            gi = seek(gi + stride);
            if (gi < slots) rb = gather_row_issue(steps[si].gather, wt);
            const GatherArgs &g = steps[cs].gather;
            if (cs != decided) {
                decided = cs;
                run = gather_decide(g, cwt);
            }
            if (run) gather_wave(g, cwt, cur);
        }
        return;
    }
    CountSink sink;
    for (int64_t item = t0 + bid; item < t1; item += nbid) {
        const PStep &st = steps[find_step(steps, first, count, item)];
        if (kind == kStepPlot && st.kind == kStepPlot) {
            sink.use(st.plot, counters);
            // mode 3: any corner tile (the single persistent launch)
            plot_tile_rule<mode == 3 ? -1 : mode>(st.plot, item - st.tile_base, reinterpret_cast<float *>(lds),
                      reinterpret_cast<double *>(lds + kPlotLineWords), sink.cnt);
        } else if (kind == kStepContract) {
            const int64_t u0 = (item - st.tile_base) * st.per_tile;
            contract_range<mode>(st.ca, u0, min(st.units, u0 + st.per_tile));
        } else if (kind == kStepCount) {
            count_tile(st.gather, item - st.tile_base);
        } else if (kind == kStepList) {
            row_list_tile(st.list, item - st.tile_base);
        } else {
            const int64_t u0 = (item - st.tile_base) * st.per_tile, u1 = min(st.units, u0 + st.per_tile);
            for (int64_t i = u0 + threadIdx.x; i < u1; i += blockDim.x) gp(st.fill_ptr)[i] = 0u;
        }
        __syncthreads();
    }
    if (kind == kStepPlot) sink.finish();
}


// Minimum waves per SIMD of a grouped kernel: the MFMA paths' own, else
// left to the compiler.
template <int KIND>
constexpr int group_occupancy() {
    return KIND % 10 == kStepGemm ? gemm_occupancy(KIND / 10) : 1;
}

template <int KIND>
__global__ __launch_bounds__(256, group_occupancy<KIND>()) void k_group(
    const PStep *__restrict__ steps, int first, int count, int64_t t0, int64_t t1, int flags,
    PlotCounters *counters) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[group_lds_words<KIND>()];
    group_run<KIND>(steps, first, count, t0, t1, flags, counters, lds, blockIdx.x, gridDim.x);
}

// Fused pass pairs of one level: one tile per workgroup of 1024 threads,
// with a uniform copy of its step's arguments (C, when not null, replaces
// their output pointer: one step launched on its own).
__global__ __launch_bounds__(1024, 1) void k_fused_group(const PStep *__restrict__ steps, int first, int count,
                                                         int64_t t0, int64_t t1, uint32_t *C) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[kFusedLdsWords];
    for (int64_t item = t0 + blockIdx.x; item < t1; item += gridDim.x) {
        const int si = __builtin_amdgcn_readfirstlane(find_step(steps, first, count, item));
        FusedArgs f = steps[si].fused;
        if (C) f.C = C;
        fused_tile(f, item - steps[si].tile_base, lds);
        __syncthreads();
    }
}

hipError_t launch_fused(const PStep *d_step, int64_t n_tiles, uint32_t *C, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(n_tiles < (1 << 20) ? n_tiles : (1 << 20));
    hipLaunchKernelGGL(k_fused_group, dim3(grid), dim3(1024), 0, s, d_step, 0, 1, (int64_t)0, n_tiles, C);
    return hipGetLastError();
}

// Workgroups of the persistent sparse-pass loop: every CU's worth.
static int64_t gather_grid() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, cus = 256, per_cu = 1;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_group<kStepGather>, 256, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        cached = cus * per_cu;
    }
    return cached;
}

hipError_t launch_group(int kind, int mode, const PStep *d_steps, int first, int count, int64_t t0, int64_t t1,
                        int flags, PlotCounters *counters, hipStream_t s) {
    if (t1 <= t0) return hipSuccess;
    const int64_t nt = t1 - t0;
    if (kind == kStepGemm && (mode < 0 || mode > 3)) return hipErrorInvalidValue;
    const int64_t cap = kind == kStepGather ? gather_grid() : ((int64_t)1 << 20);
    const dim3 grid((unsigned)(kind == kStepGemm ? gemm_grid(nt, mode) : (nt < cap ? nt : cap)));
#define PA_GROUP(K) hipLaunchKernelGGL(k_group<K>, grid, dim3(256), 0, s, d_steps, first, count, t0, t1, flags, counters)
    switch (kind) {
        case kStepPlot:
            if (mode == 1) PA_GROUP(kStepPlot + 10);      // centre-rule plots
            else if (mode == 2) PA_GROUP(kStepPlot + 20); // fixed-axis-walking trivariate corner plots
            else PA_GROUP(kStepPlot);
            break;
        case kStepGemm:
            if (mode == 1) PA_GROUP(kStepGemm + 10);
            else if (mode == 2) PA_GROUP(kStepGemm + 20);
            else if (mode == 3) PA_GROUP(kStepGemm + 30);
            else PA_GROUP(kStepGemm);
            break;
        case kStepContract:
            if (mode == kModeStreamK) PA_GROUP(kStepContract + 10 * kModeStreamK);
            else if (mode == kModeStreamW) PA_GROUP(kStepContract + 10 * kModeStreamW);
            else PA_GROUP(kStepContract + 10 * kModeBits);
            break;
        case kStepGather: PA_GROUP(kStepGather); break;
        case kStepCount: PA_GROUP(kStepCount); break;
        case kStepList: PA_GROUP(kStepList); break;
        case kStepFused:
            hipLaunchKernelGGL(k_fused_group, grid, dim3(1024), 0, s, d_steps, first, count, t0, t1,
                               static_cast<uint32_t *>(nullptr));
            break;
        default: PA_GROUP(kStepFill); break;
    }
#undef PA_GROUP
    return hipGetLastError();
}

// ------------------------------------------------- persistent executor
// One launch runs the whole step table.  The grouped executor's launches
// become chunks of work: chunk c of group g is items t0 + c chunk .. of that
// group (at most `chunk` of them), run by one workgroup with the grouped
// kernel's own tile loop (group_run).  Workgroups take chunks from one
// counter in table order, i.e. by ascending dependency level.  Before its
// first chunk of a level L > 0 a workgroup waits until every item of level
// L - 1 is done (one done counter per level): every step depends on lower
// levels only, the levels finish in order, and every chunk of a lower level
// was taken earlier by a running workgroup, so the waits end whether or not
// all workgroups are resident at once.  A wait is bounded by
// state->wait_limit polls (2^26 unless the host set another bound; a
// negative bound gives up at the first wait, so that tests reach this path
// with every kernel exiting): then `abort` is set and every workgroup leaves.
// Coherence across XCDs: after a chunk, the workgroup barrier orders its
// waves' stores and one thread's agent-scope release (the done-count add)
// writes them back from the XCD's L2; the waiting thread's agent-scope
// acquire, once its polls succeed, invalidates the stale lines of its CU and
// XCD before the workgroup reads the level's inputs.
constexpr int kPersistLdsWords = kGemmLdsWords > kPlotLdsWords ? kGemmLdsWords : kPlotLdsWords;

__global__ __launch_bounds__(256, 2) void k_persist(const PStep *__restrict__ steps,
                                                    const PGroup *__restrict__ groups, int ngroups,
                                                    int64_t nchunks, const int64_t *__restrict__ level_items,
                                                    unsigned long long *level_done, PersistState *state,
                                                    PlotCounters *counters) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[kPersistLdsWords];
    __shared__ long long s_chunk;
    __shared__ int s_ok;
    const long long limit = __hip_atomic_load(&state->wait_limit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int known = -1;       // levels up to `known` are complete (uniform)
    for (;;) {
        if (threadIdx.x == 0)
            s_chunk = (long long)__hip_atomic_fetch_add(&state->queue, 1ull, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int64_t c = s_chunk;
        if (c >= nchunks) break;
        // the group of chunk c: a scalar binary search over the chunk bases
        int gi = 0, gh = ngroups - 1;
        while (gi < gh) {
            const int mid = (gi + gh + 1) >> 1;
            if (gp(groups)[mid].cbase <= c) gi = mid;
            else gh = mid - 1;
        }
        gi = __builtin_amdgcn_readfirstlane(gi);
        const PA_G PGroup *g = gp(groups) + gi;
        const int level = g->level;
        if (level > 0 && known < level - 1) {
            if (threadIdx.x == 0) {
                int ok = 1;
                const unsigned long long need = (unsigned long long)gp(level_items)[level - 1];
                long long spins = 0;
                if (limit < 0) ok = 0;
                while (ok && __hip_atomic_load(&level_done[level - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                                 need) {
                    if (__hip_atomic_load(&state->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
                    else if (++spins > limit) ok = 0;
                    else __builtin_amdgcn_s_sleep(1);
                }
                if (!ok) __hip_atomic_store(&state->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                s_ok = ok;
            }
            __syncthreads();
            if (!s_ok) break;
            known = level - 1;
        }
        const int64_t i0 = g->t0 + (c - g->cbase) * g->chunk;
        const int64_t i1 = min(g->t1, i0 + g->chunk);
        const int first = g->first, count = g->count;
        switch (g->kind + 10 * g->mode) {
            case kStepPlot:
            case kStepPlot + 20:
                group_run<kStepPlot + 30>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u);
                break;
            case kStepGemm: group_run<kStepGemm>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u); break;
            case kStepGemm + 10:
                group_run<kStepGemm + 10>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u);
                break;
            case kStepContract + 10 * kModeStreamK:
                group_run<kStepContract + 10 * kModeStreamK>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u);
                break;
            case kStepContract + 10 * kModeStreamW:
                group_run<kStepContract + 10 * kModeStreamW>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u);
                break;
            case kStepContract + 10 * kModeBits:
                group_run<kStepContract + 10 * kModeBits>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u);
                break;
            default: group_run<kStepFill>(steps, first, count, i0, i1, 0, counters, lds, 0u, 1u); break;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&level_done[level], (unsigned long long)(i1 - i0), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_persist_reset(PersistState *state, unsigned long long *level_done, int nlevels) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nlevels; i += gridDim.x * blockDim.x) level_done[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        state->queue = 0ull;
        state->abort = 0u;
    }
}

hipError_t launch_persist_reset(PersistState *state, unsigned long long *level_done, int nlevels, hipStream_t s) {
    hipLaunchKernelGGL(k_persist_reset, grid_for(nlevels > 0 ? nlevels : 1), dim3(256), 0, s, state, level_done,
                       nlevels);
    return hipGetLastError();
}

// Default persistent grid: as many workgroups as fit on the device at once.
int persist_default_workgroups() {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    cached = cus * per_cu;
    return cached;
}

hipError_t launch_persist(const PStep *d_steps, const PGroup *d_groups, int ngroups, int64_t nchunks,
                          const int64_t *level_items, unsigned long long *level_done, PersistState *state,
                          PlotCounters *counters, int n_workgroups, hipStream_t s) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_persist, dim3((unsigned)n_workgroups), dim3(256), 0, s, d_steps, d_groups, ngroups, nchunks,
                       level_items, level_done, state, counters);
    return hipGetLastError();
}

}  // namespace pa
