// gfx950 kernels of the pixel array method: corner plotting with FP32
// evaluation and FP64 escalation, bitwise OR-of-AND contractions, and a dense
// Boolean contraction on int8 MFMA with int32 accumulation.
//
// Build flags (see build.py): -O3 --offload-arch=gfx950 -ffp-contract=off
// (no implicit FMA: every fused multiply-add below is an explicit fma/fmaf).
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "pa_internal.h"

namespace pa {

// ------------------------------------------------------------------ helpers
// Blocks for `total` threads, capped (the kernels loop over the rest).
static dim3 grid_for(int64_t total) {
    int64_t blocks = (total + 255) / 256;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    if (blocks < 1) blocks = 1;
    return dim3((unsigned)blocks);
}

__device__ __forceinline__ int find_by_base(const PlotRel *rels, int nrel, int64_t idx, bool lines) {
    int lo = 0, hi = nrel - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int64_t b = lines ? rels[mid].line_base : rels[mid].word_base;
        if (b <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Canonical FP64 value of a relation at a point given in DECLARED variable
// order: nested Horner, last declared variable outermost, fma at every step.
// c is the dense table c[e0 + (d+1)*(e1 + (d+1)*e2)].
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

// ------------------------------------------------------------ plot: lines
// For every corner line (fixed corner indices on the non-packed storage axes)
// of an FP32-mode relation: the univariate coefficients a_t of the relation
// restricted to the line (in the packed variable), rounded to FP32, and the
// FP32 error bound E of evaluating them by Horner at any corner of the line.
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
// A corner is escalated unless E < |p^| <= FLT_MAX; otherwise
// |f_exact| > E - gamma S >= |f64 - f_exact|, so sign(p^) = sign(f64) != 0.
__global__ void k_plot_lines(const PlotRel *__restrict__ rels, int nrel, int64_t total_lines) {
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total_lines;
       gid += (int64_t)gridDim.x * blockDim.x) {
    const PlotRel &R = rels[find_by_base(rels, nrel, gid, true)];
    const int64_t L = gid - R.line_base;
    if (L >= R.n_lines) continue;
    const int n = R.n, d = R.d, D1 = d + 1;
    const int pk = R.perm[n - 1];                 // declared index of the packed variable
    double xd[kMaxA] = {0.0, 0.0, 0.0};
    int64_t rem = L;
    for (int s = n - 2; s >= 0; --s) {
        const int64_t dim = R.res[s] + 1;
        const int64_t i = rem % dim;
        rem /= dim;
        xd[R.perm[s]] = R.ax[s][i];
    }
    double a[kMaxD + 1], sab[kMaxD + 1];
    for (int t = 0; t <= kMaxD; ++t) { a[t] = 0.0; sab[t] = 0.0; }
    const int e2max = (n > 2) ? d : 0;
    for (int e2 = 0; e2 <= e2max; ++e2) {
        const int e1max = (n > 1) ? d - e2 : 0;
        for (int e1 = 0; e1 <= e1max; ++e1) {
            for (int e0 = 0; e0 <= d - e1 - e2; ++e0) {
                const double c = R.coef[e0 + D1 * (e1 + D1 * e2)];
                const int e[3] = {e0, e1, e2};
                double term = c;
                for (int v = 0; v < n; ++v) {
                    if (v == pk) continue;
                    for (int q = 0; q < e[v]; ++q) term *= xd[v];
                }
                a[e[pk]] += term;
                sab[e[pk]] += fabs(term);
            }
        }
    }
    const double V = fmax(1.0, R.vmax);
    double S = 0.0, Vp = 1.0;
    for (int t = 0; t <= d; ++t) { S += sab[t] * Vp; Vp *= V; }
    const double u = 0x1p-24;
    const double K = 2.0 * d + 1.0;
    const double gam = K * u / (1.0 - K * u);
    const double E = (gam + 0x1p-40) * S * (1.0 + 0x1p-30) + 0x1p-100 * (1.0 + S) * Vp;
    float Ef = (float)E;
    if ((double)Ef < E) Ef = nextafterf(Ef, INFINITY);
    float *dst = R.lines + L * (kMaxD + 2);
    for (int t = 0; t <= d; ++t) dst[t] = (float)a[t];
    dst[kMaxD + 1] = Ef;
  }
}

// ------------------------------------------------------------ plot: cells
// One thread per output word: 32 cells along the packed axis at fixed cell
// indices on the other axes.  The cell is set iff its 2^n corners include
// f <= 0 and f >= 0 (closed cells; a NaN corner counts as neither).
// A corner is evaluated by every thread whose cells touch it; only its owner
// counts it (lower cell on every axis, or the last cell where there is none).
__global__ void k_plot_cells(const PlotRel *__restrict__ rels, int nrel, int64_t total_words,
                             PlotCounters *__restrict__ counters) {
  unsigned long long nflag = 0, ndis = 0, ndis_unf = 0;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < total_words; g0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gid = g0 + threadIdx.x;
    if (gid < total_words) {
        const PlotRel &R = rels[find_by_base(rels, nrel, gid, false)];
        const int64_t local = gid - R.word_base;
        const int64_t row = local / R.row_words;
        const int64_t w = local % R.row_words;
        const int n = R.n, d = R.d;
        const int rp = R.res[n - 1];
        uint32_t word = 0;
        if (w * 32 < rp) {
            int cidx[kMaxA] = {0, 0, 0};
            int64_t rem = row;
            for (int s = n - 2; s >= 0; --s) { cidx[s] = (int)(rem % R.res[s]); rem /= R.res[s]; }
            const int k0 = (int)(w * 32);
            const int kmax = min(32, rp - k0);         // cells in this word
            uint64_t cl = 0, cg = 0;
            const int nlines = 1 << (n - 1);
            for (int dl = 0; dl < nlines; ++dl) {
                int li[kMaxA] = {0, 0, 0};
                int64_t L = 0;
                for (int s = 0; s < n - 1; ++s) {
                    li[s] = cidx[s] + ((dl >> s) & 1);
                    L = L * (R.res[s] + 1) + li[s];
                }
                double xdec[kMaxA] = {0.0, 0.0, 0.0};
                bool line_owned = true;
                for (int s = 0; s < n - 1; ++s) {
                    xdec[R.perm[s]] = R.ax[s][li[s]];
                    line_owned &= (((dl >> s) & 1) == 0) || (li[s] == R.res[s]);
                }
                const int pk = R.perm[n - 1];
                uint64_t LE = 0, GE = 0;
                if (R.mode == PA_PLOT_FP32_ESCALATE) {
                    const float *ln = R.lines + L * (kMaxD + 2);
                    float ca[kMaxD + 1];
                    for (int t = 0; t <= kMaxD; ++t) ca[t] = (t <= d) ? ln[t] : 0.0f;
                    const float E = ln[kMaxD + 1];
                    for (int kk = 0; kk <= kmax; ++kk) {
                        const float x = R.axf[n - 1][k0 + kk];
                        float f = ca[d];
                        for (int t = d - 1; t >= 0; --t) f = fmaf(f, x, ca[t]);
                        const float af = fabsf(f);
                        const bool ok = (af > E) && (af <= FLT_MAX);
                        const bool own = line_owned && (kk < kmax || k0 + kk == rp);
                        bool le, ge;
                        if (ok && !R.audit) {
                            le = f < 0.0f;
                            ge = f > 0.0f;
                        } else {
                            xdec[pk] = R.ax[n - 1][k0 + kk];
                            const double f64 = canon_eval(R.coef, n, d, xdec);
                            le = f64 <= 0.0;
                            ge = f64 >= 0.0;
                            if (R.audit) {
                                const int s32 = (f > 0.0f) - (f < 0.0f);
                                const int s64 = (f64 > 0.0) - (f64 < 0.0);
                                const bool dis = (s32 != s64) || (f != f) || (f64 != f64);
                                ndis += dis && own;
                                if (ok) ndis_unf += dis && own;
                                if (ok) { le = f < 0.0f; ge = f > 0.0f; }
                            }
                        }
                        nflag += (!ok) && own;
                        LE |= (uint64_t)le << kk;
                        GE |= (uint64_t)ge << kk;
                    }
                } else {
                    for (int kk = 0; kk <= kmax; ++kk) {
                        xdec[pk] = R.ax[n - 1][k0 + kk];
                        const double f64 = canon_eval(R.coef, n, d, xdec);
                        LE |= (uint64_t)(f64 <= 0.0) << kk;
                        GE |= (uint64_t)(f64 >= 0.0) << kk;
                    }
                }
                cl |= LE | (LE >> 1);
                cg |= GE | (GE >> 1);
            }
            const uint32_t valid = (kmax == 32) ? 0xFFFFFFFFu : ((1u << kmax) - 1u);
            word = (uint32_t)(cl & cg) & valid;
        }
        R.out[local] = word;
    }
  }
    // counters: one atomic per wave, only when something was counted
    const unsigned long long any = __ballot(nflag != 0 || ndis != 0 || ndis_unf != 0);
    if (any && counters) {
        if (nflag) atomicAdd(&counters->flagged, nflag);
        if (ndis) atomicAdd(&counters->disagree, ndis);
        if (ndis_unf) atomicAdd(&counters->disagree_unflagged, ndis_unf);
    }
}

hipError_t launch_plot(const PlotRel *d_rels, int nrel, int64_t total_lines, int64_t total_words,
                       int mode_any_fp32, PlotCounters *d_counters, hipStream_t s, int *n_launches) {
    if (mode_any_fp32 && total_lines > 0) {
        hipLaunchKernelGGL(k_plot_lines, grid_for(total_lines), dim3(256), 0, s, d_rels, nrel, total_lines);
        if (n_launches) ++*n_launches;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (total_words > 0) {
        hipLaunchKernelGGL(k_plot_cells, grid_for(total_words), dim3(256), 0, s, d_rels, nrel, total_words,
                           d_counters);
        if (n_launches) ++*n_launches;
    }
    return hipGetLastError();
}

// --------------------------------------------------- bitwise contractions
__device__ __forceinline__ void decode_out(const ContractArgs &a, int64_t row, int64_t bit, int64_t *c) {
    if (a.nout > 0) c[a.nout - 1] = bit;
    int64_t rem = row;
    for (int i = a.nout - 2; i >= 0; --i) { c[i] = rem % a.out_dim[i]; rem /= a.out_dim[i]; }
}

// General mode: one thread per output bit; every latent entry visited bit by
// bit (any layouts).
__global__ void k_contract_bits(ContractArgs a, int64_t total) {
  // grid-stride over whole blocks: every wave keeps 64 consecutive bits
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < total; g0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gid = g0 + threadIdx.x;
    const int64_t rowbits = a.c_row_words * 32;
    const int64_t row = gid / rowbits, bit = gid % rowbits;
    bool valid;
    if (a.nout == 0) valid = (gid == 0);
    else valid = (row < a.n_out_rows) && (bit < a.out_dim[a.nout - 1]);
    unsigned acc = 0;
    if (valid) {
        int64_t c[kMaxDim];
        decode_out(a, row, bit, c);
        int64_t baseA = 0, baseB = 0;
        for (int i = 0; i < a.nout; ++i) { baseA += c[i] * a.a_str[i]; baseB += c[i] * a.b_str[i]; }
        const int64_t pa_out = (a.a_pk_out >= 0) ? c[a.a_pk_out] : 0;
        const int64_t pb_out = (a.b_pk_out >= 0) ? c[a.b_pk_out] : 0;
        int64_t kidx[kMaxDim];
        for (int j = 0; j < a.nk; ++j) kidx[j] = 0;
        int64_t offA = 0, offB = 0;
        for (;;) {
            const int64_t pa = (a.a_pk_k >= 0) ? kidx[a.a_pk_k] : pa_out;
            const int64_t pb = (a.b_pk_k >= 0) ? kidx[a.b_pk_k] : pb_out;
            const unsigned ba = (a.A[baseA + offA + (pa >> 5)] >> (pa & 31)) & 1u;
            const unsigned bb = a.B ? ((a.B[baseB + offB + (pb >> 5)] >> (pb & 31)) & 1u) : 1u;
            if (ba & bb) { acc = 1; break; }
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
            if (j < 0) break;
        }
    }
    const unsigned long long bits = __ballot(acc != 0);
    if ((threadIdx.x & 63) == 0 && gid < (a.nout == 0 ? 1 : a.n_out_rows * rowbits)) {
        if (a.nout == 0) {
            a.C[0] = (uint32_t)(bits & 1ull);
        } else {
            uint32_t *dst = a.C + row * a.c_row_words + bit / 32;
            dst[0] = (uint32_t)bits;
            dst[1] = (uint32_t)(bits >> 32);
        }
    }
  }
}

// Stream mode K: A and B are both bit-packed along the same latent variable;
// words are AND-ed along it (16 bytes at a time when rows allow).
template <bool VEC4>
__global__ void k_contract_stream_k(ContractArgs a, int64_t total) {
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < total; g0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gid = g0 + threadIdx.x;
    const int64_t rowbits = a.c_row_words * 32;
    const int64_t row = gid / rowbits, bit = gid % rowbits;
    bool valid;
    if (a.nout == 0) valid = (gid == 0);
    else valid = (row < a.n_out_rows) && (bit < a.out_dim[a.nout - 1]);
    uint32_t acc = 0;
    if (valid) {
        int64_t c[kMaxDim];
        decode_out(a, row, bit, c);
        int64_t baseA = 0, baseB = 0;
        for (int i = 0; i < a.nout; ++i) { baseA += c[i] * a.a_str[i]; baseB += c[i] * a.b_str[i]; }
        int64_t kidx[kMaxDim];
        for (int j = 0; j < a.nk; ++j) kidx[j] = 0;
        int64_t offA = 0, offB = 0;
        const int kp = a.a_pk_k;
        const int64_t rw = a.a_row_words;
        for (;;) {
            const uint32_t *pa = a.A + baseA + offA;
            if (a.B) {
                const uint32_t *pb = a.B + baseB + offB;
                if (VEC4) {
                    for (int64_t w = 0; w < rw; w += 4) {
                        const uint4 x = *reinterpret_cast<const uint4 *>(pa + w);
                        const uint4 y = *reinterpret_cast<const uint4 *>(pb + w);
                        acc |= (x.x & y.x) | (x.y & y.y) | (x.z & y.z) | (x.w & y.w);
                    }
                } else {
                    for (int64_t w = 0; w < rw; ++w) acc |= pa[w] & pb[w];
                }
            } else {
                if (VEC4) {
                    for (int64_t w = 0; w < rw; w += 4) {
                        const uint4 x = *reinterpret_cast<const uint4 *>(pa + w);
                        acc |= x.x | x.y | x.z | x.w;
                    }
                } else {
                    for (int64_t w = 0; w < rw; ++w) acc |= pa[w];
                }
            }
            int j = a.nk - 1;
            for (; j >= 0; --j) {
                if (j == kp) continue;
                ++kidx[j];
                offA += a.ka_str[j];
                offB += a.kb_str[j];
                if (kidx[j] < a.k_dim[j]) break;
                offA -= a.ka_str[j] * a.k_dim[j];
                offB -= a.kb_str[j] * a.k_dim[j];
                kidx[j] = 0;
            }
            if (j < 0) break;
        }
    }
    const unsigned long long bits = __ballot(acc != 0);
    if ((threadIdx.x & 63) == 0 && gid < (a.nout == 0 ? 1 : a.n_out_rows * rowbits)) {
        if (a.nout == 0) {
            a.C[0] = (uint32_t)(bits & 1ull);
        } else {
            uint32_t *dst = a.C + row * a.c_row_words + bit / 32;
            dst[0] = (uint32_t)bits;
            dst[1] = (uint32_t)(bits >> 32);
        }
    }
  }
}

// Stream mode W: A, B and C share the packed variable (an output variable);
// one thread per output word ORs the AND of whole words over the latent
// entries.
__global__ void k_contract_stream_w(ContractArgs a, int64_t total) {
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
       gid += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = gid / a.c_row_words, wc = gid % a.c_row_words;
    const int64_t last = a.out_dim[a.nout - 1];
    uint32_t acc = 0;
    if (wc * 32 < last) {
        int64_t c[kMaxDim];
        decode_out(a, row, 0, c);
        int64_t baseA = wc, baseB = wc;
        for (int i = 0; i < a.nout - 1; ++i) { baseA += c[i] * a.a_str[i]; baseB += c[i] * a.b_str[i]; }
        int64_t kidx[kMaxDim];
        for (int j = 0; j < a.nk; ++j) kidx[j] = 0;
        int64_t offA = 0, offB = 0;
        for (;;) {
            const uint32_t x = a.A[baseA + offA];
            acc |= a.B ? (x & a.B[baseB + offB]) : x;
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
            if (j < 0) break;
        }
    }
    a.C[row * a.c_row_words + wc] = acc;
  }
}

hipError_t launch_contract(const ContractArgs &a, int mode, hipStream_t s) {
    const int64_t rowbits = a.c_row_words * 32;
    if (mode == kModeStreamW) {
        const int64_t total = a.n_out_rows * a.c_row_words;
        if (total == 0) return hipSuccess;
        hipLaunchKernelGGL(k_contract_stream_w, grid_for(total), dim3(256), 0, s, a, total);
        return hipGetLastError();
    }
    const int64_t total = (a.nout == 0) ? 64 : a.n_out_rows * rowbits;
    if (total == 0) return hipSuccess;
    const dim3 grid = grid_for(total);
    if (mode == kModeStreamK) {
        if (a.a_row_words % 4 == 0)
            hipLaunchKernelGGL(k_contract_stream_k<true>, grid, dim3(256), 0, s, a, total);
        else
            hipLaunchKernelGGL(k_contract_stream_k<false>, grid, dim3(256), 0, s, a, total);
    } else {
        hipLaunchKernelGGL(k_contract_bits, grid, dim3(256), 0, s, a, total);
    }
    return hipGetLastError();
}

// ------------------------------------------------------- MFMA contraction
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;     // 128 x 128 output tile per workgroup (4 waves of 64 x 64)
constexpr int kChunk = 8;      // K words staged per iteration (256 Boolean k)
constexpr int kPitch = 12;     // LDS row pitch in words: 16-byte reads of 8 rows hit distinct banks

__device__ __forceinline__ uint4 load_row4(const uint32_t *__restrict__ p, int64_t kw, int64_t kend, bool ok,
                                           bool vec4) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (!ok) return v;
    if (vec4) {
        if (kw + 3 < kend) return *reinterpret_cast<const uint4 *>(p + kw);
    }
    // rows are an even number of words: pairs are 8-byte aligned
    if (kw + 1 < kend) { const uint2 t = *reinterpret_cast<const uint2 *>(p + kw); v.x = t.x; v.y = t.y; }
    if (kw + 3 < kend) { const uint2 t = *reinterpret_cast<const uint2 *>(p + kw + 2); v.z = t.x; v.w = t.y; }
    return v;
}

// Spread one 32-bit word of Boolean k-entries into an int8 MFMA operand:
// byte p of dword j (j = 0..3) is bit (8p + 4h + j) of x times 2^(4h + j),
// h = lane half.  A and B use the same map, so every product is 0 or a
// positive 4^(4h+j) and an accumulated count is > 0 iff some k has both bits.
__device__ __forceinline__ v4i spread(uint32_t x, const uint32_t *m) {
    v4i r;
    r[0] = (int)(x & m[0]);
    r[1] = (int)(x & m[1]);
    r[2] = (int)(x & m[2]);
    r[3] = (int)(x & m[3]);
    return r;
}

__global__ __launch_bounds__(256) void k_gemm_mfma(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint32_t sA[2][kTile * kPitch];
    __shared__ __attribute__((aligned(16))) uint32_t sB[2][kTile * kPitch];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, l32 = lane & 31;
    int64_t t = blockIdx.x;
    const int ks = (int)(t % g.ksplit);
    t /= g.ksplit;
    const int64_t tn = t % g.tiles_n, tm = t / g.tiles_n;
    const int64_t b = blockIdx.y;
    const int64_t m0 = tm * kTile, n0 = tn * kTile;
    const int64_t Wc = g.rwc * 32;
    const int64_t kw0 = (int64_t)ks * g.kchunk;
    const int64_t kw1 = min(g.Kw, kw0 + g.kchunk);
    const bool vec4 = (g.Kw % 4) == 0;

    const int lrow = tid >> 1, lw = (tid & 1) * 4;
    const int64_t am = m0 + lrow;
    const bool a_ok = am < g.M;
    const uint32_t *aptr = g.A + b * g.sA_b + (a_ok ? am : 0) * g.Kw;
    const int64_t bn = n0 + lrow;
    const int64_t bno = bn / Wc, bj = bn % Wc;
    const bool b_ok = (bno < g.No) && (bj < g.rn);
    const uint32_t *bptr = g.B + b * g.sB_b + (b_ok ? (bno * g.rn + bj) : 0) * g.Kw;

    uint32_t msk[4];
    for (int j = 0; j < 4; ++j) msk[j] = 0x01010101u << (4 * h + j);

    v16i acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    int cur = 0;
    if (kw0 < kw1) {
        uint4 ra = load_row4(aptr, kw0 + lw, kw1, a_ok, vec4);
        uint4 rb = load_row4(bptr, kw0 + lw, kw1, b_ok, vec4);
        *reinterpret_cast<uint4 *>(&sA[0][lrow * kPitch + lw]) = ra;
        *reinterpret_cast<uint4 *>(&sB[0][lrow * kPitch + lw]) = rb;
    }
    __syncthreads();
    for (int64_t kc = kw0; kc < kw1; kc += kChunk) {
        const bool more = kc + kChunk < kw1;
        uint4 na = make_uint4(0u, 0u, 0u, 0u), nb = make_uint4(0u, 0u, 0u, 0u);
        if (more) {
            na = load_row4(aptr, kc + kChunk + lw, kw1, a_ok, vec4);
            nb = load_row4(bptr, kc + kChunk + lw, kw1, b_ok, vec4);
        }
#pragma unroll
        for (int q4 = 0; q4 < kChunk; q4 += 4) {
            uint4 a4[2], b4[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a4[i] = *reinterpret_cast<const uint4 *>(&sA[cur][(wm * 64 + i * 32 + l32) * kPitch + q4]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b4[j] = *reinterpret_cast<const uint4 *>(&sB[cur][(wn * 64 + j * 32 + l32) * kPitch + q4]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v4i opa[2], opb[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const uint32_t x = q == 0 ? a4[i].x : q == 1 ? a4[i].y : q == 2 ? a4[i].z : a4[i].w;
                    opa[i] = spread(x, msk);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint32_t y = q == 0 ? b4[j].x : q == 1 ? b4[j].y : q == 2 ? b4[j].z : b4[j].w;
                    opb[j] = spread(y, msk);
                }
                // MFMA rows index n (from B), columns index m (from A): each lane
                // then holds one column m, i.e. bits of one output row.
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(opb[j], opa[i], acc[i][j], 0, 0, 0);
            }
        }
        if (more) {
            *reinterpret_cast<uint4 *>(&sA[cur ^ 1][lrow * kPitch + lw]) = na;
            *reinterpret_cast<uint4 *>(&sB[cur ^ 1][lrow * kPitch + lw]) = nb;
        }
        __syncthreads();
        cur ^= 1;
    }
    // Epilogue: accumulator register r of a 32x32 block holds MFMA row
    // 8*(r/4) + 4*h + r%4 (our n) at MFMA column l32 (our m).
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            uint32_t mask = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                mask |= (acc[i][j][r] > 0 ? 1u : 0u) << (8 * (r >> 2) + 4 * h + (r & 3));
            mask |= __shfl_xor(mask, 32);
            if (h == 0) {
                const int64_t m = m0 + wm * 64 + i * 32 + l32;
                const int64_t n = n0 + wn * 64 + j * 32;
                const int64_t no = n / Wc, wc = (n % Wc) / 32;
                if (m < g.M && no < g.No) {
                    uint32_t *dst = g.C + b * g.sC_b + (m * g.No + no) * g.rwc + wc;
                    if (g.ksplit > 1) {
                        if (mask) atomicOr(dst, mask);
                    } else {
                        *dst = mask;
                    }
                }
            }
        }
    }
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    if (g.nbatch == 0 || g.M == 0 || g.No == 0) return hipSuccess;
    const int64_t gx = g.tiles_m * g.tiles_n * g.ksplit;
    if (gx > 0x7fffffff || g.nbatch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_mfma, dim3((unsigned)gx, (unsigned)g.nbatch), dim3(256), 0, s, g);
    return hipGetLastError();
}

// ------------------------------------------------------------ fill, count
__global__ void k_fill(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
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

hipError_t launch_popcount(const uint32_t *p, int64_t n, unsigned long long *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_popcount, dim3((unsigned)blocks), dim3(256), 0, s, p, n, out);
    return hipGetLastError();
}

}  // namespace pa
