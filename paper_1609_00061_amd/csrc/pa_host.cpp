// Host runtime of libpa.so: validation, planning (cluster tree and layouts),
// workspace management and kernel dispatch.  C ABI declared in pa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "pa.h"
#include "pa_internal.h"
#include "pa_plan.h"

namespace pa {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) return fail(PA_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// ------------------------------------------------------------------ layouts
int64_t row_words_of(int64_t d) { return d <= 0 ? 0 : 2 * ((d + 63) / 64); }

Layout make_layout(const std::vector<int> &vars, const std::vector<int64_t> &res_of_var) {
    Layout L;
    L.vars = vars;
    for (int v : vars) L.dims.push_back(res_of_var[v]);
    if (vars.empty()) {
        L.rw = 1;
        L.words = 1;
    } else {
        L.rw = row_words_of(L.dims.back());
        L.words = L.rw;
        for (size_t i = 0; i + 1 < L.dims.size(); ++i) L.words *= L.dims[i];
    }
    return L;
}

int Layout::packed() const { return vars.empty() ? -1 : vars.back(); }

// Word stride of a non-packed variable; 0 if absent or packed.
int64_t Layout::stride(int v) const {
    const int q = (int)vars.size();
    for (int s = 0; s + 1 < q; ++s) {
        if (vars[s] != v) continue;
        int64_t st = rw;
        for (int t = s + 1; t + 1 < q; ++t) st *= dims[t];
        return st;
    }
    return 0;
}

bool Layout::has(int v) const { return std::find(vars.begin(), vars.end(), v) != vars.end(); }

// --------------------------------------------------------- monomial order
// Graded-lex exponent tuples of `n` variables with total degree <= d: degree
// ascending, then lexicographically descending tuples.
static void gl_rec(int n, int D, int pos, int *cur, std::vector<std::array<int, 3>> &out) {
    if (pos == n - 1) {
        cur[pos] = D;
        std::array<int, 3> e = {0, 0, 0};
        for (int i = 0; i < n; ++i) e[i] = cur[i];
        out.push_back(e);
        return;
    }
    for (int e = D; e >= 0; --e) {
        cur[pos] = e;
        gl_rec(n, D - e, pos + 1, cur, out);
    }
}

std::vector<std::array<int, 3>> graded_lex(int n, int d) {
    std::vector<std::array<int, 3>> out;
    int cur[3] = {0, 0, 0};
    for (int D = 0; D <= d; ++D) gl_rec(n, D, 0, cur, out);
    return out;
}

int64_t n_monomials(int n, int d) {
    int64_t num = 1, den = 1;
    for (int i = 1; i <= d; ++i) { num *= (n + i); den *= i; }
    return num / den;
}

// Dense table c[e0 + (d+1)(e1 + (d+1) e2)] of the declared-order coefficients.
std::vector<double> dense_coef(const pa_relation &r) {
    const int D1 = r.degree + 1;
    std::vector<double> c((size_t)D1 * D1 * D1, 0.0);
    auto exps = graded_lex(r.arity, r.degree);
    for (size_t m = 0; m < exps.size(); ++m) {
        const auto &e = exps[m];
        c[e[0] + D1 * (e[1] + D1 * e[2])] = r.coef[m];
    }
    return c;
}

// Pixel boundaries x_k = lo + k * ((hi - lo) / r), k = 0..r (eqn Pixel_def,
// 0-based corners): the kernels form k * step and then lo + that in FP64,
// each rounded (no contraction), and take the nearest float for FP32.
double axis_step(double lo, double hi, int r) { return (hi - lo) / (double)r; }

// -------------------------------------------------------------- validation
int validate_relation(const pa_relation &r, const pa_axis *axes_of_vars, int n_vars_total, const char *who) {
    if (r.arity < 1 || r.arity > PA_MAX_ARITY)
        return fail(PA_EINVAL, std::string(who) + ": arity must be 1..3");
    if (r.degree < 0 || r.degree > PA_MAX_DEGREE)
        return fail(PA_EINVAL, std::string(who) + ": degree must be 0..4");
    if (!r.vars || !r.coef) return fail(PA_EINVAL, std::string(who) + ": null vars or coef");
    if (r.target < PA_TARGET_EQ || r.target > PA_TARGET_LT)
        return fail(PA_EINVAL, std::string(who) + ": target must be PA_TARGET_EQ, _LE or _LT");
    for (int i = 0; i < r.arity; ++i) {
        if (n_vars_total >= 0 && (r.vars[i] < 0 || r.vars[i] >= n_vars_total))
            return fail(PA_EINVAL, std::string(who) + ": variable id out of range");
        for (int j = 0; j < i; ++j)
            if (r.vars[i] == r.vars[j]) return fail(PA_EINVAL, std::string(who) + ": repeated variable");
    }
    if (axes_of_vars) {
        for (int i = 0; i < r.arity; ++i) {
            const pa_axis &a = axes_of_vars[i];
            if (a.res < 2) return fail(PA_EINVAL, std::string(who) + ": resolution must be >= 2");
            if (!std::isfinite(a.lo) || !std::isfinite(a.hi) || !(a.lo <= a.hi))
                return fail(PA_EINVAL, std::string(who) + ": need finite lo <= hi");
        }
    }
    return PA_OK;
}

int check_bitarray(const pa_bitarray *a, const std::vector<int64_t> &dims, const char *who) {
    if (!a) return fail(PA_EINVAL, std::string(who) + ": null array");
    if (a->ndim != (int)dims.size()) return fail(PA_EINVAL, std::string(who) + ": rank mismatch");
    for (size_t i = 0; i < dims.size(); ++i)
        if (a->dims[i] != dims[i]) return fail(PA_EINVAL, std::string(who) + ": dims mismatch");
    const int64_t rw = dims.empty() ? 1 : row_words_of(dims.back());
    if (!dims.empty() && a->row_words != rw) return fail(PA_EINVAL, std::string(who) + ": row_words must be 2*ceil(d/64)");
    if (!a->data) return fail(PA_EINVAL, std::string(who) + ": null data");
    return PA_OK;
}

// ------------------------------------------------------------- workspace
int Workspace::ensure(size_t bytes) {
    if (bytes <= cap) return PA_OK;
    if (external) return fail(PA_ENOMEM, "workspace too small: need " + std::to_string(bytes) + " bytes");
    if (ptr) {
        (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
    if (hipMalloc(&ptr, bytes) != hipSuccess) {
        ptr = nullptr;
        return fail(PA_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    cap = bytes;
    return PA_OK;
}

Workspace::~Workspace() {
    if (ptr && !external) (void)hipFree(ptr);
}

}  // namespace pa

// ====================================================================== ABI
using namespace pa;

extern "C" const char *pa_last_error(void) { return pa::g_err.c_str(); }

extern "C" int64_t pa_row_words(int32_t d) { return pa::row_words_of(d); }

extern "C" int64_t pa_array_words(int32_t ndim, const int32_t *dims) {
    if (ndim <= 0) return 1;
    int64_t w = pa::row_words_of(dims[ndim - 1]);
    for (int i = 0; i + 1 < ndim; ++i) w *= dims[i];
    return w;
}
