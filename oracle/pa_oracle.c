/*
 * pa_oracle.c -- plain, slow CPU oracle for the pixel array method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.  Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 * -pthread (no FMA contraction, IEEE semantics, no flush-to-zero).
 *
 * What it computes (Ch. 3 of the paper, "Mathematical foundations"):
 *   - axis discretization: each port with bounds [a, b) and resolution r is cut
 *     into r pixels of width delta = (b - a) / r (eqn Pixel_def); the pixel
 *     boundaries ("corners") are x_k = a + k * delta, k = 0..r, the same step
 *     form the paper's sample code uses for pixel centres (App. A);
 *   - a canonical FP64 value of a polynomial relation at a corner (nested
 *     Horner with correctly rounded fma; this sequence *is* the definition of
 *     the FP64 value that every implementation must reproduce bit for bit);
 *   - the corner sign-change plot: a pixel (closed cell) is set iff among its
 *     2^n corners one has f <= 0 and one has f >= 0 (the corner plotting
 *     method of the library; the paper allows any sufficiently fast and accurate plotting
 *     method, Sec. 3.6); a NaN corner counts as neither;
 *   - generalized array multiplication (Alg. "Generalized array
 *     multiplication", eqn GAM): A'(e') = OR over link entries e projecting to
 *     e' of AND_i A_i(e_i), both as a pairwise contraction of two arrays and
 *     as the whole-diagram formula with short-circuit AND/OR.
 *
 * Arrays are one byte per entry, row-major over the declared variable order
 * (deliberately a different layout from the GPU's bit-packed arrays).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 4         /* max arity of a relation */
#define ORC_MAXD 6         /* max total degree */
#define ORC_MAXV 64        /* max variables in a system */
#define ORC_MAXDIM 16      /* max rank of an array in a contraction */

/* ------------------------------------------------------------------ axes */
/* Corners of one axis: x_k = lo + k * ((hi - lo) / r), k = 0..r (eqn Pixel_def). */
int orc_axis(double lo, double hi, int r, double *x) {
    if (r < 1 || !(lo <= hi)) return -1;
    double delta = (hi - lo) / (double)r;
    for (int k = 0; k <= r; ++k) {
        double t = (double)k * delta;
        x[k] = lo + t;
    }
    return 0;
}

/* --------------------------------------------------------- monomial order */
/* Graded-lex order of exponent tuples (e_0..e_{n-1}) with sum <= d: total degree
 * ascending, then lexicographically descending tuples.  Returns the count. */
static int enum_fixed(int n, int D, int pos, int *cur, int (*out)[ORC_MAXN], int cnt) {
    if (pos == n - 1) {
        cur[pos] = D;
        memcpy(out[cnt], cur, sizeof(int) * ORC_MAXN);
        return cnt + 1;
    }
    for (int e = D; e >= 0; --e) {
        cur[pos] = e;
        cnt = enum_fixed(n, D - e, pos + 1, cur, out, cnt);
    }
    return cnt;
}

static int enum_monomials(int n, int d, int (*out)[ORC_MAXN]) {
    int cur[ORC_MAXN] = {0};
    int cnt = 0;
    if (n == 0) { memset(out[0], 0, sizeof(int) * ORC_MAXN); return 1; }
    for (int D = 0; D <= d; ++D) cnt = enum_fixed(n, D, 0, cur, out, cnt);
    return cnt;
}

long orc_n_monomials(int n, int d) {
    long num = 1, den = 1;            /* C(n+d, d) */
    for (int i = 1; i <= d; ++i) { num *= (n + i); den *= i; }
    return num / den;
}

typedef struct {
    int n, d, nm;
    int exps[512][ORC_MAXN];
    int slot[2401];                 /* (d+1)-ary exponent key -> monomial index */
    const double *coef;
} poly_t;

static int exp_key(const poly_t *p, const int *e) {
    int k = 0;
    for (int j = p->n - 1; j >= 0; --j) k = k * (p->d + 1) + e[j];
    return k;
}

static int poly_init(poly_t *p, int n, int d, const double *coef) {
    if (n < 1 || n > ORC_MAXN || d < 0 || d > ORC_MAXD) return -1;
    if (orc_n_monomials(n, d) > 512) return -1;
    p->n = n; p->d = d; p->coef = coef;
    p->nm = enum_monomials(n, d, p->exps);
    for (int m = 0; m < p->nm; ++m) p->slot[exp_key(p, p->exps[m])] = m;
    return 0;
}

static double coef_of(const poly_t *p, const int *e) {
    return p->coef[p->slot[exp_key(p, e)]];
}

/* Canonical nested Horner.  With the variables x_0..x_{n-1} in declared order,
 *   f = sum_i A_i(x_0..x_{n-2}) x_{n-1}^i,  deg A_i <= d - i,
 * evaluated as p = A_d; p = fma(p, x_{n-1}, A_i) for i = d-1..0, with every A_i
 * evaluated by the same rule one variable down.  `e` holds the exponents fixed
 * so far for x_m..x_{n-1}. */
static double horner(const poly_t *p, int m, int budget, int *e, const double *x) {
    if (m == 0) return coef_of(p, e);
    e[m - 1] = budget;
    for (int j = 0; j < m - 1; ++j) e[j] = 0;
    double acc = horner(p, m - 1, 0, e, x);
    for (int i = budget - 1; i >= 0; --i) {
        e[m - 1] = i;
        double a = horner(p, m - 1, budget - i, e, x);
        e[m - 1] = i;
        acc = fma(acc, x[m - 1], a);
    }
    return acc;
}

double orc_eval(int n, int d, const double *coef, const double *x) {
    poly_t p;
    if (poly_init(&p, n, d, coef)) return NAN;
    int e[ORC_MAXN] = {0};
    return horner(&p, n, d, e, x);
}

/* ------------------------------------------------------------------ plot */
typedef struct {
    const poly_t *p;
    const double *const *ax;      /* corner tables per declared variable */
    const int *res;
    double *vals;                 /* corner grid, row-major over (r_j + 1) */
    long n_corners, begin, end;
} eval_job;

static void *eval_worker(void *arg) {
    eval_job *j = (eval_job *)arg;
    int n = j->p->n;
    for (long c = j->begin; c < j->end; ++c) {
        long rem = c;
        double x[ORC_MAXN];
        for (int a = n - 1; a >= 0; --a) {
            long k = rem % (j->res[a] + 1);
            rem /= (j->res[a] + 1);
            x[a] = j->ax[a][k];
        }
        int e[ORC_MAXN] = {0};
        j->vals[c] = horner(j->p, n, j->p->d, e, x);
    }
    return NULL;
}

/* FP64 value at every corner of the grid, row-major over (r_0+1, ..., r_{n-1}+1). */
int orc_corner_values(int n, int d, const double *coef, const double *lo, const double *hi,
                      const int *res, double *vals, int nthreads) {
    poly_t *p = (poly_t *)malloc(sizeof(poly_t));
    if (!p || poly_init(p, n, d, coef)) { free(p); return -1; }
    double *ax[ORC_MAXN];
    long nc = 1;
    for (int a = 0; a < n; ++a) {
        if (res[a] < 1) { free(p); return -1; }
        ax[a] = (double *)malloc(sizeof(double) * (res[a] + 1));
        if (orc_axis(lo[a], hi[a], res[a], ax[a])) { free(p); return -1; }
        nc *= res[a] + 1;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    eval_job jobs[64];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].p = p; jobs[t].ax = (const double *const *)ax; jobs[t].res = res;
        jobs[t].vals = vals; jobs[t].n_corners = nc;
        jobs[t].begin = nc * t / nthreads; jobs[t].end = nc * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, eval_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int a = 0; a < n; ++a) free(ax[a]);
    free(p);
    return 0;
}

/* Corner sign-change plot: cell (i_0..i_{n-1}) is set iff its 2^n corners
 * (i_a or i_a + 1 on every axis) include one with f <= 0 and one with f >= 0.
 * out: one byte per cell, row-major over (r_0, ..., r_{n-1}).
 * *n_zero receives the number of corners with f == 0 exactly. */
int orc_plot(int n, int d, const double *coef, const double *lo, const double *hi,
             const int *res, unsigned char *out, long long *n_zero, int nthreads) {
    long nc = 1, ncell = 1;
    for (int a = 0; a < n; ++a) { nc *= res[a] + 1; ncell *= res[a]; }
    double *vals = (double *)malloc(sizeof(double) * nc);
    if (!vals) return -2;
    if (orc_corner_values(n, d, coef, lo, hi, res, vals, nthreads)) { free(vals); return -1; }
    long long z = 0;
    for (long c = 0; c < nc; ++c) z += (vals[c] == 0.0);
    if (n_zero) *n_zero = z;
    for (long cell = 0; cell < ncell; ++cell) {
        long rem = cell;
        int idx[ORC_MAXN];
        for (int a = n - 1; a >= 0; --a) { idx[a] = (int)(rem % res[a]); rem /= res[a]; }
        int le = 0, ge = 0;
        for (int corner = 0; corner < (1 << n); ++corner) {
            long off = 0;
            for (int a = 0; a < n; ++a) off = off * (res[a] + 1) + idx[a] + ((corner >> a) & 1);
            double f = vals[off];
            if (f <= 0.0) le = 1;
            if (f >= 0.0) ge = 1;
        }
        out[cell] = (unsigned char)(le && ge);
    }
    free(vals);
    return 0;
}

/* Corner plot of an inequality (Sec. 3.2: relations f <= 0 and f < 0, the
 * target subsets (-inf, 0] and (-inf, 0) of Def. "functionally_defined"),
 * by the same corner sampling as orc_plot: a cell (closed) is set iff one of
 * its 2^n corners satisfies the inequality, target 1: f <= 0, target 2:
 * f < 0 (a NaN corner satisfies neither).  Such a corner is a point of the
 * closed cell in the relation.  out: one byte per cell, as orc_plot. */
int orc_plot_ineq(int n, int d, const double *coef, const double *lo, const double *hi,
                  const int *res, int target, unsigned char *out, int nthreads) {
    if (target != 1 && target != 2) return -1;
    long nc = 1, ncell = 1;
    for (int a = 0; a < n; ++a) { nc *= res[a] + 1; ncell *= res[a]; }
    double *vals = (double *)malloc(sizeof(double) * nc);
    if (!vals) return -2;
    if (orc_corner_values(n, d, coef, lo, hi, res, vals, nthreads)) { free(vals); return -1; }
    for (long cell = 0; cell < ncell; ++cell) {
        long rem = cell;
        int idx[ORC_MAXN];
        for (int a = n - 1; a >= 0; --a) { idx[a] = (int)(rem % res[a]); rem /= res[a]; }
        int hit = 0;
        for (int corner = 0; corner < (1 << n); ++corner) {
            long off = 0;
            for (int a = 0; a < n; ++a) off = off * (res[a] + 1) + idx[a] + ((corner >> a) & 1);
            double f = vals[off];
            if (target == 1 ? (f <= 0.0) : (f < 0.0)) hit = 1;
        }
        out[cell] = (unsigned char)hit;
    }
    free(vals);
    return 0;
}

/* Centre of pixel k of one axis: lo + (k + 1/2) * ((hi - lo) / r), k = 0..r-1
 * (eqn Pixel_def, 0-based; the sample code's centre form in App. A); the
 * step, the product and the sum are each rounded once. */
int orc_centers(double lo, double hi, int r, double *c) {
    if (r < 1 || !(lo <= hi)) return -1;
    double delta = (hi - lo) / (double)r;
    for (int k = 0; k < r; ++k) {
        double t = ((double)k + 0.5) * delta;
        c[k] = lo + t;
    }
    return 0;
}

/* epsilon-tolerance sample-in-center plot (Def. sample_in_center): cell e is
 * set iff the {c_e}-error of the relation achieves eps, i.e. the distance
 * from f(c_e) to the target subset S is at most eps (Def. plot_error:
 * "achieves u" means some distance in [0, u]).  Target 0, S = {0}: |f| <= eps;
 * target 1, S = (-inf, 0]: f <= eps; target 2, S = (-inf, 0): the distances
 * to S form the open ray (f, inf) when f >= 0, so f < eps.  A NaN value
 * achieves nothing.  f(c_e) is the canonical FP64 value (orc_eval's Horner)
 * at the FP64 centre.  out: one byte per cell, row-major over (r_0..r_{n-1}). */
typedef struct {
    const poly_t *p;
    const double *const *cx;
    const int *res;
    double eps;
    int target;
    unsigned char *out;
    long begin, end;
} center_job;

static void *center_worker(void *arg) {
    center_job *j = (center_job *)arg;
    int n = j->p->n;
    for (long cell = j->begin; cell < j->end; ++cell) {
        long rem = cell;
        double x[ORC_MAXN];
        for (int a = n - 1; a >= 0; --a) {
            long k = rem % j->res[a];
            rem /= j->res[a];
            x[a] = j->cx[a][k];
        }
        int e[ORC_MAXN] = {0};
        double f = horner(j->p, n, j->p->d, e, x);
        int on;
        if (j->target == 0) on = fabs(f) <= j->eps;
        else if (j->target == 1) on = f <= j->eps;
        else on = f < j->eps;
        j->out[cell] = (unsigned char)on;
    }
    return NULL;
}

int orc_plot_center(int n, int d, const double *coef, const double *lo, const double *hi, const int *res,
                    double eps, int target, unsigned char *out, int nthreads) {
    if (target < 0 || target > 2 || !(eps >= 0.0)) return -1;
    poly_t *p = (poly_t *)malloc(sizeof(poly_t));
    if (!p || poly_init(p, n, d, coef)) { free(p); return -1; }
    double *cx[ORC_MAXN];
    long ncell = 1;
    for (int a = 0; a < n; ++a) {
        if (res[a] < 1) { free(p); return -1; }
        cx[a] = (double *)malloc(sizeof(double) * res[a]);
        if (orc_centers(lo[a], hi[a], res[a], cx[a])) { free(p); return -1; }
        ncell *= res[a];
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    center_job jobs[64];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].p = p; jobs[t].cx = (const double *const *)cx; jobs[t].res = res;
        jobs[t].eps = eps; jobs[t].target = target; jobs[t].out = out;
        jobs[t].begin = ncell * t / nthreads; jobs[t].end = ncell * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, center_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int a = 0; a < n; ++a) free(cx[a]);
    free(p);
    return 0;
}

/* ------------------------------------------------------ pairwise contraction */
/* C(out_vars) = OR over all entries of vars(A) u vars(B) projecting to the
 * output entry of A(a_vars) AND B(b_vars): generalized array multiplication of
 * a two-pack cluster (Alg. "Generalized array multiplication" restricted to
 * two inner packs).  var_res[v] = resolution of variable v.  Output vars must
 * be a subset of vars(A) u vars(B) and distinct.
 *
 * Written as the i-k-j loop of a Boolean matrix product: the shared
 * variables play k, the variables only A has i, those only B has j.  For
 * every set entry of A (i, k) the loop visits the set entries of B with the
 * same k and sets C at the output entry their union projects to.  To find
 * those B entries the set entries of B are first listed as (k, j) pairs
 * sorted by k; a B without variables of its own is read directly.
 *
 * The entries of A are split into contiguous ranges, one per thread.  Each
 * output byte is only ever set to 1 (the OR of the semiring), so the threads
 * write with relaxed atomic stores and the result does not depend on how the
 * range is split or on the thread count. */
typedef struct { long k, j; } kj_pair;

static int kj_cmp(const void *x, const void *y) {
    const kj_pair *p = (const kj_pair *)x, *q = (const kj_pair *)y;
    if (p->k != q->k) return p->k < q->k ? -1 : 1;
    return (p->j > q->j) - (p->j < q->j);
}

typedef struct {
    const unsigned char *A, *B;
    unsigned char *C;
    int na, nb, nc, nbx, nsh;
    const int *a_vars, *b_vars, *c_vars, *var_res;
    int bx[ORC_MAXDIM], sh[ORC_MAXDIM];   /* variables only in B; variables in both */
    const kj_pair *pairs;                 /* set entries of B sorted by k (nbx > 0) */
    long npairs;
    long begin, end;
} contract_job;

static void *contract_worker(void *arg) {
    contract_job *j = (contract_job *)arg;
    int val[ORC_MAXV];
    for (long ea = j->begin; ea < j->end; ++ea) {
        if (!j->A[ea]) continue;
        long rem = ea;
        for (int i = j->na - 1; i >= 0; --i) {
            val[j->a_vars[i]] = (int)(rem % j->var_res[j->a_vars[i]]);
            rem /= j->var_res[j->a_vars[i]];
        }
        if (j->nbx == 0) {               /* every variable of B is bound by A */
            long ib = 0;
            for (int i = 0; i < j->nb; ++i) ib = ib * j->var_res[j->b_vars[i]] + val[j->b_vars[i]];
            if (!j->B[ib]) continue;
            long ic = 0;
            for (int i = 0; i < j->nc; ++i) ic = ic * j->var_res[j->c_vars[i]] + val[j->c_vars[i]];
            __atomic_store_n(&j->C[ic], (unsigned char)1, __ATOMIC_RELAXED);
            continue;
        }
        long k = 0;
        for (int i = 0; i < j->nsh; ++i) k = k * j->var_res[j->sh[i]] + val[j->sh[i]];
        long lo = 0, hi = j->npairs;     /* first pair with key >= k */
        while (lo < hi) {
            long mid = lo + (hi - lo) / 2;
            if (j->pairs[mid].k < k) lo = mid + 1; else hi = mid;
        }
        for (long p = lo; p < j->npairs && j->pairs[p].k == k; ++p) {
            long r2 = j->pairs[p].j;
            for (int i = j->nbx - 1; i >= 0; --i) {
                val[j->bx[i]] = (int)(r2 % j->var_res[j->bx[i]]);
                r2 /= j->var_res[j->bx[i]];
            }
            long ic = 0;
            for (int i = 0; i < j->nc; ++i) ic = ic * j->var_res[j->c_vars[i]] + val[j->c_vars[i]];
            __atomic_store_n(&j->C[ic], (unsigned char)1, __ATOMIC_RELAXED);
        }
    }
    return NULL;
}

int orc_contract(const unsigned char *A, int na, const int *a_vars,
                 const unsigned char *B, int nb, const int *b_vars,
                 int nc, const int *c_vars, const int *var_res, unsigned char *C, int nthreads) {
    int in_a[ORC_MAXV] = {0}, in_b[ORC_MAXV] = {0};
    for (int i = 0; i < na; ++i) { if (a_vars[i] < 0 || a_vars[i] >= ORC_MAXV || in_a[a_vars[i]]) return -1; in_a[a_vars[i]] = 1; }
    for (int i = 0; i < nb; ++i) { if (b_vars[i] < 0 || b_vars[i] >= ORC_MAXV || in_b[b_vars[i]]) return -1; in_b[b_vars[i]] = 1; }
    for (int i = 0; i < nc; ++i) if (c_vars[i] < 0 || c_vars[i] >= ORC_MAXV || !(in_a[c_vars[i]] || in_b[c_vars[i]])) return -1;
    if (na > ORC_MAXDIM || nb > ORC_MAXDIM || nc > ORC_MAXDIM) return -1;
    contract_job base;
    memset(&base, 0, sizeof(base));
    base.A = A; base.B = B; base.C = C;
    base.na = na; base.nb = nb; base.nc = nc;
    base.a_vars = a_vars; base.b_vars = b_vars; base.c_vars = c_vars; base.var_res = var_res;
    for (int i = 0; i < nb; ++i) {
        if (in_a[b_vars[i]]) base.sh[base.nsh++] = b_vars[i];
        else base.bx[base.nbx++] = b_vars[i];
    }
    long sizeA = 1, sizeB = 1, sizeC = 1;
    for (int i = 0; i < na; ++i) sizeA *= var_res[a_vars[i]];
    for (int i = 0; i < nb; ++i) sizeB *= var_res[b_vars[i]];
    for (int i = 0; i < nc; ++i) sizeC *= var_res[c_vars[i]];
    memset(C, 0, (size_t)sizeC);
    kj_pair *pairs = NULL;
    if (base.nbx > 0) {
        long n = 0;
        for (long eb = 0; eb < sizeB; ++eb) n += (B[eb] != 0);
        pairs = (kj_pair *)malloc(sizeof(kj_pair) * (size_t)(n > 0 ? n : 1));
        if (!pairs) return -2;
        int val[ORC_MAXV];
        long t = 0;
        for (long eb = 0; eb < sizeB; ++eb) {
            if (!B[eb]) continue;
            long rem = eb;
            for (int i = nb - 1; i >= 0; --i) { val[b_vars[i]] = (int)(rem % var_res[b_vars[i]]); rem /= var_res[b_vars[i]]; }
            long k = 0, j = 0;
            for (int i = 0; i < base.nsh; ++i) k = k * var_res[base.sh[i]] + val[base.sh[i]];
            for (int i = 0; i < base.nbx; ++i) j = j * var_res[base.bx[i]] + val[base.bx[i]];
            pairs[t].k = k; pairs[t].j = j; ++t;
        }
        qsort(pairs, (size_t)n, sizeof(kj_pair), kj_cmp);
        base.pairs = pairs;
        base.npairs = n;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    contract_job jobs[64];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = base;
        jobs[t].begin = sizeA * t / nthreads;
        jobs[t].end = sizeA * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, contract_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(pairs);
    return 0;
}

/* ------------------------------------- pairwise contraction, count semiring */
/* Generalized array multiplication of a two-pack cluster in the semiring N of
 * natural numbers (footnote on semirings in Sec. 2.2, Notation of Ch. 3: the
 * same formula with + and * of N): C(e') = sum over the entries of
 * vars(A) u vars(B) projecting to e' of A(e_A) * B(e_B).  Entries are uint64;
 * sums and products saturate at UINT64_MAX.  Plain nested loops over every
 * entry of A and, for each nonzero one, every entry of the variables only B
 * has (no index structure: the inputs here are small).  Single-threaded. */
static uint64_t sat_add(uint64_t a, uint64_t b) { return a > UINT64_MAX - b ? UINT64_MAX : a + b; }
static uint64_t sat_mul(uint64_t a, uint64_t b) { return (a != 0 && b > UINT64_MAX / a) ? UINT64_MAX : a * b; }

int orc_contract_count(const uint64_t *A, int na, const int *a_vars, const uint64_t *B, int nb, const int *b_vars,
                       int nc, const int *c_vars, const int *var_res, uint64_t *C) {
    int in_a[ORC_MAXV] = {0}, in_b[ORC_MAXV] = {0};
    for (int i = 0; i < na; ++i) { if (a_vars[i] < 0 || a_vars[i] >= ORC_MAXV || in_a[a_vars[i]]) return -1; in_a[a_vars[i]] = 1; }
    for (int i = 0; i < nb; ++i) { if (b_vars[i] < 0 || b_vars[i] >= ORC_MAXV || in_b[b_vars[i]]) return -1; in_b[b_vars[i]] = 1; }
    for (int i = 0; i < nc; ++i) if (c_vars[i] < 0 || c_vars[i] >= ORC_MAXV || !(in_a[c_vars[i]] || in_b[c_vars[i]])) return -1;
    if (na > ORC_MAXDIM || nb > ORC_MAXDIM || nc > ORC_MAXDIM) return -1;
    int bx[ORC_MAXDIM], nbx = 0;
    for (int i = 0; i < nb; ++i) if (!in_a[b_vars[i]]) bx[nbx++] = b_vars[i];
    long sizeA = 1, sizeBX = 1, sizeC = 1;
    for (int i = 0; i < na; ++i) sizeA *= var_res[a_vars[i]];
    for (int i = 0; i < nbx; ++i) sizeBX *= var_res[bx[i]];
    for (int i = 0; i < nc; ++i) sizeC *= var_res[c_vars[i]];
    for (long i = 0; i < sizeC; ++i) C[i] = 0;
    int val[ORC_MAXV];
    for (long ea = 0; ea < sizeA; ++ea) {
        if (!A[ea]) continue;
        long rem = ea;
        for (int i = na - 1; i >= 0; --i) { val[a_vars[i]] = (int)(rem % var_res[a_vars[i]]); rem /= var_res[a_vars[i]]; }
        for (long eb = 0; eb < sizeBX; ++eb) {
            long r2 = eb;
            for (int i = nbx - 1; i >= 0; --i) { val[bx[i]] = (int)(r2 % var_res[bx[i]]); r2 /= var_res[bx[i]]; }
            long ib = 0;
            for (int i = 0; i < nb; ++i) ib = ib * var_res[b_vars[i]] + val[b_vars[i]];
            if (!B[ib]) continue;
            long ic = 0;
            for (int i = 0; i < nc; ++i) ic = ic * var_res[c_vars[i]] + val[c_vars[i]];
            C[ic] = sat_add(C[ic], sat_mul(A[ea], B[ib]));
        }
    }
    return 0;
}

/* --------------------------------------------------- whole-diagram formula */
/* eqn GAM for a whole wiring diagram with short-circuit evaluation: variables
 * are assigned one at a time (exposed ones first, in the order given, then the
 * latent ones by increasing id); a relation is checked as soon as all its
 * variables are assigned and a zero prunes the branch (AND); the first full
 * assignment found sets the output entry and ends the search below it (OR).
 * This visits exactly the terms of eqn GAM that can still be nonzero. */
typedef struct {
    int n_vars, n_rel, n_exp;
    const int *var_res;
    const int *rel_nd;
    const int *rel_vars[64];
    const unsigned char *rel_data[64];
    int order[ORC_MAXV];                 /* assignment order of variables */
    int check_at[ORC_MAXV][64];          /* relations completed at depth t */
    int n_check_at[ORC_MAXV];
} solve_ctx;

static int rel_holds(const solve_ctx *s, int r, const int *val) {
    long idx = 0;
    for (int i = 0; i < s->rel_nd[r]; ++i) {
        int v = s->rel_vars[r][i];
        idx = idx * s->var_res[v] + val[v];
    }
    return s->rel_data[r][idx] != 0;
}

static int search(const solve_ctx *s, int depth, int *val) {
    if (depth == s->n_vars) return 1;
    int v = s->order[depth];
    for (int k = 0; k < s->var_res[v]; ++k) {
        val[v] = k;
        int ok = 1;
        for (int c = 0; c < s->n_check_at[depth] && ok; ++c) ok = rel_holds(s, s->check_at[depth][c], val);
        if (ok && search(s, depth + 1, val)) return 1;
    }
    return 0;
}

static int solve_setup(solve_ctx *s, int n_vars, const int *var_res, int n_rel, const int *rel_nd,
                       const int *rel_vars_flat, const unsigned char *const *rel_data,
                       int n_exp, const int *exposed) {
    if (n_vars > ORC_MAXV || n_rel > 64 || n_exp > n_vars) return -1;
    s->n_vars = n_vars; s->n_rel = n_rel; s->n_exp = n_exp;
    s->var_res = var_res; s->rel_nd = rel_nd;
    int off = 0;
    for (int r = 0; r < n_rel; ++r) { s->rel_vars[r] = rel_vars_flat + off; s->rel_data[r] = rel_data[r]; off += rel_nd[r]; }
    int used[ORC_MAXV] = {0}, pos[ORC_MAXV];
    int t = 0;
    for (int i = 0; i < n_exp; ++i) { if (used[exposed[i]]) return -1; used[exposed[i]] = 1; s->order[t++] = exposed[i]; }
    for (int v = 0; v < n_vars; ++v) if (!used[v]) s->order[t++] = v;
    for (int i = 0; i < n_vars; ++i) pos[s->order[i]] = i;
    memset(s->n_check_at, 0, sizeof(s->n_check_at));
    for (int r = 0; r < n_rel; ++r) {
        int last = -1;
        for (int i = 0; i < rel_nd[r]; ++i) if (pos[s->rel_vars[r][i]] > last) last = pos[s->rel_vars[r][i]];
        if (last < 0) return -1;
        s->check_at[last][s->n_check_at[last]++] = r;
    }
    return 0;
}

/* Evaluate the output entries listed in `entries` (n_entries rows of n_exp
 * indices, in the exposed order); out[i] = A'(entries[i]). */
typedef struct { const solve_ctx *s; const int *entries; unsigned char *out; long begin, end; } solve_job;

static void *solve_worker(void *arg) {
    solve_job *j = (solve_job *)arg;
    const solve_ctx *s = j->s;
    int val[ORC_MAXV];
    for (long e = j->begin; e < j->end; ++e) {
        int ok = 1;
        for (int i = 0; i < s->n_exp; ++i) {
            val[s->order[i]] = j->entries[e * s->n_exp + i];
            for (int c = 0; c < s->n_check_at[i] && ok; ++c) ok = rel_holds(s, s->check_at[i][c], val);
        }
        /* relations whose variables are all exposed were checked above; they
         * may only be checked once all their variables are assigned, which the
         * check_at table guarantees */
        j->out[e] = (unsigned char)(ok && search(s, s->n_exp, val));
    }
    return NULL;
}

int orc_solve_entries(int n_vars, const int *var_res, int n_rel, const int *rel_nd,
                      const int *rel_vars_flat, const unsigned char *const *rel_data,
                      int n_exp, const int *exposed, long n_entries, const int *entries,
                      unsigned char *out, int nthreads) {
    solve_ctx *s = (solve_ctx *)malloc(sizeof(solve_ctx));
    if (!s) return -2;
    if (solve_setup(s, n_vars, var_res, n_rel, rel_nd, rel_vars_flat, rel_data, n_exp, exposed)) { free(s); return -1; }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    solve_job jobs[64];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].s = s; jobs[t].entries = entries; jobs[t].out = out;
        jobs[t].begin = n_entries * t / nthreads; jobs[t].end = n_entries * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, solve_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(s);
    return 0;
}
