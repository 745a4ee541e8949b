/*
 * CPU oracle for the FMM-based NUFFT / INUFFT of Gumerov & Duraiswami,
 * "Fast Multipole Method based filtering of non-uniformly sampled data".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, table or constant
 * with the GPU library.
 *
 * Every routine is a plain, slow, direct evaluation of a closed form printed
 * in the paper, in IEEE binary64 with compensated (Neumaier) summation.  The
 * one place that uses more precision is the reduction of the FP64 radian
 * value y_j to grid units s_j = N y_j / (2 pi), done in binary128: the paper
 * treats y_j and x_k = 2 pi k / N as exact reals, and a binary64 reduction
 * would already lose about 1e-12 at N = 2^16 (the phase N y_j is large).
 *
 * Grid units.  s_j = m_j + theta_j with integer m_j in [0, N) and
 * theta_j in [-1/2, 1/2].  x_k corresponds to s = k exactly, so every
 * difference y_j - x_k is 2 pi ((m_j - k) + theta_j) / N with an exact
 * integer part.  For the sign bookkeeping of the inverse a point is also
 * given the representative s'_j = m'_j + theta_j in [0, N), where m'_j = N
 * when m_j = 0 and theta_j < 0, and m'_j = m_j otherwise.
 *
 * Complex arrays are interleaved (re, im) binary64, the layout of numpy
 * complex128.
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

/* Neumaier's compensated sum: the running error of every addition is kept
 * exactly and added back at the end. */
typedef struct {
    double s, c;
} nsum;

static inline void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nsum_get(const nsum *a) { return a->s + a->c; }

/* d = n + (a - b) with n an integer and a, b in [-1/2, 1/2]; the difference
 * a - b is formed exactly as a two-term sum so that d carries one rounding. */
static inline double int_plus_diff(int64_t n, double a, double b)
{
    double hi = a - b;
    double bb = hi - a;
    double lo = (a - (hi - bb)) + (-b - bb);
    return ((double)n + hi) + lo;
}

/* Integer offset n reduced to (-N/2, N/2]. */
static inline int64_t wrap_half(int64_t n, int64_t N)
{
    n %= N;
    if (2 * n > N)
        n -= N;
    else if (2 * n <= -N)
        n += N;
    return n;
}

static void set_threads(int nthreads)
{
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
}

/* Threads a parallel region of the oracle uses (for reporting). */
int or_max_threads(int nthreads)
{
    set_threads(nthreads);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------ grid units */

/* s_j = N y_j / (2 pi) in binary128; m_j = nearest integer mod N,
 * theta_j = s_j - nearest integer (binary64).  Problem statement of
 * Section 2: x_k = 2 pi k / N, y_j arbitrary.
 *
 * |theta_j| < 1e-200 is returned as 0, an exact hit.  The kernel of
 * Eq. (p2) is smooth in y (every entry moves by at most 2 pi |theta_j|, far
 * below the rounding of any binary64 result), while its closed form (p4)
 * divides a vanishing F_j by a vanishing sine there, which underflows to
 * 0/0 for subnormal theta_j. */
void or_grid_units(int64_t N, int64_t M, const double *y, int64_t *m,
                   double *theta)
{
    const __float128 scale = (__float128)N / (2 * M_PIq);
    for (int64_t j = 0; j < M; ++j) {
        __float128 s = (__float128)y[j] * scale;
        __float128 n = floorq(s + 0.5Q);
        theta[j] = (double)(s - n);
        if (fabs(theta[j]) < 1e-200)
            theta[j] = 0.0;
        int64_t ni = (int64_t)fmodq(n, (__float128)N);
        if (ni < 0)
            ni += N;
        m[j] = ni;
    }
}

/* ---------------------------------------------------------------- forward */

/* One target of Eq. (p4)-(p5):
 *   g = F * sum_k G(y - x_k) f_k,  F = (e^{i N y} - 1) / N,
 *   G(t) = 1 / (e^{it} - 1) = -(1 + i cot(t/2)) / 2.
 * With y = 2 pi (m + theta) / N:  e^{iNy} - 1 = e^{2 pi i theta} - 1
 * = 2i sin(pi theta) e^{i pi theta}, and t/2 = pi d / N with d the grid
 * offset (m - k) + theta taken in (-N/2, N/2] + theta.
 * theta == 0 is an exact hit y = x_m: K_jk reduces to the Kronecker delta
 * (the sum of Eq. (p2) over n), so g = f_m. */
static void fwd_one(int64_t N, const double *f, int64_t m, double th,
                    double *out)
{
    if (th == 0.0) {
        out[0] = f[2 * m];
        out[1] = f[2 * m + 1];
        return;
    }
    nsum Sr = {0, 0}, Si = {0, 0}, Hr = {0, 0}, Hi = {0, 0};
    const double dN = (double)N;
    for (int64_t k = 0; k < N; ++k) {
        int64_t n = wrap_half(m - k, N);
        double d = (double)n + th;
        double sn, cs;
        sincos(M_PI * (d / dN), &sn, &cs);
        double ct = cs / sn;
        double fr = f[2 * k], fi = f[2 * k + 1];
        nsum_add(&Sr, fr);
        nsum_add(&Si, fi);
        nsum_add(&Hr, fr * ct);
        nsum_add(&Hi, fi * ct);
    }
    /* sum_k G f_k = -(S + i H) / 2 */
    double sr = nsum_get(&Sr), si = nsum_get(&Si);
    double hr = nsum_get(&Hr), hi = nsum_get(&Hi);
    double Gr = -0.5 * (sr - hi), Gi = -0.5 * (si + hr);
    double sp, cp;
    sincos(M_PI * th, &sp, &cp);
    double Fr = -2.0 * sp * sp / dN, Fi = 2.0 * sp * cp / dN;
    out[0] = Fr * Gr - Fi * Gi;
    out[1] = Fr * Gi + Fi * Gr;
}

/* g = K f with K_jk of Eq. (p2), evaluated through its closed form (p4). */
void or_fwd_kernel(int64_t N, int64_t M, const double *y, const double *f,
                   double *g, int nthreads)
{
    int64_t *m = malloc(sizeof(int64_t) * (size_t)M);
    double *th = malloc(sizeof(double) * (size_t)M);
    or_grid_units(N, M, y, m, th);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j)
        fwd_one(N, f, m[j], th[j], g + 2 * j);
    free(m);
    free(th);
}

/* The same sum at the selected targets sel[0..nsel) only. */
void or_fwd_kernel_at(int64_t N, int64_t M, const double *y, const double *f,
                      int64_t nsel, const int64_t *sel, double *gsel,
                      int nthreads)
{
    (void)M;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nsel; ++i) {
        int64_t m;
        double th;
        or_grid_units(N, 1, y + sel[i], &m, &th);
        fwd_one(N, f, m, th, gsel + 2 * i);
    }
}

/* The matrix K of Eq. (p2) itself, K[j][k] (row-major, M x N complex), each
 * entry in the closed form (p4)-(p5) the forward sums: F_j G(y_j - x_k),
 * with F_j = 2i sin(pi theta_j) e^{i pi theta_j} / N and
 * G(t) = -(1 + i cot(t/2)) / 2; a point on the grid (theta_j == 0) gives
 * the Kronecker delta. */
void or_kmatrix(int64_t N, int64_t M, const double *y, double *K, int nthreads)
{
    int64_t *m = malloc(sizeof(int64_t) * (size_t)(M ? M : 1));
    double *th = malloc(sizeof(double) * (size_t)(M ? M : 1));
    or_grid_units(N, M, y, m, th);
    const double dN = (double)N;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; ++j) {
        double *row = K + 2 * (size_t)j * (size_t)N;
        if (th[j] == 0.0) {
            for (int64_t k = 0; k < N; ++k) {
                row[2 * k] = k == m[j] ? 1.0 : 0.0;
                row[2 * k + 1] = 0.0;
            }
            continue;
        }
        double sp, cp;
        sincos(M_PI * th[j], &sp, &cp);
        const double Fr = -2.0 * sp * sp / dN, Fi = 2.0 * sp * cp / dN;
        for (int64_t k = 0; k < N; ++k) {
            const double d = (double)wrap_half(m[j] - k, N) + th[j];
            double sn, cs;
            sincos(M_PI * (d / dN), &sn, &cs);
            const double Gr = -0.5, Gi = -0.5 * (cs / sn);
            row[2 * k] = Fr * Gr - Fi * Gi;
            row[2 * k + 1] = Fr * Gi + Fi * Gr;
        }
    }
    free(m);
    free(th);
}

/* Adjoint of Eq. (p2): f_k = sum_j conj(K_jk) g_j at the grid points
 * k = ks[i] (all k = 0..N-1 when ks is NULL; nk outputs), with K_jk in
 * its closed form (p4)-(p5), K_jk = F_j G(y_j - x_k): the conjugate of the
 * same product fwd_one forms, term by term over j.  A point on the grid
 * (theta_j == 0, y_j = x_{m_j}) has K_jk = delta(k, m_j). */
void or_adj_at(int64_t N, int64_t M, const double *y, const double *g, int64_t nk,
               const int64_t *ks, double *f, int nthreads)
{
    int64_t *m = malloc(sizeof(int64_t) * (size_t)(M ? M : 1));
    double *th = malloc(sizeof(double) * (size_t)(M ? M : 1));
    double *F = malloc(sizeof(double) * 2 * (size_t)(M ? M : 1));
    or_grid_units(N, M, y, m, th);
    const double dN = (double)N;
    for (int64_t j = 0; j < M; ++j) {
        double sp, cp;
        sincos(M_PI * th[j], &sp, &cp);
        F[2 * j] = -2.0 * sp * sp / dN;   /* F_j = 2i sin(pi th) e^{i pi th} / N */
        F[2 * j + 1] = 2.0 * sp * cp / dN;
    }
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nk; ++i) {
        const int64_t k = ks ? ks[i] : i;
        nsum ar = {0, 0}, ai = {0, 0};
        for (int64_t j = 0; j < M; ++j) {
            const double gr = g[2 * j], gi = g[2 * j + 1];
            if (th[j] == 0.0) {
                if (m[j] == k) {
                    nsum_add(&ar, gr);
                    nsum_add(&ai, gi);
                }
                continue;
            }
            /* G(y_j - x_k) = -(1 + i cot(pi d / N)) / 2, d = (m_j - k) + th_j */
            const double d = (double)wrap_half(m[j] - k, N) + th[j];
            double sn, cs;
            sincos(M_PI * (d / dN), &sn, &cs);
            const double ct = cs / sn;
            const double Gr = -0.5, Gi = -0.5 * ct;
            const double Kr = F[2 * j] * Gr - F[2 * j + 1] * Gi;
            const double Ki = F[2 * j] * Gi + F[2 * j + 1] * Gr;
            /* conj(K) g */
            nsum_add(&ar, Kr * gr);
            nsum_add(&ar, Ki * gi);
            nsum_add(&ai, Kr * gi);
            nsum_add(&ai, -Ki * gr);
        }
        f[2 * i] = nsum_get(&ar);
        f[2 * i + 1] = nsum_get(&ai);
    }
    free(m);
    free(th);
    free(F);
}

/* Eq. (p1): g_j = f(y_j) = sum_{n=0}^{N-1} c_n e^{i n y_j}, the band-limited
 * interpolant evaluated term by term.  e^{i n y_j} = e^{2 pi i n s_j / N} is
 * split into the exact root of unity e^{2 pi i ((n m_j) mod N) / N} (table
 * rounded from binary128) and e^{2 pi i n theta_j / N}. */
void or_eval_series(int64_t N, int64_t M, const double *y, const double *c,
                    double *g, int nthreads)
{
    int64_t *m = malloc(sizeof(int64_t) * (size_t)M);
    double *th = malloc(sizeof(double) * (size_t)M);
    double *tab = malloc(sizeof(double) * 2 * (size_t)N);
    or_grid_units(N, M, y, m, th);
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < N; ++r) {
        __float128 a = 2 * M_PIq * (__float128)r / (__float128)N;
        tab[2 * r] = (double)cosq(a);
        tab[2 * r + 1] = (double)sinq(a);
    }
    const double dN = (double)N;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j) {
        nsum ar = {0, 0}, ai = {0, 0};
        for (int64_t n = 0; n < N; ++n) {
            int64_t r = (int64_t)(((__int128)n * m[j]) % N);
            double sn, cs;
            sincos(2.0 * M_PI * (((double)n * th[j]) / dN), &sn, &cs);
            double er = tab[2 * r] * cs - tab[2 * r + 1] * sn;
            double ei = tab[2 * r] * sn + tab[2 * r + 1] * cs;
            double cr = c[2 * n], ci = c[2 * n + 1];
            nsum_add(&ar, cr * er);
            nsum_add(&ar, -ci * ei);
            nsum_add(&ai, cr * ei);
            nsum_add(&ai, ci * er);
        }
        g[2 * j] = nsum_get(&ar);
        g[2 * j + 1] = nsum_get(&ai);
    }
    free(m);
    free(th);
    free(tab);
}

/* ---------------------------------------------------------------- inverse */

struct pt {
    int64_t m;
    double th;
};

static int pt_cmp(const void *a, const void *b)
{
    const struct pt *p = a, *q = b;
    if (p->m != q->m)
        return p->m < q->m ? -1 : 1;
    return (p->th > q->th) - (p->th < q->th);
}

/* Representative s' = m' + theta in [0, N) (see the file header). */
static inline int64_t rep_int(int64_t m, double th, int64_t N)
{
    return (m == 0 && th < 0.0) ? N : m;
}

/* log |2 sin(pi d / N)| for a grid offset d = n + (fa - fb), n reduced
 * first (|sin| has period N in d), split as E ln 2 + main + corr:
 *   - d and x = d / N are carried as double-double pairs, and the argument
 *     a = pi x as ah + al with pi = M_PI + PI_LO; the tail al enters to
 *     first order as al cot(ah) (corr);
 *   - |2 sin(ah)| = mant 2^E with mant in [1/2, 1), main = log(mant).
 * Callers sum E exactly, main and corr apart, and combine them once: the
 * rounding of pi alone would otherwise shift every term the same way (a
 * drift of 3.9e-17 N ln 2 over N terms), and rounding log|2 sin| whole
 * (terms up to ~12) costs an ulp of the term. */
static const double PI_LO = 1.2246467991473532e-16; /* pi - M_PI */

typedef struct {
    int64_t e;   /* sum of the binary exponents */
    nsum main;   /* sum of log(mant) */
    nsum corr;   /* sum of the argument tails */
} logsum;

static inline void logsum_add(logsum *ls, int64_t n, double fa, double fb, int64_t N)
{
    const double nd = (double)wrap_half(n, N);
    /* hi + lo = fa - fb exactly */
    const double hi = fa - fb;
    const double bb = hi - fa;
    const double lo = (fa - (hi - bb)) + (-fb - bb);
    /* dh + dl = nd + hi + lo */
    const double dh = nd + hi;
    const double bv = dh - nd;
    const double dl = ((nd - (dh - bv)) + (hi - bv)) + lo;
    /* q + ql = (dh + dl) / N */
    const double Nd = (double)N;
    const double q = dh / Nd;
    const double ql = (fma(-q, Nd, dh) + dl) / Nd;
    /* ah + al = pi (q + ql) */
    const double ah = M_PI * q;
    const double al = fma(M_PI, q, -ah) + M_PI * ql + PI_LO * q;
    double sn, cs;
    sincos(ah, &sn, &cs);
    int e;
    const double mant = frexp(fabs(2.0 * sn), &e);
    ls->e += e;
    nsum_add(&ls->main, log(mant));
    nsum_add(&ls->corr, al * (cs / sn));
}

/* E ln 2 and the sum of log(mant) are each large and cancel to an O(1)
 * result: they are combined in binary128 from the unrounded compensated
 * pairs (s, c). */
static inline double logsum_get(const logsum *ls)
{
    const __float128 v = (__float128)ls->e * M_LN2q + (__float128)ls->main.s +
                         (__float128)ls->main.c + (__float128)ls->corr.s +
                         (__float128)ls->corr.c;
    return (double)v;
}

/* Sums behind the coefficients of Eq. (p8), rescaled by 2^N (the rescaling
 * cancels in the product C_k D_j):
 *   logC[k] = sum_j log|2 sin((x_k - y_j)/2)|,
 *   logD[j] = -sum_{i != j} log|2 sin((y_j - y_i)/2)|,
 * and the sign counts negC[k] = #{j : s'_j > k},
 * negD[j] = #{i : s'_i > s'_j}.  A target k with an exact hit s'_j == k
 * gets logC = -inf.  Only the entries listed in ks / js are computed
 * (pass nk = N, ks = NULL for all). */
void or_logsums_at(int64_t N, const double *y, int64_t nk, const int64_t *ks,
                   double *logC, int64_t *negC, int64_t nj, const int64_t *js,
                   double *logD, int64_t *negD, int nthreads)
{
    int64_t *m = malloc(sizeof(int64_t) * (size_t)N);
    double *th = malloc(sizeof(double) * (size_t)N);
    or_grid_units(N, N, y, m, th);
    for (int64_t j = 0; j < N; ++j)
        m[j] = rep_int(m[j], th[j], N);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < nk; ++i) {
        int64_t k = ks ? ks[i] : i;
        logsum acc = {0, {0, 0}, {0, 0}};
        int64_t neg = 0;
        int hit = 0;
        for (int64_t j = 0; j < N; ++j) {
            /* x_k - y_j in grid units: (k - m'_j) - theta_j */
            if (m[j] == k && th[j] == 0.0) {
                hit = 1;
                continue;
            }
            logsum_add(&acc, k - m[j], 0.0, th[j], N);
            if (m[j] > k || (m[j] == k && th[j] > 0.0))
                ++neg;
        }
        logC[i] = hit ? -INFINITY : logsum_get(&acc);
        negC[i] = neg;
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < nj; ++t) {
        int64_t j = js ? js[t] : t;
        logsum acc = {0, {0, 0}, {0, 0}};
        int64_t neg = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (i == j)
                continue;
            /* y_j - y_i in grid units: (m'_j - m'_i) + (theta_j - theta_i) */
            double d = int_plus_diff(m[j] - m[i], th[j], th[i]);
            if (d < 0.0)
                ++neg;
            logsum_add(&acc, m[j] - m[i], th[j], th[i], N);
        }
        logD[t] = -logsum_get(&acc);
        negD[t] = neg;
    }
    free(m);
    free(th);
}

/* Inverse interpolation, Eq. (p6)/(p8), M = N:
 *   f_k = C_k sum_j G(x_k - y_j) D_j g_j,
 *   C_k = (-1)^k prod_j sin((x_k - y_j)/2),
 *   D_j = 2i e^{-iNy_j/2} / prod_{k != j} sin((y_j - y_k)/2).
 * Evaluated as Chat_k = 2^N C_k and Dhat_j = 2^{-N} D_j from the log-sums
 * above.  e^{-iNy_j/2} = e^{-i pi s'_j} = (-1)^{m'_j} e^{-i pi theta_j}; the
 * sign of prod sin(pi (k - s'_j)/N) over j is (-1)^{#{j: s'_j > k}}, and
 * likewise for the denominator of D_j.  An exact hit theta_j == 0 makes
 * C_{m_j} vanish and G singular; the limit is f_{m_j} = g_j.
 * Returns 0, 4 if two points coincide, 5 if a coefficient leaves the binary64
 * range. */
int or_inv(int64_t N, const double *y, const double *g, double *f,
           int nthreads)
{
    int64_t *m = malloc(sizeof(int64_t) * (size_t)N);
    double *th = malloc(sizeof(double) * (size_t)N);
    double *logC = malloc(sizeof(double) * (size_t)N);
    double *logD = malloc(sizeof(double) * (size_t)N);
    int64_t *negC = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *negD = malloc(sizeof(int64_t) * (size_t)N);
    double *w = malloc(sizeof(double) * 2 * (size_t)N);
    int status = 0;

    or_grid_units(N, N, y, m, th);
    int64_t *mr = malloc(sizeof(int64_t) * (size_t)N);
    for (int64_t j = 0; j < N; ++j)
        mr[j] = rep_int(m[j], th[j], N);

    /* two coincident points make the interpolation problem singular */
    {
        struct pt *p = malloc(sizeof(struct pt) * (size_t)N);
        for (int64_t j = 0; j < N; ++j) {
            p[j].m = mr[j];
            p[j].th = th[j];
        }
        qsort(p, (size_t)N, sizeof(struct pt), pt_cmp);
        for (int64_t j = 1; j < N; ++j)
            if (p[j].m == p[j - 1].m && p[j].th == p[j - 1].th)
                status = 4;
        free(p);
    }
    if (status)
        goto done;

    or_logsums_at(N, y, N, NULL, logC, negC, N, NULL, logD, negD, nthreads);

    /* w_j = Dhat_j g_j */
    for (int64_t j = 0; j < N; ++j) {
        if (logD[j] > 700.0) {
            status = 5;
            goto done;
        }
        double mag = exp(logD[j]);
        double sgn = (((mr[j] + negD[j]) & 1) ? -1.0 : 1.0);
        double sp, cp;
        sincos(M_PI * th[j], &sp, &cp);
        /* i e^{-i pi theta} = sin(pi theta) + i cos(pi theta) */
        double dr = sgn * mag * sp, di = sgn * mag * cp;
        double gr = g[2 * j], gi = g[2 * j + 1];
        w[2 * j] = dr * gr - di * gi;
        w[2 * j + 1] = dr * gi + di * gr;
    }
    for (int64_t k = 0; k < N; ++k)
        if (logC[k] > 700.0) {
            status = 5;
            goto done;
        }

    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < N; ++k) {
        if (logC[k] == -INFINITY) /* overwritten by the hit below */
            continue;
        nsum Wr = {0, 0}, Wi = {0, 0}, Hr = {0, 0}, Hi = {0, 0};
        for (int64_t j = 0; j < N; ++j) {
            /* (x_k - y_j)/2 = pi d / N with d = (k - m'_j) - theta_j */
            double d = int_plus_diff(wrap_half(k - mr[j], N), 0.0, th[j]);
            double sn, cs;
            sincos(M_PI * (d / (double)N), &sn, &cs);
            double ct = cs / sn;
            nsum_add(&Wr, w[2 * j]);
            nsum_add(&Wi, w[2 * j + 1]);
            nsum_add(&Hr, w[2 * j] * ct);
            nsum_add(&Hi, w[2 * j + 1] * ct);
        }
        /* sum_j G w_j = -(W + i H)/2 */
        double Gr = -0.5 * (nsum_get(&Wr) - nsum_get(&Hi));
        double Gi = -0.5 * (nsum_get(&Wi) + nsum_get(&Hr));
        double C = exp(logC[k]) * (((k + negC[k]) & 1) ? -1.0 : 1.0);
        f[2 * k] = C * Gr;
        f[2 * k + 1] = C * Gi;
    }
    for (int64_t j = 0; j < N; ++j)
        if (th[j] == 0.0) {
            f[2 * m[j]] = g[2 * j];
            f[2 * m[j] + 1] = g[2 * j + 1];
        }

done:
    free(m);
    free(mr);
    free(th);
    free(logC);
    free(logD);
    free(negC);
    free(negD);
    free(w);
    return status;
}

/* Chat_k (k in ks) and Dhat_j (j in js) of Eq. (p8), rescaled by 2^N:
 *   Chat_k = (-1)^(k + #{j: s_j > k}) exp(logC_k)       (0 at an exact hit),
 *   Dhat_j = (-1)^(m'_j + #{i: s_i > s_j}) exp(logD_j) i e^{-i pi theta_j},
 * from the direct log-sums above (the same composition as or_inv). */
void or_coeffs_at(int64_t N, const double *y, int64_t nk, const int64_t *ks,
                  double *chat, int64_t nj, const int64_t *js, double *dhat,
                  int nthreads)
{
    double *logC = malloc(sizeof(double) * (size_t)(nk ? nk : 1));
    double *logD = malloc(sizeof(double) * (size_t)(nj ? nj : 1));
    int64_t *negC = malloc(sizeof(int64_t) * (size_t)(nk ? nk : 1));
    int64_t *negD = malloc(sizeof(int64_t) * (size_t)(nj ? nj : 1));
    or_logsums_at(N, y, nk, ks, logC, negC, nj, js, logD, negD, nthreads);
    for (int64_t i = 0; i < nk; ++i) {
        const int64_t k = ks[i];
        chat[i] = logC[i] == -INFINITY
                      ? 0.0
                      : exp(logC[i]) * (((k + negC[i]) & 1) ? -1.0 : 1.0);
    }
    for (int64_t t = 0; t < nj; ++t) {
        int64_t m;
        double th;
        or_grid_units(N, 1, y + js[t], &m, &th);
        const int64_t mr = rep_int(m, th, N);
        const double sgn = (((mr + negD[t]) & 1) ? -1.0 : 1.0) * exp(logD[t]);
        double sp, cp;
        sincos(M_PI * th, &sp, &cp);
        dhat[2 * t] = sgn * sp;
        dhat[2 * t + 1] = sgn * cp;
    }
    free(logC);
    free(logD);
    free(negC);
    free(negD);
}
