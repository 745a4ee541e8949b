// Host side of the FMM-based NUFFT / INUFFT: parameter selection, operator
// tables, plans, launches and the C ABI declared in include/fmmnufft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fmmnufft.h"
#include "fmm_kernels.h"
#include "tree_kernels.h"

using namespace fn;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

#define HIPCHK(expr)                                                           \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(FN_EHIP, "%s: %s (%s:%d)", #expr,                      \
                        hipGetErrorString(e_), __FILE__, __LINE__);            \
    } while (0)

// ---------------------------------------------------- caching device memory
//
// Plans are created and destroyed per one-shot call; freed blocks are kept
// per size and handed out again so that repeated calls do not pay for
// hipMalloc / hipFree.

namespace {
std::mutex g_pool_mu;
std::multimap<size_t, void *> g_pool;

size_t round_bytes(size_t n) { return (n + 255) & ~size_t(255); }

void *pool_get(size_t bytes)
{
    bytes = round_bytes(bytes ? bytes : 1);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pool.find(bytes);
        if (it != g_pool.end()) {
            void *p = it->second;
            g_pool.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return nullptr;
    return p;
}

void pool_put(void *p, size_t bytes)
{
    if (!p)
        return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.emplace(round_bytes(bytes ? bytes : 1), p);
}

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};
} // namespace

// ------------------------------------------------- parameters (Section 2.3)

// Eq. (18.2) as printed uses 3 pi / (10 eps); balancing the two halves of
// Eq. (18) gives 10 / (3 pi eps).  The larger of the two is taken.
static void trunc_numbers(double eps, int lmax, int *p, int *q)
{
    const double x = std::max(3.0 * M_PI / (10.0 * eps), 10.0 / (3.0 * M_PI * eps));
    *q = std::max(1, (int)std::ceil(0.5 * std::log2(x)));
    *p = std::max(2, (int)std::ceil(std::log(x) / std::log(3.0) +
                                     lmax / std::log2(3.0) + 1.0));
}

// Depth: Eq. (25) with the offset measured by the paper (l_max = log2 N - 5
// for N = M, Section 3.2), generalised to N != M through log2 sqrt(N M).
static int default_depth(int64_t N, int64_t M, int dtype)
{
    (void)dtype;
    const double lg = 0.5 * std::log2((double)N * (double)M);
    int l = (int)std::lround(lg) - 5;
    if (const char *e = getenv("FN_LEAF_OFFSET"))
        l = (int)std::lround(lg) - atoi(e);
    return std::min(24, std::max(2, l));
}

static int round8(int x) { return (x + 7) & ~7; }

static double eps_floor(int dtype) { return dtype == FN_C64 ? 1e-7 : 1e-15; }

// ------------------------------------------------------ operator tables

// |B_2m| = 2 (2m)! zeta(2m) / (2 pi)^(2m)  (m >= 1), zeta by direct
// summation with an Euler-Maclaurin tail, in long double.
static long double bernoulli_abs(int m)
{
    const int s = 2 * m;
    const int K = 64;
    long double z = 0;
    for (int k = K - 1; k >= 1; --k)
        z += powl((long double)k, -(long double)s);
    const long double Kl = K;
    z += powl(Kl, 1.0L - s) / (s - 1) + 0.5L * powl(Kl, -(long double)s);
    // Bernoulli-number corrections of the tail: B_2 s/2!, B_4 s(s+1)(s+2)/4!, ...
    const long double B[] = {1.0L / 6, -1.0L / 30, 1.0L / 42, -1.0L / 30, 5.0L / 66};
    long double fac = 1, rise = s;
    for (int j = 1; j <= 5; ++j) {
        fac *= (2 * j - 1) * (2 * j);
        z += B[j - 1] / fac * rise * powl(Kl, -(long double)(s + 2 * j - 1));
        rise *= (long double)(s + 2 * j - 1) * (s + 2 * j);
    }
    long double r = 2 * z;
    const long double twopi = 6.283185307179586476925286766559L;
    for (int i = 1; i <= s; ++i)
        r *= (long double)i / twopi;
    return r;
}

static long double binom(int n, int k)
{
    if (k < 0 || k > n)
        return 0;
    long double r = 1;
    for (int i = 1; i <= k; ++i)
        r = r * (n - k + i) / i;
    return r;
}

static long double factl(int n)
{
    long double r = 1;
    for (int i = 2; i <= n; ++i)
        r *= i;
    return r;
}

struct Tables {
    std::vector<long double> m2m, l2l, m2l, bin, reg1, reg2;
};

// M2M (child at c_p + s r_p/2 -> parent):  a^P_n = sum_{m<=n} C(n,m) 2^-n s^(n-m) a^C_m
// L2L (parent -> child):                   b^C_m = sum_{n>=m} C(n,m) 2^-n s^(n-m) b^P_n
// M2L cot (1/t kernel, delta = (c_t - c_s)/r):
//                    b_n = sum_m (-1)^n C(m+n, n) delta^-(m+n+1) a_m
// M2L log (log|t| kernel):
//                    b_0 = a_0 log|delta| - sum_{m>=1} (a_m/m) delta^-m
//                    b_n = a_0 (-1)^(n+1) / (n delta^n)
//                          - sum_{m>=1} (a_m/m) C(m+n-1, n) (-1)^n delta^-(m+n)
// Regular part at level 2 (Eq. p20 and its log analogue) in the variable
// u = (y - x_c)/(pi/4), with A_t the moments of Omega_1 (reg1) or of the
// opposite quarter (reg2) about the centre x_c in units of pi/4.
static void build_tables(int P, int q, int kernel, Tables &T)
{
    const int PP = P * P;
    T.m2m.assign(2 * PP, 0);
    T.l2l.assign(2 * PP, 0);
    T.m2l.assign(4 * PP, 0);
    T.bin.assign(PP, 0);
    T.reg1.assign(PP, 0);
    T.reg2.assign(PP, 0);
    for (int c = 0; c < 2; ++c) {
        const long double s = c == 0 ? -1 : 1;
        for (int n = 0; n < P; ++n)
            for (int m = 0; m <= n; ++m) {
                long double v = binom(n, m) * powl(2.0L, -n) * powl(s, n - m);
                T.m2m[c * PP + m * P + n] = v; // [in m][out n]
                T.l2l[c * PP + n * P + m] = v; // [in n][out m]
            }
    }
    const int deltas[4] = {-6, -4, 4, 6};
    for (int di = 0; di < 4; ++di) {
        const long double d = deltas[di];
        for (int m = 0; m < P; ++m)
            for (int n = 0; n < P; ++n) {
                long double v;
                if (kernel == KER_COT) {
                    v = ((n & 1) ? -1 : 1) * binom(m + n, n) * powl(d, -(m + n + 1));
                } else if (m == 0 && n == 0) {
                    v = logl(fabsl(d));
                } else if (n == 0) {
                    v = -powl(d, -m) / m;
                } else if (m == 0) {
                    v = ((n & 1) ? 1 : -1) / (n * powl(d, n));
                } else {
                    v = -binom(m + n - 1, n) * ((n & 1) ? -1 : 1) * powl(d, -(m + n)) / m;
                }
                T.m2l[di * PP + m * P + n] = v;
            }
    }
    for (int t = 0; t < P; ++t)
        for (int j = 0; j <= t; ++j)
            T.bin[t * P + j] = binom(t, j);
    const long double qpi = 0.785398163397448309615660845819875721L; // pi/4
    for (int m = 1; m <= q; ++m) {
        const long double B = bernoulli_abs(m);
        const long double four_m = powl(4.0L, m) - 1;
        const int top = kernel == KER_COT ? 2 * m - 1 : 2 * m;
        for (int lo = 0; lo <= top; ++lo) {
            const int t = (kernel == KER_COT ? 2 * m - 1 : 2 * m) - lo;
            if (lo >= P || t >= P)
                continue;
            const long double w = kernel == KER_COT ? B / m : B / (2 * m);
            const long double kap = -(powl(qpi, lo) / factl(lo)) * w *
                                    (powl(-qpi, t) / factl(t));
            T.reg1[t * P + lo] = kap;
            T.reg2[t * P + lo] = kap * four_m;
        }
    }
}

// ------------------------------------------------------------------ plan

struct fn_plan {
    int kind = 0, dtype = 0;
    int64_t N = 0, M = 0;
    int p = 0, q = 0, l = 0, P = 0;
    double eps = 0;
    int lr = 2;                   // subtree root level of k_down_eval
    // sorted point set (targets of the forward, sources of the inverse)
    Buf off, sm, sth, sperm;
    Buf work;
    int nwork = 0;
    // k_up band structure
    UpArgs<float, cx<float>> bands_f; // only the band fields are used
    int up_grid = 0;
    size_t up_smem = 0, dn_smem = 0;
    Buf cnt;
    // cot expansions and operators (element type R = double or float)
    Buf mp, loc2, S, tabs;
    size_t tab_m2m = 0, tab_l2l = 0, tab_m2l = 0, tab_bin = 0, tab_reg1 = 0,
           tab_reg2 = 0;
    // inverse
    Buf hit, chat, dhat, wsorted;
    std::vector<Buf *> all()
    {
        return {&off, &sm, &sth, &sperm, &work, &cnt, &mp, &loc2, &S, &tabs,
                &hit, &chat, &dhat, &wsorted};
    }
};

static bool alloc(Buf &b, size_t bytes)
{
    b.n = bytes;
    b.p = pool_get(bytes);
    return b.p != nullptr;
}

static void release(Buf &b)
{
    pool_put(b.p, b.n);
    b.p = nullptr;
    b.n = 0;
}

static void release_plan(fn_plan *P)
{
    for (Buf *b : P->all())
        release(*b);
}

// Bands of k_up: climbs of at most dmax levels from the leaves to level 2.
template <typename BandArgs>
static void make_bands(int l, int dmax, BandArgs &a, int *grid, int *ncnt)
{
    int nb = 0, lo = l;
    while (true) {
        int d = std::min(dmax, lo - 2);
        a.band_lo[nb] = lo;
        a.band_d[nb] = d;
        ++nb;
        lo -= d;
        if (lo == 2)
            break;
    }
    a.nbands = nb;
    // counters: band k (k >= 1) has 2^(band_lo[k] - band_d[k]) nodes; the
    // final stage has one.
    int off = 0;
    a.cnt_off[0] = 0;
    for (int k = 1; k < nb; ++k) {
        a.cnt_off[k] = off;
        off += 1 << (a.band_lo[k] - a.band_d[k]);
    }
    a.cnt_off[nb] = off;
    off += 1;
    *ncnt = off;
    *grid = 1 << (l - a.band_d[0]);
}

template <typename R>
static int upload_tables(fn_plan *P, int kernel, int Pn, int q, hipStream_t st)
{
    Tables T;
    build_tables(Pn, q, kernel, T);
    std::vector<R> h;
    auto push = [&](const std::vector<long double> &v) {
        size_t o = h.size();
        for (long double x : v)
            h.push_back((R)x);
        return o;
    };
    P->tab_m2m = push(T.m2m);
    P->tab_l2l = push(T.l2l);
    P->tab_m2l = push(T.m2l);
    P->tab_bin = push(T.bin);
    P->tab_reg1 = push(T.reg1);
    P->tab_reg2 = push(T.reg2);
    if (!alloc(P->tabs, h.size() * sizeof(R)))
        return fail(FN_ENOMEM, "table allocation failed");
    HIPCHK(hipMemcpyAsync(P->tabs.p, h.data(), h.size() * sizeof(R),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st)); // h goes out of scope
    return FN_OK;
}

// Double-double N / (2 pi): 1/(2 pi) = ONE_OVER_2PI_HI + ONE_OVER_2PI_LO.
static const double ONE_OVER_2PI_HI = 0x1.45f306dc9c883p-3;
static const double ONE_OVER_2PI_LO = -0x1.6b01ec5417056p-57;

static void n_over_2pi(int64_t N, double *hi, double *lo)
{
#pragma clang fp contract(off)
    const double n = (double)N;
    double p = n * ONE_OVER_2PI_HI;
    double e = std::fma(n, ONE_OVER_2PI_HI, -p);
    e = std::fma(n, ONE_OVER_2PI_LO, e);
    *hi = p + e;
    *lo = e - (*hi - p);
}

static int grid_for(int64_t n, int block = 256)
{
    int64_t g = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// Sort a point set into the leaves.  deterministic = order inside a leaf by
// position (inverse); otherwise arbitrary (forward).  Also fills the hit map
// when requested.  Synchronises.
static int build_tree(fn_plan *P, int64_t n, const double *y, bool deterministic,
                      bool want_hit, hipStream_t st)
{
    const int64_t nleaf = int64_t(1) << P->l;
    Buf um, uth, ukey, count, cursor, flags, gm, gth, gperm, gkey;
    auto cleanup = [&]() {
        for (Buf *b : {&um, &uth, &ukey, &count, &cursor, &flags, &gm, &gth,
                       &gperm, &gkey})
            release(*b);
    };
    bool ok = alloc(um, n * 4) && alloc(uth, n * 8) && alloc(ukey, n * 4) &&
              alloc(count, nleaf * 4) && alloc(cursor, nleaf * 4) &&
              alloc(flags, 4) && alloc(P->off, (nleaf + 1) * 4) &&
              alloc(P->sm, n * 4) && alloc(P->sth, n * 8) &&
              alloc(P->sperm, n * 4);
    if (ok && deterministic)
        ok = alloc(gm, n * 4) && alloc(gth, n * 8) && alloc(gperm, n * 4) &&
             alloc(gkey, n * 4);
    if (ok && want_hit)
        ok = alloc(P->hit, P->N * 4);
    if (!ok) {
        cleanup();
        return fail(FN_ENOMEM, "workspace allocation failed (%lld points)", (long long)n);
    }
    double chi, clo;
    n_over_2pi(P->N, &chi, &clo);
    int rc = FN_OK;
#define TRY(expr)                                                              \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            rc = fail(FN_EHIP, "%s: %s", #expr, hipGetErrorString(e_));        \
            goto out;                                                          \
        }                                                                      \
    } while (0)
    {
        TRY(hipMemsetAsync(count.p, 0, nleaf * 4, st));
        TRY(hipMemsetAsync(flags.p, 0, 4, st));
        if (want_hit)
            TRY(hipMemsetAsync(P->hit.p, 0xff, P->N * 4, st));
        hipLaunchKernelGGL(k_reduce, dim3(grid_for(n)), dim3(256), 0, st, n, y,
                           chi, clo, P->N, P->l, (double)FN_Y_MAX,
                           (int32_t *)um.p, (double *)uth.p, (int32_t *)ukey.p,
                           (int32_t *)count.p,
                           want_hit ? (int32_t *)P->hit.p : nullptr,
                           (int *)flags.p);
        TRY(hipGetLastError());
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st,
                           (const int32_t *)count.p, (int32_t *)P->off.p,
                           (int32_t *)cursor.p, nleaf);
        TRY(hipGetLastError());
        if (!deterministic) {
            hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(256), 0, st, n,
                               (const int32_t *)um.p, (const double *)uth.p,
                               (const int32_t *)ukey.p, (int32_t *)cursor.p,
                               (int32_t *)P->sm.p, (double *)P->sth.p,
                               (int32_t *)P->sperm.p, nullptr);
            TRY(hipGetLastError());
        } else {
            hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(256), 0, st, n,
                               (const int32_t *)um.p, (const double *)uth.p,
                               (const int32_t *)ukey.p, (int32_t *)cursor.p,
                               (int32_t *)gm.p, (double *)gth.p,
                               (int32_t *)gperm.p, (int32_t *)gkey.p);
            TRY(hipGetLastError());
            hipLaunchKernelGGL(k_rank, dim3(grid_for(n)), dim3(256), 0, st, n,
                               (const int32_t *)gm.p, (const double *)gth.p,
                               (const int32_t *)gperm.p, (const int32_t *)gkey.p,
                               (const int32_t *)P->off.p, (int32_t *)P->sm.p,
                               (double *)P->sth.p, (int32_t *)P->sperm.p,
                               (int *)flags.p);
            TRY(hipGetLastError());
        }
        int hflags = 0;
        TRY(hipMemcpyAsync(&hflags, flags.p, 4, hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        if (hflags & FLAG_BAD_Y) {
            rc = fail(FN_EINVAL, "y holds a non-finite value or |y| > %g", FN_Y_MAX);
            goto out;
        }
        if (hflags & FLAG_DUP) {
            rc = fail(FN_ESINGULAR, "two points y_j coincide on the circle");
            goto out;
        }
    }
out:
#undef TRY
    cleanup();
    return rc;
}

// Work items of k_down_eval: one per subtree of level lr holding targets,
// split so that no item has more than tmax sorted targets.
static int build_work(fn_plan *P, bool sorted_targets, bool uniform_targets,
                      hipStream_t st)
{
    const int64_t nleaf = int64_t(1) << P->l;
    const int s = P->l - P->lr;
    std::vector<int32_t> off(nleaf + 1);
    HIPCHK(hipMemcpyAsync(off.data(), P->off.p, (nleaf + 1) * 4,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int32_t tmax = 2048;
    std::vector<WorkItem> items;
    const int64_t nroot = int64_t(1) << P->lr;
    for (int64_t R = 0; R < nroot; ++R) {
        int32_t t0 = 0, t1 = 0, u0 = 0, u1 = 0;
        if (sorted_targets) {
            t0 = off[R << s];
            t1 = off[(R + 1) << s];
        }
        if (uniform_targets) {
            u0 = (int32_t)((R * P->N + nroot - 1) >> P->lr);
            u1 = (int32_t)(((R + 1) * P->N + nroot - 1) >> P->lr);
        }
        if (t1 == t0 && u1 == u0)
            continue;
        if (sorted_targets && !uniform_targets) {
            for (int32_t a = t0; a < t1; a += tmax)
                items.push_back({R, a, std::min(t1, a + tmax), 0, 0});
        } else {
            items.push_back({R, t0, t1, u0, u1});
        }
    }
    P->nwork = (int)items.size();
    if (!alloc(P->work, std::max<size_t>(1, items.size()) * sizeof(WorkItem)))
        return fail(FN_ENOMEM, "work list allocation failed");
    if (!items.empty()) {
        HIPCHK(hipMemcpyAsync(P->work.p, items.data(), items.size() * sizeof(WorkItem),
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return FN_OK;
}

static constexpr int UP_DMAX = 4;
static constexpr int DN_S = 4;

// Expansion storage and k_up / k_down_eval launch shapes for one FMM.
template <typename R, typename V>
static int setup_fmm(fn_plan *P, int kernel, int Pn, int q, Buf &mp, Buf &loc2,
                     Buf &S, Buf &cnt, UpArgs<R, V> &ua, int *up_grid,
                     size_t *up_smem, size_t *dn_smem, hipStream_t st)
{
    int ncnt = 0;
    make_bands(P->l, UP_DMAX, ua, up_grid, &ncnt);
    const int64_t nmp = lev_off(P->l + 1, Pn);
    if (!alloc(mp, nmp * sizeof(V)) || !alloc(loc2, 4 * Pn * sizeof(V)) ||
        !alloc(S, sizeof(V)) || !alloc(cnt, ncnt * 4))
        return fail(FN_ENOMEM, "expansion allocation failed");
    HIPCHK(hipMemsetAsync(cnt.p, 0, ncnt * 4, st));
    const int d0 = ua.band_d[0];
    const int nbot = 1 << std::max(d0, 0);
    *up_smem = (size_t)std::max(nbot + std::max(nbot / 2, 1), 8) * Pn * sizeof(V);
    *dn_smem = (size_t)2 * ((size_t)1 << (P->l - P->lr)) * Pn * sizeof(V);
    (void)kernel;
    (void)q;
    return FN_OK;
}

// --------------------------------------------------------- forward plan

template <typename R>
static int plan_fwd_impl(fn_plan *P, const double *y, hipStream_t st)
{
    int rc = build_tree(P, P->M, y, false, false, st);
    if (rc)
        return rc;
    P->lr = std::max(2, P->l - DN_S);
    rc = build_work(P, true, false, st);
    if (rc)
        return rc;
    rc = upload_tables<R>(P, KER_COT, P->P, P->q, st);
    if (rc)
        return rc;
    UpArgs<R, cx<R>> ua{};
    rc = setup_fmm<R, cx<R>>(P, KER_COT, P->P, P->q, P->mp, P->loc2, P->S, P->cnt,
                             ua, &P->up_grid, &P->up_smem, &P->dn_smem, st);
    if (rc)
        return rc;
    std::memcpy(P->bands_f.band_lo, ua.band_lo, sizeof ua.band_lo);
    std::memcpy(P->bands_f.band_d, ua.band_d, sizeof ua.band_d);
    std::memcpy(P->bands_f.cnt_off, ua.cnt_off, sizeof ua.cnt_off);
    P->bands_f.nbands = ua.nbands;
    HIPCHK(hipStreamSynchronize(st));
    return FN_OK;
}

template <typename R, typename A>
static void copy_bands(const fn_plan *P, A &a)
{
    std::memcpy(a.band_lo, P->bands_f.band_lo, sizeof a.band_lo);
    std::memcpy(a.band_d, P->bands_f.band_d, sizeof a.band_d);
    std::memcpy(a.cnt_off, P->bands_f.cnt_off, sizeof a.cnt_off);
    a.nbands = P->bands_f.nbands;
}

template <typename R>
static int exec_fwd(fn_plan *P, const void *in, void *out, hipStream_t st)
{
    using V = cx<R>;
    const R *tabs = (const R *)P->tabs.p;
    UpArgs<R, V> ua{};
    copy_bands<R>(P, ua);
    ua.N = P->N;
    ua.l = P->l;
    ua.P = P->P;
    ua.cnt = (int *)P->cnt.p;
    ua.f_uniform = (const cx<R> *)in;
    ua.mp = (V *)P->mp.p;
    ua.loc2 = (V *)P->loc2.p;
    ua.S = (V *)P->S.p;
    ua.m2m = tabs + P->tab_m2m;
    ua.bin = tabs + P->tab_bin;
    ua.reg1 = tabs + P->tab_reg1;
    ua.reg2 = tabs + P->tab_reg2;
    hipLaunchKernelGGL((k_up<R, V, KER_COT, SET_UNIFORM>), dim3(P->up_grid),
                       dim3(BLOCK), P->up_smem, st, ua);
    HIPCHK(hipGetLastError());
    if (P->nwork == 0)
        return FN_OK;
    DownArgs<R, V> da{};
    da.N = P->N;
    da.l = P->l;
    da.P = P->P;
    da.lr = P->lr;
    da.work = (const WorkItem *)P->work.p;
    da.mp = (const V *)P->mp.p;
    da.loc2 = (const V *)P->loc2.p;
    da.l2l = tabs + P->tab_l2l;
    da.m2l = tabs + P->tab_m2l;
    da.f_uniform = (const cx<R> *)in;
    da.tgt = {(const int32_t *)P->off.p, (const int32_t *)P->sm.p,
              (const double *)P->sth.p, (const int32_t *)P->sperm.p};
    da.out = (cx<R> *)out;
    da.S = (const V *)P->S.p;
    da.f_hit = (const cx<R> *)in;
    hipLaunchKernelGGL((k_down_eval<R, V, KER_COT, SET_UNIFORM, EPI_FWD>),
                       dim3(P->nwork), dim3(BLOCK), P->dn_smem, st, da);
    HIPCHK(hipGetLastError());
    return FN_OK;
}

// --------------------------------------------------------- inverse plan

// The log-kernel FMM of the plan: logC_k at the uniform points and logD_j
// at the sorted sources, then Chat and Dhat (Eq. p8).
static int plan_inv_logs(fn_plan *P, hipStream_t st)
{
    using R = double;
    using V = double;
    // parameters of the log FMM: the log-sums are absolute errors of log|C|,
    // log|D|, i.e. relative errors of f, so they get a tenth of eps.
    const double eps_log = std::max(P->eps * 0.1, 1e-15);
    int plog, qlog;
    trunc_numbers(eps_log, P->l, &plog, &qlog);
    const int Plog = round8(std::max(plog, 2 * qlog + 1));
    fn_plan tmp; // tables of the log kernel
    int rc = upload_tables<R>(&tmp, KER_LOG, Plog, qlog, st);
    if (rc) {
        release_plan(&tmp);
        return rc;
    }
    Buf mp, loc2, S, cnt, logc, logd, flags;
    UpArgs<R, V> ua{};
    int up_grid;
    size_t up_smem, dn_smem;
    auto cleanup = [&]() {
        for (Buf *b : {&mp, &loc2, &S, &cnt, &logc, &logd, &flags})
            release(*b);
        release_plan(&tmp);
    };
    rc = setup_fmm<R, V>(P, KER_LOG, Plog, qlog, mp, loc2, S, cnt, ua, &up_grid,
                         &up_smem, &dn_smem, st);
    if (!rc && !(alloc(logc, P->N * 8) && alloc(logd, P->N * 8) && alloc(flags, 4)))
        rc = fail(FN_ENOMEM, "log-sum allocation failed");
    if (rc) {
        cleanup();
        return rc;
    }
    const R *tabs = (const R *)tmp.tabs.p;
    ua.N = P->N;
    ua.l = P->l;
    ua.P = Plog;
    ua.cnt = (int *)cnt.p;
    ua.src = {(const int32_t *)P->off.p, (const int32_t *)P->sm.p,
              (const double *)P->sth.p, (const int32_t *)P->sperm.p};
    ua.mp = (V *)mp.p;
    ua.loc2 = (V *)loc2.p;
    ua.S = (V *)S.p;
    ua.m2m = tabs + tmp.tab_m2m;
    ua.bin = tabs + tmp.tab_bin;
    ua.reg1 = tabs + tmp.tab_reg1;
    ua.reg2 = tabs + tmp.tab_reg2;
    ua.logc1 = std::log(2.0 * M_PI / (double)P->N);
    ua.logc2 = std::log(2.0);
    hipLaunchKernelGGL((k_up<R, V, KER_LOG, SET_SORTED>), dim3(up_grid),
                       dim3(BLOCK), up_smem, st, ua);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        DownArgs<R, V> da{};
        da.N = P->N;
        da.l = P->l;
        da.P = Plog;
        da.lr = P->lr;
        da.work = (const WorkItem *)P->work.p;
        da.mp = (const V *)mp.p;
        da.loc2 = (const V *)loc2.p;
        da.l2l = tabs + tmp.tab_l2l;
        da.m2l = tabs + tmp.tab_m2l;
        da.src = ua.src;
        da.tgt = ua.src;
        da.logc = (double *)logc.p;
        da.logd = (double *)logd.p;
        da.logself = std::log(2.0 * M_PI / (double)P->N);
        hipLaunchKernelGGL((k_down_eval<R, V, KER_LOG, SET_SORTED, EPI_LOGCD>),
                           dim3(P->nwork), dim3(BLOCK), dn_smem, st, da);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemsetAsync(flags.p, 0, 4, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_coeffs, dim3(grid_for(P->N)), dim3(256), 0, st, P->N,
                           (const double *)logc.p, (const double *)logd.p,
                           (const int32_t *)P->sm.p, (const double *)P->sth.p,
                           (const int32_t *)P->hit.p, (double *)P->chat.p,
                           (cx<double> *)P->dhat.p, (int *)flags.p);
        e = hipGetLastError();
    }
    int hflags = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&hflags, flags.p, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess)
        return fail(FN_EHIP, "inverse plan: %s", hipGetErrorString(e));
    if (hflags & FLAG_RANGE)
        return fail(FN_ERANGE, "|C_k| or |D_j| leaves the binary64 range: the "
                               "point set is too ill-conditioned for the inverse");
    return FN_OK;
}

template <typename R>
static int plan_inv_impl(fn_plan *P, const double *y, hipStream_t st)
{
    int rc = build_tree(P, P->N, y, true, true, st);
    if (rc)
        return rc;
    P->lr = std::max(2, P->l - DN_S);
    rc = build_work(P, true, true, st);
    if (rc)
        return rc;
    if (!alloc(P->chat, P->N * 8) || !alloc(P->dhat, P->N * 16) ||
        !alloc(P->wsorted, P->N * 2 * sizeof(R)))
        return fail(FN_ENOMEM, "inverse coefficient allocation failed");
    rc = plan_inv_logs(P, st);
    if (rc)
        return rc;
    rc = upload_tables<R>(P, KER_COT, P->P, P->q, st);
    if (rc)
        return rc;
    UpArgs<R, cx<R>> ua{};
    rc = setup_fmm<R, cx<R>>(P, KER_COT, P->P, P->q, P->mp, P->loc2, P->S, P->cnt,
                             ua, &P->up_grid, &P->up_smem, &P->dn_smem, st);
    if (rc)
        return rc;
    std::memcpy(P->bands_f.band_lo, ua.band_lo, sizeof ua.band_lo);
    std::memcpy(P->bands_f.band_d, ua.band_d, sizeof ua.band_d);
    std::memcpy(P->bands_f.cnt_off, ua.cnt_off, sizeof ua.cnt_off);
    P->bands_f.nbands = ua.nbands;
    HIPCHK(hipStreamSynchronize(st));
    return FN_OK;
}

template <typename R>
static int exec_inv(fn_plan *P, const void *in, void *out, hipStream_t st)
{
    using V = cx<R>;
    const R *tabs = (const R *)P->tabs.p;
    UpArgs<R, V> ua{};
    copy_bands<R>(P, ua);
    ua.N = P->N;
    ua.l = P->l;
    ua.P = P->P;
    ua.cnt = (int *)P->cnt.p;
    ua.src = {(const int32_t *)P->off.p, (const int32_t *)P->sm.p,
              (const double *)P->sth.p, (const int32_t *)P->sperm.p};
    ua.dhat = (const cx<double> *)P->dhat.p;
    ua.gin = (const cx<R> *)in;
    ua.w_out = (cx<R> *)P->wsorted.p;
    ua.mp = (V *)P->mp.p;
    ua.loc2 = (V *)P->loc2.p;
    ua.S = (V *)P->S.p;
    ua.m2m = tabs + P->tab_m2m;
    ua.bin = tabs + P->tab_bin;
    ua.reg1 = tabs + P->tab_reg1;
    ua.reg2 = tabs + P->tab_reg2;
    hipLaunchKernelGGL((k_up<R, V, KER_COT, SET_SORTED>), dim3(P->up_grid),
                       dim3(BLOCK), P->up_smem, st, ua);
    HIPCHK(hipGetLastError());
    DownArgs<R, V> da{};
    da.N = P->N;
    da.l = P->l;
    da.P = P->P;
    da.lr = P->lr;
    da.work = (const WorkItem *)P->work.p;
    da.mp = (const V *)P->mp.p;
    da.loc2 = (const V *)P->loc2.p;
    da.l2l = tabs + P->tab_l2l;
    da.m2l = tabs + P->tab_m2l;
    da.src = ua.src;
    da.w_sorted = (const cx<R> *)P->wsorted.p;
    da.out = (cx<R> *)out;
    da.S = (const V *)P->S.p;
    da.chat = (const double *)P->chat.p;
    da.hit = (const int32_t *)P->hit.p;
    da.gin = (const cx<R> *)in;
    hipLaunchKernelGGL((k_down_eval<R, V, KER_COT, SET_SORTED, EPI_INV>),
                       dim3(P->nwork), dim3(BLOCK), P->dn_smem, st, da);
    HIPCHK(hipGetLastError());
    return FN_OK;
}

// ------------------------------------------------------------------ ABI

static int check_common(int64_t N, int64_t M, double eps, int dtype)
{
    if (N < 1 || N > INT32_MAX - 1)
        return fail(FN_EINVAL, "N = %lld out of range [1, 2^31 - 2]", (long long)N);
    if (M < 1 || M > INT32_MAX - 1)
        return fail(FN_EINVAL, "M = %lld out of range [1, 2^31 - 2]", (long long)M);
    if (dtype != FN_C128 && dtype != FN_C64)
        return fail(FN_EINVAL, "unknown dtype %d", dtype);
    if (!(eps > 0.0) || !std::isfinite(eps) || eps >= 1.0)
        return fail(FN_EINVAL, "eps = %g must be finite and in (0, 1)", eps);
    if (eps < eps_floor(dtype))
        return fail(FN_EPREC, "eps = %g is below the floor %g of this precision path",
                    eps, eps_floor(dtype));
    return FN_OK;
}

static void choose(int64_t N, int64_t M, double eps, int dtype, int32_t p_in,
                   int32_t q_in, int32_t l_in, int *p, int *q, int *l)
{
    *l = l_in > 0 ? l_in : default_depth(N, M, dtype);
    int pp, qq;
    trunc_numbers(eps, *l, &pp, &qq);
    *p = p_in > 0 ? p_in : pp;
    *q = q_in > 0 ? q_in : qq;
}

static int plan_common(fn_plan **out, int kind, int64_t N, int64_t M,
                       const double *y, double eps, int dtype, int32_t p_in,
                       int32_t q_in, int32_t l_in, void *stream)
{
    if (!out)
        return fail(FN_EINVAL, "plan pointer is NULL");
    *out = nullptr;
    int rc = check_common(N, M, eps, dtype);
    if (rc)
        return rc;
    if (!y)
        return fail(FN_EINVAL, "y is NULL");
    if (l_in > 24 || p_in > 64 || q_in > 30)
        return fail(FN_EINVAL, "explicit parameters out of range (lmax <= 24, p <= 64, q <= 30)");
    fn_plan *P = new fn_plan();
    P->kind = kind;
    P->dtype = dtype;
    P->N = N;
    P->M = M;
    P->eps = eps;
    choose(N, M, eps, dtype, p_in, q_in, l_in, &P->p, &P->q, &P->l);
    P->P = round8(std::max(P->p, 2 * P->q));
    if (P->P > 64) {
        delete P;
        return fail(FN_EINVAL, "expansion length %d exceeds 64", P->P);
    }
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0)
        rc = dtype == FN_C128 ? plan_fwd_impl<double>(P, y, st)
                              : plan_fwd_impl<float>(P, y, st);
    else
        rc = dtype == FN_C128 ? plan_inv_impl<double>(P, y, st)
                              : plan_inv_impl<float>(P, y, st);
    if (rc) {
        (void)hipStreamSynchronize(st);
        release_plan(P);
        delete P;
        return rc;
    }
    *out = P;
    return FN_OK;
}

extern "C" {

int nufft_plan_fwd_ex(fn_plan **plan, int64_t N, int64_t M, const double *y,
                      double eps, int dtype, int32_t p, int32_t q, int32_t lmax,
                      void *stream)
{
    return plan_common(plan, 0, N, M, y, eps, dtype, p, q, lmax, stream);
}

int nufft_plan_inv_ex(fn_plan **plan, int64_t N, const double *y, double eps,
                      int dtype, int32_t p, int32_t q, int32_t lmax, void *stream)
{
    return plan_common(plan, 1, N, N, y, eps, dtype, p, q, lmax, stream);
}

int nufft_plan_fwd(fn_plan **plan, int64_t N, int64_t M, const double *y,
                   double eps, int dtype, void *stream)
{
    return plan_common(plan, 0, N, M, y, eps, dtype, 0, 0, 0, stream);
}

int nufft_plan_inv(fn_plan **plan, int64_t N, const double *y, double eps,
                   int dtype, void *stream)
{
    return plan_common(plan, 1, N, N, y, eps, dtype, 0, 0, 0, stream);
}

int nufft_execute(fn_plan *plan, const void *in, void *out, void *stream)
{
    if (!plan)
        return fail(FN_EINVAL, "plan is NULL");
    if (!in || !out)
        return fail(FN_EINVAL, "input or output pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (plan->kind == 0)
        return plan->dtype == FN_C128 ? exec_fwd<double>(plan, in, out, st)
                                      : exec_fwd<float>(plan, in, out, st);
    return plan->dtype == FN_C128 ? exec_inv<double>(plan, in, out, st)
                                  : exec_inv<float>(plan, in, out, st);
}

int nufft_destroy(fn_plan *plan)
{
    if (!plan)
        return FN_OK;
    hipError_t e = hipDeviceSynchronize();
    release_plan(plan);
    delete plan;
    if (e != hipSuccess)
        return fail(FN_EHIP, "hipDeviceSynchronize: %s", hipGetErrorString(e));
    return FN_OK;
}

int nufft_plan_get_info(const fn_plan *plan, fn_plan_info *info)
{
    if (!plan || !info)
        return fail(FN_EINVAL, "NULL argument");
    info->N = plan->N;
    info->M = plan->M;
    info->kind = plan->kind;
    info->dtype = plan->dtype;
    info->p = plan->p;
    info->q = plan->q;
    info->lmax = plan->l;
    info->nterms = plan->P;
    info->eps = plan->eps;
    return FN_OK;
}

int nufft_select_params(int64_t N, int64_t M, double eps, int dtype, int32_t *p,
                        int32_t *q, int32_t *lmax)
{
    int rc = check_common(N, M, eps, dtype);
    if (rc)
        return rc;
    int pp, qq, ll;
    choose(N, M, eps, dtype, 0, 0, 0, &pp, &qq, &ll);
    if (p)
        *p = pp;
    if (q)
        *q = qq;
    if (lmax)
        *lmax = ll;
    return FN_OK;
}

int nufft_fwd(int64_t N, int64_t M, const double *y, const void *f, void *g,
              double eps, int dtype, void *stream)
{
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    fn_plan *P = nullptr;
    int rc = nufft_plan_fwd(&P, N, M, y, eps, dtype, stream);
    if (rc)
        return rc;
    rc = nufft_execute(P, f, g, stream);
    int rc2 = nufft_destroy(P);
    return rc ? rc : rc2;
}

int inufft(int64_t N, const double *y, const void *g, void *f, double eps,
           int dtype, void *stream)
{
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    fn_plan *P = nullptr;
    int rc = nufft_plan_inv(&P, N, y, eps, dtype, stream);
    if (rc)
        return rc;
    rc = nufft_execute(P, g, f, stream);
    int rc2 = nufft_destroy(P);
    return rc ? rc : rc2;
}

const char *nufft_last_error(void) { return g_err.c_str(); }

} // extern "C"
