// Host side of the FMM-based NUFFT / INUFFT: parameter selection, operator
// tables, plans, launches and the C ABI declared in include/fmmnufft.h.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fmmnufft.h"
#include "fmm_kernels.h"
#include "solver_kernels.h"
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
    try { // never throws: callers may have released resources already
        g_err = buf;
    } catch (...) {
    }
    return status;
}

#define HIPCHK(expr)                                                           \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(FN_EHIP, "%s: %s (%s:%d)", #expr,                      \
                        hipGetErrorString(e_), __FILE__, __LINE__);            \
    } while (0)

// No C++ exception crosses the C ABI: every entry point's body runs inside
// FN_API_BEGIN / FN_API_END, which turn a failed host allocation into
// FN_ENOMEM and anything else into FN_EHIP.
static int fail_nothrow(int status, const char *msg) noexcept
{
    try {
        g_err = msg;
    } catch (...) {
    }
    return status;
}

#define FN_API_BEGIN try {
#define FN_API_END                                                             \
    }                                                                          \
    catch (const std::bad_alloc &)                                             \
    {                                                                          \
        return fail_nothrow(FN_ENOMEM, "host memory allocation failed");       \
    }                                                                          \
    catch (...)                                                                \
    {                                                                          \
        return fail_nothrow(FN_EHIP, "unexpected C++ exception in the library"); \
    }

// ---------------------------------------------------- caching device memory
//
// Plans are created and destroyed per one-shot call; freed blocks are kept
// per size and handed out again so that repeated calls do not pay for
// hipMalloc / hipFree.  The pool holds at most POOL_CAP bytes of free
// blocks (a block returned beyond that is freed at once), and a failed
// hipMalloc first frees every cached block and tries again, so the cache
// never starves the caller's own allocations.  nufft_release_cache frees
// the cached blocks on demand.

namespace {
std::mutex g_pool_mu;
thread_local hipError_t g_alloc_err = hipSuccess; // last failed hipMalloc
std::multimap<size_t, void *> g_pool;
size_t g_pool_bytes = 0;                           // free bytes held
constexpr size_t POOL_CAP = size_t(8) << 30;

size_t round_bytes(size_t n) { return (n + 255) & ~size_t(255); }

// Frees every cached block; returns the bytes released.  hipFree waits for
// the device, and a cached block is in no plan's use.
size_t pool_trim()
{
    std::multimap<size_t, void *> blocks;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        blocks.swap(g_pool);
        g_pool_bytes = 0;
    }
    size_t n = 0;
    for (auto &b : blocks) {
        (void)hipFree(b.second);
        n += b.first;
    }
    return n;
}

void *pool_get(size_t bytes)
{
    bytes = round_bytes(bytes ? bytes : 1);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pool.find(bytes);
        if (it != g_pool.end()) {
            void *p = it->second;
            g_pool.erase(it);
            g_pool_bytes -= bytes;
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError(); // clear it before the retry
        if (pool_trim() > 0)
            e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        g_alloc_err = e;
        return nullptr;
    }
    return p;
}

void pool_put(void *p, size_t bytes)
{
    if (!p)
        return;
    bytes = round_bytes(bytes ? bytes : 1);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (g_pool_bytes + bytes <= POOL_CAP) {
            g_pool.emplace(bytes, p);
            g_pool_bytes += bytes;
            return;
        }
    }
    (void)hipFree(p);
}

struct Buf {
    void *p = nullptr;
    size_t n = 0;
    bool arena = false; // carved from an Arena chunk (not returned alone)
};

// Bump allocation from large pooled chunks, for the many small workspaces
// of a batch of transforms; the chunks go back to the pool with the batch.
// A fixed arena (the allocation-free entry point) carves one given region
// and never grows: a request beyond it fails and sets `overflow`.
struct Arena {
    std::vector<Buf> chunks;
    size_t used = 0; // bytes used in the last chunk (or the fixed region)
    unsigned char *fixed = nullptr;
    size_t fixed_cap = 0;
    bool overflow = false;
    // operator tables built into the fixed region by this call (key, where)
    long tab_key = -1;
    void *tab_base = nullptr;
    size_t tab_off[8] = {0};
};
thread_local Arena *g_arena = nullptr;
constexpr size_t ARENA_CHUNK = size_t(64) << 20;

void *arena_get(Arena &A, size_t bytes)
{
    bytes = round_bytes(bytes ? bytes : 1);
    if (A.fixed) {
        if (bytes > A.fixed_cap - A.used) {
            A.overflow = true;
            return nullptr;
        }
        void *p = A.fixed + A.used;
        A.used += bytes;
        return p;
    }
    if (A.chunks.empty() || A.used + bytes > A.chunks.back().n) {
        Buf c;
        c.n = std::max(ARENA_CHUNK, bytes);
        c.p = pool_get(c.n);
        if (!c.p)
            return nullptr;
        A.chunks.push_back(c);
        A.used = 0;
    }
    void *p = (unsigned char *)A.chunks.back().p + A.used;
    A.used += bytes;
    return p;
}
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
// for N = M, Section 3.2), generalised to N != M through lg = log2 sqrt(N M).
static int paper_depth(int64_t N, int64_t M)
{
    const double lg = 0.5 * std::log2((double)N * (double)M);
    return std::min(24, std::max(2, (int)std::lround(lg) - 5));
}

// Depth of a plan (kind 0 forward, 1 inverse, 2 adjoint, whose sources are
// the M points and whose tree is the inverse's): lg minus a leaf offset
// measured on MI355X for one-shot transforms (binary64 and mixed agree).
// Forward: 4 below lg = 14, 5 up to lg = 17, then 6 (leaves of about 64
// targets: its near field runs on staged uniform sources and is cheap next
// to the translations).  Inverse: 4 below lg = 17, then 5 (its sorted-source
// and log near fields cost more per pair).  FN_LEAF_OFFSET overrides both.
// The mixed path also keeps at most 128 sources per leaf (defaults and
// autotuned depths alike).  Its moment and near-field sums are blocked with
// binary64 totals, so deeper leaves stay accurate too, but with few targets
// the cost model alone would pick trees of thousands of sources per leaf.
// Smallest depth that keeps at most 128 sources per leaf on the mixed path
// (2 on the binary64 path).
static int mixed_min_depth(int64_t N, int dtype)
{
    int l = 2;
    if (dtype == FN_C64)
        while (l < 24 && (N >> l) > 128)
            ++l;
    return l;
}

static int default_depth(int64_t N, int64_t M, int kind, int dtype)
{
    const double lg = 0.5 * std::log2((double)N * (double)M);
    const int r = (int)std::lround(lg);
    int off = kind == 0 ? (r < 14 ? 4 : (r < 18 ? 5 : 6)) : (r < 17 ? 4 : 5);
    if (const char *e = getenv("FN_LEAF_OFFSET"))
        off = atoi(e);
    const int l = std::min(24, std::max(2, r - off));
    return std::max(l, mixed_min_depth(kind == 2 ? M : N, dtype));
}

// Largest |log|Chat_k|| and |log|Dhat_j|| an inverse plan accepts on the
// mixed path (FN_ERANGE beyond).
static constexpr double LOG_MAX_C64 = 60.0;

static double eps_floor(int dtype) { return dtype == FN_C64 ? 1e-7 : 1e-15; }

// The precision floor eps_th of a path (Section 3.1), the accuracy that
// eps = FN_EPS_MACHINE requests.  Binary64: the maximum error for f = 1
// grows with the size through the rounding of the grid-unit reduction and
// of the sums; measured on MI355X at N = M = 2^3 ... 2^20 (uniform y, 5.6e-16
// ... 2.8e-15), it follows 1.4e-16 log2 sqrt(N M) within 25 %.  Binary32
// data: the relative l2 floor of the mixed path, 2e-7 at 2^20.
static double eps_th(int64_t N, int64_t M, int dtype)
{
    if (dtype == FN_C64)
        return 2e-7;
    const double lg = 0.5 * std::log2((double)N * (double)M);
    return 1.4e-16 * std::max(4.0, lg);
}

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

struct Tables {
    std::vector<long double> m2m, l2l, m2l4, m2l6, regR, regL, reg1, reg2;
};

// M2M (child at c_p + s r_p/2 -> parent):  a^P_n = sum_{m<=n} C(n,m) 2^-n s^(n-m) a^C_m
// L2L (parent -> child):                   b^C_m = sum_{n>=m} C(n,m) 2^-n s^(n-m) b^P_n
// Only the left child (s = -1) is stored; the right one differs by (-1)^(n-m).
// M2L cot (1/t kernel, delta = (c_t - c_s)/r):
//                    b_n = sum_m (-1)^n C(m+n, n) delta^-(m+n+1) a_m
// M2L log (log|t| kernel):
//                    b_0 = a_0 log|delta| - sum_{m>=1} (a_m/m) delta^-m
//                    b_n = a_0 (-1)^(n+1) / (n delta^n)
//                          - sum_{m>=1} (a_m/m) C(m+n-1, n) (-1)^n delta^-(m+n)
// Only delta = +4 and +6 are stored; delta < 0 follows from the sign pattern.
// Regular part at level 2 (Eq. p20 and its log analogue) in the variable
// u = (y - x_c)/(pi/4), with A_t the moments of Omega_1 (reg1) or of the
// opposite quarter (reg2) about the centre x_c in units of pi/4.
// Multipole sizes are PU, local sizes PD.
static void build_tables(int PU, int PD, int q, int kernel, Tables &T)
{
    T.m2m.assign(PU * PU, 0);
    T.regR.assign(PU * PD, 0);
    T.regL.assign(PU * PD, 0);
    T.l2l.assign(PD * PD, 0);
    T.m2l4.assign(PD * PD, 0);
    T.m2l6.assign(PD * PD, 0);
    T.reg1.assign(PU * PD, 0);
    T.reg2.assign(PU * PD, 0);
    const int NB = 2 * std::max(PU, PD) + 2;
    std::vector<long double> C(NB * NB, 0);
    for (int n = 0; n < NB; ++n) {
        C[n * NB] = 1;
        for (int k = 1; k <= n; ++k)
            C[n * NB + k] = C[(n - 1) * NB + k - 1] + (k < n ? C[(n - 1) * NB + k] : 0);
    }
    auto binom = [&](int n, int k) -> long double {
        return (k < 0 || k > n) ? 0 : C[n * NB + k];
    };
    auto shiftc = [&](int n, int m) -> long double { // C(n,m) 2^-n (-1)^(n-m)
        return binom(n, m) * ldexpl(1.0L, -n) * (((n - m) & 1) ? -1 : 1);
    };
    for (int n = 0; n < PU; ++n)
        for (int m = 0; m <= n; ++m)
            T.m2m[m * PU + n] = shiftc(n, m); // [in m][out n]
    for (int n = 0; n < PD; ++n)
        for (int m = 0; m <= n; ++m)
            T.l2l[n * PD + m] = shiftc(n, m); // [in n][out m]
    for (int di = 0; di < 2; ++di) {
        const long double d = di == 0 ? 4 : 6;
        std::vector<long double> &Mt = di == 0 ? T.m2l4 : T.m2l6;
        std::vector<long double> ip(2 * PD + 2, 1);
        for (int j = 1; j < 2 * PD + 2; ++j)
            ip[j] = ip[j - 1] / d; // d^-j
        for (int m = 0; m < PD; ++m)
            for (int n = 0; n < PD; ++n) {
                long double v;
                if (kernel == KER_COT) {
                    v = ((n & 1) ? -1 : 1) * binom(m + n, n) * ip[m + n + 1];
                } else if (m == 0 && n == 0) {
                    v = logl(d);
                } else if (n == 0) {
                    v = -ip[m] / m;
                } else if (m == 0) {
                    v = ((n & 1) ? 1 : -1) * ip[n] / n;
                } else {
                    v = -binom(m + n - 1, n) * ((n & 1) ? -1 : 1) * ip[m + n] / m;
                }
                Mt[m * PD + n] = v;
            }
    }
    const long double qpi = 0.785398163397448309615660845819875721L; // pi/4
    std::vector<long double> fac(2 * PU + 4, 1);
    for (int i = 1; i < (int)fac.size(); ++i)
        fac[i] = fac[i - 1] * i;
    for (int m = 1; m <= q; ++m) {
        const long double B = bernoulli_abs(m);
        const long double four_m = powl(4.0L, m) - 1;
        const int top = kernel == KER_COT ? 2 * m - 1 : 2 * m;
        for (int lo = 0; lo <= top; ++lo) {
            const int t = top - lo;
            if (lo >= PD || t >= PU)
                continue;
            const long double w = kernel == KER_COT ? B / m : B / (2 * m);
            const long double kap = -(powl(qpi, lo) / fac[lo]) * w *
                                    (powl(-qpi, t) / fac[t]);
            T.reg1[t * PD + lo] = kap;
            T.reg2[t * PD + lo] = kap * four_m;
        }
    }
    // the neighbours' moments about the quarter's centre: a quarter's
    // moments shifted by +-2 half-widths, (v +- 2)^t = sum_j C(t,j) (+-2)^(t-j) v^j,
    // composed with reg1 (right neighbour: +2; left: -2)
    for (int j = 0; j < PU; ++j)
        for (int lo = 0; lo < PD; ++lo) {
            long double r = 0, l = 0;
            for (int t = j; t < PU; ++t) {
                const long double c = T.reg1[t * PD + lo] * binom(t, j) * ldexpl(1.0L, t - j);
                r += c;
                l += ((t - j) & 1) ? -c : c;
            }
            T.regR[j * PD + lo] = r;
            T.regL[j * PD + lo] = l;
        }
}

// Device copies of the tables, built once per (precision, kernel, PU, PD,
// q, device) and kept for the life of the process.
struct TableSet {
    void *base = nullptr;
    size_t off[8] = {0};
};

static std::mutex g_tab_mu;
static std::map<std::tuple<int, int, int, int, int, int>, TableSet> g_tab_cache;

template <typename R>
static int get_tables(int kernel, int PU, int PD, int q, OpTables<R> *out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const auto key = std::make_tuple((int)sizeof(R), kernel, PU, PD, q, dev);
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tab_cache.find(key);
    if (it == g_tab_cache.end() && g_arena && g_arena->fixed) {
        // allocation-free call: tables not built yet by another call go
        // into the call's own region (built again by the next such call)
        Arena &A = *g_arena;
        const long fkey = (((long)sizeof(R) * 2 + kernel) * 65 + PU) * 65 * 31 + PD * 31 + q;
        if (A.tab_key == fkey) {
            const R *b = (const R *)A.tab_base;
            *out = {b + A.tab_off[0], b + A.tab_off[1], b + A.tab_off[2], b + A.tab_off[3],
                    b + A.tab_off[4], b + A.tab_off[5], b + A.tab_off[6], b + A.tab_off[7]};
            return FN_OK;
        }
        Tables T;
        build_tables(PU, PD, q, kernel, T);
        std::vector<R> h;
        size_t off[8];
        const std::vector<long double> *parts[8] = {&T.m2m, &T.l2l,  &T.m2l4, &T.m2l6,
                                                    &T.regR, &T.regL, &T.reg1, &T.reg2};
        for (int i = 0; i < 8; ++i) {
            off[i] = h.size();
            for (long double x : *parts[i])
                h.push_back((R)x);
        }
        R *b = (R *)arena_get(A, h.size() * sizeof(R));
        if (!b)
            return fail(FN_ENOMEM, "no room for the operator tables");
        HIPCHK(hipMemcpy(b, h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice));
        A.tab_key = fkey;
        A.tab_base = b;
        for (int i = 0; i < 8; ++i)
            A.tab_off[i] = off[i];
        *out = {b + off[0], b + off[1], b + off[2], b + off[3], b + off[4], b + off[5],
                b + off[6], b + off[7]};
        return FN_OK;
    }
    if (it == g_tab_cache.end()) {
        Tables T;
        build_tables(PU, PD, q, kernel, T);
        std::vector<R> h;
        TableSet ts;
        const std::vector<long double> *parts[8] = {&T.m2m, &T.l2l,  &T.m2l4, &T.m2l6,
                                                    &T.regR, &T.regL, &T.reg1, &T.reg2};
        for (int i = 0; i < 8; ++i) {
            ts.off[i] = h.size();
            for (long double x : *parts[i])
                h.push_back((R)x);
        }
        HIPCHK(hipMalloc(&ts.base, h.size() * sizeof(R)));
        HIPCHK(hipMemcpy(ts.base, h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice));
        it = g_tab_cache.emplace(key, ts).first;
    }
    const R *b = (const R *)it->second.base;
    const size_t *o = it->second.off;
    *out = {b + o[0], b + o[1], b + o[2], b + o[3], b + o[4], b + o[5], b + o[6], b + o[7]};
    return FN_OK;
}

// ------------------------------------------------------------------ plan

static constexpr int MAX_BANDS = 12;

struct Band {
    int lb, d, first, grid;
    size_t smem;
};

// Workspace and launch shapes of one FMM (cot or log kernel) on a tree.
struct FmmSetup {
    int PU = 0, PD = 0, q = 0;
    int RSu = 0, RSd = 0;          // LDS row strides (elements of R)
    Buf mp, loc2, S;
    // M2L results of every box of levels 3..l (PD per box, packed per
    // level); the leaf level becomes the leaf locals (read by the evaluation)
    Buf pre;
    int nbands = 0;
    Band band[MAX_BANDS];
    size_t m2l_smem = 0; // M2L kernel (with the level-2 regular part)
    size_t dn_smem = 0; // evaluation kernel
    size_t tr_smem = 0; // translation kernel
    int rows_buf = 0, rows_src = 0, near_bytes = 0, grp_lds = 0;
    int stage_cap = 0; // first upward band: sorted sources staged in LDS
};

struct fn_plan {
    int kind = 0, dtype = 0; // kind 0 forward, 1 inverse, 2 adjoint
    int64_t N = 0, M = 0;
    int p = 0, q = 0, l = 0;
    bool p_explicit = false;
    double eps = 0;
    int lr = 2; // subtree root level of k_down_eval
    // points sorted into the leaves (targets of the forward, sources of the
    // inverse and of the adjoint)
    Buf off, sm, sth, sperm, skey;
    Buf spt; // forward: sorted target records (instead of sm, sth, sperm, skey)
    Buf work, nwork_dev;
    int nwork = 0;  // grid of k_down_eval: the largest possible work list
    FmmSetup cot;
    // inverse
    Buf hit, chat, dhat, wsorted;
    // error flags of the setup kernels, read once at the end of the plan;
    // set to 0 by the first launch of the sort unless flags_ready (a slot
    // of a batch's flag array, cleared by the batch)
    Buf flags;
    bool flags_ready = false;
    // (measurement) events around the inverse setup's log-sum FMM passes,
    // recorded when timing is on, and their durations (ms; -1 if not taken)
    // (tev 0..3: the inverse setup's log-sum FMM; 4, 5: the sort of the plan)
    hipEvent_t tev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    float tms[4] = {-1.f, -1.f, -1.f, -1.f};
    int log_terms = 0, log_mterms = 0; // log-sum FMM expansion lengths
    // spectral plans (Eq. p1): the uniform DFT by rocFFT around the FMM
    bool spec = false;
    rocfft_plan fft = nullptr; // owned unless it came from the plan cache
    bool fft_cached = false;
    rocfft_execution_info fft_info = nullptr;
    Buf fft_work, spec_buf; // rocFFT's work buffer; the N grid values f_k
    // temporaries of the setup, released after its synchronisation
    std::vector<Buf> tmp;
    hipStream_t stream = nullptr; // stream of the last call
    std::vector<Buf *> all()
    {
        return {&off, &sm, &sth, &sperm, &skey, &spt, &work, &nwork_dev, &cot.mp, &cot.loc2,
                &cot.pre, &cot.S, &hit, &chat, &dhat, &wsorted, &flags, &fft_work, &spec_buf};
    }
};

static bool alloc(Buf &b, size_t bytes)
{
    b.n = bytes;
    b.arena = g_arena != nullptr;
    b.p = b.arena ? arena_get(*g_arena, bytes) : pool_get(bytes);
    return b.p != nullptr;
}

static void release(Buf &b)
{
    if (!b.arena)
        pool_put(b.p, b.n);
    b = Buf{};
}

static void release_tmp(fn_plan *P)
{
    for (Buf &b : P->tmp)
        release(b);
    P->tmp.clear();
}

static void drop_events(fn_plan *P)
{
    for (hipEvent_t &e : P->tev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
}

static void release_plan(fn_plan *P)
{
    for (Buf *b : P->all())
        release(*b);
    release_tmp(P);
    drop_events(P);
    if (P->fft_info)
        (void)rocfft_execution_info_destroy(P->fft_info);
    if (P->fft && !P->fft_cached)
        (void)rocfft_plan_destroy(P->fft);
    P->fft_info = nullptr;
    P->fft = nullptr;
    P->fft_cached = false;
}

// A temporary of the setup: kept until the plan's synchronisation.
static void *tmp_alloc(fn_plan *P, size_t bytes)
{
    Buf b;
    if (!alloc(b, bytes))
        return nullptr;
    P->tmp.push_back(b);
    return b.p;
}

static int round16(int x) { return std::min(64, std::max(16, (x + 15) & ~15)); }

// LDS per workgroup of the current device (cached per device).
static size_t lds_limit()
{
    static std::mutex mu;
    static std::map<int, size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 64 * 1024;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end())
        return it->second;
    int v = 0;
    size_t r = 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
        r = (size_t)v;
    cache[dev] = r;
    return r;
}

// LDS row stride: nc * P elements of size es, padded so that a row's start
// moves by 4 nc banks (of 64) from one row to the next: the matrix-core
// B-operand loads of a wavefront then hit distinct banks.
static int row_stride(int nc, int P, int es)
{
    const int w0 = nc * P * es / 4;
    const int pad_w = ((4 * nc - w0) % 64 + 64) % 64;
    return nc * P + pad_w * 4 / es;
}

static size_t down_lds(int s, int lr, int RS, int es, int *rows_buf, int *rows_src)
{
    const int nA = lr - 2;
    *rows_buf = std::max(1 << s, nA + 1);
    *rows_src = std::max((1 << s) + 6, 3 * nA);
    return (size_t)(2 * *rows_buf + *rows_src) * RS * es;
}

// Subtree root level of k_down_eval: subtrees of at most 4 levels whose
// workspace fits in LDS.
static int choose_lr(int l, int nc, int PD, int es)
{
    const size_t lim = lds_limit();
    const int RS = row_stride(nc, PD, es);
    for (int s = std::min(4, l - 2); s >= 0; --s) {
        int rb, rsrc;
        // the translation kernel also holds the PD x PD L2L table
        if (down_lds(s, l - s, RS, es, &rb, &rsrc) + (size_t)PD * PD * es <= lim)
            return l - s;
    }
    return l;
}

// Uniform sources: the number B of grid points in every leaf when all
// leaves hold the same number and 4 <= B <= 64, B a multiple of 4 (the
// matrix-core P2M, with the band's weights staged in LDS); else 0.
static int uniform_leaf_pts(const fn_plan *P)
{
    const int64_t B = P->N >> P->l;
    return ((B << P->l) == P->N && B >= 4 && B <= 64 && B % 4 == 0) ? (int)B : 0;
}

template <typename R, typename V>
static int setup_fmm(fn_plan *P, int kernel, int PU, int PD, int q, bool sorted_src,
                     FmmSetup &F, hipStream_t st)
{
    constexpr int NC = ncomp<V>::value;
    const int es = sizeof(R);
    F.PU = PU;
    F.PD = PD;
    F.q = q;
    F.RSu = row_stride(NC, PU, es);
    F.RSd = row_stride(NC, PD, es);
    const size_t lim = lds_limit();
    // bands of the upward pass: the leaves' band, then bands of at most 5
    // levels down to level 2 (the last one has 4 workgroups, one per
    // quarter).  The leaves' band spans 5 levels, except where the cot
    // kernel stages coordinates, powers and complex weights (sorted sources,
    // and a uniform grid with unequal leaves), which for 32 leaves would
    // cost occupancy: 4 there (measured at 2^20: 5 levels take 3 us off the
    // forward's pass and 7 us off the log-sums', and add 2 us to the
    // inverse's)
    // a uniform grid with unequal leaves is staged like sorted sources
    const bool uni_staged = !sorted_src && kernel == KER_COT && uniform_leaf_pts(P) == 0;
    const int d_first = (kernel == KER_COT && (sorted_src || uni_staged)) ? 4 : 5;
    const int d_rest = 5;
    F.nbands = 0;
    int lb = P->l;
    bool first = true;
    do {
        const int d = std::min(first ? d_first : d_rest, lb - 2);
        F.band[F.nbands++] = {lb, d, first ? 1 : 0, 1 << (lb - d),
                              (size_t)(1 << d) * F.RSu * es};
        lb -= d;
        first = false;
    } while (lb > 2);
    // every band: the level buffer of its bottom level, and the buffer of
    // the level above it, which in the first band holds the staged sources
    // until the P2M is done (uniform grid with an equal number B in every
    // leaf: the weights; sorted sources: coordinates and weights of up to
    // 1.25 times the mean count plus 64; a uniform grid with unequal
    // leaves: coordinates and weights of its at most ceil(N / 2^l) points
    // per leaf; else they are read in place)
    for (int b = 0; b < F.nbands; ++b) {
        const int nbot = 1 << F.band[b].d;
        size_t bytes = (size_t)std::max(nbot / 2, 1) * F.RSu * es;
        if (b == 0 && !sorted_src && kernel == KER_COT && uniform_leaf_pts(P) > 0) {
            bytes = std::max(bytes, (size_t)nbot *
                                        uni_stage_stride(uniform_leaf_pts(P), es) * es);
        } else if (b == 0 && (sorted_src || uni_staged)) {
            const int64_t nsrc = P->kind == 2 ? P->M : P->N; // the adjoint's are y
            const int64_t mean = (nsrc + (int64_t(1) << P->l) - 1) >> P->l;
            // coordinate, its fourth power, and (cot) the complex weight
            const size_t per = es * (kernel == KER_COT ? 4 : 2);
            const size_t room = lim > F.band[0].smem + 4 * (size_t)(nbot + 1) + 64
                                    ? lim - F.band[0].smem - 4 * (size_t)(nbot + 1) - 64
                                    : 0;
            const int64_t want = sorted_src ? nbot * mean + nbot * mean / 4 + 64 : nbot * mean + 4;
            int64_t cap = std::min<int64_t>(want, (int64_t)(room / per) - 4);
            cap = std::min<int64_t>(cap, 4096) & ~int64_t(3);
            F.stage_cap = cap >= 64 ? (int)cap : 0;
            // the sources (cap rounded up to 4), then the nbot + 1 leaf offsets
            if (F.stage_cap)
                bytes = std::max(bytes, (size_t)((F.stage_cap + 3) & ~3) * per +
                                            4 * (size_t)(nbot + 1));
        }
        F.band[b].smem += bytes;
    }
    for (int b = 0; b < F.nbands; ++b)
        if (F.band[b].smem > lim)
            return fail(FN_EINVAL, "expansion length %d needs %zu bytes of LDS", PU,
                        F.band[b].smem);
    const int s = P->l - P->lr;
    F.dn_smem = down_lds(s, P->lr, F.RSd, es, &F.rows_buf, &F.rows_src);
    // the translation kernel: its two level buffers and the L2L table; the
    // M2L kernel: the source rows and the output rows of its boxes
    F.tr_smem = (size_t)2 * F.rows_buf * F.RSd * es + (size_t)PD * PD * es;
    // (block 0: the four level-2 multipoles and the regular part's partial
    // sums, 4 PU + 4 BLOCK values)
    F.m2l_smem = std::max((size_t)(M2L_BOXES + 6) * F.RSd * es,
                          (4 * (size_t)PU + 4 * BLOCK) * sizeof(V));
    if (F.tr_smem > lim || F.m2l_smem > lim)
        return fail(FN_EINVAL, "expansion length %d needs %zu bytes of LDS", PD,
                    std::max(F.tr_smem, F.m2l_smem));
    // the evaluation stages its near-field sources after the leaf locals:
    // for sorted sources, room for 1.25 times the mean count of the
    // subtree's leaves and its two neighbours (16 bytes of position, plus
    // the weight for the cot kernel), within 48 KiB (four workgroups per
    // compute unit); a subtree beyond it reads its sources in place
    const size_t loc_bytes = (size_t)F.rows_buf * F.RSd * es;
    if (sorted_src) {
        const int64_t nsrc = P->kind == 2 ? P->M : P->N;
        const int64_t mean = (nsrc + (int64_t(1) << P->l) - 1) >> P->l;
        const int64_t want = (((int64_t(1) << s) + 2) * mean * 5) / 4 + 64;
        const size_t per = 16 + (kernel == KER_COT ? 2 * (size_t)es : 0);
        const size_t need = loc_bytes + (size_t)want * per + 4 * (((size_t)1 << s) + 4);
        F.dn_smem = std::max(F.dn_smem, std::min(need, std::min(lim, (size_t)48 << 10)));
    }
    F.near_bytes = (int)(F.dn_smem - loc_bytes);
    // the forward evaluation's grouping of targets by leaf, after the rest
    F.grp_lds = (int)F.dn_smem;
    if (!sorted_src && kernel == KER_COT)
        F.dn_smem += 4 * (((size_t)1 << s) + 1 + FWD_TMAX);
    const int64_t nmp = lev_off(P->l + 1, PU);
    if (!alloc(F.mp, nmp * sizeof(V)) || !alloc(F.loc2, 4 * PD * sizeof(V)) ||
        !alloc(F.S, sizeof(V)) || !alloc(F.pre, lev_off(P->l + 1, PD) * sizeof(V)))
        return fail(FN_ENOMEM, "expansion allocation failed");
    (void)kernel;
    (void)st;
    return FN_OK;
}

template <typename R, typename V>
static void fill_up(const fn_plan *P, const FmmSetup &F, const OpTables<R> &T,
                    UpArgs<R, V> &ua)
{
    ua.N = P->N;
    ua.l = P->l;
    ua.RS = F.RSu;
    ua.PD = F.PD;
    ua.leaf_pts = uniform_leaf_pts(P);
    ua.stage_cap = F.stage_cap;
    ua.src_leaf = (const int32_t *)P->skey.p;
    ua.mp = (V *)F.mp.p;
    ua.loc2 = (V *)F.loc2.p;
    ua.S = (V *)F.S.p;
    ua.T = T;
}

template <typename R, typename V>
static void fill_down(const fn_plan *P, const FmmSetup &F, const OpTables<R> &T,
                      DownArgs<R, V> &da)
{
    da.N = P->N;
    da.l = P->l;
    da.lr = P->lr;
    da.RS = F.RSd;
    da.rows_buf = F.rows_buf;
    da.rows_src = F.rows_src;
    da.near_bytes = F.near_bytes;
    da.grp_lds = F.grp_lds;
    da.work = (const WorkItem *)P->work.p;
    da.nwork = (const int32_t *)P->nwork_dev.p;
    da.mp = (const V *)F.mp.p;
    da.PU = F.PU;
    da.loc2 = (const V *)F.loc2.p;
    da.S = (const V *)F.S.p;
    da.T = T;
    da.flags = (const int *)P->flags.p;
    da.pre = (V *)F.pre.p;
    da.leaf_loc = (V *)F.pre.p + lev_off(P->l, F.PD);
}

// Launches with the expansion lengths as template arguments.
#define FN_DISPATCH16(val, NAME, ...)                                          \
    switch (val) {                                                             \
    case 16: { constexpr int NAME = 16; __VA_ARGS__; } break;                  \
    case 32: { constexpr int NAME = 32; __VA_ARGS__; } break;                  \
    case 48: { constexpr int NAME = 48; __VA_ARGS__; } break;                  \
    default: { constexpr int NAME = 64; __VA_ARGS__; } break;                  \
    }

// The upward pass: the bands (the level-2 regular part runs with the M2L
// kernel of the downward pass).  ua must be filled except for the band
// fields.
template <typename R, typename V, int KER, int SRC>
static int launch_up(const FmmSetup &F, UpArgs<R, V> ua, hipStream_t st)
{
    for (int b = 0; b < F.nbands; ++b) {
        ua.lb = F.band[b].lb;
        ua.d = F.band[b].d;
        ua.first_band = F.band[b].first;
        FN_DISPATCH16(F.PU, PU_,
                      hipLaunchKernelGGL((k_up_band<R, V, KER, SRC, PU_>),
                                         dim3(F.band[b].grid), dim3(BLOCK),
                                         F.band[b].smem, st, ua));
        HIPCHK(hipGetLastError());
    }
    return FN_OK;
}

template <typename R, typename V, int KER, int SRC, int EPI>
// The downward pass: its translations (which = 1: the M2L of every box with
// the level-2 regular part, then the subtrees' L2L), its evaluation kernel
// (which = 2), or both (which < 0).  ua: the regular part's arguments.
static int launch_down(const fn_plan *P, const FmmSetup &F, const DownArgs<R, V> &da,
                       const UpArgs<R, V> &ua, hipStream_t st, int which = -1)
{
    if (which != 2) {
        FN_DISPATCH16(F.PD, PD_,
                      hipLaunchKernelGGL((k_m2l<R, V, KER, PD_>), dim3(m2l_blocks(P->l) + 1),
                                         dim3(BLOCK), F.m2l_smem, st, da, ua));
        HIPCHK(hipGetLastError());
    }
    if (P->nwork == 0)
        return FN_OK;
    if (which != 2) {
        FN_DISPATCH16(F.PD, PD_,
                      hipLaunchKernelGGL((k_down_trans<R, V, KER, SRC, EPI, PD_>),
                                         dim3(P->nwork), dim3(BLOCK), F.tr_smem, st, da));
        HIPCHK(hipGetLastError());
    }
    if (which != 1) {
        FN_DISPATCH16(F.PD, PD_,
                      hipLaunchKernelGGL((k_down_eval<R, V, KER, SRC, EPI, PD_>),
                                         dim3(P->nwork), dim3(BLOCK), F.dn_smem, st, da));
        HIPCHK(hipGetLastError());
    }
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

// Largest leaf the inverse accepts: 16 times the mean occupancy (at least
// 512).  A jittered grid stays near the mean; denser leaves mean a point set
// far too clustered for the inverse.
static int32_t dense_max(int64_t N, int l)
{
    const int64_t mean = (N + (int64_t(1) << l) - 1) >> l;
    return (int32_t)std::min<int64_t>(INT32_MAX, std::max<int64_t>(512, 16 * mean));
}

static constexpr int SORT_LDS_BINS = 32768; // LDS histogram limit (128 KB)

// The sort of a point set by the level-(l - keyshift) box (the leaves for
// keyshift = 0): a counting sort with per-block LDS histograms when the keys
// fit in LDS, with global atomics otherwise.  It is split into its workspace
// and arguments (prepare_tree) and its launches (launch_tree), so that a
// batch of sorts can share launches.
struct TreeJob {
    SortArgs a{};
    bool lds_path = true;
    bool leaf_order = false;               // k_leaf_order after the placement
    bool rank = false;                     // ... ordering every leaf (inverse)
    OrderArgs ord{};
    int32_t *tsum = nullptr;               // tile sums of the multi-pass scan
    const WorkArgs *work = nullptr;        // work list built with the scan
};

static int prepare_tree(fn_plan *P, int64_t n, const double *y, int keyshift,
                        bool deterministic, bool want_hit, bool records, TreeJob *J)
{
    // Sorted arrays by leaf (!records): the counting sort runs on the boxes
    // of level l - ks (at most 2^ORDER_MAX_SHIFT leaves each, never below
    // the subtree roots of level lr), with a small key range and one
    // k_leaf_order workgroup per key for the leaves
    J->leaf_order = !records;
    J->rank = deterministic;
    if (!records)
        keyshift = std::max(0, std::min(P->l - P->lr, ORDER_MAX_SHIFT));
    const int nbins = 1 << (P->l - keyshift);
    J->lds_path = nbins <= SORT_LDS_BINS;
    const bool lds_path = J->lds_path;
    SortArgs &a = J->a;
    a.n = n;
    a.y = y;
    n_over_2pi(P->N, &a.c_hi, &a.c_lo);
    a.N = P->N;
    a.invN = 1.0 / (double)P->N;
    a.l = P->l;
    a.keyshift = keyshift;
    a.ymax = FN_Y_MAX;
    a.nbins = nbins;
    // histogram blocks: more of them (fuller chip) when the histograms are
    // small; the column scan takes at most 256
    a.nblk = !lds_path ? 0
             : nbins <= 4096
                 ? (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + 4095) / 4096))
                 : (int)std::max<int64_t>(1, std::min<int64_t>(128, (n + 8191) / 8192));
    a.chunk = lds_path ? (n + a.nblk - 1) / a.nblk : 0;
    // unsorted grid units and keys: only the global-atomic path stores them
    a.um = lds_path ? nullptr : (int32_t *)tmp_alloc(P, n * 4);
    a.uth = lds_path ? nullptr : (double *)tmp_alloc(P, n * 8);
    a.ukey = lds_path ? nullptr : (int32_t *)tmp_alloc(P, n * 4);
    a.H = lds_path ? (int32_t *)tmp_alloc(P, (size_t)nbins * a.nblk * 4) : nullptr;
    a.tot = (int32_t *)tmp_alloc(P, (size_t)nbins * 4);
    a.cursor = lds_path ? nullptr : (int32_t *)tmp_alloc(P, (size_t)nbins * 4);
    J->tsum = (int32_t *)tmp_alloc(P, ((nbins + SCAN_TILE - 1) / SCAN_TILE) * 4);
    // sorted points: (m, perm, th) records by key; or, by leaf, separate
    // arrays plus every point's leaf, from records by key and their offsets
    // (workspace) and a scratch copy for keys too large for LDS
    const int64_t nleaf = int64_t(1) << P->l;
    SortedPt *grec = nullptr, *gtmp = nullptr;
    int32_t *koff = nullptr;
    if (!records) {
        grec = (SortedPt *)tmp_alloc(P, n * sizeof(SortedPt));
        gtmp = (SortedPt *)tmp_alloc(P, n * sizeof(SortedPt));
        koff = (int32_t *)tmp_alloc(P, ((size_t)nbins + 1) * 4);
    }
    const bool sorted_ok =
        records ? alloc(P->spt, n * sizeof(SortedPt))
                : (grec && gtmp && koff && alloc(P->skey, n * 4) && alloc(P->sm, n * 4) &&
                   alloc(P->sth, n * 8) && alloc(P->sperm, n * 4));
    if ((!lds_path && (!a.um || !a.uth || !a.ukey || !a.cursor)) || (lds_path && !a.H) ||
        !a.tot || !J->tsum || !sorted_ok ||
        !alloc(P->off, ((size_t)(records ? nbins : nleaf) + 1) * 4) ||
        (want_hit && !alloc(P->hit, P->N * 4)))
        return fail(FN_ENOMEM, "workspace allocation failed (%lld points)", (long long)n);
    if ((nbins + SCAN_TILE - 1) / SCAN_TILE > 4096)
        return fail(FN_EINVAL, "tree too large for the scan (%d leaves)", nbins);
    a.off = records ? (int32_t *)P->off.p : koff;
    a.sm = nullptr;
    a.sth = nullptr;
    a.sperm = nullptr;
    a.skey = nullptr;
    a.spt = records ? (SortedPt *)P->spt.p : grec;
    a.hit = want_hit ? (int32_t *)P->hit.p : nullptr;
    a.flags = (int *)P->flags.p;
    if (!records) {
        OrderArgs &o = J->ord;
        o.nkey = nbins;
        o.ks = keyshift;
        o.l = P->l;
        o.N = P->N;
        o.invN = 1.0 / (double)P->N;
        o.rec = grec;
        o.tmp = gtmp;
        o.koff = koff;
        o.off = (int32_t *)P->off.p;
        o.dense_max = deterministic ? dense_max(P->N, P->l) : INT32_MAX;
        o.sm = (int32_t *)P->sm.p;
        o.sth = (double *)P->sth.p;
        o.sperm = (int32_t *)P->sperm.p;
        o.skey = (int32_t *)P->skey.p;
        o.flags = (int *)P->flags.p;
    }
    return FN_OK;
}

// Enqueues the sort of one point set; errors land in P->flags.
static int launch_tree(fn_plan *P, const TreeJob &J, hipStream_t st)
{
    const SortArgs &a = J.a;
    const int nbins = a.nbins;
    // the flags cleared and the hit table filled before the first kernel
    // that writes them (k_place, k_reduce): by k_hist, else by one launch
    // (either is cheaper on the host than a memset each)
    const bool need_init = a.hit || !P->flags_ready;
    if (need_init && !J.lds_path) {
        const int64_t nhit = a.hit ? P->N : 0;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nhit + 255) / 256));
        hipLaunchKernelGGL(k_init, dim3(grid), dim3(256), 0, st,
                           P->flags_ready ? nullptr : (int *)P->flags.p, 1, a.hit, nhit);
        HIPCHK(hipGetLastError());
    }
    if (J.lds_path) {
        // grid units and keys are computed inside the histogram and
        // placement passes
        SortArgs ha = a;
        ha.init_flags = P->flags_ready ? 0 : 1;
        ha.nhit = a.hit ? P->N : 0;
        hipLaunchKernelGGL(k_hist, dim3(a.nblk), dim3(SORT_THREADS), (size_t)nbins * 4, st, ha);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_colscan, dim3((nbins + CS_COLS - 1) / CS_COLS), dim3(CS_THREADS),
                           0, st, a);
    } else {
        HIPCHK(hipMemsetAsync(a.tot, 0, (size_t)nbins * 4, st));
        hipLaunchKernelGGL(k_reduce, dim3(grid_for(a.n)), dim3(256), 0, st, a.n, a.y,
                           a.c_hi, a.c_lo, a.N, a.l, a.keyshift, a.ymax, a.um, a.uth,
                           a.ukey, a.tot, a.hit, a.flags);
    }
    HIPCHK(hipGetLastError());
    // off = exclusive scan of the key totals; cursor copy for the atomic path
    if (nbins <= SCAN1_MAX && J.work) {
        // the work list comes out of the same launch
        hipLaunchKernelGGL(k_scan_work, dim3(1), dim3(1024), SCAN1_SMEM + 4096, st,
                           (const int32_t *)a.tot, nbins, a.off, a.cursor, *J.work);
        HIPCHK(hipGetLastError());
    } else if (nbins <= SCAN1_MAX) {
        hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(1024), SCAN1_SMEM, st,
                           (const int32_t *)a.tot, nbins, a.off, a.cursor);
        HIPCHK(hipGetLastError());
    } else {
        const int nt = (int)((nbins + SCAN_TILE - 1) / SCAN_TILE);
        hipLaunchKernelGGL(k_scan_sums, dim3(nt), dim3(256), 0, st, (const int32_t *)a.tot,
                           (int64_t)nbins, J.tsum);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, J.tsum, nt, a.off + nbins);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(256), 0, st, (const int32_t *)a.tot,
                           (int64_t)nbins, (const int32_t *)J.tsum, a.off, a.cursor);
        HIPCHK(hipGetLastError());
        if (J.work) {
            hipLaunchKernelGGL(k_work, dim3(1), dim3(1024), 0, st, *J.work);
            HIPCHK(hipGetLastError());
        }
    }
    P->flags_ready = true;
    if (J.lds_path && a.spt && !a.skey && nbins <= 4 * SORT_THREADS &&
        a.chunk <= PLACE_REC_MAX) {
        // records staged in LDS in their destination order, then written
        const size_t smem = (size_t)PLACE_REC_MAX * (sizeof(SortedPt) + 4) +
                            (3 * (size_t)nbins + 32) * 4;
        hipLaunchKernelGGL(k_place_rec, dim3(a.nblk), dim3(SORT_THREADS), smem, st, a);
    } else if (J.lds_path) {
        hipLaunchKernelGGL(k_place, dim3(a.nblk), dim3(SORT_THREADS), (size_t)nbins * 4, st, a);
    } else {
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(a.n)), dim3(256), 0, st, a.n,
                           (const int32_t *)a.um, (const double *)a.uth,
                           (const int32_t *)a.ukey, a.cursor, a.sm, a.sth, a.sperm, a.skey,
                           a.spt);
    }
    HIPCHK(hipGetLastError());
    if (J.leaf_order) {
        if (J.rank)
            hipLaunchKernelGGL(k_leaf_order<true>, dim3((unsigned)J.ord.nkey),
                               dim3(ORDER_THREADS), 0, st, J.ord);
        else
            hipLaunchKernelGGL(k_leaf_order<false>, dim3((unsigned)J.ord.nkey),
                               dim3(ORDER_THREADS), 0, st, J.ord);
        HIPCHK(hipGetLastError());
    }
    return FN_OK;
}

// Sort of the points into the leaves, ranked inside each leaf by position
// (inverse; keyshift must be 0) when `deterministic`; otherwise the order
// inside a key is arbitrary (forward).  Fills the hit map when asked.
// Enqueues only; errors land in P->flags.
// With w (from prepare_work), the work list of the downward pass is built
// right after the scan of the sort.
// Measurement switch (nufft_set_timing): plans created while it is on record
// events around their sort and the inverse setup's log-sum FMM passes.
static std::atomic<int> g_timing{0};

static int build_tree(fn_plan *P, int64_t n, const double *y, int keyshift,
                      bool deterministic, bool want_hit, bool records, hipStream_t st,
                      WorkArgs *w = nullptr)
{
    TreeJob J;
    int rc = prepare_tree(P, n, y, keyshift, deterministic, want_hit, records, &J);
    if (rc)
        return rc;
    if (w) {
        // the work list reads the offsets of the sort's keys (level
        // l - keyshift, at or below the subtree roots)
        w->off = (const int32_t *)J.a.off;
        w->sh = P->l - J.a.keyshift - P->lr;
        J.work = w;
    }
    const bool timed = g_timing.load() != 0;
    if (timed) {
        for (int i = 4; i < 6; ++i)
            if (!P->tev[i] && hipEventCreate(&P->tev[i]) != hipSuccess) {
                P->tev[i] = nullptr;
                return fail(FN_EHIP, "event creation failed");
            }
        HIPCHK(hipEventRecord(P->tev[4], st));
    }
    rc = launch_tree(P, J, st);
    if (!rc && timed)
        HIPCHK(hipEventRecord(P->tev[5], st));
    return rc;
}

// Work list of k_down_eval, built on the device: subtree roots of level lr;
// P->off indexes the sorted points at level lr + sh.  The grid is sized for
// the largest possible list.
static int prepare_work(fn_plan *P, int sh, bool uniform, int64_t npts, WorkArgs *w)
{
    const int32_t tmax = FWD_TMAX;
    const int64_t nroot = int64_t(1) << P->lr;
    const int64_t maxitems = uniform ? nroot : nroot + npts / tmax + 1;
    if (maxitems > INT32_MAX)
        return fail(FN_EINVAL, "work list too long");
    P->nwork = (int)maxitems;
    if (!alloc(P->work, maxitems * sizeof(WorkItem)) || !alloc(P->nwork_dev, 4))
        return fail(FN_ENOMEM, "work list allocation failed");
    *w = {nroot, sh, (const int32_t *)P->off.p, uniform ? 1 : 0, P->N, P->lr, tmax,
          (WorkItem *)P->work.p, (int32_t *)P->nwork_dev.p};
    return FN_OK;
}

// The one synchronisation of a plan: waits for the setup, reads the error
// flags and releases the temporaries.
// Pinned host memory per host thread for the flag read-backs (a copy into
// pageable memory takes a much slower, staged path): at least `bytes`,
// grown on demand and held until the process ends; nullptr if it cannot be
// had (the read-back then goes to pageable memory).
// Slot 0 serves the flag read-backs, slot 1 the I/O tables of one-shot
// batches (each call synchronises before it returns, so the next call on
// the thread may reuse the memory).
static void *pinned_scratch(size_t bytes, int slot = 0)
{
    if (g_arena && g_arena->fixed)
        return nullptr; // allocation-free call: pageable read-back

    static thread_local void *buf[2] = {nullptr, nullptr};
    static thread_local size_t cap[2] = {0, 0};
    if (bytes > cap[slot]) {
        if (buf[slot])
            (void)hipHostFree(buf[slot]);
        buf[slot] = nullptr;
        cap[slot] = 0;
        const size_t want = std::max<size_t>(bytes, 256);
        if (hipHostMalloc(&buf[slot], want, hipHostMallocPortable) != hipSuccess) {
            buf[slot] = nullptr;
            return nullptr;
        }
        cap[slot] = want;
    }
    return buf[slot];
}

// Fine-grained (coherent) pinned host words per host thread that a kernel
// writes the error flags into, with their device address; allocated once
// and held until the process ends.  nullptr if they cannot be had (the
// flags are then copied).
static int *flag_mirror(int **dev)
{
    if (g_arena && g_arena->fixed)
        return nullptr; // allocation-free call
    static thread_local int *host = nullptr, *devp = nullptr;
    static thread_local bool tried = false;
    if (!tried) {
        tried = true;
        void *h = nullptr, *d = nullptr;
        if (hipHostMalloc(&h, 256, hipHostMallocCoherent | hipHostMallocPortable |
                                       hipHostMallocMapped) == hipSuccess) {
            if (hipHostGetDevicePointer(&d, h, 0) == hipSuccess) {
                host = (int *)h;
                devp = (int *)d;
            } else {
                (void)hipHostFree(h);
            }
        }
    }
    *dev = devp;
    return host;
}

static int finish_plan(fn_plan *P, hipStream_t st)
{
    int hstack = 0;
    int *dmirror = nullptr;
    int *hw = flag_mirror(&dmirror);
    hipError_t e;
    if (hw) {
        *hw = -1; // overwritten by the kernel
        hipLaunchKernelGGL(k_flags_out, dim3(1), dim3(64), 0, st, (const int *)P->flags.p, 1,
                           dmirror);
        e = hipGetLastError();
    } else {
        hw = (int *)pinned_scratch(4);
        if (!hw)
            hw = &hstack;
        e = hipMemcpyAsync(hw, P->flags.p, 4, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    const int hflags = *(volatile int *)hw;
    if (e == hipSuccess && P->tev[0]) {
        for (int i = 0; i < 3; ++i)
            if (hipEventElapsedTime(&P->tms[i], P->tev[i], P->tev[i + 1]) != hipSuccess)
                P->tms[i] = -1.f;
    }
    if (e == hipSuccess && P->tev[4] &&
        hipEventElapsedTime(&P->tms[3], P->tev[4], P->tev[5]) != hipSuccess)
        P->tms[3] = -1.f;
    drop_events(P);
    release_tmp(P);
    if (e != hipSuccess)
        return fail(FN_EHIP, "plan setup: %s", hipGetErrorString(e));
    if (hflags & FLAG_BAD_Y)
        return fail(FN_EINVAL, "y holds a non-finite value or |y| > %g", FN_Y_MAX);
    if (hflags & FLAG_DUP)
        return fail(FN_ESINGULAR, "two points y_j coincide on the circle");
    if (hflags & FLAG_DENSE)
        return fail(FN_ERANGE, "a leaf holds more than %d points: the point set is "
                               "too clustered for the inverse", dense_max(P->N, P->l));
    if (hflags & FLAG_RANGE)
        return fail(FN_ERANGE, "|C_k| or |D_j| leaves the range of %s: the point set "
                               "is too ill-conditioned for the inverse%s",
                    P->dtype == FN_C64 ? "the mixed path (exp(+-60))" : "binary64",
                    P->dtype == FN_C64 ? " on this path (FN_C128 has exp(+-700))" : "");
    return FN_OK;
}

// Expansion lengths of the cot FMM for (p, q).
// Terms of the translations for a relative l2 target eps.  Eq. (18.2)
// carries a factor 2^lmax from Eq. (17), a bound on the maximum error summed
// over all leaves for unit sources; the relative l2 error does not add up
// over leaves, and 3^-p per box pair decides it.  Calibrated on the oracle
// at N = M = 2^20 (binary64: 32 terms reach the rounding floor at 1e-12,
// 16 terms give 8.7e-11; binary32: 16 terms reach its 1.8e-7 floor).
static int p_calibrated(double eps)
{
    const double x = 10.0 / (3.0 * M_PI * eps);
    return (int)std::ceil(std::log(x) / std::log(3.0)) + 3;
}

// Expansion lengths of the cot FMM: locals and translations PD, multipoles
// PU >= 2q (the level-2 moments of the regular part).
static void cot_lengths(const fn_plan *P, int *PU, int *PD)
{
    const int p = P->p_explicit ? P->p : std::min(P->p, p_calibrated(P->eps));
    *PD = round16(p);
    *PU = round16(std::max(*PD, 2 * P->q));
}

// --------------------------------------------------------- forward plan

template <typename R>
static int plan_fwd_impl(fn_plan *P, const double *y, hipStream_t st)
{
    int PU, PD;
    cot_lengths(P, &PU, &PD);
    P->lr = choose_lr(P->l, 2, PD, sizeof(R));
    // targets grouped by leaf: the lanes of a wavefront then share the
    // leaf locals and near-field sources they read
    // every workspace is allocated before the first launch (the sort); the
    // targets are sorted by subtree (the evaluation groups each work item's
    // targets by leaf in LDS)
    WorkArgs w;
    int rc = prepare_work(P, 0, false, P->M, &w);
    if (rc)
        return rc;
    rc = setup_fmm<R, cx<R>>(P, KER_COT, PU, PD, P->q, false, P->cot, st);
    if (rc)
        return rc;
    OpTables<R> T;
    rc = get_tables<R>(KER_COT, PU, PD, P->q, &T);
    if (rc)
        return rc;
    return build_tree(P, P->M, y, P->l - P->lr, false, false, true, st, &w);
}

template <typename R>
static int exec_fwd(fn_plan *P, const void *in, void *out, int phase,
                    hipStream_t st)
{
    using V = cx<R>;
    const FmmSetup &F = P->cot;
    OpTables<R> T;
    int rc = get_tables<R>(KER_COT, F.PU, F.PD, F.q, &T);
    if (rc)
        return rc;
    UpArgs<R, V> ua{};
    fill_up(P, F, T, ua);
    ua.f_uniform = (const cx<R> *)in;
    if (phase <= 0) {
        rc = launch_up<R, V, KER_COT, SET_UNIFORM>(F, ua, st);
        if (rc)
            return rc;
    }
    if (phase == 0)
        return FN_OK;
    DownArgs<R, V> da{};
    fill_down(P, F, T, da);
    da.f_uniform = (const cx<R> *)in;
    da.tgt_pt = (const SortedPt *)P->spt.p;
    da.out = (cx<R> *)out;
    da.f_hit = (const cx<R> *)in;
    return launch_down<R, V, KER_COT, SET_UNIFORM, EPI_FWD>(P, F, da, ua, st, phase);
}

// --------------------------------------------------------- inverse plan

// Event timing of the inverse setup's log-sum FMM (measurement only; off
// unless nufft_set_timing turns it on).

// The log-kernel FMM of the plan: log|Chat_k| at the uniform points and
// log|Dhat_j| at the sorted sources, and from them (in the evaluation's
// epilogue) Chat and Dhat (Eq. p8).  Enqueues only.
static int plan_inv_logs(fn_plan *P, hipStream_t st)
{
    using R = double;
    using V = double;
    // the log-sums are absolute errors of log|C|, log|D|, i.e. relative
    // errors of f, so they get a tenth of eps
    const double eps_log = std::max(P->eps * 0.1, 1e-15);
    int plog, qlog;
    trunc_numbers(eps_log, P->l, &plog, &qlog);
    const int PD = round16(std::min(plog, p_calibrated(eps_log)));
    const int PU = round16(std::max(PD, 2 * qlog + 1));
    OpTables<R> T;
    int rc = get_tables<R>(KER_LOG, PU, PD, qlog, &T);
    if (rc)
        return rc;
    FmmSetup F;
    rc = setup_fmm<R, V>(P, KER_LOG, PU, PD, qlog, true, F, st);
    // the log FMM's workspace lives until the plan's synchronisation
    for (Buf *b : {&F.mp, &F.loc2, &F.S, &F.pre})
        if (b->p)
            P->tmp.push_back(*b);
    if (rc)
        return rc;
    const SortedSet src = {(const int32_t *)P->off.p, (const int32_t *)P->sm.p,
                           (const double *)P->sth.p, (const int32_t *)P->sperm.p};
    UpArgs<R, V> ua{};
    fill_up(P, F, T, ua);
    ua.src = src;
    ua.leaf_pts = 0;
    ua.logc1 = std::log(2.0 * M_PI / (double)P->N);
    ua.logc2 = std::log(2.0);
    P->log_terms = PD;
    P->log_mterms = PU;
    const bool timed = g_timing.load() != 0;
    if (timed)
        for (int i = 0; i < 4; ++i)
            if (hipEventCreate(&P->tev[i]) != hipSuccess) {
                drop_events(P);
                return fail(FN_EHIP, "event creation failed");
            }
    if (timed)
        HIPCHK(hipEventRecord(P->tev[0], st));
    rc = launch_up<R, V, KER_LOG, SET_SORTED>(F, ua, st);
    if (rc)
        return rc;
    if (timed)
        HIPCHK(hipEventRecord(P->tev[1], st));
    DownArgs<R, V> da{};
    fill_down(P, F, T, da);
    da.src = src;
    da.tgt = src;
    da.tgt_leaf = (const int32_t *)P->skey.p;
    da.hit = (const int32_t *)P->hit.p;
    da.chat_out = (double *)P->chat.p;
    da.dhat_out = (cx<double> *)P->dhat.p;
    da.flags_out = (int *)P->flags.p;
    da.logself = std::log(2.0 * M_PI / (double)P->N);
    // binary64 holds exp(+-700); the mixed path stores w_j = Dhat_j g_j in
    // binary32 (about exp(+-87)), which leaves |g_j| a range of exp(+-27)
    da.log_max = P->dtype == FN_C64 ? LOG_MAX_C64 : 700.0;
    // the evaluation's epilogue forms Chat and Dhat
    rc = launch_down<R, V, KER_LOG, SET_SORTED, EPI_LOGCD>(P, F, da, ua, st, 1);
    if (rc)
        return rc;
    if (timed)
        HIPCHK(hipEventRecord(P->tev[2], st));
    rc = launch_down<R, V, KER_LOG, SET_SORTED, EPI_LOGCD>(P, F, da, ua, st, 2);
    if (rc)
        return rc;
    if (timed)
        HIPCHK(hipEventRecord(P->tev[3], st));
    return FN_OK;
}

template <typename R>
static int plan_inv_impl(fn_plan *P, const double *y, hipStream_t st)
{
    int PU, PD;
    cot_lengths(P, &PU, &PD);
    // one subtree level serves the log FMM (binary64, real, at most 64
    // terms) and the cot FMM
    P->lr = std::max(choose_lr(P->l, 2, PD, sizeof(R)), choose_lr(P->l, 1, 64, 8));
    WorkArgs w;
    int rc = prepare_work(P, P->l - P->lr, true, P->N, &w);
    if (rc)
        return rc;
    rc = build_tree(P, P->N, y, 0, true, true, false, st, &w);
    if (rc)
        return rc;
    if (!alloc(P->chat, P->N * 8) || !alloc(P->dhat, P->N * 16) ||
        !alloc(P->wsorted, P->N * 2 * sizeof(R)))
        return fail(FN_ENOMEM, "inverse coefficient allocation failed");
    rc = plan_inv_logs(P, st);
    if (rc)
        return rc;
    rc = setup_fmm<R, cx<R>>(P, KER_COT, PU, PD, P->q, true, P->cot, st);
    if (rc)
        return rc;
    OpTables<R> T;
    rc = get_tables<R>(KER_COT, PU, PD, P->q, &T);
    if (rc)
        return rc;
    return FN_OK;
}

template <typename R>
static int exec_inv(fn_plan *P, const void *in, void *out, int phase,
                    hipStream_t st)
{
    using V = cx<R>;
    const FmmSetup &F = P->cot;
    OpTables<R> T;
    int rc = get_tables<R>(KER_COT, F.PU, F.PD, F.q, &T);
    if (rc)
        return rc;
    const SortedSet src = {(const int32_t *)P->off.p, (const int32_t *)P->sm.p,
                           (const double *)P->sth.p, (const int32_t *)P->sperm.p};
    UpArgs<R, V> ua{};
    fill_up(P, F, T, ua);
    ua.src = src;
    ua.leaf_pts = 0;
    ua.w_sorted = (const cx<R> *)P->wsorted.p;
    if (phase <= 0) {
        hipLaunchKernelGGL((k_weights<R>), dim3(grid_for(P->N)), dim3(256), 0, st, P->N,
                           (const cx<double> *)P->dhat.p, (const int32_t *)P->sperm.p,
                           (const cx<R> *)in, (cx<R> *)P->wsorted.p);
        HIPCHK(hipGetLastError());
        rc = launch_up<R, V, KER_COT, SET_SORTED>(F, ua, st);
        if (rc)
            return rc;
    }
    if (phase == 0)
        return FN_OK;
    DownArgs<R, V> da{};
    fill_down(P, F, T, da);
    da.src = src;
    da.w_sorted = (const cx<R> *)P->wsorted.p;
    da.out = (cx<R> *)out;
    da.chat = (const double *)P->chat.p;
    da.hit = (const int32_t *)P->hit.p;
    da.gin = (const cx<R> *)in;
    return launch_down<R, V, KER_COT, SET_SORTED, EPI_INV>(P, F, da, ua, st, phase);
}

// --------------------------------------------------------- adjoint plan
//
// f_k = sum_j conj(K_jk) g_j (k = 0..N-1, j = 0..M-1), the adjoint of
// Eq. (p2).  conj(K_jk) = conj(F_j) G(x_k - y_j), since conj(G(t)) = G(-t):
// the cot FMM of the inverse (Section 2, roles of x and y swapped) with
// weights conj(F_j) g_j and no C_k factor, f_k = -(W + i h_k) / 2.  The M
// points are sorted into the leaves like the inverse's sources, without the
// inverse's ranking (no signs are needed, and coincident points are
// allowed).

template <typename R>
static int plan_adj_impl(fn_plan *P, const double *y, hipStream_t st)
{
    int PU, PD;
    cot_lengths(P, &PU, &PD);
    P->lr = choose_lr(P->l, 2, PD, sizeof(R));
    // every workspace is allocated before the first launch (the sort)
    WorkArgs w;
    int rc = prepare_work(P, P->l - P->lr, true, P->N, &w);
    if (rc)
        return rc;
    rc = setup_fmm<R, cx<R>>(P, KER_COT, PU, PD, P->q, true, P->cot, st);
    if (rc)
        return rc;
    if (!alloc(P->wsorted, P->M * 2 * sizeof(R)))
        return fail(FN_ENOMEM, "adjoint weight allocation failed");
    OpTables<R> T;
    rc = get_tables<R>(KER_COT, PU, PD, P->q, &T);
    if (rc)
        return rc;
    return build_tree(P, P->M, y, 0, false, false, false, st, &w);
}

template <typename R>
static int exec_adj(fn_plan *P, const void *in, void *out, int phase, hipStream_t st)
{
    using V = cx<R>;
    const FmmSetup &F = P->cot;
    OpTables<R> T;
    int rc = get_tables<R>(KER_COT, F.PU, F.PD, F.q, &T);
    if (rc)
        return rc;
    const SortedSet src = {(const int32_t *)P->off.p, (const int32_t *)P->sm.p,
                           (const double *)P->sth.p, (const int32_t *)P->sperm.p};
    UpArgs<R, V> ua{};
    fill_up(P, F, T, ua);
    ua.src = src;
    ua.leaf_pts = 0;
    ua.w_sorted = (const cx<R> *)P->wsorted.p;
    if (phase <= 0) {
        hipLaunchKernelGGL((k_adj_weights<R>), dim3(grid_for(P->M)), dim3(256), 0, st, P->M,
                           P->N, (const double *)P->sth.p, (const int32_t *)P->sperm.p,
                           (const cx<R> *)in, (cx<R> *)P->wsorted.p);
        HIPCHK(hipGetLastError());
        rc = launch_up<R, V, KER_COT, SET_SORTED>(F, ua, st);
        if (rc)
            return rc;
    }
    if (phase == 0)
        return FN_OK;
    DownArgs<R, V> da{};
    fill_down(P, F, T, da);
    da.src = src;
    da.w_sorted = (const cx<R> *)P->wsorted.p;
    da.out = (cx<R> *)out;
    rc = launch_down<R, V, KER_COT, SET_SORTED, EPI_ADJ>(P, F, da, ua, st, phase);
    if (rc || phase == 1)
        return rc;
    hipLaunchKernelGGL((k_adj_hits<R>), dim3(grid_for(P->M)), dim3(256), 0, st, P->M,
                       (const int32_t *)P->sm.p, (const double *)P->sth.p,
                       (const int32_t *)P->sperm.p, (const cx<R> *)in, (cx<R> *)out);
    HIPCHK(hipGetLastError());
    return FN_OK;
}

// ------------------------------------------------------- spectral plans
//
// Eq. (p1): f(x) = sum_{n<N} c_n e^{inx}.  The spectral forward evaluates
// g_j = f(y_j) from the coefficients: f_k = sum_n c_n e^{2 pi i n k / N} on
// the grid (rocFFT's unscaled backward DFT), then g = K f.  The spectral
// inverse (M = N) returns the coefficients of the interpolant through the
// g_j: f = L g, then c_n = (1/N) sum_k f_k e^{-2 pi i n k / N} (rocFFT's
// forward DFT with the scale 1/N).  The uniform DFT is a library step: the
// paper puts it beside the FMM, which is the part it accelerates.

static std::once_flag g_fft_once;
static rocfft_status g_fft_setup = rocfft_status_success;

#define FFTCHK(expr)                                                           \
    do {                                                                       \
        const rocfft_status e_ = (expr);                                       \
        if (e_ != rocfft_status_success)                                       \
            return fail(FN_EHIP, "%s: rocFFT status %d", #expr, (int)e_);      \
    } while (0)

// rocFFT plans by (device, N, dtype, direction), created once and shared by
// every spectral plan and one-shot call (creating one takes milliseconds;
// each user keeps its own execution info and work buffer, so shared plans
// may run at once on different streams).  At most FFT_CACHE_MAX are kept;
// beyond that a spectral plan owns its rocFFT plan.
static std::mutex g_fft_mu;
static std::map<std::tuple<int, int64_t, int, int>, rocfft_plan> g_fft_cache;
static constexpr size_t FFT_CACHE_MAX = 64;

static rocfft_status create_fft(int64_t N, int dtype, int kind, rocfft_plan *out)
{
    const size_t len = (size_t)N;
    const rocfft_precision prec =
        dtype == FN_C128 ? rocfft_precision_double : rocfft_precision_single;
    if (kind == 0) // c -> f in place in spec_buf, unscaled e^{+2 pi i n k / N}
        return rocfft_plan_create(out, rocfft_placement_inplace,
                                  rocfft_transform_type_complex_inverse, prec, 1, &len, 1,
                                  nullptr);
    // f (spec_buf) -> c, e^{-2 pi i n k / N} / N
    rocfft_plan_description d = nullptr;
    rocfft_status e = rocfft_plan_description_create(&d);
    if (e != rocfft_status_success)
        return e;
    e = rocfft_plan_description_set_scale_factor(d, 1.0 / (double)N);
    if (e == rocfft_status_success)
        e = rocfft_plan_create(out, rocfft_placement_notinplace,
                               rocfft_transform_type_complex_forward, prec, 1, &len, 1, d);
    (void)rocfft_plan_description_destroy(d);
    return e;
}

// rocFFT plan of a spectral plan; the work buffer and the grid values are
// allocated with the plan's workspace.
static int setup_spec(fn_plan *P)
{
    std::call_once(g_fft_once, [] { g_fft_setup = rocfft_setup(); });
    FFTCHK(g_fft_setup);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, P->N, P->dtype, P->kind == 0 ? 0 : 1);
    {
        std::lock_guard<std::mutex> lk(g_fft_mu);
        auto it = g_fft_cache.find(key);
        if (it != g_fft_cache.end()) {
            P->fft = it->second;
            P->fft_cached = true;
        } else {
            FFTCHK(create_fft(P->N, P->dtype, P->kind, &P->fft));
            if (g_fft_cache.size() < FFT_CACHE_MAX) {
                g_fft_cache[key] = P->fft;
                P->fft_cached = true;
            }
        }
    }
    size_t wbytes = 0;
    FFTCHK(rocfft_plan_get_work_buffer_size(P->fft, &wbytes));
    FFTCHK(rocfft_execution_info_create(&P->fft_info));
    const size_t es = P->dtype == FN_C128 ? 16 : 8;
    if (!alloc(P->spec_buf, (size_t)P->N * es) || (wbytes && !alloc(P->fft_work, wbytes)))
        return fail(FN_ENOMEM, "spectral workspace allocation failed");
    if (wbytes)
        FFTCHK(rocfft_execution_info_set_work_buffer(P->fft_info, P->fft_work.p, wbytes));
    P->spec = true;
    return FN_OK;
}

static int run_fft(fn_plan *P, void *in, void *out, hipStream_t st)
{
    FFTCHK(rocfft_execution_info_set_stream(P->fft_info, st));
    void *ib[1] = {in}, *ob[1] = {out};
    FFTCHK(rocfft_execute(P->fft, ib, out ? ob : nullptr, P->fft_info));
    return FN_OK;
}

// ------------------------------------------------------ least squares
//
// f = argmin ||K f - g||_2 for M points and any M (the square inverse of
// Eq. p6 needs M = N and a well-conditioned point set): conjugate gradients
// on the normal equations K^H K f = K^H g (CGNR), each iteration one forward
// and one adjoint transform, the norms summed in binary64 on the device and
// read back once per iteration.

static int execute(fn_plan *plan, const void *in, void *out, int phase, void *stream);

struct Lsq {
    Buf r, s, p, q, part;
    double *hpart = nullptr; // pinned read-back of the partial sums
};

template <typename R>
static int lsq_sqnorm(const void *x, int64_t n, Lsq &L, hipStream_t st, double *out)
{
    hipLaunchKernelGGL((k_sqnorm<R>), dim3(SOLVE_BLOCKS), dim3(256), 0, st, n,
                       (const cx<R> *)x, (double *)L.part.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(L.hpart, L.part.p, SOLVE_BLOCKS * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double sum = 0.0;
    for (int b = 0; b < SOLVE_BLOCKS; ++b)
        sum += L.hpart[b];
    *out = sum;
    return FN_OK;
}

template <typename R>
static int lsq_run(fn_plan *Pf, fn_plan *Pa, const void *g, void *f, double tol,
                   int32_t maxiter, Lsq &L, hipStream_t st, int32_t *iters, double *resid)
{
    const int64_t N = Pf->N, M = Pf->M;
    const size_t es = sizeof(cx<R>);
    // f = 0, r = g, s = K^H r, p = s
    HIPCHK(hipMemsetAsync(f, 0, (size_t)N * es, st));
    HIPCHK(hipMemcpyAsync(L.r.p, g, (size_t)M * es, hipMemcpyDeviceToDevice, st));
    int rc = execute(Pa, L.r.p, L.s.p, -1, st);
    if (rc)
        return rc;
    HIPCHK(hipMemcpyAsync(L.p.p, L.s.p, (size_t)N * es, hipMemcpyDeviceToDevice, st));
    double gamma = 0.0, gamma0 = 0.0;
    rc = lsq_sqnorm<R>(L.s.p, N, L, st, &gamma);
    if (rc)
        return rc;
    gamma0 = gamma;
    int32_t k = 0;
    double res = gamma0 > 0.0 ? 1.0 : 0.0;
    const int gN = grid_for(N), gM = grid_for(M);
    while (k < maxiter && res > tol) {
        rc = execute(Pf, L.p.p, L.q.p, -1, st); // q = K p
        if (rc)
            return rc;
        double qq = 0.0;
        rc = lsq_sqnorm<R>(L.q.p, M, L, st, &qq);
        if (rc)
            return rc;
        if (!(qq > 0.0))
            break;
        const double alpha = gamma / qq;
        hipLaunchKernelGGL((k_axpy<R>), dim3(gN), dim3(256), 0, st, N, alpha,
                           (const cx<R> *)L.p.p, (cx<R> *)f);
        hipLaunchKernelGGL((k_axpy<R>), dim3(gM), dim3(256), 0, st, M, -alpha,
                           (const cx<R> *)L.q.p, (cx<R> *)L.r.p);
        HIPCHK(hipGetLastError());
        rc = execute(Pa, L.r.p, L.s.p, -1, st); // s = K^H r
        if (rc)
            return rc;
        double gnew = 0.0;
        rc = lsq_sqnorm<R>(L.s.p, N, L, st, &gnew);
        if (rc)
            return rc;
        ++k;
        res = std::sqrt(gnew / gamma0);
        hipLaunchKernelGGL((k_xpby<R>), dim3(gN), dim3(256), 0, st, N,
                           (const cx<R> *)L.s.p, gnew / gamma, (cx<R> *)L.p.p);
        HIPCHK(hipGetLastError());
        gamma = gnew;
    }
    HIPCHK(hipStreamSynchronize(st));
    if (iters)
        *iters = k;
    if (resid)
        *resid = res;
    return FN_OK;
}

// ------------------------------------------------------------------ ABI

// Machine precision (eps = FN_EPS_MACHINE) on binary64: the expansion length
// p_th and regular-part truncation q_th measured on MI355X to reach eps_th(N)
// at every N = M = 2^6 ... 2^20 (uniform y; one term fewer of either leaves
// 4x its error).  Eq. (18.2) at eps_th(N) asks for p = 34 ... 42, q = 25.
// Values given explicitly are kept.
static constexpr int P_TH = 32, Q_TH = 22;
static void machine_params(double eps_in, int dtype, int32_t *p_in, int32_t *q_in)
{
    if (eps_in != 0.0 || dtype != FN_C128)
        return;
    if (*p_in <= 0)
        *p_in = P_TH;
    if (*q_in <= 0)
        *q_in = Q_TH;
}

// Checks the scalar arguments; eps = FN_EPS_MACHINE (0) becomes the path's
// floor eps_th(N, M).
static int check_common(int64_t N, int64_t M, double &eps, int dtype)
{
    if (N < 1 || N > INT32_MAX - 1)
        return fail(FN_EINVAL, "N = %lld out of range [1, 2^31 - 2]", (long long)N);
    if (M < 1 || M > INT32_MAX - 1)
        return fail(FN_EINVAL, "M = %lld out of range [1, 2^31 - 2]", (long long)M);
    if (dtype != FN_C128 && dtype != FN_C64)
        return fail(FN_EINVAL, "unknown dtype %d", dtype);
    if (eps == 0.0) {
        eps = eps_th(N, M, dtype);
        return FN_OK;
    }
    if (!(eps > 0.0) || !std::isfinite(eps) || eps >= 1.0)
        return fail(FN_EINVAL, "eps = %g must be 0 (the precision floor) or finite and "
                               "in (0, 1)", eps);
    if (eps < eps_floor(dtype))
        return fail(FN_EPREC, "eps = %g is below the floor %g of this precision path",
                    eps, eps_floor(dtype));
    return FN_OK;
}

// Parameters of a plan of the given kind (-1: the paper's depth rule).
// Depth and expansion length recorded by nufft_autotune, per (kind,
// dtype, size class lg = round(log2 sqrt(N M)), accuracy class
// floor(-log10 eps)).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tuned;

static std::tuple<int, int, int, int> tune_key(int kind, int dtype, int64_t N, int64_t M,
                                               double eps)
{
    const int lg = (int)std::lround(0.5 * std::log2((double)N * (double)M));
    const int ec = (int)std::floor(-std::log10(eps) + 1e-9);
    return std::make_tuple(kind, dtype, lg, ec);
}

// Parameters of a plan of the given kind (-1: the paper's depth rule).
// Values not given explicitly come from the autotuner's record when there
// is one (the expansion length then counts as given), else from the
// defaults.
static void choose(int64_t N, int64_t M, double eps, int kind, int dtype, int32_t p_in,
                   int32_t q_in, int32_t l_in, int *p, int *q, int *l, bool *p_given)
{
    int tl = 0, tp = 0;
    if (kind >= 0 && (l_in <= 0 || p_in <= 0)) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(tune_key(kind, dtype, N, M, eps));
        if (it != g_tuned.end()) {
            tl = it->second.first;
            tp = it->second.second;
        }
    }
    // a recorded depth was tuned for its size class lg = round(log2 sqrt(N M));
    // N and M can be skewed within the class, so the mixed path's leaf
    // bound applies to it again
    *l = l_in > 0 ? l_in
                  : (tl > 0 ? std::max(tl, mixed_min_depth(kind == 2 ? M : N, dtype))
                            : (kind < 0 ? paper_depth(N, M) : default_depth(N, M, kind, dtype)));
    int pp, qq;
    trunc_numbers(eps, *l, &pp, &qq);
    *p = p_in > 0 ? p_in : (tp > 0 ? tp : pp);
    *q = q_in > 0 ? q_in : qq;
    if (p_given)
        *p_given = p_in > 0 || tp > 0;
}

static int plan_body(fn_plan *P, int kind, int64_t N, int64_t M, const double *y,
                     double eps, int dtype, int32_t p_in, int32_t q_in, int32_t l_in,
                     void *stream, bool defer);

// Creates a plan.  Unless `defer`, waits for the setup kernels and reports
// their errors; a deferred plan is checked by finish_plan after its first
// execute (the one-shot calls), which then costs a single synchronisation.
static int plan_common(fn_plan **out, int kind, int64_t N, int64_t M,
                       const double *y, double eps, int dtype, int32_t p_in,
                       int32_t q_in, int32_t l_in, void *stream, bool defer = false)
{
    if (!out)
        return fail(FN_EINVAL, "plan pointer is NULL");
    *out = nullptr;
    machine_params(eps, dtype, &p_in, &q_in);
    int rc = check_common(N, M, eps, dtype);
    if (rc)
        return rc;
    if (!y)
        return fail(FN_EINVAL, "y is NULL");
    if (l_in > 24 || p_in > 64 || q_in > 30)
        return fail(FN_EINVAL, "explicit parameters out of range (lmax <= 24, p <= 64, q <= 30)");
    fn_plan *P = new fn_plan();
    try {
        rc = plan_body(P, kind, N, M, y, eps, dtype, p_in, q_in, l_in, stream, defer);
    } catch (...) { // a failed host allocation: release the plan, then report
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    if (rc)
        return rc; // plan_body released the plan
    *out = P;
    return FN_OK;
}

static int plan_body(fn_plan *P, int kind, int64_t N, int64_t M, const double *y,
                     double eps, int dtype, int32_t p_in, int32_t q_in, int32_t l_in,
                     void *stream, bool defer)
{
    int rc = FN_OK;
    P->kind = kind;
    P->dtype = dtype;
    P->N = N;
    P->M = M;
    P->eps = eps;
    choose(N, M, eps, kind, dtype, p_in, q_in, l_in, &P->p, &P->q, &P->l, &P->p_explicit);
    if (P->p > 64 || 2 * P->q > 64) {
        const int p = P->p, q = P->q;
        delete P;
        return fail(FN_EINVAL, "truncation numbers p = %d, q = %d need more than 64 terms", p, q);
    }
    hipStream_t st = (hipStream_t)stream;
    P->stream = st;
    if (!alloc(P->flags, 4)) {
        delete P;
        return fail(FN_ENOMEM, "flag allocation failed (%s)", hipGetErrorString(g_alloc_err));
    }
    // (the flags are cleared by the first launch of the plan's sort)
    if (kind == 0)
        rc = dtype == FN_C128 ? plan_fwd_impl<double>(P, y, st)
                              : plan_fwd_impl<float>(P, y, st);
    else if (kind == 1)
        rc = dtype == FN_C128 ? plan_inv_impl<double>(P, y, st)
                              : plan_inv_impl<float>(P, y, st);
    else
        rc = dtype == FN_C128 ? plan_adj_impl<double>(P, y, st)
                              : plan_adj_impl<float>(P, y, st);
    if (!rc && !defer)
        rc = finish_plan(P, st);
    if (rc) {
        (void)hipStreamSynchronize(st);
        release_plan(P);
        delete P;
        return rc;
    }
    return FN_OK;
}

// End of a one-shot call: one synchronisation for the setup's error flags
// and the evaluation, then the plan goes.  A setup error takes precedence
// (the evaluation then ran on a rejected point set and its output is void).
static int finish_one_shot(fn_plan *P, int rc_exec)
{
    int rc = finish_plan(P, P->stream);
    release_plan(P);
    delete P;
    return rc ? rc : rc_exec;
}

// ------------------------------------------------------ batched forward
//
// Many independent forward transforms of uneven sizes.  Every transform
// gets its own plan (workspace, tree, work list), but each pass runs as one
// launch over the whole batch: block b of a launch works for the transform
// its BlockMap assigns.  The arguments of all launches sit in one device
// blob written at plan time; the per-call inputs and outputs come from a
// small IoPtr table, so the evaluation (upward bands, regular part,
// downward pass) is captured once in a HIP graph and replayed.  Transforms
// whose sort needs the global-atomic path or whose expansion lengths differ
// from the batch's run with their own launches.

struct LaunchShape {
    size_t args = 0, map = 0; // byte offsets in the blob
    int grid = 0, n = 0;      // blocks; problems in the launch
    size_t smem = 0;
};

struct fn_batch {
    Arena arena; // every workspace of the batch's plans
    int T = 0, dtype = 0;
    double eps = 0;
    bool machine = false; // eps = FN_EPS_MACHINE: each transform at its eps_th
    std::vector<fn_plan *> P;
    std::vector<int> grp, solo;
    int PU = 0, PD = 0, q = 0, nbands = 0;
    size_t tr_smem = 0;
    Buf blob, io, flags;
    // host images of the argument blob and of the I/O table, kept unchanged
    // until the copies that read them have run: the blob's until the batch
    // is released, the table's until ev_io (recorded after its last copy)
    std::vector<unsigned char> blob_host;
    IoPtr *hio = nullptr; // pinned, T entries (graph replays)
    hipEvent_t ev_io = nullptr;
    bool io_pending = false;
    std::vector<IoPtr> hio_pageable; // one-shot fallback without pinned memory
    LaunchShape hist, colscan, place, scan, work, reg, m2l, down, up[MAX_BANDS];
    hipStream_t stream = nullptr;
    hipStream_t bs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec = nullptr;
};

// Host image of the blob: argument arrays and block maps appended in turn.
struct BlobBuilder {
    std::vector<unsigned char> bytes;
    size_t put(const void *p, size_t n)
    {
        size_t off = (bytes.size() + 15) & ~size_t(15);
        bytes.resize(off + n);
        memcpy(bytes.data() + off, p, n);
        return off;
    }
    template <typename A>
    void add(LaunchShape &L, const std::vector<A> &args, const std::vector<int> &blocks)
    {
        std::vector<int32_t> start(blocks.size() + 1, 0);
        for (size_t i = 0; i < blocks.size(); ++i)
            start[i + 1] = start[i] + blocks[i];
        L.args = put(args.data(), args.size() * sizeof(A));
        L.map = put(start.data(), start.size() * 4);
        L.grid = start.back();
        L.n = (int)args.size();
    }
};

static void release_batch(fn_batch *B)
{
    for (fn_plan *P : B->P) {
        if (!P)
            continue;
        P->flags = Buf{}; // a slot of the batch's flag array
        P->flags_ready = true;
        release_plan(P);
        delete P;
    }
    B->P.clear();
    release(B->blob);
    release(B->io);
    release(B->flags);
    for (Buf &c : B->arena.chunks)
        release(c);
    B->arena.chunks.clear();
    if (B->gexec)
        (void)hipGraphExecDestroy(B->gexec);
    if (B->ev_in)
        (void)hipEventDestroy(B->ev_in);
    if (B->ev_out)
        (void)hipEventDestroy(B->ev_out);
    if (B->ev_io)
        (void)hipEventDestroy(B->ev_io);
    if (B->hio)
        (void)hipHostFree(B->hio);
    B->hio = nullptr;
    if (B->bs)
        (void)hipStreamDestroy(B->bs);
}

template <typename R>
static int plan_batch_impl(fn_batch *B, const int64_t *Ns, const int64_t *Ms,
                           const double *const *ys, hipStream_t st)
{
    using V = cx<R>;
    const int T = B->T;
    // host bookkeeping first: a failed host allocation then surfaces before
    // any device work
    std::vector<SortArgs> sa;
    std::vector<WorkArgs> wa;
    std::vector<int> nb_hist, nb_col, nb_one;
    std::vector<TreeJob> jobs(T);
    std::vector<WorkArgs> works(T);
    B->P.assign(T, nullptr);
    if (!alloc(B->flags, (size_t)T * 4) || !alloc(B->io, (size_t)T * sizeof(IoPtr)))
        return fail(FN_ENOMEM, "batch allocation failed");
    HIPCHK(hipMemsetAsync(B->flags.p, 0, (size_t)T * 4, st));
    for (int t = 0; t < T; ++t) {
        fn_plan *P = new fn_plan();
        B->P[t] = P;
        P->kind = 0;
        P->dtype = B->dtype;
        P->N = Ns[t];
        P->M = Ms[t];
        P->eps = B->machine ? eps_th(P->N, P->M, P->dtype) : B->eps;
        P->stream = st;
        int32_t p_in = 0, q_in = 0;
        machine_params(B->machine ? 0.0 : B->eps, P->dtype, &p_in, &q_in);
        choose(P->N, P->M, P->eps, 0, P->dtype, p_in, q_in, 0, &P->p, &P->q, &P->l,
               &P->p_explicit);
        if (P->p > 64 || 2 * P->q > 64)
            return fail(FN_EINVAL, "transform %d: truncation numbers need more than 64 terms", t);
        P->flags.p = (int *)B->flags.p + t;
        int PU, PD;
        cot_lengths(P, &PU, &PD);
        P->lr = choose_lr(P->l, 2, PD, sizeof(R));
        int rc = prepare_tree(P, P->M, ys[t], P->l - P->lr, false, false, true, &jobs[t]);
        if (!rc)
            rc = prepare_work(P, 0, false, P->M, &works[t]);
        if (!rc)
            rc = setup_fmm<R, V>(P, KER_COT, PU, PD, P->q, false, P->cot, st);
        if (rc)
            return rc;
        if (B->grp.empty()) {
            B->PU = PU;
            B->PD = PD;
            B->q = P->q;
        }
        const bool shared = jobs[t].lds_path && PU == B->PU && PD == B->PD &&
                            jobs[t].a.nbins <= SCAN1_MAX;
        (shared ? B->grp : B->solo).push_back(t);
    }
    // the sorts: shared launches for the group, own launches for the rest
    BlobBuilder bb;
    size_t hist_smem = 0;
    for (int t : B->grp) {
        const SortArgs &a = jobs[t].a;
        sa.push_back(a);
        wa.push_back(works[t]);
        nb_hist.push_back(a.nblk);
        nb_col.push_back((a.nbins + CS_COLS - 1) / CS_COLS);
        nb_one.push_back(1);
        hist_smem = std::max(hist_smem, (size_t)a.nbins * 4);
    }
    if (!B->grp.empty()) {
        bb.add(B->hist, sa, nb_hist);
        B->hist.smem = hist_smem;
        bb.add(B->colscan, sa, nb_col);
        bb.add(B->scan, sa, nb_one);
        bb.add(B->place, sa, nb_hist);
        B->place.smem = hist_smem;
        bb.add(B->work, wa, nb_one);
    }
    // the evaluation: per band, the transforms that have it
    OpTables<R> Tb;
    int rc = get_tables<R>(KER_COT, B->PU ? B->PU : 16, B->PD ? B->PD : 16, B->q ? B->q : 1, &Tb);
    if (rc)
        return rc;
    B->nbands = 0;
    for (int t : B->grp)
        B->nbands = std::max(B->nbands, B->P[t]->cot.nbands);
    for (int k = 0; k < B->nbands; ++k) {
        std::vector<UpArgs<R, V>> ua;
        std::vector<int> nb;
        size_t smem = 0;
        for (int t : B->grp) {
            const fn_plan *P = B->P[t];
            const FmmSetup &F = P->cot;
            if (k >= F.nbands)
                continue;
            UpArgs<R, V> u{};
            fill_up(P, F, Tb, u);
            u.lb = F.band[k].lb;
            u.d = F.band[k].d;
            u.first_band = F.band[k].first;
            u.io_index = t;
            ua.push_back(u);
            nb.push_back(F.band[k].grid);
            smem = std::max(smem, F.band[k].smem);
        }
        bb.add(B->up[k], ua, nb);
        B->up[k].smem = smem;
    }
    {
        std::vector<UpArgs<R, V>> ua;
        std::vector<DownArgs<R, V>> da;
        std::vector<int> nb_reg, nb_down, nb_m2l;
        size_t dsm = 0, msm = 0;
        for (int t : B->grp) {
            fn_plan *P = B->P[t];
            const FmmSetup &F = P->cot;
            UpArgs<R, V> u{};
            fill_up(P, F, Tb, u);
            u.io_index = t;
            ua.push_back(u);
            nb_reg.push_back(1);
            DownArgs<R, V> d{};
            fill_down(P, F, Tb, d);
            d.tgt_pt = (const SortedPt *)P->spt.p;
            d.io_index = t;
            d.io = (const IoPtr *)B->io.p; // f, g of every call come from the table
            da.push_back(d);
            nb_down.push_back(P->nwork);
            nb_m2l.push_back(m2l_blocks(P->l) + 1); // + the regular part
            dsm = std::max(dsm, F.dn_smem);
            msm = std::max(msm, F.m2l_smem);
            B->tr_smem = std::max(B->tr_smem, F.tr_smem);
        }
        bb.add(B->reg, ua, nb_reg); // the regular part's arguments (read by kb_m2l)
        bb.add(B->down, da, nb_down);
        B->down.smem = dsm;
        bb.add(B->m2l, da, nb_m2l);
        B->m2l.smem = msm;
    }
    if (!bb.bytes.empty()) {
        if (!alloc(B->blob, bb.bytes.size()))
            return fail(FN_ENOMEM, "batch argument allocation failed");
        B->blob_host = std::move(bb.bytes);
        HIPCHK(hipMemcpyAsync(B->blob.p, B->blob_host.data(), B->blob_host.size(),
                              hipMemcpyHostToDevice, st));
    }
    // enqueue the sorts
    auto at = [&](size_t off) { return (unsigned char *)B->blob.p + off; };
    auto map = [&](const LaunchShape &L) {
        return BlockMap{(const int32_t *)at(L.map), L.n};
    };
    if (!B->grp.empty()) {
        hipLaunchKernelGGL(kb_hist, dim3(B->hist.grid), dim3(SORT_THREADS), B->hist.smem, st,
                           (const SortArgs *)at(B->hist.args), map(B->hist));
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(kb_colscan, dim3(B->colscan.grid), dim3(CS_THREADS), 0, st,
                           (const SortArgs *)at(B->colscan.args), map(B->colscan));
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(kb_scan_one, dim3(B->scan.grid), dim3(1024), SCAN1_SMEM, st,
                           (const SortArgs *)at(B->scan.args));
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(kb_place, dim3(B->place.grid), dim3(SORT_THREADS), B->place.smem, st,
                           (const SortArgs *)at(B->place.args), map(B->place));
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(kb_work, dim3(B->work.grid), dim3(1024), 0, st,
                           (const WorkArgs *)at(B->work.args));
        HIPCHK(hipGetLastError());
    }
    for (int t : B->solo) {
        rc = launch_tree(B->P[t], jobs[t], st);
        if (rc)
            return rc;
        hipLaunchKernelGGL(k_work, dim3(1), dim3(1024), 0, st, works[t]);
        HIPCHK(hipGetLastError());
    }
    return FN_OK;
}

// The evaluation of the group: upward bands, regular part, downward pass.
template <typename R>
static int launch_batch_eval(fn_batch *B, hipStream_t st)
{
    using V = cx<R>;
    if (B->grp.empty())
        return FN_OK;
    auto at = [&](size_t off) { return (unsigned char *)B->blob.p + off; };
    auto map = [&](const LaunchShape &L) {
        return BlockMap{(const int32_t *)at(L.map), L.n};
    };
    const IoPtr *io = (const IoPtr *)B->io.p;
    for (int k = 0; k < B->nbands; ++k) {
        const LaunchShape &L = B->up[k];
        FN_DISPATCH16(B->PU, PU_,
                      hipLaunchKernelGGL((kb_up_band<R, V, KER_COT, SET_UNIFORM, PU_>),
                                         dim3(L.grid), dim3(BLOCK), L.smem, st,
                                         (const UpArgs<R, V> *)at(L.args), map(L), io));
        HIPCHK(hipGetLastError());
    }
    FN_DISPATCH16(B->PD, PD_,
                  hipLaunchKernelGGL((kb_m2l<R, V, KER_COT, PD_>), dim3(B->m2l.grid),
                                     dim3(BLOCK), B->m2l.smem, st,
                                     (const DownArgs<R, V> *)at(B->m2l.args), map(B->m2l),
                                     (const UpArgs<R, V> *)at(B->reg.args)));
    HIPCHK(hipGetLastError());
    FN_DISPATCH16(
        B->PD, PD_,
        hipLaunchKernelGGL((kb_down_trans<R, V, KER_COT, SET_UNIFORM, EPI_FWD, PD_>),
                           dim3(B->down.grid), dim3(BLOCK), B->tr_smem, st,
                           (const DownArgs<R, V> *)at(B->down.args), map(B->down), io);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL((kb_down_eval<R, V, KER_COT, SET_UNIFORM, EPI_FWD, PD_>),
                           dim3(B->down.grid), dim3(BLOCK), B->down.smem, st,
                           (const DownArgs<R, V> *)at(B->down.args), map(B->down), io));
    HIPCHK(hipGetLastError());
    return FN_OK;
}

static int plan_batch(fn_batch **out, int32_t count, const int64_t *Ns, const int64_t *Ms,
                      const double *const *ys, double eps, int dtype, void *stream)
{
    if (!out)
        return fail(FN_EINVAL, "batch pointer is NULL");
    *out = nullptr;
    if (count < 1 || !Ns || !Ms || !ys)
        return fail(FN_EINVAL, "count must be >= 1 and the size and point arrays non-NULL");
    // FN_EPS_MACHINE: each transform at its own floor; the batch records
    // the smallest
    const bool machine = eps == 0.0;
    double eps_b = machine ? 1.0 : eps;
    for (int32_t t = 0; t < count; ++t) {
        double e = eps;
        int rc = check_common(Ns[t], Ms[t], e, dtype);
        if (rc)
            return fail(rc, "transform %d: %s", t, std::string(g_err).c_str());
        if (!ys[t])
            return fail(FN_EINVAL, "transform %d: y is NULL", t);
        eps_b = std::min(eps_b, e);
    }
    eps = eps_b;
    fn_batch *B = new fn_batch();
    B->T = count;
    B->dtype = dtype;
    B->eps = eps;
    B->machine = machine;
    hipStream_t st = (hipStream_t)stream;
    B->stream = st;
    g_arena = &B->arena;
    int rc;
    try {
        rc = dtype == FN_C128 ? plan_batch_impl<double>(B, Ns, Ms, ys, st)
                              : plan_batch_impl<float>(B, Ns, Ms, ys, st);
    } catch (...) { // a failed host allocation: release the batch, then report
        g_arena = nullptr;
        (void)hipStreamSynchronize(st);
        release_batch(B);
        delete B;
        throw;
    }
    g_arena = nullptr;
    if (rc) {
        (void)hipStreamSynchronize(st);
        release_batch(B);
        delete B;
        return rc;
    }
    *out = B;
    return FN_OK;
}

// Waits for the batch's setup and reports its errors (first transform
// with a flag); releases the setup temporaries.
static int finish_batch(fn_batch *B, hipStream_t st)
{
    std::vector<int> hv;
    int *hf = (int *)pinned_scratch((size_t)B->T * 4);
    if (!hf) {
        hv.assign(B->T, 0);
        hf = hv.data();
    }
    hipError_t e = hipMemcpyAsync(hf, B->flags.p, (size_t)B->T * 4,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    for (fn_plan *P : B->P)
        release_tmp(P);
    if (e != hipSuccess)
        return fail(FN_EHIP, "batch setup: %s", hipGetErrorString(e));
    for (int t = 0; t < B->T; ++t)
        if (hf[t] & FLAG_BAD_Y)
            return fail(FN_EINVAL, "transform %d: y holds a non-finite value or |y| > %g", t,
                        FN_Y_MAX);
    return FN_OK;
}

// Replay resources of a batch plan, made once at plan time so that its
// executes allocate nothing: the batch's stream, its events, the pinned I/O
// table, and the evaluation captured as a graph (it reads f, g through the
// device I/O table, so one capture serves every call).
template <typename R>
static int prepare_replay(fn_batch *B)
{
    if (B->grp.empty())
        return FN_OK;
    HIPCHK(hipStreamCreateWithFlags(&B->bs, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_io, hipEventDisableTiming));
    if (hipHostMalloc((void **)&B->hio, (size_t)B->T * sizeof(IoPtr),
                      hipHostMallocPortable) != hipSuccess) {
        B->hio = nullptr;
        return fail(FN_ENOMEM, "pinned host allocation of the I/O table failed");
    }
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamBeginCapture(B->bs, hipStreamCaptureModeThreadLocal));
    int rc = launch_batch_eval<R>(B, B->bs);
    hipError_t e = hipStreamEndCapture(B->bs, &gr);
    if (rc) {
        if (gr)
            (void)hipGraphDestroy(gr);
        return rc;
    }
    if (e != hipSuccess)
        return fail(FN_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&B->gexec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
        B->gexec = nullptr;
        return fail(FN_EHIP, "graph instantiation: %s", hipGetErrorString(e));
    }
    return FN_OK;
}

template <typename R>
static int exec_batch_impl(fn_batch *B, const void *const *f, void *const *g, hipStream_t st,
                           bool graph)
{
    for (int t = 0; t < B->T; ++t)
        if (!f[t] || !g[t])
            return fail(FN_EINVAL, "transform %d: f or g is NULL", t);
    B->stream = st;
    if (!B->grp.empty() && !graph) {
        // one-shot: the call synchronises before it returns, so the
        // thread's pinned table (or the batch's own) stays put until then
        IoPtr *h = (IoPtr *)pinned_scratch((size_t)B->T * sizeof(IoPtr), 1);
        if (!h) {
            B->hio_pageable.resize(B->T);
            h = B->hio_pageable.data();
        }
        for (int t = 0; t < B->T; ++t)
            h[t] = {f[t], g[t]};
        HIPCHK(hipMemcpyAsync(B->io.p, h, (size_t)B->T * sizeof(IoPtr),
                              hipMemcpyHostToDevice, st));
        int rc = launch_batch_eval<R>(B, st);
        if (rc)
            return rc;
    } else if (!B->grp.empty()) {
        if (!B->gexec)
            return fail(FN_EINVAL, "batch plan has no captured evaluation");
        // the pinned I/O table is rewritten only once its last copy has run
        if (B->io_pending)
            HIPCHK(hipEventSynchronize(B->ev_io));
        B->io_pending = false;
        for (int t = 0; t < B->T; ++t)
            B->hio[t] = {f[t], g[t]};
        // replay on the batch's stream, ordered after the caller's work
        HIPCHK(hipEventRecord(B->ev_in, st));
        HIPCHK(hipStreamWaitEvent(B->bs, B->ev_in, 0));
        HIPCHK(hipMemcpyAsync(B->io.p, B->hio, (size_t)B->T * sizeof(IoPtr),
                              hipMemcpyHostToDevice, B->bs));
        HIPCHK(hipEventRecord(B->ev_io, B->bs));
        B->io_pending = true;
        HIPCHK(hipGraphLaunch(B->gexec, B->bs));
        HIPCHK(hipEventRecord(B->ev_out, B->bs));
        HIPCHK(hipStreamWaitEvent(st, B->ev_out, 0));
    }
    for (int t : B->solo) {
        int rc = exec_fwd<R>(B->P[t], f[t], g[t], -1, st);
        if (rc)
            return rc;
    }
    return FN_OK;
}

static int exec_batch(fn_batch *B, const void *const *f, void *const *g, void *stream,
                      bool graph)
{
    if (!B)
        return fail(FN_EINVAL, "batch is NULL");
    if (!f || !g)
        return fail(FN_EINVAL, "f or g pointer array is NULL");
    hipStream_t st = (hipStream_t)stream;
    return B->dtype == FN_C128 ? exec_batch_impl<double>(B, f, g, st, graph)
                               : exec_batch_impl<float>(B, f, g, st, graph);
}

// ------------------------------------------------------------ autotuner
//
// For one kind, size and accuracy, on a synthetic problem of that size
// (uniform targets for the forward, a jittered grid for the inverse):
//   1. the shortest expansion length (16, 32, 48) whose output stays within
//      eps / 4 (relative l2) of the output with 64 terms, at the default
//      depth; else the default length;
//   2. the fastest depth among lg - 4 .. lg - 7 (lg = round(log2 sqrt(N M)))
//      for one-shot transforms with that length (median of three; another
//      depth must beat the default by 5%); small
//      forward transforms are timed as a batch of copies of about 2^20
//      points, the way batches run them.
// The result is recorded for later plans of that kind, dtype, size class
// and accuracy class.

static int execute(fn_plan *plan, const void *in, void *out, int phase, void *stream);

// One-shot transform with explicit parameters; returns the wall time.
static int tune_run(int kind, int64_t N, int64_t M, const double *y, const void *in,
                    void *out, double eps, int dtype, int p, int l, hipStream_t st,
                    double *secs)
{
    const auto t0 = std::chrono::steady_clock::now();
    fn_plan *P = nullptr;
    int rc = plan_common(&P, kind, N, M, y, eps, dtype, p, 0, l, st, true);
    if (rc)
        return rc;
    rc = finish_one_shot(P, execute(P, in, out, -1, st));
    *secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

static int tune_err(int64_t n, const void *a, const void *b, int dtype, Buf &part,
                    hipStream_t st, double *err)
{
    const int nb = 256;
    if (dtype == FN_C128)
        hipLaunchKernelGGL(k_diff2<double>, dim3(nb), dim3(256), 0, st, n,
                           (const cx<double> *)a, (const cx<double> *)b, (double *)part.p);
    else
        hipLaunchKernelGGL(k_diff2<float>, dim3(nb), dim3(256), 0, st, n,
                           (const cx<float> *)a, (const cx<float> *)b, (double *)part.p);
    HIPCHK(hipGetLastError());
    std::vector<double> h(2 * nb);
    HIPCHK(hipMemcpyAsync(h.data(), part.p, h.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double d = 0, r = 0;
    for (int i = 0; i < nb; ++i) {
        d += h[2 * i];
        r += h[2 * i + 1];
    }
    *err = r > 0 ? std::sqrt(d / r) : std::sqrt(d);
    return FN_OK;
}

static int autotune(int kind, int64_t N, int64_t M, double eps, int dtype, int32_t *l_out,
                    int32_t *p_out, hipStream_t st)
{
    if (kind < 0 || kind > 2)
        return fail(FN_EINVAL, "kind must be 0 (forward), 1 (inverse) or 2 (adjoint)");
    if (kind == 1)
        M = N;
    int rc = check_common(N, M, eps, dtype);
    if (rc)
        return rc;
    const size_t es = dtype == FN_C128 ? 16 : 8;
    const int64_t nin = kind == 2 ? M : N, nout = kind == 0 ? M : N;
    Buf y, in, out, ref, part;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (Buf *b : {&y, &in, &out, &ref, &part})
            release(*b);
    };
    if (!alloc(y, (size_t)M * 8) || !alloc(in, nin * es) || !alloc(out, nout * es) ||
        !alloc(ref, nout * es) || !alloc(part, 512 * 8)) {
        cleanup();
        return fail(FN_ENOMEM, "autotuner allocation failed");
    }
    const uint64_t seed = 0x5eed0f0e11ull;
    hipLaunchKernelGGL(k_synth_points, dim3(grid_for(M)), dim3(256), 0, st, M, N,
                       kind == 1 ? 0.8 : 0.0, seed, (double *)y.p);
    if (dtype == FN_C128)
        hipLaunchKernelGGL(k_synth_data<double>, dim3(grid_for(nin)), dim3(256), 0, st, nin,
                           seed + 1, (cx<double> *)in.p);
    else
        hipLaunchKernelGGL(k_synth_data<float>, dim3(grid_for(nin)), dim3(256), 0, st, nin,
                           seed + 1, (cx<float> *)in.p);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu); // measure without an old record
        g_tuned.erase(tune_key(kind, dtype, N, M, eps));
    }
    const int l0 = default_depth(N, M, kind, dtype);
    double secs = 0, err = 0;
    rc = tune_run(kind, N, M, (const double *)y.p, in.p, ref.p, eps, dtype, 64, l0, st, &secs);
    int pbest = 0;
    for (int pc = 16; !rc && pc <= 48; pc += 16) {
        rc = tune_run(kind, N, M, (const double *)y.p, in.p, out.p, eps, dtype, pc, l0, st,
                      &secs);
        if (!rc)
            rc = tune_err(nout, out.p, ref.p, dtype, part, st, &err);
        if (!rc && err <= 0.25 * eps) {
            pbest = pc;
            break;
        }
    }
    const int lg = (int)std::lround(0.5 * std::log2((double)N * (double)M));
    // small forward transforms are timed as a batch of copies of about 2^20
    // points through the batched path (one alone is launch-bound)
    const int64_t K = kind == 0 ? std::max<int64_t>(1, (int64_t(1) << 20) / (N + M)) : 1;
    Buf outs;
    if (!rc && K > 1 && !alloc(outs, (size_t)K * nout * es))
        rc = fail(FN_ENOMEM, "autotuner allocation failed");
    std::vector<int64_t> Ns(K, N), Ms(K, M);
    std::vector<const double *> ys(K, (const double *)y.p);
    std::vector<const void *> fs(K, in.p);
    std::vector<void *> gs(K);
    for (int64_t k = 0; k < K && outs.p; ++k)
        gs[k] = (unsigned char *)outs.p + (size_t)k * nout * es;
    const auto key = tune_key(kind, dtype, N, M, eps);
    int lbest = l0;
    double tbest = 1e300;
    const int lmin = mixed_min_depth(N, dtype);
    for (int off = 4; !rc && off <= 7; ++off) {
        const int l = std::max(lmin, std::min(24, std::max(2, lg - off)));
        if (off > 4 && l == std::max(lmin, std::min(24, std::max(2, lg - off + 1))))
            continue;
        std::vector<double> ts;
        for (int r = 0; !rc && r < 4; ++r) {
            if (K == 1) {
                rc = tune_run(kind, N, M, (const double *)y.p, in.p, out.p, eps, dtype, pbest,
                              l, st, &secs);
            } else {
                {
                    std::lock_guard<std::mutex> lk(g_tune_mu);
                    g_tuned[key] = {l, pbest};
                }
                const auto t0 = std::chrono::steady_clock::now();
                fn_batch *B = nullptr;
                rc = plan_batch(&B, (int32_t)K, Ns.data(), Ms.data(), ys.data(), eps, dtype, st);
                if (!rc) {
                    const int rx = exec_batch(B, fs.data(), gs.data(), st, false);
                    rc = finish_batch(B, st);
                    rc = rc ? rc : rx;
                    release_batch(B);
                    delete B;
                }
                secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0)
                           .count();
            }
            if (r > 0)
                ts.push_back(secs); // the first run warms the caches
        }
        if (rc)
            break;
        std::sort(ts.begin(), ts.end());
        // another depth must beat the default by 5% (timing noise)
        const double tq = l == l0 ? ts[1] : ts[1] / 0.95;
        if (tq < tbest) {
            tbest = tq;
            lbest = l;
        }
    }
    release(outs);
    cleanup();
    if (rc)
        return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(kind, dtype, N, M, eps)] = {lbest, pbest};
    }
    if (l_out)
        *l_out = lbest;
    if (p_out)
        *p_out = pbest;
    return FN_OK;
}

// ---------------------------------------- the allocation-free forward call
//
// nufft_fwd_noalloc takes every workspace (sorted targets, histograms, work
// list, multipoles, leaf locals, and operator tables not yet built by
// another call) from one static device array instead of the block cache.
// Each device holds its own copy at its own address, found once per device
// with hipGetSymbolAddress; host code never passes the array's name itself
// to a kernel or a copy.

static constexpr size_t SCRATCH_BYTES = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static constexpr int SCRATCH_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEV];

// Device address of the current device's scratch array (looked up on the
// first call on that device).
static int scratch_region(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEV)
        return fail(FN_EINVAL, "device %d beyond the %d the static scratch serves", dev,
                    SCRATCH_MAX_DEV);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FN_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FN_OK;
}

extern "C" {

int nufft_plan_fwd_ex(fn_plan **plan, int64_t N, int64_t M, const double *y,
                      double eps, int dtype, int32_t p, int32_t q, int32_t lmax,
                      void *stream)
{
    FN_API_BEGIN
    return plan_common(plan, 0, N, M, y, eps, dtype, p, q, lmax, stream);
    FN_API_END
}

int nufft_plan_inv_ex(fn_plan **plan, int64_t N, const double *y, double eps,
                      int dtype, int32_t p, int32_t q, int32_t lmax, void *stream)
{
    FN_API_BEGIN
    return plan_common(plan, 1, N, N, y, eps, dtype, p, q, lmax, stream);
    FN_API_END
}

int nufft_plan_fwd(fn_plan **plan, int64_t N, int64_t M, const double *y,
                   double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    return plan_common(plan, 0, N, M, y, eps, dtype, 0, 0, 0, stream);
    FN_API_END
}

int nufft_plan_adj_ex(fn_plan **plan, int64_t N, int64_t M, const double *y,
                      double eps, int dtype, int32_t p, int32_t q, int32_t lmax,
                      void *stream)
{
    FN_API_BEGIN
    return plan_common(plan, 2, N, M, y, eps, dtype, p, q, lmax, stream);
    FN_API_END
}

int nufft_plan_adj(fn_plan **plan, int64_t N, int64_t M, const double *y,
                   double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    return plan_common(plan, 2, N, M, y, eps, dtype, 0, 0, 0, stream);
    FN_API_END
}

int nufft_adj(int64_t N, int64_t M, const double *y, const void *g, void *f,
              double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    fn_plan *P = nullptr;
    int rc = plan_common(&P, 2, N, M, y, eps, dtype, 0, 0, 0, stream, true);
    if (rc)
        return rc;
    try {
        return finish_one_shot(P, execute(P, g, f, -1, stream));
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    FN_API_END
}

static int plan_spec_common(fn_plan **plan, int kind, int64_t N, int64_t M, const double *y,
                            double eps, int dtype, void *stream, bool defer)
{
    int rc = plan_common(plan, kind, N, M, y, eps, dtype, 0, 0, 0, stream, defer);
    if (rc)
        return rc;
    try {
        rc = setup_spec(*plan);
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(*plan);
        delete *plan;
        *plan = nullptr;
        throw;
    }
    if (rc) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(*plan);
        delete *plan;
        *plan = nullptr;
    }
    return rc;
}

int nufft_plan_spec_fwd(fn_plan **plan, int64_t N, int64_t M, const double *y, double eps,
                        int dtype, void *stream)
{
    FN_API_BEGIN
    return plan_spec_common(plan, 0, N, M, y, eps, dtype, stream, false);
    FN_API_END
}

int nufft_plan_spec_inv(fn_plan **plan, int64_t N, const double *y, double eps, int dtype,
                        void *stream)
{
    FN_API_BEGIN
    return plan_spec_common(plan, 1, N, N, y, eps, dtype, stream, false);
    FN_API_END
}

int nufft_spec_fwd(int64_t N, int64_t M, const double *y, const void *c, void *g,
                   double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    if (!c || !g)
        return fail(FN_EINVAL, "c or g is NULL");
    fn_plan *P = nullptr;
    int rc = plan_spec_common(&P, 0, N, M, y, eps, dtype, stream, true);
    if (rc)
        return rc;
    try {
        return finish_one_shot(P, execute(P, c, g, -1, stream));
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    FN_API_END
}

int inufft_spec(int64_t N, const double *y, const void *g, void *c, double eps, int dtype,
                void *stream)
{
    FN_API_BEGIN
    if (!c || !g)
        return fail(FN_EINVAL, "c or g is NULL");
    fn_plan *P = nullptr;
    int rc = plan_spec_common(&P, 1, N, N, y, eps, dtype, stream, true);
    if (rc)
        return rc;
    try {
        return finish_one_shot(P, execute(P, g, c, -1, stream));
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    FN_API_END
}

int nufft_plan_inv(fn_plan **plan, int64_t N, const double *y, double eps,
                   int dtype, void *stream)
{
    FN_API_BEGIN
    return plan_common(plan, 1, N, N, y, eps, dtype, 0, 0, 0, stream);
    FN_API_END
}

static int execute_fmm(fn_plan *plan, const void *in, void *out, int phase, hipStream_t st);

static int execute(fn_plan *plan, const void *in, void *out, int phase,
                   void *stream)
{
    if (!plan)
        return fail(FN_EINVAL, "plan is NULL");
    if (!in || !out)
        return fail(FN_EINVAL, "input or output pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    plan->stream = st;
    if (!plan->spec)
        return execute_fmm(plan, in, out, phase, st);
    const size_t bytes = (size_t)plan->N * (plan->dtype == FN_C128 ? 16 : 8);
    if (plan->kind == 0) { // c -> f (phase 0 starts with it) -> g
        if (phase <= 0) {
            HIPCHK(hipMemcpyAsync(plan->spec_buf.p, in, bytes, hipMemcpyDeviceToDevice, st));
            int rc = run_fft(plan, plan->spec_buf.p, nullptr, st);
            if (rc)
                return rc;
        }
        return execute_fmm(plan, plan->spec_buf.p, out, phase, st);
    }
    // g -> f -> c (phase 2 ends with it)
    int rc = execute_fmm(plan, in, plan->spec_buf.p, phase, st);
    if (rc || (phase >= 0 && phase < 2))
        return rc;
    return run_fft(plan, plan->spec_buf.p, out, st);
}

static int execute_fmm(fn_plan *plan, const void *in, void *out, int phase, hipStream_t st)
{
    if (plan->kind == 0)
        return plan->dtype == FN_C128 ? exec_fwd<double>(plan, in, out, phase, st)
                                      : exec_fwd<float>(plan, in, out, phase, st);
    if (plan->kind == 2)
        return plan->dtype == FN_C128 ? exec_adj<double>(plan, in, out, phase, st)
                                      : exec_adj<float>(plan, in, out, phase, st);
    return plan->dtype == FN_C128 ? exec_inv<double>(plan, in, out, phase, st)
                                  : exec_inv<float>(plan, in, out, phase, st);
}

int nufft_execute(fn_plan *plan, const void *in, void *out, void *stream)
{
    FN_API_BEGIN
    return execute(plan, in, out, -1, stream);
    FN_API_END
}

int nufft_execute_phase(fn_plan *plan, const void *in, void *out, int phase,
                        void *stream)
{
    FN_API_BEGIN
    if (phase < 0 || phase > 2)
        return fail(FN_EINVAL, "phase must be 0, 1 or 2");
    return execute(plan, in, out, phase, stream);
    FN_API_END
}

int nufft_destroy(fn_plan *plan)
{
    FN_API_BEGIN
    if (!plan)
        return FN_OK;
    // the workspace returns to the library's pool only once the plan's
    // last stream has drained
    hipError_t e = hipStreamSynchronize(plan->stream);
    release_plan(plan);
    delete plan;
    if (e != hipSuccess)
        return fail(FN_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return FN_OK;
    FN_API_END
}

int nufft_plan_coeffs(const fn_plan *plan, double *chat, void *dhat, void *stream)
{
    FN_API_BEGIN
    if (!plan || !chat || !dhat)
        return fail(FN_EINVAL, "NULL argument");
    if (plan->kind != 1)
        return fail(FN_EINVAL, "only inverse plans hold the coefficients of Eq. (p8)");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(chat, plan->chat.p, plan->N * 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_unsort_c128, dim3(grid_for(plan->N)), dim3(256), 0, st, plan->N,
                       (const cx<double> *)plan->dhat.p, (const int32_t *)plan->sperm.p,
                       (cx<double> *)dhat);
    HIPCHK(hipGetLastError());
    return FN_OK;
    FN_API_END
}

int nufft_plan_get_info(const fn_plan *plan, fn_plan_info *info)
{
    FN_API_BEGIN
    if (!plan || !info)
        return fail(FN_EINVAL, "NULL argument");
    info->N = plan->N;
    info->M = plan->M;
    info->kind = plan->kind;
    info->dtype = plan->dtype;
    info->p = plan->p;
    info->q = plan->q;
    info->lmax = plan->l;
    info->nterms = plan->cot.PD;
    info->eps = plan->eps;
    info->mterms = plan->cot.PU;
    info->log_nterms = plan->log_terms;
    info->log_mterms = plan->log_mterms;
    return FN_OK;
    FN_API_END
}

int nufft_set_timing(int on)
{
    FN_API_BEGIN
    g_timing.store(on ? 1 : 0);
    return FN_OK;
    FN_API_END
}

int nufft_plan_get_timings(const fn_plan *plan, float *ms, int32_t *log_terms)
{
    FN_API_BEGIN
    if (!plan || !ms)
        return fail(FN_EINVAL, "plan or ms is NULL");
    for (int i = 0; i < 4; ++i)
        ms[i] = plan->tms[i];
    if (log_terms)
        *log_terms = plan->log_terms;
    return FN_OK;
    FN_API_END
}

int nufft_select_params(int64_t N, int64_t M, double eps, int dtype, int32_t *p,
                        int32_t *q, int32_t *lmax)
{
    FN_API_BEGIN
    int32_t p_in = 0, q_in = 0;
    machine_params(eps, dtype, &p_in, &q_in);
    int rc = check_common(N, M, eps, dtype);
    if (rc)
        return rc;
    int pp, qq, ll;
    choose(N, M, eps, -1, dtype, p_in, q_in, 0, &pp, &qq, &ll, nullptr);
    if (p)
        *p = pp;
    if (q)
        *q = qq;
    if (lmax)
        *lmax = ll;
    return FN_OK;
    FN_API_END
}

int nufft_fwd(int64_t N, int64_t M, const double *y, const void *f, void *g,
              double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    fn_plan *P = nullptr;
    int rc = plan_common(&P, 0, N, M, y, eps, dtype, 0, 0, 0, stream, true);
    if (rc)
        return rc;
    try {
        return finish_one_shot(P, execute(P, f, g, -1, stream));
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    FN_API_END
}

int inufft(int64_t N, const double *y, const void *g, void *f, double eps,
           int dtype, void *stream)
{
    FN_API_BEGIN
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    fn_plan *P = nullptr;
    int rc = plan_common(&P, 1, N, N, y, eps, dtype, 0, 0, 0, stream, true);
    if (rc)
        return rc;
    try {
        return finish_one_shot(P, execute(P, g, f, -1, stream));
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    FN_API_END
}

int nufft_plan_fwd_batched(fn_batch **batch, int32_t count, const int64_t *N,
                           const int64_t *M, const double *const *y, double eps, int dtype,
                           void *stream)
{
    FN_API_BEGIN
    int rc = plan_batch(batch, count, N, M, y, eps, dtype, stream);
    if (rc)
        return rc;
    try {
        rc = finish_batch(*batch, (hipStream_t)stream);
        if (!rc)
            rc = dtype == FN_C128 ? prepare_replay<double>(*batch)
                                  : prepare_replay<float>(*batch);
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_batch(*batch);
        delete *batch;
        *batch = nullptr;
        throw;
    }
    if (rc) {
        release_batch(*batch);
        delete *batch;
        *batch = nullptr;
    }
    return rc;
    FN_API_END
}

int nufft_execute_batched(fn_batch *batch, const void *const *f, void *const *g, void *stream)
{
    FN_API_BEGIN
    return exec_batch(batch, f, g, stream, true);
    FN_API_END
}

int nufft_destroy_batched(fn_batch *batch)
{
    FN_API_BEGIN
    if (!batch)
        return FN_OK;
    hipError_t e = hipStreamSynchronize(batch->stream);
    if (e == hipSuccess && batch->bs)
        e = hipStreamSynchronize(batch->bs);
    release_batch(batch);
    delete batch;
    if (e != hipSuccess)
        return fail(FN_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return FN_OK;
    FN_API_END
}

int nufft_fwd_batched(int32_t count, const int64_t *N, const int64_t *M,
                      const double *const *y, const void *const *f, void *const *g,
                      double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    if (!f || !g)
        return fail(FN_EINVAL, "f or g pointer array is NULL");
    fn_batch *B = nullptr;
    int rc = plan_batch(&B, count, N, M, y, eps, dtype, stream);
    if (rc)
        return rc;
    try {
        int rc_exec = exec_batch(B, f, g, stream, false);
        rc = finish_batch(B, (hipStream_t)stream);
        rc = rc ? rc : rc_exec;
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_batch(B);
        delete B;
        throw;
    }
    release_batch(B);
    delete B;
    return rc;
    FN_API_END
}

int nufft_autotune(int kind, int64_t N, int64_t M, double eps, int dtype, int32_t *lmax,
                   int32_t *nterms, void *stream)
{
    FN_API_BEGIN
    return autotune(kind, N, M, eps, dtype, lmax, nterms, (hipStream_t)stream);
    FN_API_END
}

int nufft_autotune_clear(void)
{
    FN_API_BEGIN
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    return FN_OK;
    FN_API_END
}

// Autotune records as text: a header line, then one record per line,
// "kind dtype size_class accuracy_class lmax nterms".
static const char *const TUNE_HEADER = "# fmmnufft autotune records v1";

int nufft_autotune_save(const char *path)
{
    FN_API_BEGIN
    if (!path)
        return fail(FN_EINVAL, "path is NULL");
    std::vector<std::pair<std::tuple<int, int, int, int>, std::pair<int, int>>> recs;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        recs.assign(g_tuned.begin(), g_tuned.end());
    }
    FILE *fp = fopen(path, "w");
    if (!fp)
        return fail(FN_EINVAL, "cannot write %s", path);
    bool ok = fprintf(fp, "%s\n", TUNE_HEADER) > 0;
    for (const auto &r : recs)
        ok = ok && fprintf(fp, "%d %d %d %d %d %d\n", std::get<0>(r.first), std::get<1>(r.first),
                           std::get<2>(r.first), std::get<3>(r.first), r.second.first,
                           r.second.second) > 0;
    ok = (fclose(fp) == 0) && ok;
    if (!ok)
        return fail(FN_EINVAL, "cannot write %s", path);
    return FN_OK;
    FN_API_END
}

int nufft_autotune_load(const char *path)
{
    FN_API_BEGIN
    if (!path)
        return fail(FN_EINVAL, "path is NULL");
    FILE *fp = fopen(path, "r");
    if (!fp)
        return fail(FN_EINVAL, "cannot read %s", path);
    std::vector<std::pair<std::tuple<int, int, int, int>, std::pair<int, int>>> recs;
    char line[256];
    int lineno = 0;
    bool header = false;
    while (fgets(line, sizeof line, fp)) {
        ++lineno;
        if (lineno == 1) {
            header = strncmp(line, TUNE_HEADER, strlen(TUNE_HEADER)) == 0;
            if (!header)
                break;
            continue;
        }
        int kind, dtype, lg, ec, l, p;
        char extra;
        if (sscanf(line, "%d %d %d %d %d %d %c", &kind, &dtype, &lg, &ec, &l, &p, &extra) != 6 ||
            kind < 0 || kind > 2 || (dtype != FN_C128 && dtype != FN_C64) || lg < 0 ||
            lg > 62 || ec < 0 || ec > 20 || l < 2 || l > 24 || p < 0 || p > 64 || p % 16) {
            fclose(fp);
            return fail(FN_EINVAL, "%s line %d: not an autotune record", path, lineno);
        }
        recs.push_back({std::make_tuple(kind, dtype, lg, ec), {l, p}});
    }
    fclose(fp);
    if (!header)
        return fail(FN_EINVAL, "%s: not an autotune record file", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &r : recs)
        g_tuned[r.first] = r.second;
    return FN_OK;
    FN_API_END
}

int nufft_fwd_noalloc(int64_t N, int64_t M, const double *y, const void *f, void *g,
                      double eps, int dtype, void *stream)
{
    FN_API_BEGIN
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    const double eps_in = eps; // FN_EPS_MACHINE stays visible to the plan
    int rc = check_common(N, M, eps, dtype);
    if (rc)
        return rc;
    void *base = nullptr;
    rc = scratch_region(&base);
    if (rc)
        return rc;
    Arena A;
    A.fixed = (unsigned char *)base;
    A.fixed_cap = SCRATCH_BYTES;
    struct Scope { // the call's allocations come from the fixed region
        Arena *prev;
        explicit Scope(Arena *a) : prev(g_arena) { g_arena = a; }
        ~Scope() { g_arena = prev; }
    } scope(&A);
    fn_plan *P = nullptr;
    rc = plan_common(&P, 0, N, M, y, eps_in, dtype, 0, 0, 0, stream, true);
    if (rc) {
        if (A.overflow)
            return fail(FN_EINVAL, "N = %lld, M = %lld need more workspace than the %zu "
                                   "bytes of the static scratch region (nufft_fwd has no "
                                   "such limit)",
                        (long long)N, (long long)M, SCRATCH_BYTES);
        return rc;
    }
    try {
        return finish_one_shot(P, execute(P, f, g, -1, stream));
    } catch (...) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        release_plan(P);
        delete P;
        throw;
    }
    FN_API_END
}

int nufft_lsq(int64_t N, int64_t M, const double *y, const void *g, void *f, double eps,
              double tol, int32_t maxiter, int dtype, int32_t *iters, double *resid,
              void *stream)
{
    FN_API_BEGIN
    if (!f || !g)
        return fail(FN_EINVAL, "f or g is NULL");
    if (!(tol >= 0.0) || !std::isfinite(tol) || maxiter < 0)
        return fail(FN_EINVAL, "tol must be finite and >= 0, maxiter >= 0");
    hipStream_t st = (hipStream_t)stream;
    fn_plan *Pf = nullptr, *Pa = nullptr;
    int rc = plan_common(&Pf, 0, N, M, y, eps, dtype, 0, 0, 0, stream);
    if (rc)
        return rc;
    rc = plan_common(&Pa, 2, N, M, y, eps, dtype, 0, 0, 0, stream);
    if (rc) {
        release_plan(Pf);
        delete Pf;
        return rc;
    }
    Lsq L;
    const size_t es = dtype == FN_C128 ? 16 : 8;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (Buf *b : {&L.r, &L.s, &L.p, &L.q, &L.part})
            release(*b);
        release_plan(Pf);
        delete Pf;
        release_plan(Pa);
        delete Pa;
    };
    try {
        L.hpart = (double *)pinned_scratch(SOLVE_BLOCKS * sizeof(double));
        if (!alloc(L.r, (size_t)M * es) || !alloc(L.q, (size_t)M * es) ||
            !alloc(L.s, (size_t)N * es) || !alloc(L.p, (size_t)N * es) ||
            !alloc(L.part, SOLVE_BLOCKS * sizeof(double)) || !L.hpart)
            rc = fail(FN_ENOMEM, "least-squares workspace allocation failed");
        else
            rc = dtype == FN_C128
                     ? lsq_run<double>(Pf, Pa, g, f, tol, maxiter, L, st, iters, resid)
                     : lsq_run<float>(Pf, Pa, g, f, tol, maxiter, L, st, iters, resid);
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    return rc;
    FN_API_END
}

int nufft_release_cache(void)
{
    FN_API_BEGIN
    (void)pool_trim();
    return FN_OK;
    FN_API_END
}

const char *nufft_last_error(void) { return g_err.c_str(); }

} // extern "C"
