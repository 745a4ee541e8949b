// The circular-tree FMM of Sections 2.1-2.4 as HIP kernels for gfx950.
//
// One engine serves three sums, all over a 2 pi-periodic kernel split at
// tree level 2 into the neighbourhood Omega_1 (the quarter arc P_n of the
// target and its two neighbours) and the opposite quarter Omega_2:
//
//   cot kernel (Eq. p9):  h(tau) = sum_sigma w_sigma cot(pi (tau - sigma)/N)
//        = (N/pi) sum_{Omega_1} w / (tau - sigma~)      singular part, MLFMM
//          - sum_l (d_l / l!) (y - x_c)^l                regular part, Eq. p20
//   log kernel: sum_sigma log|2 sin(pi (tau - sigma)/N)|  (the logarithms of
//        the products of Eq. p8), split the same way: log|t| over Omega_1 by
//        the MLFMM, and the term-wise integrals of Eq. (10) and (11) (divided
//        by 2) as the regular part.
//
// Kernels:
//   k_up         P2M at the leaves and M2M to level 2, by bands of levels;
//                the last workgroup to finish a band's subtree carries on
//                with the parent subtree (no grid-wide wait), and the last
//                one overall turns the level-2 moments into the level-2
//                local polynomial of the regular part (Eq. p20).
//   k_down_eval  for one subtree of the finest levels: the local expansion
//                of its root from level 2 down (L2L + M2L over interaction
//                lists), the subtree's locals, then every target in it:
//                L2P + near-field P2P + the transform's epilogue.
#pragma once

#include "fmm_device.h"

namespace fn {

enum { KER_COT = 0, KER_LOG = 1 };
enum { SET_UNIFORM = 0, SET_SORTED = 1 };
enum { EPI_FWD = 0, EPI_INV = 1, EPI_LOGCD = 2 };

constexpr int MAX_BANDS = 16;
constexpr int CH = 8;          // moments per thread in P2M
constexpr int BLOCK = 256;

// Points sorted by leaf: off[b]..off[b+1] index the points of leaf b.
struct SortedSet {
    const int32_t *off;
    const int32_t *m;   // integer part of the representative (0..N)
    const double *th;   // fraction in [-1/2, 1/2]
    const int32_t *perm;// sorted position -> input index
};

template <typename V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ double vzero<double>() { return 0.0; }
template <>
__device__ __forceinline__ float vzero<float>() { return 0.0f; }
template <>
__device__ __forceinline__ cx<double> vzero<cx<double>>() { return {0.0, 0.0}; }
template <>
__device__ __forceinline__ cx<float> vzero<cx<float>>() { return {0.0f, 0.0f}; }

template <typename R>
__device__ __forceinline__ void vfma(cx<R> &acc, R t, cx<R> a)
{
    acc.re = fma(t, a.re, acc.re);
    acc.im = fma(t, a.im, acc.im);
}
template <typename R>
__device__ __forceinline__ void vfma(R &acc, R t, R a) { acc = fma(t, a, acc); }

template <typename R>
__device__ __forceinline__ cx<R> vscale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ R vscale(R a, R s) { return a * s; }

template <typename R>
__device__ __forceinline__ void vadd(cx<R> &a, cx<R> b)
{
    a.re += b.re;
    a.im += b.im;
}
template <typename R>
__device__ __forceinline__ void vadd(R &a, R b) { a += b; }

// ------------------------------------------------------------------ k_up

// Operator tables (type R) shared by all plans with the same (P, q, kernel):
//   m2m  [P in m][P out n]  M2M for the left child (centre c_p - r_p/2):
//                           C(n,m) 2^-n (-1)^(n-m); the right child differs
//                           by (-1)^(n-m)
//   l2l  [P in n][P out m]  L2L to the left child, same coefficients
//   m2l4, m2l6 [P in m][P out n]  M2L for delta = (c_t - c_s)/r = +4, +6;
//                           delta = -4, -6 differ by (-1)^(m+n+1) (cot
//                           kernel) or (-1)^(m+n) (log kernel)
//   bin  [P][P]             C(t, j) at [t][j]
//   reg1, reg2 [P t][P lo]  level-2 regular part (Eq. p20 and its log analogue)
template <typename R>
struct OpTables {
    const R *m2m, *l2l, *m2l4, *m2l6, *bin, *reg1, *reg2;
};

template <typename R, typename V>
struct UpArgs {
    int64_t N;
    int l, P, nbands;
    int band_lo[MAX_BANDS]; // bottom level of each band
    int band_d[MAX_BANDS];  // levels the band climbs
    int cnt_off[MAX_BANDS + 1];
    int *cnt;               // arrival counters, zero between launches
    // sources
    SortedSet src;
    const cx<R> *f_uniform;      // forward: f_k at the uniform points
    const cx<double> *dhat;      // inverse: Dhat_j in sorted order
    const cx<R> *gin;            // inverse: g_j in input order
    cx<R> *w_out;                // inverse: w_j = Dhat_j g_j (sorted)
    // outputs
    V *mp;                       // multipoles, levels 2..l
    V *loc2;                     // level-2 local polynomials, 4 x P
    V *S;                        // sum of the weights (cot kernel)
    OpTables<R> T;
    double logc1, logc2;         // log kernel: log(2 pi / N), log 2
};

// P2M at leaf b (cot or log kernel) for CH consecutive moments m0..m0+CH-1.
// Moments are a_m = sum w (sigma - c)^m / r^m over the leaf's sources; the
// log kernel takes unit weights minus the uniform density of one point per
// grid unit (whose moments are 2r/(m+1) for even m).
template <typename R, typename V, int KER, int SRC>
__device__ __forceinline__ void p2m_chunk(const UpArgs<R, V> &a, int64_t b,
                                          int m0, V *acc, bool store_w)
{
    const int l = a.l;
    const int64_t N = a.N;
    for (int c = 0; c < CH; ++c)
        acc[c] = vzero<V>();
    if constexpr (SRC == SET_UNIFORM) {
        const int64_t k0 = uni_start(b, l, N), k1 = uni_start(b + 1, l, N);
        for (int64_t k = k0; k < k1; ++k) {
            R v = (R)rel_coord(k, 0.0, b, l, N);
            R pw = ipow(v, m0);
            V w;
            if constexpr (KER == KER_COT)
                w = a.f_uniform[k];
            else
                w = R(1);
            for (int c = 0; c < CH; ++c) {
                vfma(acc[c], pw, w);
                pw *= v;
            }
        }
    } else {
        const int32_t t0 = a.src.off[b], t1 = a.src.off[b + 1];
        for (int32_t t = t0; t < t1; ++t) {
            R v = (R)rel_coord(a.src.m[t], a.src.th[t], b, l, N);
            R pw = ipow(v, m0);
            V w;
            if constexpr (KER == KER_COT) {
                cx<double> d = a.dhat[t];
                cx<R> g = a.gin[a.src.perm[t]];
                w = {(R)(d.re * (double)g.re - d.im * (double)g.im),
                     (R)(d.re * (double)g.im + d.im * (double)g.re)};
                if (store_w)
                    a.w_out[t] = w;
            } else {
                w = R(1);
            }
            for (int c = 0; c < CH; ++c) {
                vfma(acc[c], pw, w);
                pw *= v;
            }
        }
    }
    if constexpr (KER == KER_LOG) {
        const double r = ldexp((double)N, -(l + 1));
        for (int c = 0; c < CH; ++c) {
            int m = m0 + c;
            if ((m & 1) == 0)
                acc[c] -= (R)(2.0 * r / (double)(m + 1));
        }
    }
}

template <typename R, typename V, int KER, int SRC>
__global__ void __launch_bounds__(BLOCK) k_up(UpArgs<R, V> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = a.P;
    R *tm2m = reinterpret_cast<R *>(smem_raw);
    V *buf0 = reinterpret_cast<V *>(tm2m + P * P);
    __shared__ int s_last;
    const int tid = threadIdx.x;
    int band = 0;
    int64_t node = blockIdx.x;

    for (int i = tid; i < P * P; i += BLOCK)
        tm2m[i] = a.T.m2m[i];

    for (;;) {
        const int lb = a.band_lo[band];
        const int d = a.band_d[band];
        const int nbot = 1 << d;
        const int64_t first = node << d;
        V *buf1 = buf0 + (size_t)nbot * P;
        if (band == 0) {
            const int nch = P / CH;
            V *g = a.mp + lev_off(lb, P);
            for (int idx = tid; idx < nbot * nch; idx += BLOCK) {
                const int i = idx / nch, ch = idx - i * nch;
                V acc[CH];
                p2m_chunk<R, V, KER, SRC>(a, first + i, ch * CH, acc, ch == 0);
                for (int c = 0; c < CH; ++c) {
                    buf0[i * P + ch * CH + c] = acc[c];
                    g[(first + i) * P + ch * CH + c] = acc[c];
                }
            }
        } else {
            const V *g = a.mp + lev_off(lb, P) + first * P;
            for (int idx = tid; idx < nbot * P; idx += BLOCK)
                buf0[idx] = g[idx];
        }
        __syncthreads();

        // M2M up the band: a^parent_n = sum_c sum_{m<=n} M2M_c[m][n] a^c_m
        V *cur = buf0, *nxt = buf1;
        int n = nbot;
        for (int lev = lb - 1; lev >= lb - d; --lev) {
            n >>= 1;
            const int64_t pfirst = first >> (lb - lev);
            V *g = a.mp + lev_off(lev, P) + pfirst * P;
            for (int idx = tid; idx < n * P; idx += BLOCK) {
                const int i = idx / P, nn = idx - i * P;
                const V *cl = cur + (size_t)(2 * i) * P;
                const V *cr = cl + P;
                V al = vzero<V>(), ar = vzero<V>();
                for (int m = nn; m >= 0; m -= 2) {   // n - m even
                    const R t = tm2m[m * P + nn];
                    vfma(al, t, cl[m]);
                    vfma(ar, t, cr[m]);
                }
                for (int m = nn - 1; m >= 0; m -= 2) { // n - m odd
                    const R t = tm2m[m * P + nn];
                    vfma(al, t, cl[m]);
                    vfma(ar, -t, cr[m]);
                }
                vadd(al, ar);
                nxt[idx] = al;
                g[idx] = al;
            }
            __syncthreads();
            V *t = cur;
            cur = nxt;
            nxt = t;
        }

        // hand the subtree root to the parent band
        __threadfence();
        __syncthreads();
        const int nb1 = band + 1;
        const int dn = (nb1 < a.nbands) ? a.band_d[nb1] : 2;
        const int64_t parent = node >> dn;
        if (tid == 0) {
            int *c = a.cnt + a.cnt_off[nb1] + parent;
            int old = atomicAdd(c, 1);
            s_last = (old == (1 << dn) - 1);
            if (s_last)
                atomicExch(c, 0);
        }
        __syncthreads();
        if (!s_last)
            return;
        __threadfence();
        node = parent;
        band = nb1;
        if (band == a.nbands)
            break;
    }

    // ---- level 2: regular part of Eq. (p20) as the level-2 local polynomial
    V *a2 = buf0;          // [4][P] level-2 moments about the quarter centres
    V *A1 = buf0 + 4 * P;  // [4][P] moments of Omega_1(P_n) about c_n
    for (int idx = tid; idx < 4 * P; idx += BLOCK)
        a2[idx] = a.mp[idx];
    __syncthreads();
    for (int idx = tid; idx < 4 * P; idx += BLOCK) {
        const int q = idx / P, t = idx - q * P;
        // (v + 2i)^t expanded, i = -1, 0, +1 (unwrapped neighbours)
        V acc = a2[q * P + t];
        const V *lft = a2 + ((q + 3) & 3) * P;
        const V *rgt = a2 + ((q + 1) & 3) * P;
        R pw = R(1);
        for (int j = t; j >= 0; --j) {
            R cb = a.T.bin[t * P + j] * pw;
            vfma(acc, cb, rgt[j]);
            vfma(acc, ((t - j) & 1) ? -cb : cb, lft[j]);
            pw *= R(2);
        }
        A1[idx] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < 4 * P; idx += BLOCK) {
        const int q = idx / P, lo = idx - q * P;
        const V *o = a2 + ((q + 2) & 3) * P;
        const V *n1 = A1 + q * P;
        V acc = vzero<V>();
        for (int t = 0; t < P; ++t) {
            vfma(acc, a.T.reg1[t * P + lo], n1[t]);
            vfma(acc, a.T.reg2[t * P + lo], o[t]);
        }
        if constexpr (KER == KER_LOG) {
            if (lo == 0)
                acc += (R)(a.logc1 * (double)n1[0] + a.logc2 * (double)o[0]);
        }
        a.loc2[idx] = acc;
    }
    if constexpr (KER == KER_COT) {
        if (tid == 0) {
            V s = a2[0];
            vadd(s, a2[P]);
            vadd(s, a2[2 * P]);
            vadd(s, a2[3 * P]);
            *a.S = s;
        }
    }
}

// ------------------------------------------------------------ k_down_eval

struct WorkItem {
    int64_t root;      // subtree root at level lr
    int32_t t0, t1;    // sorted-target range
    int32_t u0, u1;    // uniform-target range
};

template <typename R, typename V>
struct DownArgs {
    int64_t N;
    int l, P, lr;
    int nbuf;                // rows of each LDS local buffer: max(2^s, lr)
    int near_cap;            // LDS slots for the forward near-field sources
    const WorkItem *work;
    const V *mp;
    const V *loc2;
    OpTables<R> T;
    // sources of the near field
    SortedSet src;
    const cx<R> *f_uniform;
    const cx<R> *w_sorted;
    // targets
    SortedSet tgt;
    // epilogues
    cx<R> *out;              // FWD: g (input order); INV: f
    const V *S;              // sum of the weights
    const cx<R> *f_hit;      // FWD: f (exact hits)
    const double *chat;      // INV: Chat_k
    const int32_t *hit;      // INV: source index j with y_j = x_k, or -1
    const cx<R> *gin;        // INV: g (input order)
    double *logc, *logd;     // LOGCD outputs
    double logself;          // LOGCD: log(2 pi / N), the excluded self term
};

// M2L of the three interaction-list boxes of box B at level lev onto output
// coefficient n (left child: source offsets -2, +2, +3 boxes, i.e. delta =
// +4, -4, -6; right child: -3, -2, +2, i.e. delta = +6, +4, -4).  srcrow(o)
// returns the multipole of box B + o.  cot coefficients are in units of h:
// the 1/t M2L carries (N/pi)/r = 2^(lev+1)/pi.  The log kernel adds
// a_0 log r to the constant term (its tables hold log|delta|).
template <typename R, typename V, int KER, typename SrcRow>
__device__ __forceinline__ V m2l_coeff(const R *t4, const R *t6, int P,
                                       int lev, int64_t B, int n, int64_t N,
                                       SrcRow srcrow)
{
    // sign of T_{-delta} relative to T_delta: (-1)^(m+n+1) (cot), (-1)^(m+n) (log)
    const bool neg_odd = ((n + (KER == KER_COT ? 1 : 0)) & 1) != 0;
    V pos = vzero<V>(), neg = vzero<V>();
    R a0 = R(0);
    const bool left = (B & 1) == 0;
    const V *s_p4 = srcrow(-2);              // delta = +4: offset -2
    const V *s_m4 = srcrow(2);               // delta = -4: offset +2
    const V *s_6 = srcrow(left ? 3 : -3);    // delta = -6 (left) / +6 (right)
    for (int m = 0; m < P; ++m) {
        const R a4 = t4[m * P + n];
        const R a6 = t6[m * P + n];
        vfma(pos, a4, s_p4[m]);
        // T_{-4}[m][n] = +-(-1)^m T_4[m][n]
        const R sm = (m & 1) ? -a4 : a4;
        vfma(neg, sm, s_m4[m]);
        if (left) {
            const R s6 = (m & 1) ? -a6 : a6;
            vfma(neg, s6, s_6[m]);
        } else {
            vfma(pos, a6, s_6[m]);
        }
    }
    if (neg_odd)
        neg = vscale(neg, R(-1));
    vadd(pos, neg);
    if constexpr (KER == KER_COT) {
        return vscale(pos, (R)(ldexp(2.0, lev) / 3.14159265358979323846));
    } else {
        if (n == 0) {
            a0 = (R)((double)s_p4[0] + (double)s_m4[0] + (double)s_6[0]);
            pos += a0 * (R)log(ldexp((double)N, -(lev + 1)));
        }
        return pos;
    }
}

template <typename R, typename V>
__device__ __forceinline__ V horner(const V *c, int P, R u)
{
    V acc = c[P - 1];
    for (int n = P - 2; n >= 0; --n) {
        V t = vscale(acc, u);
        vadd(t, c[n]);
        acc = t;
    }
    return acc;
}

// 1/d to full binary64 (or binary32) precision: hardware reciprocal refined
// by Newton steps.
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float d)
{
    float r = __builtin_amdgcn_rcpf(d);
    float e = fmaf(-d, r, 1.0f);
    return fmaf(r, e, r);
}

// Near field of the cot kernel: sum over the sources of leaves b-1, b, b+1
// (unwrapped around the circle) of w / (tau - sigma~).
template <typename R, typename V, int SRC>
__device__ __forceinline__ cx<R> near_cot(const DownArgs<R, V> &a, int64_t tm,
                                          double tth, int64_t leaf,
                                          const cx<R> *fs, int64_t K0)
{
    const int64_t N = a.N;
    const int64_t nleaf = int64_t(1) << a.l;
    cx<R> acc = {R(0), R(0)};
    if constexpr (SRC == SET_UNIFORM) {
        if (fs) { // sources staged in LDS from unwrapped index K0 on
            auto ustart = [&](int64_t b) {
                if (b < 0)
                    return uni_start(b + nleaf, a.l, N) - N;
                if (b > nleaf)
                    return uni_start(b - nleaf, a.l, N) + N;
                return uni_start(b, a.l, N);
            };
            const int64_t k0 = ustart(leaf - 1), k1 = ustart(leaf + 2);
            for (int64_t k = k0; k < k1; ++k) {
                const R rd = recip((R)((double)(tm - k) + tth));
                const cx<R> w = fs[k - K0];
                acc.re = fma(w.re, rd, acc.re);
                acc.im = fma(w.im, rd, acc.im);
            }
            return acc;
        }
    }
    for (int dl = -1; dl <= 1; ++dl) {
        int64_t b = leaf + dl, shift = 0;
        if (b < 0) {
            b += nleaf;
            shift = -N;
        } else if (b >= nleaf) {
            b -= nleaf;
            shift = N;
        }
        if constexpr (SRC == SET_UNIFORM) {
            const int64_t k0 = uni_start(b, a.l, N), k1 = uni_start(b + 1, a.l, N);
            for (int64_t k = k0; k < k1; ++k) {
                const R rd = recip((R)((double)(tm - k - shift) + tth));
                const cx<R> w = a.f_uniform[k];
                acc.re = fma(w.re, rd, acc.re);
                acc.im = fma(w.im, rd, acc.im);
            }
        } else {
            const int32_t t0 = a.src.off[b], t1 = a.src.off[b + 1];
            for (int32_t t = t0; t < t1; ++t) {
                const double d = grid_diff(tm - a.src.m[t] - shift, tth, a.src.th[t]);
                const R rd = recip((R)d);
                const cx<R> w = a.w_sorted[t];
                acc.re = fma(w.re, rd, acc.re);
                acc.im = fma(w.im, rd, acc.im);
            }
        }
    }
    return acc;
}

// Near field of the log kernel with the uniform background removed:
// sum log|tau - sigma~| over the sources of leaves b-1..b+1 (skipping the
// source `self`), minus the integral of log|tau - sigma| over those leaves.
template <typename R, typename V>
__device__ __forceinline__ double near_log(const DownArgs<R, V> &a, int64_t tm,
                                           double tth, int64_t leaf,
                                           int32_t self)
{
    const int64_t N = a.N;
    const int l = a.l;
    const int64_t nleaf = int64_t(1) << l;
    double acc = 0.0;
    for (int dl = -1; dl <= 1; ++dl) {
        int64_t b = leaf + dl, shift = 0;
        if (b < 0) {
            b += nleaf;
            shift = -N;
        } else if (b >= nleaf) {
            b -= nleaf;
            shift = N;
        }
        const int32_t t0 = a.src.off[b], t1 = a.src.off[b + 1];
        for (int32_t t = t0; t < t1; ++t) {
            if (t == self)
                continue;
            double d = grid_diff(tm - a.src.m[t] - shift, tth, a.src.th[t]);
            acc += log(fabs(d));
        }
    }
    // integral over [(leaf-1) N/2^l, (leaf+2) N/2^l) (unwrapped)
    const double sc = ldexp(1.0, -l);
    double lo = (double)((leaf - 1) * N - (tm << l)) * sc - tth;
    double hi = (double)((leaf + 2) * N - (tm << l)) * sc - tth;
    return acc - (xlogx_m_x(hi) - xlogx_m_x(lo));
}

template <typename R, typename V, int KER, int SRC, int EPI>
__global__ void __launch_bounds__(BLOCK) k_down_eval(DownArgs<R, V> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int P = a.P;
    const int s = a.l - a.lr;
    const int PP = P * P;
    R *t4 = reinterpret_cast<R *>(smem_raw);
    R *t6 = t4 + PP;
    R *tll = t6 + PP;
    V *bufA = reinterpret_cast<V *>(tll + PP);
    V *bufB = bufA + (size_t)a.nbuf * P;
    V *srcs = bufB + (size_t)a.nbuf * P;       // (2^s + 6) x P
    // near-field staging reuses the source buffer once the translations are
    // done (near_cap slots of cx<R>)
    cx<R> *fs = reinterpret_cast<cx<R> *>(srcs);
    const int tid = threadIdx.x;
    const WorkItem w = a.work[blockIdx.x];
    const int64_t R0 = w.root;
    const int lr = a.lr;
    const int64_t N = a.N;

    for (int i = tid; i < PP; i += BLOCK) {
        t4[i] = a.T.m2l4[i];
        t6[i] = a.T.m2l6[i];
        tll[i] = a.T.l2l[i];
    }
    __syncthreads();

    // ---- local expansion of the subtree root R0 (level lr).  The local of
    // a box is the sum over its ancestors A_L (L = 2..lr) of the M2L result
    // at A_L (the regular-part polynomial for L = 2) shifted straight from
    // the centre of A_L to the centre of R0:
    //   u_A = rho u_R + delta,  b^R_n = sum_{n'>=n} C(n',n) rho^n delta^(n'-n) b^A_n'.
    const int nL = lr - 1; // levels 2..lr
    V *X = bufA;           // X[L-2][n]
    V *Y = bufB;
    for (int idx = tid; idx < nL * P; idx += BLOCK) {
        const int li = idx / P, n = idx - li * P;
        const int L = li + 2;
        const int64_t A = R0 >> (lr - L);
        if (L == 2) {
            X[idx] = a.loc2[A * P + n];
        } else {
            const int64_t mask = (int64_t(1) << L) - 1;
            const V *base = a.mp + lev_off(L, P);
            X[idx] = m2l_coeff<R, V, KER>(t4, t6, P, L, A, n, N, [&](int o) {
                return base + ((A + o) & mask) * P;
            });
        }
    }
    __syncthreads();
    for (int idx = tid; idx < nL * P; idx += BLOCK) {
        const int li = idx / P, n = idx - li * P;
        const int L = li + 2;
        const int64_t A = R0 >> (lr - L);
        const int sh = lr - L;
        // rho = 2^-sh; delta = ((2 R0 + 1) - (2A + 1) 2^sh) / 2^sh
        const R rho2 = (R)ldexp(2.0, -sh);                     // 2 rho
        const R md2 = (R)(-2.0 * ldexp((double)((2 * R0 + 1) - ((2 * A + 1) << sh)), -sh));
        // C(n',n) = tll[n'][n] 2^n' (-1)^(n'-n) = tll[n'][n] 2^n (-2)^(n'-n)
        const V *x = X + li * P;
        V acc = vzero<V>();
        R pw = R(1);
        for (int np = n; np < P; ++np) {
            vfma(acc, tll[np * P + n] * pw, x[np]);
            pw *= md2;
        }
        Y[idx] = vscale(acc, ipow(rho2, n));
    }
    __syncthreads();
    V *cur = bufA, *nxt = bufB;
    for (int n = tid; n < P; n += BLOCK) {
        V acc = Y[n];
        for (int li = 1; li < nL; ++li)
            vadd(acc, Y[li * P + n]);
        cur[n] = acc; // X is no longer needed
    }
    __syncthreads();

    // ---- the subtree's levels: L2L from the parent + M2L from the level's
    // interaction lists (sources staged in LDS)
    for (int lev = lr + 1; lev <= a.l; ++lev) {
        const int nb = 1 << (lev - lr);
        const int64_t first = R0 << (lev - lr);
        const int64_t mask = (int64_t(1) << lev) - 1;
        const V *base = a.mp + lev_off(lev, P);
        for (int idx = tid; idx < (nb + 6) * P; idx += BLOCK) {
            const int i = idx / P, m = idx - i * P;
            srcs[idx] = base[((first - 3 + i) & mask) * P + m];
        }
        __syncthreads();
        for (int idx = tid; idx < nb * P; idx += BLOCK) {
            const int i = idx / P, n = idx - i * P;
            const int64_t B = first + i;
            const V *par = cur + (size_t)(i >> 1) * P;
            V acc = vzero<V>();
            if ((B & 1) == 0) {
                for (int m = n; m < P; ++m)
                    vfma(acc, tll[m * P + n], par[m]);
            } else {
                for (int m = n; m < P; ++m) {
                    const R t = tll[m * P + n];
                    vfma(acc, ((m - n) & 1) ? -t : t, par[m]);
                }
            }
            V far = m2l_coeff<R, V, KER>(t4, t6, P, lev, B, n, N, [&](int o) {
                return srcs + (size_t)(i + 3 + o) * P;
            });
            vadd(acc, far);
            nxt[idx] = acc;
        }
        __syncthreads();
        V *t = cur;
        cur = nxt;
        nxt = t;
    }
    const V *leafloc = cur;
    const int64_t leaf0 = R0 << s;

    if constexpr (EPI == EPI_FWD) {
        // stage the near-field sources of the subtree (uniform sources)
        const cx<R> *fsp = nullptr;
        int64_t K0 = 0;
        if constexpr (SRC == SET_UNIFORM) {
            const int64_t nleaf = int64_t(1) << a.l;
            auto ustart = [&](int64_t b) {
                if (b < 0)
                    return uni_start(b + nleaf, a.l, N) - N;
                if (b > nleaf)
                    return uni_start(b - nleaf, a.l, N) + N;
                return uni_start(b, a.l, N);
            };
            K0 = ustart(leaf0 - 1);
            const int64_t K1 = ustart(leaf0 + (1 << s) + 1);
            if (K1 - K0 <= a.near_cap) {
                for (int64_t i = tid; i < K1 - K0; i += BLOCK) {
                    int64_t k = K0 + i;
                    k = k < 0 ? k + N : (k >= N ? k - N : k);
                    fs[i] = a.f_uniform[k];
                }
                fsp = fs;
            }
            __syncthreads();
        }
        const V S = *a.S;
        const double hscale = (double)N / 3.14159265358979323846;
        for (int32_t t = w.t0 + tid; t < w.t1; t += BLOCK) {
            const int64_t tm = a.tgt.m[t];
            const double th = a.tgt.th[t];
            const int32_t j = a.tgt.perm[t];
            if (th == 0.0) { // exact hit: K_jk is the Kronecker delta
                a.out[j] = a.f_hit[tm == N ? 0 : tm];
                continue;
            }
            const int64_t leaf = box_of(tm, th, a.l, N);
            const R u = (R)rel_coord(tm, th, leaf, a.l, N);
            V h = horner<R, V>(leafloc + (leaf - leaf0) * P, P, u);
            cx<R> nr = near_cot<R, V, SRC>(a, tm, th, leaf, fsp, K0);
            double hr = (double)h.re + hscale * (double)nr.re;
            double hi = (double)h.im + hscale * (double)nr.im;
            // g = -(F/2)(S + i h), F = 2i sin(pi th) e^{i pi th} / N
            double sp = sinpi(th), cp = cospi(th);
            double Fr = -2.0 * sp * sp / (double)N, Fi = 2.0 * sp * cp / (double)N;
            double Ar = (double)S.re - hi, Ai = (double)S.im + hr;
            cx<R> g = {(R)(-0.5 * (Fr * Ar - Fi * Ai)), (R)(-0.5 * (Fr * Ai + Fi * Ar))};
            a.out[j] = g;
        }
    } else if constexpr (EPI == EPI_INV) {
        const V W = *a.S;
        const double hscale = (double)N / 3.14159265358979323846;
        for (int32_t k = w.u0 + tid; k < w.u1; k += BLOCK) {
            const int32_t hj = a.hit[k];
            if (hj >= 0) { // exact hit: C_k = 0 and f_k = g_j
                a.out[k] = a.gin[hj];
                continue;
            }
            const int64_t leaf = box_of(k, 0.0, a.l, N);
            const R u = (R)rel_coord(k, 0.0, leaf, a.l, N);
            V h = horner<R, V>(leafloc + (leaf - leaf0) * P, P, u);
            cx<R> nr = near_cot<R, V, SRC>(a, k, 0.0, leaf, nullptr, 0);
            double hr = (double)h.re + hscale * (double)nr.re;
            double hi = (double)h.im + hscale * (double)nr.im;
            // f = -(C/2)(W + i h)
            const double C = a.chat[k];
            a.out[k] = {(R)(-0.5 * C * ((double)W.re - hi)),
                        (R)(-0.5 * C * ((double)W.im + hr))};
        }
    } else { // EPI_LOGCD
        for (int32_t k = w.u0 + tid; k < w.u1; k += BLOCK) {
            const int64_t leaf = box_of(k, 0.0, a.l, N);
            const R u = (R)rel_coord(k, 0.0, leaf, a.l, N);
            V far = horner<R, V>(leafloc + (leaf - leaf0) * P, P, u);
            a.logc[k] = (double)far + near_log<R, V>(a, k, 0.0, leaf, -1);
        }
        for (int32_t t = w.t0 + tid; t < w.t1; t += BLOCK) {
            const int64_t tm = a.tgt.m[t];
            const double th = a.tgt.th[t];
            const int64_t leaf = box_of(tm, th, a.l, N);
            const R u = (R)rel_coord(tm, th, leaf, a.l, N);
            V far = horner<R, V>(leafloc + (leaf - leaf0) * P, P, u);
            // the net count of Omega_1 carried log(2 pi / N) for the point
            // itself, whose log|t| term the near field skips
            a.logd[t] = -((double)far + near_log<R, V>(a, tm, th, leaf, t) - a.logself);
        }
    }
}

} // namespace fn
