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
    // operators
    const R *m2m;                // [2][P in][P out]
    const R *bin;                // [P][P] binomial C(t, j) at [t][j]
    const R *reg1, *reg2;        // [P t][P lo]
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
    V *buf0 = reinterpret_cast<V *>(smem_raw);
    __shared__ int s_last;
    const int P = a.P;
    const int tid = threadIdx.x;
    int band = 0;
    int64_t node = blockIdx.x;

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
                V acc = vzero<V>();
                for (int c = 0; c < 2; ++c) {
                    const R *T = a.m2m + (size_t)c * P * P;
                    const V *ch = cur + (size_t)(2 * i + c) * P;
                    for (int m = 0; m <= nn; ++m)
                        vfma(acc, T[m * P + nn], ch[m]);
                }
                nxt[idx] = acc;
                g[idx] = acc;
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
            R cb = a.bin[t * P + j] * pw;
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
            vfma(acc, a.reg1[t * P + lo], n1[t]);
            vfma(acc, a.reg2[t * P + lo], o[t]);
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
    const WorkItem *work;
    const V *mp;
    const V *loc2;
    const R *l2l;     // [2][P in][P out]
    const R *m2l;     // [4][P in][P out], offsets delta = -6, -4, 4, 6
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

// Local expansion coefficient n of box B at level lev: L2L from the parent
// local plus M2L from the interaction list (left child: source offsets
// -2, +2, +3 boxes; right child: -3, -2, +2).  cot kernel coefficients are
// in units of h: M2L carries (N/pi)/r = 2^(lev+1)/pi.  The log kernel adds
// a_0 log r to the constant term (the M2L table holds log|delta|).
template <typename R, typename V, int KER>
__device__ __forceinline__ V down_coeff(const DownArgs<R, V> &a, int lev,
                                        int64_t B, int n, const V *ploc)
{
    const int P = a.P;
    V acc = vzero<V>();
    const R *T = a.l2l + (size_t)(B & 1) * P * P;
    for (int m = n; m < P; ++m)
        vfma(acc, T[m * P + n], ploc[m]);
    const int64_t mask = (int64_t(1) << lev) - 1;
    int offs[3], didx[3];
    if ((B & 1) == 0) {
        offs[0] = -2; didx[0] = 2;  // delta = +4
        offs[1] = 2;  didx[1] = 1;  // delta = -4
        offs[2] = 3;  didx[2] = 0;  // delta = -6
    } else {
        offs[0] = -3; didx[0] = 3;  // delta = +6
        offs[1] = -2; didx[1] = 2;  // delta = +4
        offs[2] = 2;  didx[2] = 1;  // delta = -4
    }
    V far = vzero<V>();
    R a0sum = R(0);
    for (int i = 0; i < 3; ++i) {
        const V *as = a.mp + lev_off(lev, P) + ((B + offs[i]) & mask) * P;
        const R *M = a.m2l + (size_t)didx[i] * P * P;
        for (int m = 0; m < P; ++m)
            vfma(far, M[m * P + n], as[m]);
        if constexpr (KER == KER_LOG)
            a0sum += as[0];
    }
    if constexpr (KER == KER_COT) {
        const R sc = (R)(ldexp(2.0, lev) / 3.14159265358979323846);
        vfma(acc, sc, far);
    } else {
        acc += far;
        if (n == 0)
            acc += a0sum * (R)log(ldexp((double)a.N, -(lev + 1)));
    }
    return acc;
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

// Near field of the cot kernel: sum over the sources of leaves b-1, b, b+1
// (unwrapped around the circle) of w / (tau - sigma~).
template <typename R, typename V, int SRC>
__device__ __forceinline__ cx<R> near_cot(const DownArgs<R, V> &a, int64_t tm,
                                          double tth, int64_t leaf)
{
    const int64_t N = a.N;
    const int64_t nleaf = int64_t(1) << a.l;
    cx<R> acc = {R(0), R(0)};
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
                double d = (double)(tm - k - shift) + tth;
                R rd = R(1) / (R)d;
                cx<R> w = a.f_uniform[k];
                acc.re = fma(w.re, rd, acc.re);
                acc.im = fma(w.im, rd, acc.im);
            }
        } else {
            const int32_t t0 = a.src.off[b], t1 = a.src.off[b + 1];
            for (int32_t t = t0; t < t1; ++t) {
                double d = grid_diff(tm - a.src.m[t] - shift, tth, a.src.th[t]);
                R rd = R(1) / (R)d;
                cx<R> w = a.w_sorted[t];
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
    V *bufA = reinterpret_cast<V *>(smem_raw);
    V *bufB = bufA + ((size_t)1 << s) * P;
    const int tid = threadIdx.x;
    const WorkItem w = a.work[blockIdx.x];
    const int64_t R0 = w.root;
    const int lr = a.lr;

    // local of the subtree root, from level 2 down
    for (int n = tid; n < P; n += BLOCK)
        bufA[n] = a.loc2[(R0 >> (lr - 2)) * P + n];
    __syncthreads();
    V *cur = bufA, *nxt = bufB;
    for (int lev = 3; lev <= lr; ++lev) {
        const int64_t B = R0 >> (lr - lev);
        for (int n = tid; n < P; n += BLOCK)
            nxt[n] = down_coeff<R, V, KER>(a, lev, B, n, cur);
        __syncthreads();
        V *t = cur;
        cur = nxt;
        nxt = t;
    }
    // the subtree's levels
    for (int lev = lr + 1; lev <= a.l; ++lev) {
        const int nb = 1 << (lev - lr);
        const int64_t first = R0 << (lev - lr);
        for (int idx = tid; idx < nb * P; idx += BLOCK) {
            const int i = idx / P, n = idx - i * P;
            nxt[idx] = down_coeff<R, V, KER>(a, lev, first + i, n,
                                             cur + (size_t)(i >> 1) * P);
        }
        __syncthreads();
        V *t = cur;
        cur = nxt;
        nxt = t;
    }
    const V *leafloc = cur;
    const int64_t leaf0 = R0 << s;
    const int64_t N = a.N;

    if constexpr (EPI == EPI_FWD) {
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
            cx<R> nr = near_cot<R, V, SRC>(a, tm, th, leaf);
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
            cx<R> nr = near_cot<R, V, SRC>(a, k, 0.0, leaf);
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
