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
// Expansions: multipoles carry PU terms (PU >= 2q: the level-2 moments feed
// the regular part up to degree 2q - 1); locals and translations carry
// PD <= PU terms (the MLFMM truncation p, rounded up to the 16-row tiles of
// the matrix cores).  Coefficients live in LDS as rows of RS elements of
// type R (complex data interleaved re, im), RS padded so that the matrix-core
// operand loads are free of bank conflicts.
//
// Kernels:
//   k_up_band    P2M at the leaves (first band) or a load of the band's
//                bottom multipoles, then M2M up the band (matrix cores); the
//                last band ends at level 2.
//   k_m2l        the M2L of every box of levels 3..l (matrix cores), and in
//                one workgroup the level-2 local polynomial of the regular
//                part (Eq. p20) from the four level-2 multipoles.
//   k_down_trans one subtree of the finest levels: the local of its root as
//                the sum of the ancestors' M2L results shifted straight to
//                the root, then the subtree's levels, each box's M2L result
//                plus the L2L of its parent (matrix cores), down to the leaf
//                locals.
//   k_down_eval  every target of a subtree: L2P + near-field P2P + the
//                transform epilogue.
#pragma once

#include "fmm_device.h"

namespace fn {

enum { KER_COT = 0, KER_LOG = 1 };
enum { SET_UNIFORM = 0, SET_SORTED = 1 };
enum { EPI_FWD = 0, EPI_INV = 1, EPI_LOGCD = 2, EPI_ADJ = 3 };

constexpr int BLOCK = 256; // 4 wavefronts of 64
constexpr int FWD_TMAX = 2048; // forward: most targets of one work item

// Binary32 sums of the near field and of the vector P2M run over blocks of
// at most this many terms; each block's partial is added into a binary64
// total.  The rounding error of a sum then stays at that of a block,
// whatever the number of sources in a leaf.  Binary64 sums are not split.
template <typename R>
__host__ __device__ constexpr int32_t fold_len()
{
    return sizeof(R) == 8 ? INT32_MAX : 256;
}
constexpr int P2M_FOLD = 64; // sources per binary32 block of the vector P2M

// Points sorted by leaf: off[b]..off[b+1] index the points of leaf b.
struct SortedSet {
    const int32_t *off;
    const int32_t *m;    // integer part of the representative (0..N)
    const double *th;    // fraction in [-1/2, 1/2]
    const int32_t *perm; // sorted position -> input index
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

// Number of real components of a coefficient type.
template <typename V>
struct ncomp { static constexpr int value = 1; };
template <typename R>
struct ncomp<cx<R>> { static constexpr int value = 2; };

// Coefficient n of row `row` of an LDS coefficient array.
template <typename R, typename V>
__device__ __forceinline__ V ld_coef(const R *base, int RS, int row, int n)
{
    if constexpr (ncomp<V>::value == 2) {
        const R *p = base + (size_t)row * RS + 2 * n;
        return V{p[0], p[1]};
    } else {
        return base[(size_t)row * RS + n];
    }
}
template <typename R, typename V>
__device__ __forceinline__ void st_coef(R *base, int RS, int row, int n, V v)
{
    if constexpr (ncomp<V>::value == 2) {
        R *p = base + (size_t)row * RS + 2 * n;
        p[0] = v.re;
        p[1] = v.im;
    } else {
        base[(size_t)row * RS + n] = v;
    }
}

// ------------------------------------------------------------ matrix cores

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename R>
struct acc_t;
template <>
struct acc_t<double> { typedef d4 type; };
template <>
struct acc_t<float> { typedef f4 type; };

// D(16x16) += A(16x4) B(4x16).  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; it receives D rows out_row(l, r), r = 0..3, of column
// l % 16 (binary64 interleaves the rows, binary32 blocks them).
__device__ __forceinline__ d4 mma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename R>
__device__ __forceinline__ int out_row(int lane, int r)
{
    if constexpr (sizeof(R) == 8)
        return 4 * r + (lane >> 4);
    else
        return 4 * (lane >> 4) + r;
}

// Operator tables (type R) shared by all plans with the same (PU, PD, q,
// kernel), each stored [input index][output index]:
//   m2m  PU x PU   M2M from the left child (centre c_p - r_p/2):
//                  C(n,m) 2^-n (-1)^(n-m); the right child differs by (-1)^(n-m)
//   l2l  PD x PD   L2L to the left child, same coefficients
//   m2l4, m2l6 PD x PD  M2L for delta = (c_t - c_s)/r = +4, +6; delta = -4, -6
//                  differ by (-1)^(m+n+1) (cot kernel) or (-1)^(m+n) (log)
//   reg1, reg2 PU x PD  level-2 regular part (Eq. p20 and its log analogue):
//                  the weights of the moments of Omega_1 and of the opposite
//                  quarter about the quarter's centre
//   regR, regL PU x PD  reg1 composed with the shift of the right (left)
//                  neighbour's moments to the quarter's centre,
//                  regR[j][lo] = sum_{t>=j} reg1[t][lo] C(t,j) 2^(t-j), regL
//                  the same with the sign (-1)^(t-j)
template <typename R>
struct OpTables {
    const R *m2m, *l2l, *m2l4, *m2l6, *regR, *regL, *reg1, *reg2;
};

// A-operands of one 16-row tile of a square operator, held in registers:
// a[ks] = T[row = 16 rt + lane % 16][k = 4 ks + lane / 16] = tab[k][row].
template <typename R, int K>
__device__ __forceinline__ void load_tile(R (&a)[K / 4], const R *tab, int rt,
                                          int lane)
{
    const int row = 16 * rt + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < K / 4; ++ks)
        a[ks] = tab[(4 * ks + (lane >> 4)) * K + row];
}

// ------------------------------------------------------------------ k_up

template <typename R, typename V>
struct UpArgs {
    int64_t N;
    int l;          // leaf level
    int lb, d;      // this launch: bottom level and levels climbed
    int RS;         // LDS row stride (elements of R)
    int PD;         // local expansion terms (level-2 polynomial)
    int first_band;
    int leaf_pts;   // uniform sources: points per leaf if every leaf holds
                    // the same number (N divisible by 2^l, a multiple of 4
                    // up to 64), else 0
    int stage_cap;  // first band, sorted sources: sources of one launch's
                    // leaves that fit in its LDS staging area
    const int32_t *src_leaf; // sorted sources: leaf of every source
    // sources (first band)
    SortedSet src;
    const cx<R> *f_uniform;  // forward: f_k at the uniform points
    const cx<R> *w_sorted;   // inverse: w_j = Dhat_j g_j (sorted)
    // outputs
    V *mp;                   // multipoles, levels 2..l, PU per box
    V *loc2;                 // level-2 local polynomials, 4 x PD
    V *S;                    // sum of the weights (cot kernel)
    OpTables<R> T;
    double logc1, logc2;     // log kernel: log(2 pi / N), log 2
    int32_t io_index;        // batched launches: entry of the IoPtr table
};

// Inverse: w_j = Dhat_j g_j in sorted order (Eq. p6: the weights of the cot
// sum).
template <typename R>
__global__ void k_weights(int64_t n, const cx<double> *dhat, const int32_t *perm,
                          const cx<R> *g, cx<R> *w)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const cx<double> d = dhat[t];
        const cx<R> x = g[perm[t]];
        w[t] = {(R)(d.re * (double)x.re - d.im * (double)x.im),
                (R)(d.re * (double)x.im + d.im * (double)x.re)};
    }
}

// Adjoint weights in sorted order: w_t = conj(F_t) g_perm(t), with
// F = (e^{i N y} - 1) / N = 2i sin(pi th) e^{i pi th} / N (Eq. p4-p5), so
// conj(F) = -(2 / N) sin(pi th) (sin(pi th) + i cos(pi th)).
template <typename R>
__global__ void k_adj_weights(int64_t n, int64_t N, const double *sth, const int32_t *perm,
                              const cx<R> *g, cx<R> *w)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    const double th = sth[t];
    const double sp = sinpi(th), cp = cospi(th);
    const double a = -2.0 * sp / (double)N;
    const double Fr = a * sp, Fi = a * cp; // conj(F)
    const cx<R> gv = g[perm[t]];
    w[t] = {(R)(Fr * (double)gv.re - Fi * (double)gv.im),
            (R)(Fr * (double)gv.im + Fi * (double)gv.re)};
}

// Adjoint, sources on grid points: conj(K_jk) = delta(k, m_j), so f_m gets
// g_j (after the evaluation wrote f; several sources may share a point).
template <typename R>
__global__ void k_adj_hits(int64_t n, const int32_t *sm, const double *sth,
                           const int32_t *perm, const cx<R> *g, cx<R> *f)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n || sth[t] != 0.0)
        return;
    const cx<R> gv = g[perm[t]];
    R *fp = reinterpret_cast<R *>(f + sm[t]);
    atomicAdd(fp, gv.re);
    atomicAdd(fp + 1, gv.im);
}

constexpr int CHS = 4; // moments per thread in the vector P2M

// Leaf of the uniform point k: floor(k 2^l / N), from a binary64 estimate
// (off by at most one) corrected with exact integer box starts.
__device__ __forceinline__ int64_t uni_leaf(int64_t k, int l, int64_t N, double scale)
{
    int64_t b = (int64_t)((double)k * scale);
    if (uni_start(b + 1, l, N) <= k)
        ++b;
    else if (uni_start(b, l, N) > k)
        --b;
    return b;
}


// Binary64 accumulator of a binary32 moment (the vector P2M's blocks).
template <typename V>
struct wide { typedef V type; };
template <>
struct wide<cx<float>> { typedef cx<double> type; };
template <>
struct wide<float> { typedef double type; };

__device__ __forceinline__ void vacc(cx<double> &t, cx<float> v)
{
    t.re += (double)v.re;
    t.im += (double)v.im;
}
__device__ __forceinline__ void vacc(double &t, float v) { t += (double)v; }
template <typename V>
__device__ __forceinline__ V vnarrow(typename wide<V>::type t)
{
    if constexpr (ncomp<V>::value == 2)
        return {(decltype(V::re))t.re, (decltype(V::re))t.im};
    else
        return (V)t;
}

// P2M at leaf b for CHS consecutive moments m0..: a_m = sum w v^m with
// v = (sigma - c)/r.  The log kernel takes unit weights minus the uniform
// density of one point per grid unit (moments 2r/(m+1) for even m).  The
// sources are read in place (they did not fit in LDS); binary32 terms are
// summed in binary64.
template <typename R, typename V, int KER, int SRC>
__device__ __forceinline__ void p2m_chunk(const UpArgs<R, V> &a, const cx<R> *fu, int64_t b,
                                          int m0, V *acc)
{
    using W = typename wide<V>::type;
    const int l = a.l;
    const int64_t N = a.N;
    W tot[CHS];
    for (int c = 0; c < CHS; ++c)
        tot[c] = vzero<W>();
    if constexpr (SRC == SET_UNIFORM) {
        const int64_t k0 = uni_start(b, l, N), k1 = uni_start(b + 1, l, N);
        for (int64_t k = k0; k < k1; ++k) {
            R v = (R)rel_coord(k, 0.0, b, l, N);
            R pw = ipow(v, m0);
            V w;
            if constexpr (KER == KER_COT)
                w = fu[k];
            else
                w = R(1);
            for (int c = 0; c < CHS; ++c) {
                if constexpr (sizeof(R) == 8)
                    vfma(tot[c], pw, w);
                else
                    vacc(tot[c], vscale(w, pw));
                pw *= v;
            }
        }
    } else {
        const int32_t t0 = a.src.off[b], t1 = a.src.off[b + 1];
        for (int32_t t = t0; t < t1; ++t) {
            R v = (R)rel_coord(a.src.m[t], a.src.th[t], b, l, N);
            R pw = ipow(v, m0);
            V w;
            if constexpr (KER == KER_COT)
                w = a.w_sorted[t];
            else
                w = R(1);
            for (int c = 0; c < CHS; ++c) {
                if constexpr (sizeof(R) == 8)
                    vfma(tot[c], pw, w);
                else
                    vacc(tot[c], vscale(w, pw));
                pw *= v;
            }
        }
    }
    for (int c = 0; c < CHS; ++c)
        acc[c] = vnarrow<V>(tot[c]);
    if constexpr (KER == KER_LOG) {
        const double r = ldexp((double)N, -(l + 1));
        for (int c = 0; c < CHS; ++c) {
            int m = m0 + c;
            if ((m & 1) == 0)
                acc[c] -= (R)(2.0 * r / (double)(m + 1));
        }
    }
}

// P2M from sources staged in LDS: relative coordinates sv, their fourth
// powers sv4 and (cot kernel) weights sw of the sources [j0, j1) of one
// leaf, moments m0 .. m0+CHS-1 (m0 a multiple of 4).  Four sources at a
// time, their powers v^m0 = (v^4)^(m0/4) formed as independent chains (two
// squarings fewer than from v); each moment still sums its sources in
// order.  Binary32 sums run over blocks of P2M_FOLD sources, each block
// added into a binary64 total.
template <typename R, typename V, int KER, int CH>
__device__ __forceinline__ void p2m_staged(const R *sv, const R *sv4, const cx<R> *sw, int j0,
                                           int j1, int m0, double r, V *acc)
{
    static_assert(CH % 4 == 0, "chunks start at multiples of 4");
    using W = typename wide<V>::type;
    constexpr int FOLD = sizeof(R) == 8 ? INT32_MAX : P2M_FOLD;
    W tot[CH];
    for (int jb = j0; jb < j1;) {
        const int je = (j1 - jb > FOLD) ? jb + FOLD : j1;
        for (int c = 0; c < CH; ++c)
            acc[c] = vzero<V>();
        int j = jb;
        for (; j + 4 <= je; j += 4) {
            R v[4], sq[4], pw[4];
            V w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[u] = sv[j + u];
                sq[u] = sv4[j + u];
                pw[u] = R(1);
                if constexpr (KER == KER_COT)
                    w[u] = sw[j + u];
                else
                    w[u] = R(1);
            }
            for (int e = m0 >> 2; e; e >>= 1) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (e & 1)
                        pw[u] *= sq[u];
                    sq[u] *= sq[u];
                }
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    vfma(acc[c], pw[u], w[u]);
                    pw[u] *= v[u];
                }
            }
        }
        for (; j < je; ++j) {
            const R v = sv[j];
            R pw = ipow(sv4[j], m0 >> 2);
            V w;
            if constexpr (KER == KER_COT)
                w = sw[j];
            else
                w = R(1);
            for (int c = 0; c < CH; ++c) {
                vfma(acc[c], pw, w);
                pw *= v;
            }
        }
        if constexpr (sizeof(R) != 8) {
            for (int c = 0; c < CH; ++c) {
                if (jb == j0)
                    tot[c] = vzero<W>();
                vacc(tot[c], acc[c]);
            }
        }
        jb = je;
    }
    if (j1 <= j0) {
        for (int c = 0; c < CH; ++c)
            acc[c] = vzero<V>();
    } else if constexpr (sizeof(R) != 8) {
        for (int c = 0; c < CH; ++c)
            acc[c] = vnarrow<V>(tot[c]);
    }
    if constexpr (KER == KER_LOG) {
        for (int c = 0; c < CH; ++c) {
            const int m = m0 + c;
            if ((m & 1) == 0)
                acc[c] -= (R)(2.0 * r / (double)(m + 1));
        }
    }
}

// The staged P2M of a band's nbot leaves, written to the band's first level
// buffer and to the multipoles g: work items (leaf, CH consecutive
// moments).  CH = 8 when the items still fill three quarters of the
// workgroup (a source's starting power then serves 8 moments instead of 4),
// else 4.
template <typename R, typename V, int KER, int PU, int CH>
__device__ __forceinline__ void p2m_staged_items(const R *sv, const R *sv4, const cx<R> *sw,
                                                 const int32_t *soff, int nbot, double r,
                                                 R *buf0, int RS, V *g, int64_t first)
{
    constexpr int nch = PU / CH;
    for (int idx = threadIdx.x; idx < nbot * nch; idx += BLOCK) {
        const int i = idx / nch, ch = idx - i * nch;
        V acc[CH];
        p2m_staged<R, V, KER, CH>(sv, sv4, sw, soff[i], soff[i + 1], ch * CH, r, acc);
        for (int c = 0; c < CH; ++c) {
            st_coef<R, V>(buf0, RS, i, ch * CH + c, acc[c]);
            g[(first + i) * PU + ch * CH + c] = acc[c];
        }
    }
}

template <typename R, typename V, int KER, int PU>
__device__ __forceinline__ void p2m_staged_band(const R *sv, const R *sv4, const cx<R> *sw,
                                                const int32_t *soff, int nbot, double r,
                                                R *buf0, int RS, V *g, int64_t first)
{
    if (PU % 8 == 0 && nbot * (PU / 8) >= 3 * BLOCK / 4)
        p2m_staged_items<R, V, KER, PU, 8>(sv, sv4, sw, soff, nbot, r, buf0, RS, g, first);
    else
        p2m_staged_items<R, V, KER, PU, 4>(sv, sv4, sw, soff, nbot, r, buf0, RS, g, first);
}

// P2M on the matrix cores for uniform sources with B points in every leaf:
// a[m][(leaf, comp)] = sum_i v_i^m f[leaf B + i], v_i = (2i - B)/B, i.e. a
// GEMM whose operator V^T (PU x B) is the same for every leaf.  f holds the
// launch's nbot B weights, staged in LDS with leaf stride SB.  Each wave
// keeps one 16-row tile of V^T in registers (its powers formed once, as
// independent chains) and takes every column tile of that row tile.
constexpr int P2M_KMAX = 16; // B <= 64

template <typename R, typename V, int PU>
__device__ __forceinline__ void p2m_mfma(const UpArgs<R, V> &a, int64_t first,
                                         int nbot, R *buf, int RS, V *g,
                                         int lane, int wave, const R *f, int SB)
{
    constexpr int NC = 2; // cot kernel: complex weights
    using A = typename acc_t<R>::type;
    constexpr int nrt = PU / 16;
    constexpr int used = (4 / nrt) * nrt;
    if (wave >= used)
        return;
    const int B = a.leaf_pts;
    const int nks = B / 4;
    const int rt = wave % nrt;
    const int m = 16 * rt + (lane & 15); // A row of this lane
    R av[P2M_KMAX], vv[P2M_KMAX];
#pragma unroll
    for (int ks = 0; ks < P2M_KMAX; ++ks) {
        const int k = 4 * ks + (lane >> 4);
        // (steps past the leaf's points: a zero coordinate, so that their
        // powers stay finite)
        vv[ks] = ks < nks ? (R)((double)(2 * k - B) / (double)B) : R(0);
        av[ks] = R(1);
    }
    for (int e = m; e; e >>= 1) {
#pragma unroll
        for (int ks = 0; ks < P2M_KMAX; ++ks) {
            if (e & 1)
                av[ks] *= vv[ks];
            vv[ks] *= vv[ks];
        }
    }
    const int nct = (NC * nbot + 15) / 16;
    for (int ct = wave / nrt; ct < nct; ct += used / nrt) {
        const int j = 16 * ct + (lane & 15);
        const int i = j / NC, c = j % NC;
        const bool valid = i < nbot;
        const R *fp = f + (valid ? i : 0) * SB + c + (lane >> 4) * NC;
        // every operand load issued before the first matrix instruction
        // (steps past the leaf's points read its last step and add zero),
        // two accumulator chains in flight
        R bv[P2M_KMAX];
#pragma unroll
        for (int ks = 0; ks < P2M_KMAX; ++ks)
            bv[ks] = fp[4 * (ks < nks ? ks : nks - 1) * NC];
        A acc = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < P2M_KMAX; ++ks) {
            const R v = (valid && ks < nks) ? bv[ks] : R(0);
            if (ks & 1)
                acc1 = mma(av[ks], v, acc1);
            else
                acc = mma(av[ks], v, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[r] += acc1[r];
        if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * rt + out_row<R>(lane, r);
                buf[(size_t)i * RS + n * NC + c] = acc[r];
                reinterpret_cast<R *>(g)[((first + i) * PU + n) * NC + c] = acc[r];
            }
        }
    }
}

// M2M of one level inside LDS: np parents from 2 np children (rows of cur),
// written to nxt (LDS) and g (global, PU per box).  Each wave takes 16-row
// tiles of the parents' moments; its operator tile sits in registers.  The
// columns are (child, component): the right child's operator follows from
// the left one by the signs (-1)^m on the input and (-1)^n on the output,
// so both children go through one product and meet in the left child's
// lane (the right child's column is NC lanes up).  A level of few parents
// then fills twice as many columns of a tile as with one product per
// child.  The operator is lower triangular: row tile rt takes no moment of
// order 16 (rt + 1) or more, so its loop has KE = 4 (rt + 1) steps, a
// constant of the instantiation: every operand load of a column tile is
// issued before the first matrix instruction, and even and odd steps feed
// two accumulator chains.
template <typename R, typename V, int PU, int KE>
__device__ __forceinline__ void m2m_tile(const R (&am)[PU / 4], int rt, int ct0, int ctstep,
                                         int lane, int np, const R *cur, R *nxt, int RS, V *g)
{
    constexpr int NC = ncomp<V>::value;
    using A = typename acc_t<R>::type;
    const int nq = 2 * np;
    const int nct = (NC * nq + 15) / 16;
    for (int ct = ct0; ct < nct; ct += ctstep) {
        const int j = 16 * ct + (lane & 15);
        const int q = j / NC, c = j % NC;
        const bool valid = q < nq, right = (q & 1) != 0;
        const R *cq = cur + (size_t)(valid ? q : 0) * RS + c;
        R b[KE];
#pragma unroll
        for (int ks = 0; ks < KE; ++ks) {
            const int m = 4 * ks + (lane >> 4);
            b[ks] = cq[m * NC];
        }
        A acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KE; ++ks) {
            const int m = 4 * ks + (lane >> 4);
            R v = valid ? b[ks] : R(0);
            if (right && (m & 1))
                v = -v;
            if (ks & 1)
                acc1 = mma(am[ks], v, acc1);
            else
                acc0 = mma(am[ks], v, acc0);
        }
        const int p = q >> 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const R sl = acc0[r] + acc1[r];
            const R sr = __shfl_down(sl, NC);
            if (valid && !right) {
                const int n = 16 * rt + out_row<R>(lane, r);
                const R v = sl + ((n & 1) ? -sr : sr);
                nxt[(size_t)p * RS + n * NC + c] = v;
                reinterpret_cast<R *>(g)[((size_t)p * PU + n) * NC + c] = v;
            }
        }
    }
}

template <typename R, typename V, int PU>
__device__ __forceinline__ void m2m_level(const R (&am)[PU / 4], int rt,
                                          int ct0, int ctstep, int lane, int np,
                                          const R *cur, R *nxt, int RS, V *g)
{
    static_assert(PU % 16 == 0 && PU <= 64, "multipole length: 16, 32, 48 or 64");
    switch (rt) {
    case 0:
        m2m_tile<R, V, PU, 4>(am, rt, ct0, ctstep, lane, np, cur, nxt, RS, g);
        break;
    case 1:
        if constexpr (PU >= 32)
            m2m_tile<R, V, PU, 8>(am, rt, ct0, ctstep, lane, np, cur, nxt, RS, g);
        break;
    case 2:
        if constexpr (PU >= 48)
            m2m_tile<R, V, PU, 12>(am, rt, ct0, ctstep, lane, np, cur, nxt, RS, g);
        break;
    default:
        if constexpr (PU >= 64)
            m2m_tile<R, V, PU, 16>(am, rt, ct0, ctstep, lane, np, cur, nxt, RS, g);
        break;
    }
}

// One launch of the upward pass: 2^d boxes of level lb (the leaves, by P2M,
// in the first band) up to level lb - d.
// fu: the uniform sources' weights (the forward's input).
template <typename R, typename V, int KER, int SRC, int PU>
__device__ __forceinline__ void up_band_body(const UpArgs<R, V> &a, int blk, const cx<R> *fu)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *buf0 = reinterpret_cast<R *>(smem_raw);
    const int RS = a.RS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lb = a.lb, d = a.d;
    const int nbot = 1 << d;
    const int64_t first = (int64_t)blk << d;
    R *buf1 = buf0 + (size_t)nbot * RS;
    if (a.first_band) {
        V *g = a.mp + lev_off(lb, PU);
        // staging area for the sources: the second level buffer, which the
        // M2M only writes after the P2M is done with the sources
        R *stage = buf1;
        bool done = false;
        if constexpr (SRC == SET_UNIFORM && KER == KER_COT) {
            if (a.leaf_pts > 0) {
                const int bn = a.leaf_pts * 2, SB = uni_stage_stride(a.leaf_pts, sizeof(R));
                const int nf = nbot * bn;
                const R *f = reinterpret_cast<const R *>(fu) + first * bn;
                // every load of a batch in flight at once (indices clamped)
                for (int i0 = 0; i0 < nf; i0 += 8 * BLOCK) {
                    R v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int i = i0 + tid + u * BLOCK;
                        v[u] = f[i < nf ? i : nf - 1];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int i = i0 + tid + u * BLOCK;
                        if (i < nf)
                            stage[i + (SB - bn) * (i / bn)] = v[u];
                    }
                }
                __syncthreads();
                p2m_mfma<R, V, PU>(a, first, nbot, buf0, RS, g, lane, wave, stage, SB);
                done = true;
            }
        }
        if constexpr (SRC == SET_SORTED) {
            const int32_t t0 = a.src.off[first], t1 = a.src.off[first + nbot];
            if (t1 - t0 <= a.stage_cap) {
                const int cnt = t1 - t0;
                const int cap4 = (a.stage_cap + 3) & ~3;
                R *sv = stage;
                cx<R> *sw = reinterpret_cast<cx<R> *>(stage + cap4);
                // the fourth powers after the weights, then the leaves'
                // offsets from t0
                R *sv4 = stage + cap4 + (KER == KER_COT ? 2 * cap4 : 0);
                int32_t *soff = reinterpret_cast<int32_t *>(sv4 + cap4);
                const double invN = 1.0 / (double)a.N;
                if (tid <= nbot)
                    soff[tid] = a.src.off[first + tid] - t0;
                // every load of a batch in flight at once (indices clamped)
                for (int i0 = 0; i0 < cnt; i0 += 4 * BLOCK) {
                    int32_t mv[4], lv[4];
                    double tv[4];
                    cx<R> wv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        int i = i0 + tid + u * BLOCK;
                        const int32_t t = t0 + (i < cnt ? i : cnt - 1);
                        mv[u] = a.src.m[t];
                        tv[u] = a.src.th[t];
                        lv[u] = a.src_leaf[t];
                        if constexpr (KER == KER_COT)
                            wv[u] = a.w_sorted[t];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + tid + u * BLOCK;
                        if (i < cnt) {
                            const R v = (R)rel_coord_r(mv[u], tv[u], lv[u], a.l, a.N, invN);
                            const R v2 = v * v;
                            sv[i] = v;
                            sv4[i] = v2 * v2;
                            if constexpr (KER == KER_COT)
                                sw[i] = wv[u];
                        }
                    }
                }
                __syncthreads();
                p2m_staged_band<R, V, KER, PU>(sv, sv4, sw, soff, nbot,
                                               ldexp((double)a.N, -(a.l + 1)), buf0, RS, g,
                                               first);
                done = true;
            }
        }
        if constexpr (SRC == SET_UNIFORM && KER == KER_COT) {
            // a grid whose leaves hold unequal numbers of points (N not a
            // multiple of the leaf count): the band's points staged with
            // their coordinates, as sorted sources are
            const int64_t K0 = uni_start(first, a.l, a.N);
            const int64_t K1 = uni_start(first + nbot, a.l, a.N);
            if (!done && a.stage_cap > 0 && K1 - K0 <= a.stage_cap) {
                const int cnt = (int)(K1 - K0);
                const int cap4 = (a.stage_cap + 3) & ~3;
                R *sv = stage;
                cx<R> *sw = reinterpret_cast<cx<R> *>(stage + cap4);
                R *sv4 = stage + 3 * cap4;
                int32_t *soff = reinterpret_cast<int32_t *>(sv4 + cap4);
                const double invN = 1.0 / (double)a.N;
                const double lscale = ldexp(1.0, a.l) * invN;
                if (tid <= nbot)
                    soff[tid] = (int32_t)(uni_start(first + tid, a.l, a.N) - K0);
                // a point's coordinate and weight into the staging area
                const auto put = [&](int i, cx<R> w) {
                    const int64_t k = K0 + i;
                    const int64_t leaf = uni_leaf(k, a.l, a.N, lscale);
                    const R v = (R)rel_coord_r(k, 0.0, leaf, a.l, a.N, invN);
                    const R v2 = v * v;
                    sv[i] = v;
                    sv4[i] = v2 * v2;
                    sw[i] = w;
                };
                // two loads in flight at once (indices clamped); named
                // values, not an array (which the batched kernel kept in
                // scratch memory)
                for (int i0 = 0; i0 < cnt; i0 += 2 * BLOCK) {
                    const int ia = i0 + tid, ib = ia + BLOCK;
                    const cx<R> wa = fu[K0 + (ia < cnt ? ia : cnt - 1)];
                    const cx<R> wb = fu[K0 + (ib < cnt ? ib : cnt - 1)];
                    if (ia < cnt)
                        put(ia, wa);
                    if (ib < cnt)
                        put(ib, wb);
                }
                __syncthreads();
                p2m_staged_band<R, V, KER, PU>(sv, sv4, sw, soff, nbot,
                                               ldexp((double)a.N, -(a.l + 1)), buf0, RS, g,
                                               first);
                done = true;
            }
        }
        if (!done) {
            constexpr int nch = PU / CHS;
            for (int idx = tid; idx < nbot * nch; idx += BLOCK) {
                const int i = idx / nch, ch = idx - i * nch;
                V acc[CHS];
                p2m_chunk<R, V, KER, SRC>(a, fu, first + i, ch * CHS, acc);
                for (int c = 0; c < CHS; ++c) {
                    st_coef<R, V>(buf0, RS, i, ch * CHS + c, acc[c]);
                    g[(first + i) * PU + ch * CHS + c] = acc[c];
                }
            }
        }
    } else {
        const V *g = a.mp + lev_off(lb, PU) + first * PU;
        for (int idx = tid; idx < nbot * PU; idx += BLOCK)
            st_coef<R, V>(buf0, RS, idx / PU, idx % PU, g[idx]);
    }
    if (d == 0)
        return;
    // (requested before the P2M, the tile held registers through it and
    // cost occupancy)
    constexpr int nrt = PU / 16;
    const int used = (4 / nrt) * nrt;
    R am[PU / 4];
    const int rt = wave % nrt;
    if (wave < used)
        load_tile<R, PU>(am, a.T.m2m, rt, lane);
    __syncthreads();
    R *cur = buf0, *nxt = buf1;
    int n = nbot;
    for (int lev = lb - 1; lev >= lb - d; --lev) {
        n >>= 1;
        if (wave < used)
            m2m_level<R, V, PU>(am, rt, wave / nrt, 4 / nrt, lane, n, cur, nxt, RS,
                                a.mp + lev_off(lev, PU) + (first >> (lb - lev)) * PU);
        __syncthreads();
        R *t = cur;
        cur = nxt;
        nxt = t;
    }
}

template <typename R, typename V, int KER, int SRC, int PU>
__global__ void __launch_bounds__(BLOCK) k_up_band(UpArgs<R, V> a)
{
    up_band_body<R, V, KER, SRC, PU>(a, blockIdx.x, a.f_uniform);
}

// The same band of every problem of a batch in one launch.
// The forward's weights come from the IoPtr table when it is given.
template <typename R, typename V, int KER, int SRC, int PU>
__global__ void __launch_bounds__(BLOCK) kb_up_band(const UpArgs<R, V> *aa, BlockMap bm,
                                                    const IoPtr *io)
{
    int blk, nblk;
    const int t = bm_find(bm, blockIdx.x, &blk, &nblk);
    // the arguments read in place (a copy took scratch memory)
    const UpArgs<R, V> &a = aa[t];
    const cx<R> *fu = io ? reinterpret_cast<const cx<R> *>(io[a.io_index].in) : a.f_uniform;
    up_band_body<R, V, KER, SRC, PU>(a, blk, fu);
}

// Level 2 (one workgroup): the regular part of Eq. (p20) as the level-2
// local polynomial of every quarter, from the four level-2 multipoles, and
// the sum of the weights.  The moments of Omega_1(P_q) about the centre of
// P_q are quarter q's own plus its neighbours' shifted by -+2 half-widths
// ((v -+ 2)^t expanded); with that shift folded into the tables regR and
// regL, local coefficient lo of quarter q is one sum over t of
//   reg1 a_q + regR a_{q+1} + regL a_{q-1} + reg2 a_{q+2}.
// Thread (lo, c) sums the t of chunk c for all four quarters, its table
// values loaded at once (one round trip); the chunks' partial sums are then
// added in LDS.  a2: 4 PU values of LDS; part: 4 PD x (BLOCK / PD) values.
template <typename R, typename V, int KER>
__device__ __forceinline__ void regular_part(const UpArgs<R, V> &a, int PU, V *a2, V *part)
{
    const int PD = a.PD; // 16, 32, 48 or 64; PU a multiple of 16
    const int tid = threadIdx.x;
    for (int i = tid; i < 4 * PU; i += BLOCK)
        a2[i] = a.mp[i]; // level 2 is the first level of mp
    const int nch = BLOCK / PD;                 // chunks of t (4 .. 16)
    const int tlen = (PU + nch - 1) / nch;      // t values per chunk (<= 16)
    const int lo = tid % PD, ch = tid / PD;
    const int t0 = ch * tlen;
    constexpr int TMAX = 16;
    __syncthreads();
    V acc[4] = {vzero<V>(), vzero<V>(), vzero<V>(), vzero<V>()};
    // one table a pass (its loads in flight at once), so that the table
    // values take few registers: the M2L workgroups of the same kernel
    // keep their occupancy
#pragma unroll 1
    for (int pass = 0; pass < 4; ++pass) {
        const R *tab = pass == 0   ? a.T.reg1
                       : pass == 1 ? a.T.regR
                       : pass == 2 ? a.T.regL
                                   : a.T.reg2;
        // the moments the table weighs: quarter q's own, its right and its
        // left neighbour's, the opposite quarter's
        const int qs = pass == 0 ? 0 : (pass == 1 ? 1 : (pass == 2 ? 3 : 2));
        R w[TMAX];
#pragma unroll
        for (int k = 0; k < TMAX; ++k) {
            const int t = t0 + k < PU ? t0 + k : PU - 1; // clamped
            w[k] = tab[t * PD + lo];
        }
#pragma unroll
        for (int k = 0; k < TMAX; ++k) {
            const int t = t0 + k;
            if (k < tlen && t < PU) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    vfma(acc[q], w[k], a2[((q + qs) & 3) * PU + t]);
            }
        }
    }
    if (ch < nch) // (PD = 48: 240 threads in 5 chunks)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            part[(q * PD + lo) * nch + ch] = acc[q];
    __syncthreads();
    for (int idx = tid; idx < 4 * PD; idx += BLOCK) {
        const int q = idx / PD, l = idx - q * PD;
        V sum = part[idx * nch];
        for (int c = 1; c < nch; ++c)
            vadd(sum, part[idx * nch + c]);
        if constexpr (KER == KER_LOG) {
            if (l == 0) {
                // the log kernel's monopoles: Omega_1 (the quarter and its
                // neighbours) and the opposite quarter
                const double m1 = (double)a2[q * PU] + (double)a2[((q + 1) & 3) * PU] +
                                  (double)a2[((q + 3) & 3) * PU];
                sum += (R)(a.logc1 * m1 + a.logc2 * (double)a2[((q + 2) & 3) * PU]);
            }
        }
        a.loc2[idx] = sum;
    }
    if constexpr (KER == KER_COT) {
        if (tid == 0) {
            V sm = a2[0];
            for (int q = 1; q < 4; ++q)
                vadd(sm, a2[q * PU]);
            *a.S = sm;
        }
    }
}

// ------------------------------------------------------------ k_down_eval

template <typename R, typename V>
struct DownArgs {
    int64_t N;
    int l, lr;
    int RS;                  // LDS row stride (elements of R)
    int rows_buf, rows_src;  // rows of each local buffer / of the source buffer
    int near_bytes;          // LDS bytes free for the near-field sources
                             // once the leaf locals are formed
    int grp_lds;             // forward evaluation: LDS byte offset of the
                             // grouping of a work item's targets by leaf
    const WorkItem *work;
    const int32_t *nwork;    // number of valid work items (device)
    const V *mp;             // PU per box
    int PU;
    const V *loc2;           // 4 x PD
    OpTables<R> T;
    // sources of the near field
    SortedSet src;
    const cx<R> *f_uniform;
    const cx<R> *w_sorted;
    // targets
    SortedSet tgt;
    const int32_t *tgt_leaf; // LOGCD: leaf of every sorted target (required)
    const SortedPt *tgt_pt;  // FWD: sorted targets
    // epilogues
    cx<R> *out;              // FWD: g (input order); INV: f
    const V *S;              // sum of the weights
    const cx<R> *f_hit;      // FWD: f (exact hits)
    const double *chat;      // INV: Chat_k
    const int32_t *hit;      // INV: source index j with y_j = x_k, or -1
    const cx<R> *gin;        // INV: g (input order)
    double *chat_out;        // LOGCD outputs: Chat_k (uniform points) and
    cx<double> *dhat_out;    // Dhat_j (sorted sources), Eq. (p8)
    double logself;          // LOGCD: log(2 pi / N), the excluded self term
    int *flags_out;          // LOGCD: FLAG_RANGE when a log-sum leaves
    double log_max;          // [-log_max, log_max] (the range of exp in
                             // binary64, or what the binary32 weights
                             // D_j g_j of the mixed path can hold)
    const int *flags;        // setup error flags: sorted-source passes stop
                             // at FLAG_DENSE (their near field would be
                             // quadratic in the leaf size)
    int32_t io_index;        // batched launches: entry of the IoPtr table
    const IoPtr *io;         // batched launches: the table (f_uniform, f_hit
                             // and out are then io[io_index].in / .out)
    V *leaf_loc;             // local expansions of the leaves, PD per leaf
    V *pre;                  // M2L results of every box of levels 3..l, PD
                             // per box packed per level (the leaf level is
                             // leaf_loc itself: each subtree turns its
                             // leaves' M2L results into their locals)
};

// Phases of the downward pass: the translations down to the leaf locals
// (written to leaf_loc), then the evaluation at the targets (reading them).
// Split in two kernels, the evaluation runs at a much higher occupancy than
// the translations' register-held operator tiles allow.
enum { PH_TRANS = 1, PH_EVAL = 2 };

// Register-held operator tiles of one wave (row tile rt of PD rows).
template <typename R, int PD>
struct DownOps {
    R a4[PD / 4], a6[PD / 4], al[PD / 4];
};

// M2L (+ L2L) for up to 16/NC target boxes per column tile with matrix
// cores.  For target column box i:
//   out = sigma [T_4 a(i,-2) + T_-4 a(i,+2) + T_(-+6) a(i,+-3)] + L2L par(i)
// (left child: offsets -2, +2, +3; right child: -3, -2, +2).  T_-delta and
// the right-child L2L follow from T_delta and the left L2L by the sign
// patterns (-1)^m on the input (applied to the B operand) and a per-row
// sign on the output.  srcrow(i, o) -> LDS row of box i's neighbour at
// offset o; parrow(i) -> LDS row of the parent local; isleft(i), sig(i),
// lgr(i) per box; outrow(i) -> output row in outbase (rows RSo apart; LDS
// or global memory).
template <typename R, typename V, int KER, int PD, bool WITH_L2L, typename SrcRow,
          typename ParRow, typename IsLeft, typename Sigma, typename LogR,
          typename OutRow, typename OutPtr>
__device__ __forceinline__ void m2l_tiles(const DownOps<R, PD> &o, int rt, int ct0,
                                          int ctstep, int lane, int nb,
                                          const R *lds, const R *parbase, int RS,
                                          SrcRow srcrow, ParRow parrow,
                                          IsLeft isleft, Sigma sig,
                                          LogR lgr, OutRow outrow, OutPtr outbase, int RSo)
{
    constexpr int NC = ncomp<V>::value;
    using A = typename acc_t<R>::type;
    const int nct = (NC * nb + 15) / 16;
    for (int ct = ct0; ct < nct; ct += ctstep) {
        const int j = 16 * ct + (lane & 15);
        const int i = j / NC, c = j % NC;
        const bool valid = i < nb;
        const int ic = valid ? i : 0;
        const bool left = isleft(ic);
        const R *sp4 = lds + (size_t)srcrow(ic, -2) * RS + c;
        const R *sm4 = lds + (size_t)srcrow(ic, 2) * RS + c;
        const R *s6 = lds + (size_t)srcrow(ic, left ? 3 : -3) * RS + c;
        const R *sp = sp4;
        if constexpr (WITH_L2L)
            sp = parbase + (size_t)parrow(ic) * RS + c;
        A p4 = {0, 0, 0, 0}, n4 = {0, 0, 0, 0}, a6 = {0, 0, 0, 0}, al = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < PD / 4; ++ks) {
            const int m = 4 * ks + (lane >> 4);
            const bool odd = (m & 1) != 0;
            R b1 = sp4[m * NC], b2 = sm4[m * NC], b3 = s6[m * NC];
            if (!valid) {
                b1 = R(0);
                b2 = R(0);
                b3 = R(0);
            }
            if (odd) {
                b2 = -b2;
                if (left)
                    b3 = -b3;
            }
            p4 = mma(o.a4[ks], b1, p4);
            n4 = mma(o.a4[ks], b2, n4);
            a6 = mma(o.a6[ks], b3, a6);
            if constexpr (WITH_L2L) {
                // the L2L operator is triangular: output moments of row tile
                // rt take no input moment below 16 rt
                if (ks >= 4 * rt) {
                    R b4 = sp[m * NC];
                    if (!valid)
                        b4 = R(0);
                    if (odd && !left)
                        b4 = -b4;
                    al = mma(o.al[ks], b4, al);
                }
            }
        }
        if (!valid)
            continue;
        const R sg = sig(ic);
        R a0 = R(0), lr0 = R(0);
        if constexpr (KER == KER_LOG) {
            a0 = sp4[0] + sm4[0] + s6[0];
            lr0 = lgr(ic);
        }
        const auto dst = outbase + (size_t)outrow(ic) * RSo + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * rt + out_row<R>(lane, r);
            // output sign of the T_-delta family
            const bool sneg = ((n + (KER == KER_COT ? 1 : 0)) & 1) != 0;
            const R nv = sneg ? -n4[r] : n4[r];
            const R v6 = (left && sneg) ? -a6[r] : a6[r];
            R v = (p4[r] + nv + v6) * sg;
            if constexpr (KER == KER_LOG) {
                if (n == 0)
                    v += a0 * lr0;
            }
            if constexpr (WITH_L2L)
                v += (!left && (n & 1)) ? -al[r] : al[r];
            dst[n * NC] = v;
        }
    }
}

// 1/d: the binary64 hardware reciprocal is good to about 2^-24; one Newton
// step brings it to about 2^-48 relative (far inside the 1e-12 target of
// the binary64 path).  The binary32 one is within 1 ulp.
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float d)
{
    return __builtin_amdgcn_rcpf(d); // within 1 ulp on gfx950
}

// sum_{n < P} c_n u^n for the coefficients of one LDS row, as four
// interleaved Horner chains in u^4 (P a multiple of 4): a quarter of the
// dependent steps of plain Horner.
template <typename R, typename V, int P>
__device__ __forceinline__ V horner4(const R *base, int RS, int row, R u)
{
    static_assert(P % 4 == 0, "expansion length must be a multiple of 4");
    const R u2 = u * u, u4 = u2 * u2;
    V c0 = ld_coef<R, V>(base, RS, row, P - 4), c1 = ld_coef<R, V>(base, RS, row, P - 3);
    V c2 = ld_coef<R, V>(base, RS, row, P - 2), c3 = ld_coef<R, V>(base, RS, row, P - 1);
#pragma unroll 2 // fully unrolled, the loads of all P coefficients get hoisted
    for (int n = P - 8; n >= 0; n -= 4) {
        V t0 = vscale(c0, u4), t1 = vscale(c1, u4), t2 = vscale(c2, u4), t3 = vscale(c3, u4);
        vadd(t0, ld_coef<R, V>(base, RS, row, n));
        vadd(t1, ld_coef<R, V>(base, RS, row, n + 1));
        vadd(t2, ld_coef<R, V>(base, RS, row, n + 2));
        vadd(t3, ld_coef<R, V>(base, RS, row, n + 3));
        c0 = t0;
        c1 = t1;
        c2 = t2;
        c3 = t3;
    }
    // (c0 + u c1) + u^2 (c2 + u c3)
    V lo = vscale(c1, u), hi = vscale(c3, u);
    vadd(lo, c0);
    vadd(hi, c2);
    V r = vscale(hi, u2);
    vadd(r, lo);
    return r;
}

// First uniform point of leaf b for b in [-1, nleaf + 1], unwrapped.
__device__ __forceinline__ int64_t uni_start_unwrapped(int64_t b, int l, int64_t N)
{
    const int64_t nleaf = int64_t(1) << l;
    if (b < 0)
        return uni_start(b + nleaf, l, N) - N;
    if (b > nleaf)
        return uni_start(b - nleaf, l, N) + N;
    return uni_start(b, l, N);
}

// Near field of the cot kernel: sum over the sources of leaves b-1, b, b+1
// (unwrapped around the circle) of w / (tau - sigma~).  Binary32 terms are
// summed in blocks (fold_len) or straight into binary64.
template <typename R, typename V, int SRC>
__device__ __forceinline__ cx<double> near_cot(const DownArgs<R, V> &a, int64_t tm,
                                               double tth, int64_t leaf,
                                               const cx<R> *fs, int64_t K0,
                                               const cx<R> *f_uniform)
{
    const int64_t N = a.N;
    const int64_t nleaf = int64_t(1) << a.l;
    cx<double> tot = {0.0, 0.0};
    if constexpr (SRC == SET_UNIFORM) {
        if (fs) { // sources staged in LDS from unwrapped index K0 on
            const int64_t k0 = uni_start_unwrapped(leaf - 1, a.l, N);
            const int64_t k1 = uni_start_unwrapped(leaf + 2, a.l, N);
            const int32_t base = (int32_t)(tm - k0);
            const cx<R> *fp = fs + (k0 - K0);
            const int32_t cnt = (int32_t)(k1 - k0);
            for (int32_t ib = 0; ib < cnt;) {
                const int32_t ie = (cnt - ib > fold_len<R>()) ? ib + fold_len<R>() : cnt;
                // binary64: two pairs at a time, each pair over one
                // reciprocal, w0/d0 + w1/d1 = (w0 d1 + w1 d0) / (d0 d1) (no
                // distance is zero: exact hits never reach the near field);
                // binary32 keeps one reciprocal per pair, whose rounding it
                // can afford less
                cx<R> acc = {R(0), R(0)}, a1 = acc, a2 = acc, a3 = acc;
                int32_t i = ib;
                double cb = (double)(base - ib); // base - i, exact
                for (; i + 4 <= ie; i += 4, cb -= 4.0) {
                    const R d0 = (R)(cb + tth);
                    const R d1 = (R)((cb - 1.0) + tth);
                    const R d2 = (R)((cb - 2.0) + tth);
                    const R d3 = (R)((cb - 3.0) + tth);
                    const cx<R> w0 = fp[i], w1 = fp[i + 1], w2 = fp[i + 2], w3 = fp[i + 3];
                    if constexpr (sizeof(R) == 8) {
                        const R r01 = recip(d0 * d1), r23 = recip(d2 * d3);
                        acc.re = fma(fma(w0.re, d1, w1.re * d0), r01, acc.re);
                        acc.im = fma(fma(w0.im, d1, w1.im * d0), r01, acc.im);
                        a1.re = fma(fma(w2.re, d3, w3.re * d2), r23, a1.re);
                        a1.im = fma(fma(w2.im, d3, w3.im * d2), r23, a1.im);
                    } else {
                        const R r0 = recip(d0), r1 = recip(d1), r2 = recip(d2), r3 = recip(d3);
                        acc.re = fma(w0.re, r0, acc.re);
                        acc.im = fma(w0.im, r0, acc.im);
                        a1.re = fma(w1.re, r1, a1.re);
                        a1.im = fma(w1.im, r1, a1.im);
                        a2.re = fma(w2.re, r2, a2.re);
                        a2.im = fma(w2.im, r2, a2.im);
                        a3.re = fma(w3.re, r3, a3.re);
                        a3.im = fma(w3.im, r3, a3.im);
                    }
                }
                for (; i < ie; ++i) {
                    const R rd = recip((R)((double)(base - i) + tth));
                    const cx<R> w = fp[i];
                    acc.re = fma(w.re, rd, acc.re);
                    acc.im = fma(w.im, rd, acc.im);
                }
                acc.re += (a1.re + a2.re) + a3.re;
                acc.im += (a1.im + a2.im) + a3.im;
                tot.re += (double)acc.re;
                tot.im += (double)acc.im;
                ib = ie;
            }
            return tot;
        }
    }
    // sources read in place (they did not fit in LDS): each term rounded in
    // R, the sum kept in binary64
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
                const cx<R> w = f_uniform[k];
                tot.re = fma((double)w.re, (double)rd, tot.re);
                tot.im = fma((double)w.im, (double)rd, tot.im);
            }
        } else {
            const int32_t t0 = a.src.off[b], t1 = a.src.off[b + 1];
            for (int32_t t = t0; t < t1; ++t) {
                const double dd = grid_diff(tm - a.src.m[t] - shift, tth, a.src.th[t]);
                if (dd == 0.0)
                    continue; // a source on this grid point (weight 0, adjoint)
                const R rd = recip((R)dd);
                const cx<R> w = a.w_sorted[t];
                tot.re = fma((double)w.re, (double)rd, tot.re);
                tot.im = fma((double)w.im, (double)rd, tot.im);
            }
        }
    }
    return tot;
}

// Sorted sources of a subtree staged in LDS: the leaves leaf0 - 1 ..
// leaf0 + nb (unwrapped, so positions increase), as (integer grid offset
// from a base point, fraction) pairs and (cot kernel) weights.  The sources
// of staged leaf j occupy [off[j], off[j + 1]).  The offset is held as a
// binary64 value (an exact integer), interleaved with the fraction, so that
// a pair takes one 16-byte LDS read and no integer-to-binary64 conversion.
template <typename R>
struct NearStage {
    double2 *p; // {offset, fraction}
    cx<R> *w;
    int32_t *off;
    int32_t self0; // staged index of sorted point t is t + self0 (own leaves)
};

// Distance tau - sigma in grid units for integer parts tm, m (binary64,
// |tm - m| < 2^31, so their difference is exact) and fractions a, b in
// [-1/2, 1/2]: a - b and the sum each round once, so the relative error is
// at most 2^-53 (1 + 1/|d|).  GT: the target is on the grid (a = 0), and
// a - b is -b exactly, so one subtraction gives the same value.
template <bool GT>
__device__ __forceinline__ double near_dist_p(double tm, double2 p, double a)
{
    if constexpr (GT)
        return (tm - p.x) - p.y;
    else
        return (tm - p.x) + (a - p.y);
}

// Cot near field from staged sources [j0, j1): sum w / (tau - sigma)
// (GT: the target is on the grid, tth = 0).  Binary32 sums run over blocks
// of NEAR_FOLD pairs, each block's partial added into a binary64 total, so
// the rounding of the sum does not grow with the number of sources.
template <typename R, bool GT>
__device__ __forceinline__ cx<double> near_cot_staged(const NearStage<R> &ns, int32_t j0,
                                                      int32_t j1, int32_t tmr, double tth)
{
    const double tmd = (double)tmr;
    cx<double> tot = {0.0, 0.0};
    for (int32_t jb = j0; jb < j1;) {
        const int32_t je = (j1 - jb > fold_len<R>()) ? jb + fold_len<R>() : j1;
        cx<R> a0 = {R(0), R(0)}, a1 = a0, a2 = a0, a3 = a0;
        int32_t j = jb;
        // binary64: two pairs at a time, each pair over one reciprocal (no
        // distance is zero: exact hits never reach the near field); binary32
        // keeps one reciprocal per pair
        for (; j + 4 <= je; j += 4) {
            const R d0 = (R)near_dist_p<GT>(tmd, ns.p[j], tth);
            const R d1 = (R)near_dist_p<GT>(tmd, ns.p[j + 1], tth);
            const R d2 = (R)near_dist_p<GT>(tmd, ns.p[j + 2], tth);
            const R d3 = (R)near_dist_p<GT>(tmd, ns.p[j + 3], tth);
            const cx<R> w0 = ns.w[j], w1 = ns.w[j + 1], w2 = ns.w[j + 2], w3 = ns.w[j + 3];
            if constexpr (sizeof(R) == 8) {
                const R r01 = recip(d0 * d1), r23 = recip(d2 * d3);
                a0.re = fma(fma(w0.re, d1, w1.re * d0), r01, a0.re);
                a0.im = fma(fma(w0.im, d1, w1.im * d0), r01, a0.im);
                a1.re = fma(fma(w2.re, d3, w3.re * d2), r23, a1.re);
                a1.im = fma(fma(w2.im, d3, w3.im * d2), r23, a1.im);
            } else {
                const R r0 = recip(d0), r1 = recip(d1), r2 = recip(d2), r3 = recip(d3);
                a0.re = fma(w0.re, r0, a0.re);
                a0.im = fma(w0.im, r0, a0.im);
                a1.re = fma(w1.re, r1, a1.re);
                a1.im = fma(w1.im, r1, a1.im);
                a2.re = fma(w2.re, r2, a2.re);
                a2.im = fma(w2.im, r2, a2.im);
                a3.re = fma(w3.re, r3, a3.re);
                a3.im = fma(w3.im, r3, a3.im);
            }
        }
        for (; j < je; ++j) {
            const R r = recip((R)near_dist_p<GT>(tmd, ns.p[j], tth));
            const cx<R> w = ns.w[j];
            a0.re = fma(w.re, r, a0.re);
            a0.im = fma(w.im, r, a0.im);
        }
        tot.re += (double)((a0.re + a1.re) + (a2.re + a3.re));
        tot.im += (double)((a0.im + a1.im) + (a2.im + a3.im));
        jb = je;
    }
    return tot;
}

// log prod |tau - sigma| over the staged sources [j, j1), folded into
// prod x 2^expo (renormalised after every eight factors and at the end;
// every factor is below 2^31 in grid units, so eight of them stay in range).
template <typename R, bool GT>
__device__ __forceinline__ void log_prod_range(const NearStage<R> &ns, int32_t j, int32_t j1,
                                               int32_t tmr, double tth, double &prod,
                                               int &expo)
{
    const double tmd = (double)tmr;
    for (; j + 8 <= j1; j += 8) {
        double d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            d[u] = fabs(near_dist_p<GT>(tmd, ns.p[j + u], tth));
        const double q = ((d[0] * d[1]) * (d[2] * d[3])) * ((d[4] * d[5]) * (d[6] * d[7]));
        int e;
        prod = frexp(prod * q, &e);
        expo += e;
    }
    double q = 1.0;
    for (; j < j1; ++j)
        q *= fabs(near_dist_p<GT>(tmd, ns.p[j], tth));
    int e;
    prod = frexp(prod * q, &e);
    expo += e;
}

// Log near field from staged sources [j0, j1) without the source `self`
// (GT: the target is on the grid, tth = 0): the product of the distances
// |tau - sigma| as mantissa and exponent, *prod x 2^*expo with *prod in
// [1/2, 1) (1 for an empty range).  The source `self` (the target itself)
// splits the range: no test per pair.
template <typename R, bool GT>
__device__ __forceinline__ void near_prod_staged(const NearStage<R> &ns, int32_t j0, int32_t j1,
                                                 int32_t self, int32_t tmr, double tth,
                                                 double *prod, int *expo)
{
    double p = 1.0;
    int e = 0;
    if (self >= j0 && self < j1) {
        log_prod_range<R, GT>(ns, j0, self, tmr, tth, p, e);
        log_prod_range<R, GT>(ns, self + 1, j1, tmr, tth, p, e);
    } else {
        log_prod_range<R, GT>(ns, j0, j1, tmr, tth, p, e);
    }
    *prod = p;
    *expo = e;
}

// Integral of log|tau - sigma| over sigma in the leaves leaf - 1 .. leaf + 1
// (unwrapped), tau = tm + tth: the uniform background the log FMM removed.
__device__ __forceinline__ double near_log_background(int64_t tm, double tth, int64_t leaf,
                                                      int l, int64_t N)
{
    const double sc = ldexp(1.0, -l);
    double lo = (double)((leaf - 1) * N - (tm << l)) * sc - tth;
    double hi = (double)((leaf + 2) * N - (tm << l)) * sc - tth;
    return xlogx_m_x(hi) - xlogx_m_x(lo);
}

// Near field of the log kernel with the uniform background removed:
// sum log|tau - sigma~| over the sources of leaves b-1..b+1 (skipping the
// source `self`), minus the integral of log|tau - sigma| over those leaves.
// The logarithms of the distances are summed as the logarithm of their
// product, kept as mantissa x 2^exponent so that it cannot leave the range.
template <typename R, typename V>
__device__ __forceinline__ double near_log(const DownArgs<R, V> &a, int64_t tm,
                                           double tth, int64_t leaf,
                                           int32_t self)
{
    const int64_t N = a.N;
    const int l = a.l;
    const int64_t nleaf = int64_t(1) << l;
    double prod = 1.0;
    int expo = 0, cnt = 0;
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
            const double dd = grid_diff(tm - a.src.m[t] - shift, tth, a.src.th[t]);
            prod *= fabs(dd);
            if (++cnt == 8) { // renormalise: |dd| <= 2N, so 8 factors stay in range
                int e;
                prod = frexp(prod, &e);
                expo += e;
                cnt = 0;
            }
        }
    }
    const double acc = log(prod) + (double)expo * 0.69314718055994530942;
    return acc - near_log_background(tm, tth, leaf, l, N);
}

// The M2L results of the nb boxes of level lev below the subtree root R0
// (PD per box), loaded into registers (no control flow between the loads,
// so that none of them waits for another) ...
template <typename R, typename V, int PD, int NPF>
__device__ __forceinline__ void pre_fetch(V (&pf)[NPF], const V *pre, int64_t R0, int lr,
                                          int lev, int tid)
{
    const int nb = 1 << (lev - lr);
    const V *base = pre + lev_off(lev, PD) + (R0 << (lev - lr)) * PD;
    const int n = nb * PD;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        int e = tid + k * BLOCK;
        e = e < n ? e : n - 1;
        pf[k] = base[e];
    }
}

// ... and from the registers into the LDS rows 0..nb-1.
template <typename R, typename V, int PD, int NPF>
__device__ __forceinline__ void pre_stage(const V (&pf)[NPF], R *rows, int RS, int nb, int tid)
{
    const int n = nb * PD;
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int e = tid + k * BLOCK;
        if (e < n) {
            const int i = e / PD, m = e - i * PD;
            st_coef<R, V>(rows, RS, i, m, pf[k]);
        }
    }
}

// L2L of one level with matrix cores: out row i (child i of parent row
// i >> 1 of par) += L2L(par row) for nb children.  The right child's
// operator follows from the left one by the signs (-1)^m on the input and
// (-1)^n on the output; the operator is triangular, so row tile rt takes no
// input moment below 16 rt: its loop runs over steps KB = 4 rt .. PD / 4 - 1,
// KB a constant of the instantiation, with every operand load issued before
// the first matrix instruction and two accumulator chains (even and odd
// steps) in flight.
template <typename R, typename V, int PD, int KB>
__device__ __forceinline__ void l2l_tile(const R (&al)[PD / 4], int rt, int ct0, int ctstep,
                                         int lane, int nb, const R *par, R *out, int RS)
{
    constexpr int NC = ncomp<V>::value;
    constexpr int KN = PD / 4 - KB;
    using A = typename acc_t<R>::type;
    const int nct = (NC * nb + 15) / 16;
    for (int ct = ct0; ct < nct; ct += ctstep) {
        const int j = 16 * ct + (lane & 15);
        const int i = j / NC, c = j % NC;
        const bool valid = i < nb;
        const int ic = valid ? i : 0;
        const bool left = (ic & 1) == 0;
        const R *sp = par + (size_t)(ic >> 1) * RS + c;
        R b[KN];
#pragma unroll
        for (int k = 0; k < KN; ++k)
            b[k] = sp[(4 * (KB + k) + (lane >> 4)) * NC];
        A acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < KN; ++k) {
            const int m = 4 * (KB + k) + (lane >> 4);
            R v = valid ? b[k] : R(0);
            if ((m & 1) && !left)
                v = -v;
            if (k & 1)
                acc1 = mma(al[KB + k], v, acc1);
            else
                acc0 = mma(al[KB + k], v, acc0);
        }
        if (!valid)
            continue;
        R *dst = out + (size_t)ic * RS + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * rt + out_row<R>(lane, r);
            const R v = acc0[r] + acc1[r];
            dst[n * NC] += (!left && (n & 1)) ? -v : v;
        }
    }
}

template <typename R, typename V, int PD>
__device__ __forceinline__ void l2l_tiles(const R (&al)[PD / 4], int rt, int ct0, int ctstep,
                                          int lane, int nb, const R *par, R *out, int RS)
{
    static_assert(PD % 16 == 0 && PD <= 64, "local length: 16, 32, 48 or 64");
    switch (rt) {
    case 0:
        l2l_tile<R, V, PD, 0>(al, rt, ct0, ctstep, lane, nb, par, out, RS);
        break;
    case 1:
        if constexpr (PD >= 32)
            l2l_tile<R, V, PD, 4>(al, rt, ct0, ctstep, lane, nb, par, out, RS);
        break;
    case 2:
        if constexpr (PD >= 48)
            l2l_tile<R, V, PD, 8>(al, rt, ct0, ctstep, lane, nb, par, out, RS);
        break;
    default:
        if constexpr (PD >= 64)
            l2l_tile<R, V, PD, 12>(al, rt, ct0, ctstep, lane, nb, par, out, RS);
        break;
    }
}

// M2L of every box of levels 3..l (the interaction lists of Section 2.1:
// the boxes at offsets -2, +2 and +-3 of the same level, whose parents
// neighbour the box's parent), written to pre (PD per box, packed per
// level like the multipoles).  Block 0 forms the level-2 regular part
// instead (it needs only the level-2 multipoles, and runs beside the M2L
// blocks).  Block 1 + k takes up to M2L_BOXES consecutive boxes of one
// level: k = 0, 1 levels 3, 4; then level 5 + j has 2^j blocks.
constexpr int M2L_BOXES = 32;

__host__ __device__ __forceinline__ int m2l_blocks(int l)
{
    return l < 3 ? 0 : (l == 3 ? 1 : (l == 4 ? 2 : 2 + (1 << (l - 4)) - 1));
}

template <typename R, typename V, int KER, int PD>
__device__ __forceinline__ void m2l_body(const DownArgs<R, V> &a, const UpArgs<R, V> &ua,
                                         int blk)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (blk == 0) {
        V *a2 = reinterpret_cast<V *>(smem_raw);
        regular_part<R, V, KER>(ua, a.PU, a2, a2 + 4 * a.PU);
        return;
    }
    blk -= 1;
    const int RS = a.RS;
    R *srcs = reinterpret_cast<R *>(smem_raw); // M2L_BOXES + 6 rows
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int L;
    int64_t b0;
    if (blk < 2) {
        L = 3 + blk;
        b0 = 0;
    } else {
        const int k = 31 - __clz(blk - 1); // blk - 1 in [2^k, 2^(k+1))
        L = 5 + k;
        b0 = (int64_t)(blk - 1 - (1 << k)) * M2L_BOXES;
    }
    const int nb = (1 << L) < M2L_BOXES ? (1 << L) : M2L_BOXES;
    const int64_t mask = (int64_t(1) << L) - 1;
    constexpr int nrt = PD / 16;
    const int used = (4 / nrt) * nrt;
    const int rt = wave % nrt, ct0 = wave / nrt, ctstep = 4 / nrt;
    DownOps<R, PD> ops;
    if (wave < used) {
        load_tile<R, PD>(ops.a4, a.T.m2l4, rt, lane);
        load_tile<R, PD>(ops.a6, a.T.m2l6, rt, lane);
    }
    // the multipoles of boxes b0 - 3 .. b0 + nb + 2 (around the circle),
    // first PD coefficients (every load of a thread issued first)
    const V *mpl = a.mp + lev_off(L, a.PU);
    const int n = (nb + 6) * PD;
    for (int e0 = 0; e0 < n; e0 += 8 * BLOCK) {
        V r[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int e = e0 + tid + k * BLOCK;
            e = e < n ? e : n - 1;
            const int i = e / PD, m = e - i * PD;
            r[k] = mpl[((b0 - 3 + i) & mask) * a.PU + m];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = e0 + tid + k * BLOCK;
            if (e < n) {
                const int i = e / PD, m = e - i * PD;
                st_coef<R, V>(srcs, RS, i, m, r[k]);
            }
        }
    }
    __syncthreads();
    const R sgl = KER == KER_COT ? (R)(ldexp(2.0, L) / 3.14159265358979323846) : R(1);
    const R lgl = KER == KER_LOG ? (R)log(ldexp((double)a.N, -(L + 1))) : R(0);
    constexpr int NC = ncomp<V>::value;
    // results straight to memory (each box's row: PD coefficients)
    R *dst = reinterpret_cast<R *>(a.pre + lev_off(L, PD) + b0 * PD);
    if (wave < used)
        m2l_tiles<R, V, KER, PD, false>(
            ops, rt, ct0, ctstep, lane, nb, srcs, srcs, RS,
            [&](int i, int o) { return i + 3 + o; }, [&](int) { return 0; },
            [&](int i) { return ((b0 + i) & 1) == 0; }, [&](int) { return sgl; },
            [&](int) { return lgl; }, [&](int i) { return i; }, dst, PD * NC);
}

// Complex load and store through a pointer of any address space (the
// batched kernels hold global-memory pointers as such).
template <typename R, typename P>
__device__ __forceinline__ cx<R> ld_cx(P p, int64_t i)
{
    return {p[i].re, p[i].im};
}
template <typename R, typename P>
__device__ __forceinline__ void st_cx(P p, int64_t i, cx<R> v)
{
    p[i].re = v.re;
    p[i].im = v.im;
}

template <typename R, typename V, int KER, int SRC, int EPI, int PD, int PH, bool IOT = false>
__device__ __forceinline__ void down_eval_body(const DownArgs<R, V> &a, int blk)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int RS = a.RS;
    const int s = a.l - a.lr;
    R *bufA = reinterpret_cast<R *>(smem_raw);
    R *bufB = bufA + (size_t)a.rows_buf * RS;
    R *srcs = bufB + (size_t)a.rows_buf * RS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (blk >= *a.nwork)
        return; // the grid is sized for the largest possible work list
    if constexpr (SRC == SET_SORTED)
        if (*a.flags & FLAG_DENSE)
            return; // the plan fails; nothing is evaluated
    const WorkItem w = a.work[blk];
    // per-call pointers: from the batch's table in the batched kernels (IOT);
    // the table holds global-memory pointers, which the casts tell the
    // compiler (as generic pointers they would take flat loads)
    using GC = const cx<R> __attribute__((address_space(1))) *;
    using G = cx<R> __attribute__((address_space(1))) *;
    const auto f_uniform = [&]() {
        if constexpr (IOT)
            return (GC)a.io[a.io_index].in;
        else
            return a.f_uniform;
    }();
    const auto f_hit = [&]() {
        if constexpr (IOT)
            return (GC)a.io[a.io_index].in;
        else
            return a.f_hit;
    }();
    const auto out = [&]() {
        if constexpr (IOT)
            return (G)a.io[a.io_index].out;
        else
            return a.out;
    }();
    if constexpr (PH == PH_TRANS)
        if (!w.lead)
            return; // another item of the same root forms its leaf locals
    const int64_t R0 = w.root;
    const int lr = a.lr;
    const int64_t N = a.N;
    R *cur = bufA;
    if constexpr (PH == PH_TRANS) {
    constexpr int nrt = PD / 16;
    const int used = (4 / nrt) * nrt;
    const int rt = wave % nrt, ct0 = wave / nrt, ctstep = 4 / nrt;
    // the first subtree level's M2L results: in flight during the
    // ancestors' work
    constexpr int NPF = (16 * PD + BLOCK - 1) / BLOCK; // subtrees of <= 4 levels
    V pf[NPF];
    if (lr < a.l)
        pre_fetch<R, V, PD, NPF>(pf, a.pre, R0, lr, lr + 1, tid);
    R al[PD / 4];
    if (wave < used)
        load_tile<R, PD>(al, a.T.l2l, rt, lane);

    // ---- local expansion of the subtree root R0 (level lr): the sum over
    // its ancestors A_L (L = 2..lr) of the M2L result at A_L (the regular-
    // part polynomial for L = 2) shifted from the centre of A_L to that of
    // R0:  u_A = rho u_R + delta,
    //      b^R_n = sum_{n' >= n} C(n', n) rho^n delta^(n'-n) b^A_n'.
    const int nA = lr - 2; // ancestors with M2L: levels 3..lr
    // X row 0: the level-2 local of R0's quarter; row li (1..nA): the M2L
    // result of the ancestor at level li + 2 (all loads issued first)
    for (int b0 = 0; b0 < (nA + 1) * PD; b0 += 4 * BLOCK) {
        V r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int idx = b0 + tid + k * BLOCK;
            idx = idx < (nA + 1) * PD ? idx : (nA + 1) * PD - 1; // clamped: no branch
            const int li = idx / PD, n = idx - li * PD;
            r[k] = li == 0 ? a.loc2[(R0 >> (lr - 2)) * PD + n]
                           : a.pre[lev_off(li + 2, PD) + (R0 >> (lr - 2 - li)) * PD + n];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = b0 + tid + k * BLOCK;
            if (idx < (nA + 1) * PD) {
                const int li = idx / PD, n = idx - li * PD;
                st_coef<R, V>(bufA, RS, li, n, r[k]);
            }
        }
    }
    // the L2L table, for the shift below (after the two level buffers)
    R *tl2l = srcs; // PD x PD, [in n'][out n]
    {
        static_assert((PD * PD) % BLOCK == 0, "PD^2 must be a multiple of the block");
        R rl[PD * PD / BLOCK];
#pragma unroll
        for (int k = 0; k < PD * PD / BLOCK; ++k)
            rl[k] = a.T.l2l[tid + k * BLOCK];
#pragma unroll
        for (int k = 0; k < PD * PD / BLOCK; ++k)
            tl2l[tid + k * BLOCK] = rl[k];
    }
    __syncthreads();
    // shift every row of X to the root (bufB rows), then sum; consecutive
    // threads take the rows of one coefficient n, so that a wavefront's
    // sums (PD - n terms) have nearly the same length
    for (int idx = tid; idx < (nA + 1) * PD; idx += BLOCK) {
        const int n = idx / (nA + 1), li = idx - n * (nA + 1);
        const int sh = nA - li; // lr - L
        const int64_t A = R0 >> sh;
        // 2 rho = 2^(1 - sh); -2 delta with delta = ((2 R0 + 1) - (2A + 1) 2^sh) / 2^sh;
        // C(n',n) = l2l[n'][n] 2^n' (-1)^(n'-n) = l2l[n'][n] 2^n (-2)^(n'-n)
        const R rho2 = (R)ldexp(2.0, -sh);
        const R md2 = (R)(-2.0 * ldexp((double)((2 * R0 + 1) - ((2 * A + 1) << sh)), -sh));
        V acc = vzero<V>();
        R pw = R(1);
        // the table from LDS; a partial unroll keeps several reads in flight
        // without the register cost of a full one
#pragma unroll 4
        for (int np = n; np < PD; ++np) {
            vfma(acc, tl2l[np * PD + n] * pw, ld_coef<R, V>(bufA, RS, li, np));
            pw *= md2;
        }
        st_coef<R, V>(bufB, RS, li, n, vscale(acc, ipow(rho2, n)));
    }
    __syncthreads();
    // the leaf locals end in bufA after the s levels below
    cur = (s & 1) ? bufB : bufA;
    R *nxt = (s & 1) ? bufA : bufB;
    for (int n = tid; n < PD; n += BLOCK) {
        V acc = ld_coef<R, V>(bufB, RS, 0, n);
        for (int li = 1; li <= nA; ++li)
            vadd(acc, ld_coef<R, V>(bufB, RS, li, n));
        st_coef<R, V>(cur, RS, 0, n, acc);
    }
    __syncthreads();

    // ---- the subtree's levels: each box's local is its M2L result (staged
    // in the output rows) plus the L2L of its parent's local (matrix cores;
    // the next level's M2L results are fetched while this level runs)
    for (int lev = lr + 1; lev <= a.l; ++lev) {
        const int nb = 1 << (lev - lr);
        pre_stage<R, V, PD, NPF>(pf, nxt, RS, nb, tid);
        __syncthreads();
        if (lev < a.l)
            pre_fetch<R, V, PD, NPF>(pf, a.pre, R0, lr, lev + 1, tid);
        if (wave < used)
            l2l_tiles<R, V, PD>(al, rt, ct0, ctstep, lane, nb, cur, nxt, RS);
        __syncthreads();
        R *t = cur;
        cur = nxt;
        nxt = t;
    }
    } // PH_TRANS
    const int64_t leaf0 = R0 << s;
    if constexpr (PH == PH_TRANS) { // the leaf locals (in bufA) go out
        V *g = a.leaf_loc + leaf0 * PD;
        for (int idx = tid; idx < (PD << s); idx += BLOCK)
            g[idx] = ld_coef<R, V>(cur, RS, idx / PD, idx % PD);
        return;
    } else { // ... and come back for the evaluation (all loads in flight)
        const V *g = a.leaf_loc + leaf0 * PD;
        const int n = PD << s; // at most 16 PD: 4 PD / 64 per thread
        constexpr int NL = (16 * PD + BLOCK - 1) / BLOCK;
        V v[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int idx = tid + k * BLOCK;
            v[k] = g[idx < n ? idx : n - 1];
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int idx = tid + k * BLOCK;
            if (idx < n)
                st_coef<R, V>(bufA, RS, idx / PD, idx % PD, v[k]);
        }
        __syncthreads();
    }
    const R *leafloc = bufA;
    const double invN = 1.0 / (double)N;
    const double lscale = ldexp(1.0, a.l) * invN;

    // sorted near-field sources of the subtree and its two neighbour leaves,
    // staged in the LDS left free by the translations when they fit
    NearStage<R> ns{};
    bool staged = false;
    int64_t base = 0;
    if constexpr (SRC == SET_SORTED) {
        const int nb = 1 << s;
        const int64_t nleaf = int64_t(1) << a.l;
        const int64_t bl = leaf0 == 0 ? nleaf - 1 : leaf0 - 1;
        const int64_t br = leaf0 + nb == nleaf ? 0 : leaf0 + nb;
        const int32_t oL = a.src.off[bl], cL = a.src.off[bl + 1] - oL;
        const int32_t oM = a.src.off[leaf0], cM = a.src.off[leaf0 + nb] - oM;
        const int32_t oR = a.src.off[br], cR = a.src.off[br + 1] - oR;
        const int32_t total = cL + cM + cR;
        constexpr bool WS = EPI == EPI_INV || EPI == EPI_ADJ; // weights staged
        constexpr int wb = WS ? (int)sizeof(cx<R>) : 0;
        const int32_t cap = ((a.near_bytes - 4 * (nb + 4)) / (16 + wb)) & ~1;
        base = uni_start(leaf0, a.l, N);
        if (total <= cap) {
            unsigned char *fr = reinterpret_cast<unsigned char *>(bufB); // 16-byte aligned
            ns.p = reinterpret_cast<double2 *>(fr);
            ns.w = reinterpret_cast<cx<R> *>(fr + 16 * (size_t)cap);
            ns.off = reinterpret_cast<int32_t *>(fr + (16 + wb) * (size_t)cap);
            ns.self0 = cL - oM;
            const int64_t shL = leaf0 == 0 ? -N : 0, shR = leaf0 + nb == nleaf ? N : 0;
            // every load of a batch in flight at once (indices clamped)
            for (int32_t i0 = 0; i0 < total; i0 += 4 * BLOCK) {
                int32_t mv[4];
                double tv[4];
                cx<R> wv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int32_t i = i0 + tid + k * BLOCK;
                    i = i < total ? i : total - 1;
                    const int32_t t = i < cL ? oL + i
                                             : (i < cL + cM ? oM + (i - cL) : oR + (i - cL - cM));
                    mv[k] = a.src.m[t];
                    tv[k] = a.src.th[t];
                    if constexpr (WS)
                        wv[k] = a.w_sorted[t];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int32_t i = i0 + tid + k * BLOCK;
                    if (i < total) {
                        const int64_t sh = i < cL ? shL : (i < cL + cM ? 0 : shR);
                        // adjoint: a source on a grid point has weight 0
                        // (F_j = 0); it is staged a quarter unit away, so
                        // that its own grid point never divides by 0
                        ns.p[i] = make_double2((double)(mv[k] + sh - base),
                                               (EPI == EPI_ADJ && tv[k] == 0.0) ? 0.25 : tv[k]);
                        if constexpr (WS)
                            ns.w[i] = wv[k];
                    }
                }
            }
            for (int i = tid; i <= nb + 2; i += BLOCK)
                ns.off[i] = i == 0 ? 0
                                   : (i == nb + 2 ? total
                                                  : cL + (a.src.off[leaf0 + i - 1] - oM));
            staged = true;
        }
        __syncthreads();
    }

    if constexpr (EPI == EPI_FWD) {
        // stage the near-field sources of the subtree (uniform sources),
        // reusing the source buffer
        const cx<R> *fsp = nullptr;
        int64_t K0 = 0;
        if constexpr (SRC == SET_UNIFORM) {
            cx<R> *fs = reinterpret_cast<cx<R> *>(bufB);
            K0 = uni_start_unwrapped(leaf0 - 1, a.l, N);
            const int64_t K1 = uni_start_unwrapped(leaf0 + (1 << s) + 1, a.l, N);
            if (K1 - K0 <= a.near_bytes / (int)sizeof(cx<R>)) {
                const int32_t nk = (int32_t)(K1 - K0);
                // every load of a batch in flight at once (indices clamped)
                // every load of a batch in flight at once (indices clamped)
                for (int32_t i0 = 0; i0 < nk; i0 += 8 * BLOCK) {
                    cx<R> v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        int32_t i = i0 + tid + u * BLOCK;
                        i = i < nk ? i : nk - 1;
                        int64_t k = K0 + i;
                        k = k < 0 ? k + N : (k >= N ? k - N : k);
                        v[u] = ld_cx<R>(f_uniform, k);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int32_t i = i0 + tid + u * BLOCK;
                        if (i < nk)
                            fs[i] = v[u];
                    }
                }
                fsp = fs;
            }
            __syncthreads();
        }
        const V S = *a.S;
        const double hscale = (double)N / 3.14159265358979323846;
        // the targets arrive sorted by subtree only: group the item's
        // targets by leaf in LDS (a counting sort of their indices), so that
        // the lanes of a wavefront share the leaf local and the near-field
        // sources they read
        const int nb = 1 << s;
        const int32_t nt = w.t1 - w.t0; // at most FWD_TMAX
        int32_t *cnt = reinterpret_cast<int32_t *>(smem_raw + a.grp_lds); // nb + 1
        int32_t *ord = cnt + (nb + 1);                                     // nt
        for (int i = tid; i <= nb; i += BLOCK)
            cnt[i] = 0;
        __syncthreads();
        constexpr int GPT = FWD_TMAX / BLOCK; // targets per thread
        int32_t gl[GPT], gr[GPT];
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
            const int32_t i = tid + u * BLOCK;
            const SortedPt pt = a.tgt_pt[w.t0 + (i < nt ? i : nt - 1)];
            gl[u] = (int32_t)(box_of(pt.m, pt.th, a.l, N, invN) - leaf0);
        }
#pragma unroll
        for (int u = 0; u < GPT; ++u)
            gr[u] = tid + u * BLOCK < nt ? atomicAdd(&cnt[gl[u] + 1], 1) : 0;
        __syncthreads();
        if (tid == 0)
            for (int i = 1; i <= nb; ++i)
                cnt[i] += cnt[i - 1];
        __syncthreads();
        // (index in the item) + (leaf in the subtree) * 2^16
#pragma unroll
        for (int u = 0; u < GPT; ++u)
            if (tid + u * BLOCK < nt)
                ord[cnt[gl[u]] + gr[u]] = (tid + u * BLOCK) | (gl[u] << 16);
        __syncthreads();
        for (int32_t q = tid; q < nt; q += BLOCK) {
            const int32_t oq = ord[q];
            const int32_t t = w.t0 + (oq & 0xffff);
            const SortedPt pt = a.tgt_pt[t];
            const int64_t tm = pt.m;
            const double th = pt.th;
            const int32_t j = pt.perm;
            if (th == 0.0) { // exact hit: K_jk is the Kronecker delta
                st_cx<R>(out, j, ld_cx<R>(f_hit, tm == N ? 0 : tm));
                continue;
            }
            const int64_t leaf = leaf0 + (oq >> 16);
            const R u = (R)rel_coord_r(tm, th, leaf, a.l, N, invN);
            V h = horner4<R, V, PD>(leafloc, RS, (int)(leaf - leaf0), u);
            const cx<double> nr =
                near_cot<R, V, SRC>(a, tm, th, leaf, fsp, K0, (const cx<R> *)f_uniform);
            double hr = (double)h.re + hscale * nr.re;
            double hi = (double)h.im + hscale * nr.im;
            // g = -(F/2)(S + i h), F = 2i sin(pi th) e^{i pi th} / N
            double sp = sinpi(th), cp = cospi(th);
            double Fr = -2.0 * sp * sp * invN, Fi = 2.0 * sp * cp * invN;
            double Ar = (double)S.re - hi, Ai = (double)S.im + hr;
            cx<R> g = {(R)(-0.5 * (Fr * Ar - Fi * Ai)), (R)(-0.5 * (Fr * Ai + Fi * Ar))};
            st_cx<R>(out, j, g);
        }
    } else if constexpr (EPI == EPI_INV) {
        const V W = *a.S;
        const double hscale = (double)N / 3.14159265358979323846;
        for (int32_t k = w.u0 + tid; k < w.u1; k += BLOCK) {
            const int32_t hj = a.hit[k];
            if (hj >= 0) { // exact hit: C_k = 0 and f_k = g_j
                st_cx<R>(out, k, a.gin[hj]);
                continue;
            }
            const int64_t leaf = uni_leaf(k, a.l, N, lscale);
            const int il = (int)(leaf - leaf0);
            const R u = (R)rel_coord_r(k, 0.0, leaf, a.l, N, invN);
            V h = horner4<R, V, PD>(leafloc, RS, il, u);
            const cx<double> nr =
                staged ? near_cot_staged<R, true>(ns, ns.off[il], ns.off[il + 3],
                                                  (int32_t)(k - base), 0.0)
                       : near_cot<R, V, SRC>(a, k, 0.0, leaf, nullptr, 0,
                                             (const cx<R> *)f_uniform);
            double hr = (double)h.re + hscale * nr.re;
            double hi = (double)h.im + hscale * nr.im;
            // f = -(C/2)(W + i h)
            const double C = a.chat[k];
            st_cx<R>(out, k, cx<R>{(R)(-0.5 * C * ((double)W.re - hi)),
                                   (R)(-0.5 * C * ((double)W.im + hr))});
        }
    } else if constexpr (EPI == EPI_ADJ) {
        // adjoint of Eq. (p2): f_k = sum_j G(x_k - y_j) conj(F_j) g_j
        //                          = -(W + i h_k) / 2 with the weights
        // w_j = conj(F_j) g_j (sources on grid points add g_j afterwards)
        const V W = *a.S;
        const double hscale = (double)N / 3.14159265358979323846;
        for (int32_t k = w.u0 + tid; k < w.u1; k += BLOCK) {
            const int64_t leaf = uni_leaf(k, a.l, N, lscale);
            const int il = (int)(leaf - leaf0);
            const R u = (R)rel_coord_r(k, 0.0, leaf, a.l, N, invN);
            V h = horner4<R, V, PD>(leafloc, RS, il, u);
            const cx<double> nr =
                staged ? near_cot_staged<R, true>(ns, ns.off[il], ns.off[il + 3],
                                                  (int32_t)(k - base), 0.0)
                       : near_cot<R, V, SRC>(a, k, 0.0, leaf, nullptr, 0,
                                             (const cx<R> *)f_uniform);
            const double hr = (double)h.re + hscale * nr.re;
            const double hi = (double)h.im + hscale * nr.im;
            st_cx<R>(out, k, cx<R>{(R)(-0.5 * ((double)W.re - hi)),
                                   (R)(-0.5 * ((double)W.im + hr))});
        }
    } else { // EPI_LOGCD
        // log|Chat_k| and log|Dhat_j| by the FMM; then the coefficients of
        // Eq. (p8), rescaled by 2^N (the scale cancels in C_k D_j):
        //   Chat_k = (-1)^k prod_j 2 sin((x_k - y_j)/2)
        //          = (-1)^(k + #{j: s_j > k}) exp(log|Chat_k|)  (0 on a hit),
        //   Dhat_j = i e^{-i N y_j / 2} / prod_{i != j} 2 sin((y_j - y_i)/2)
        //          = i (-1)^(m_j) e^{-i pi th_j} (-1)^(#{i: s_i > s_j}) exp(log|Dhat_j|),
        // with the points sorted along the circle, so #{i: s_i > s_j} =
        // N - 1 - rank.
        for (int32_t k = w.u0 + tid; k < w.u1; k += BLOCK) {
            const int64_t leaf = uni_leaf(k, a.l, N, lscale);
            const int il = (int)(leaf - leaf0);
            const R u = (R)rel_coord_r(k, 0.0, leaf, a.l, N, invN);
            V far = horner4<R, V, PD>(leafloc, RS, il, u);
            // log|Chat_k| = lt + log(prod), prod in [1/2, 1]: |Chat_k| =
            // prod exp(lt) without the logarithm of the product (lt is at
            // most 0.7 above log|Chat_k|, and the range test below uses
            // that bound)
            double prod = 1.0, lt;
            if (staged) {
                int expo;
                near_prod_staged<R, true>(ns, ns.off[il], ns.off[il + 3], -1,
                                          (int32_t)(k - base), 0.0, &prod, &expo);
                lt = ((double)far - near_log_background(k, 0.0, leaf, a.l, N)) +
                     (double)expo * 0.69314718055994530942;
            } else {
                lt = (double)far + near_log<R, V>(a, k, 0.0, leaf, -1);
            }
            // #{j : s_j <= k}: the points of the leaves before k's leaf, plus
            // a binary search over the (sorted) points of k's leaf
            int32_t lo, hi;
            if (staged) {
                const double tmr = (double)(k - base);
                lo = ns.off[il + 1];
                hi = ns.off[il + 2];
                const int32_t j0 = lo;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    const double2 pm = ns.p[mid];
                    if (pm.x < tmr || (pm.x == tmr && pm.y <= 0.0))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                lo = a.src.off[leaf] + (lo - j0);
            } else {
                lo = a.src.off[leaf];
                hi = a.src.off[leaf + 1];
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    const int32_t mm = a.src.m[mid];
                    if (mm < k || (mm == k && a.src.th[mid] <= 0.0))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
            }
            const int64_t neg = N - lo;
            if (a.hit[k] >= 0) {
                a.chat_out[k] = 0.0;
            } else {
                // |log|Chat_k|| <= log_max for lt - 0.7 ... lt
                if (!(lt <= a.log_max && lt - 0.69314718055994530942 >= -a.log_max))
                    atomicOr(a.flags_out, FLAG_RANGE);
                a.chat_out[k] = (((k + neg) & 1) ? -prod : prod) * exp(lt);
            }
        }
        for (int32_t t = w.t0 + tid; t < w.t1; t += BLOCK) {
            const int64_t tm = a.tgt.m[t];
            const double th = a.tgt.th[t];
            const int64_t leaf = a.tgt_leaf[t]; // the sort's key of every point
            const int il = (int)(leaf - leaf0);
            const R u = (R)rel_coord_r(tm, th, leaf, a.l, N, invN);
            V far = horner4<R, V, PD>(leafloc, RS, il, u);
            // the net count of Omega_1 carried log(2 pi / N) for the point
            // itself, whose log|t| term the near field skips:
            // log|Dhat_j| = lt - log(prod), prod in [1/2, 1], so |Dhat_j| =
            // exp(lt) / prod (lt is at most 0.7 below log|Dhat_j|)
            double prod = 1.0, lt;
            if (staged) {
                int expo;
                near_prod_staged<R, false>(ns, ns.off[il], ns.off[il + 3], t + ns.self0,
                                           (int32_t)(tm - base), th, &prod, &expo);
                lt = -(((double)far - near_log_background(tm, th, leaf, a.l, N)) +
                       (double)expo * 0.69314718055994530942 - a.logself);
            } else {
                lt = -((double)far + near_log<R, V>(a, tm, th, leaf, t) - a.logself);
            }
            if (!(lt >= -a.log_max && lt + 0.69314718055994530942 <= a.log_max))
                atomicOr(a.flags_out, FLAG_RANGE);
            const double sg = (((tm + (N - 1 - t)) & 1) ? -1.0 : 1.0) * exp(lt) / prod;
            double sp, cp;
            sincospi(th, &sp, &cp);
            a.dhat_out[t] = {sg * sp, sg * cp};
        }
    }
}

// The M2L of every box (levels 3..l), one launch.
template <typename R, typename V, int KER, int PD>
__global__ void __launch_bounds__(BLOCK) k_m2l(DownArgs<R, V> a, UpArgs<R, V> ua)
{
    m2l_body<R, V, KER, PD>(a, ua, blockIdx.x);
}

// at least 4 waves per SIMD (at most 128 VGPRs) up to 32 terms (the L2L
// tile is the only operator held in registers); 2 beyond
template <typename R, typename V, int KER, int SRC, int EPI, int PD>
__global__ void __launch_bounds__(BLOCK, (PD <= 32 ? 4 : 2)) k_down_trans(DownArgs<R, V> a)
{
    down_eval_body<R, V, KER, SRC, EPI, PD, PH_TRANS>(a, blockIdx.x);
}

// at least 4 waves per SIMD (at most 128 VGPRs; the evaluation needs 64-112)
template <typename R, typename V, int KER, int SRC, int EPI, int PD>
__global__ void __launch_bounds__(BLOCK, 4) k_down_eval(DownArgs<R, V> a)
{
    down_eval_body<R, V, KER, SRC, EPI, PD, PH_EVAL>(a, blockIdx.x);
}

// The downward pass of every problem of a batch in one launch (each phase).
// The forward's input and output come from the IoPtr table the arguments
// point to (io, passed as well, is the same table).
template <typename R, typename V, int KER, int SRC, int EPI, int PD, int PH>
__device__ __forceinline__ void down_batched(const DownArgs<R, V> *aa, BlockMap bm,
                                             const IoPtr *io)
{
    int blk, nblk;
    const int t = bm_find(bm, blockIdx.x, &blk, &nblk);
    // the arguments read in place (a copy of them ended up in scratch
    // memory); the per-call pointers come from the table they point to
    down_eval_body<R, V, KER, SRC, EPI, PD, PH, true>(aa[t], blk);
}

template <typename R, typename V, int KER, int PD>
__global__ void __launch_bounds__(BLOCK) kb_m2l(const DownArgs<R, V> *aa, BlockMap bm,
                                                const UpArgs<R, V> *uu)
{
    int blk, nblk;
    const int t = bm_find(bm, blockIdx.x, &blk, &nblk);
    m2l_body<R, V, KER, PD>(aa[t], uu[t], blk);
}

template <typename R, typename V, int KER, int SRC, int EPI, int PD>
__global__ void __launch_bounds__(BLOCK) kb_down_trans(const DownArgs<R, V> *aa, BlockMap bm,
                                                       const IoPtr *io)
{
    down_batched<R, V, KER, SRC, EPI, PD, PH_TRANS>(aa, bm, io);
}

template <typename R, typename V, int KER, int SRC, int EPI, int PD>
__global__ void __launch_bounds__(BLOCK, 4) kb_down_eval(const DownArgs<R, V> *aa,
                                                         BlockMap bm, const IoPtr *io)
{
    down_batched<R, V, KER, SRC, EPI, PD, PH_EVAL>(aa, bm, io);
}

} // namespace fn
