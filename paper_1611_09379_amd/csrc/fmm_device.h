// Device-side building blocks of the circular-tree FMM (gfx950).
//
// Geometry is kept in grid units: a point y in radians is s = N y / (2 pi),
// stored as an exact integer part m and a binary64 fraction th in
// [-1/2, 1/2], with the representative s = m + th in [0, N) (m may equal N
// when th < 0).  The uniform points x_k = 2 pi k / N are s = k.  Level L of
// the binary tree (Section 2.1) splits [0, N) into 2^L equal arcs; box b of
// level L has centre c = (b + 1/2) N / 2^L and half-width r = N / 2^(L+1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fn {

// Error flags the setup kernels raise (one int in device memory).
enum {
    FLAG_BAD_Y = 1, // non-finite or too large y
    FLAG_DUP = 2,   // two points coincide (inverse)
    FLAG_RANGE = 4, // |C_k| or |D_j| outside the binary64 range (inverse)
    FLAG_DENSE = 8  // a leaf far denser than the average (inverse)
};

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// First multipole / local coefficient of level L in the packed per-level
// arrays (levels 2..lmax, 2^L boxes each).
// Leaf stride (elements) of uniform-grid weights staged in LDS for the
// matrix-core P2M: B complex weights per leaf, padded so that consecutive
// leaves start 8 elements apart modulo the 256-byte bank cycle.
__host__ __device__ __forceinline__ int uni_stage_stride(int B, int es)
{
    const int W = 256 / es;
    return 2 * B + (((8 - 2 * B) % W) + W) % W;
}

__host__ __device__ __forceinline__ int64_t lev_off(int L, int P)
{
    return ((int64_t(1) << L) - 4) * (int64_t)P;
}

// floor((m + th) 2^L / N), clamped to [0, 2^L): the level-L box of the
// point s = m + th (0 <= m <= N, |th| <= 1/2).  A binary64 estimate (with
// invN = 1/N rounded, off by at most one) is corrected by exact comparisons:
// b N - m 2^L is an exact integer (below 2^53) and th 2^L an exact binary64
// value.  The sort and the evaluation both use this function, so they always
// agree.
__device__ __forceinline__ int64_t box_of(int64_t m, double th, int L, int64_t N, double invN)
{
    const int64_t A = m << L;
    const double tl = ldexp(th, L);
    int64_t b = (int64_t)floor(((double)A + tl) * invN);
    // s >= b N / 2^L  <=>  b N - A <= tl
    if ((double)(b * N - A) > tl)
        --b;
    else if ((double)((b + 1) * N - A) <= tl)
        ++b;
    const int64_t nb = int64_t(1) << L;
    return b < 0 ? 0 : (b >= nb ? nb - 1 : b);
}

// A sorted target of the forward transform: grid units and input index.
struct alignas(16) SortedPt {
    int32_t m;
    int32_t perm;
    double th;
};

// (s - c) / r for the point s = m + th and box b of level L.
__device__ __forceinline__ double rel_coord(int64_t m, double th, int64_t b,
                                            int L, int64_t N)
{
    int64_t num = (m << (L + 1)) - (2 * b + 1) * N;
    return ((double)num + ldexp(th, L + 1)) / (double)N;
}

// rel_coord with the division replaced by a product with invN = 1 / N.
__device__ __forceinline__ double rel_coord_r(int64_t m, double th, int64_t b,
                                              int L, int64_t N, double invN)
{
    int64_t num = (m << (L + 1)) - (2 * b + 1) * N;
    return ((double)num + ldexp(th, L + 1)) * invN;
}

// First uniform point k of box b at level L: ceil(b N / 2^L).
__device__ __forceinline__ int64_t uni_start(int64_t b, int L, int64_t N)
{
    return (b * N + (int64_t(1) << L) - 1) >> L;
}

// Integer power by squaring (v^e, e >= 0).
template <typename R>
__device__ __forceinline__ R ipow(R v, int e)
{
    R r = R(1);
    while (e) {
        if (e & 1)
            r *= v;
        v *= v;
        e >>= 1;
    }
    return r;
}

// d = n + (a - b) with one rounding (a, b in [-1/2, 1/2]); the difference
// a - b is carried as an exact two-term sum.
__device__ __forceinline__ double grid_diff(int64_t n, double a, double b)
{
    double hi = a - b;
    double bb = hi - a;
    double lo = (a - (hi - bb)) + (-b - bb);
    return ((double)n + hi) + lo;
}

// Antiderivative of log|u|: u log|u| - u (0 at u = 0).
__device__ __forceinline__ double xlogx_m_x(double u)
{
    return u == 0.0 ? 0.0 : u * log(fabs(u)) - u;
}

// Launch of one kernel over several problems: block b of the grid belongs
// to problem t with start[t] <= b < start[t + 1] and is its local block
// b - start[t].
struct BlockMap {
    const int32_t *start; // T + 1 entries
    int T;
};

__device__ __forceinline__ int bm_find(const BlockMap &bm, int b, int *local, int *count)
{
    int lo = 0, hi = bm.T; // largest t with start[t] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bm.start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    *local = b - bm.start[lo];
    *count = bm.start[lo + 1] - bm.start[lo];
    return lo;
}

// Input and output of one problem of a batch, read by the batched
// evaluation launches (so that their arguments stay fixed from call to call).
struct IoPtr {
    const void *in;
    void *out;
};

// One workgroup's share of the downward pass: a subtree root of level lr,
// a range of sorted targets and a range of uniform targets.
struct WorkItem {
    int64_t root;
    int32_t t0, t1;
    int32_t u0, u1;
    int32_t lead; // the first item of its root (forms the root's leaf locals)
    int32_t pad;
};

} // namespace fn
