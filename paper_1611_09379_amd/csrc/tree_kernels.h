// Setup step ("setting the data structure", Section 3.3): reduction of the
// points to grid units, the sort of the points into the leaves of the
// circular binary tree (Section 2.1), and for the inverse the assembly of
// C_k and D_j of Eq. (p8) from their log-sums.
#pragma once

#include "fmm_device.h"

namespace fn {

// s = y (c_hi + c_lo) in double-double, split into the nearest integer n
// and the remainder th.  Contraction stays off: fusing p - n with
// p = y c_hi into one fma would count the rounding error of y c_hi twice.
// (Returned by value: outputs through pointers would put the caller's
// locals in scratch memory around the call.)
constexpr double HIT_SNAP = 0x1p-100; // grid units

struct GridUnits {
    double n, th;
};
__device__ __noinline__ GridUnits grid_units(double y, double c_hi, double c_lo)
{
#pragma clang fp contract(off)
    double p = y * c_hi;
    double e = fma(y, c_hi, -p);
    e = fma(y, c_lo, e);
    double n = rint(p);
    return {n, (p - n) + e};
}

// y -> (m, th): s = y N / (2 pi) in double-double from the double-double
// constant N/(2 pi) = c_hi + c_lo; m = nearest integer mod N, th = s -
// nearest integer in [-1/2, 1/2]; the representative in [0, N) uses m = N
// when m = 0 and th < 0.  A fraction below HIT_SNAP in magnitude becomes 0:
// such a point is an exact hit (Eq. p2 then gives g_j = f_m up to a term of
// order th, far below any tolerance), where 1/th would leave the binary32
// (and near 1e-308 the binary64) range.  Returns false for a non-finite or
// too large y.
__device__ __forceinline__ bool reduce_point(double yy, double c_hi, double c_lo,
                                             int64_t N, double invN, double ymax,
                                             int64_t *m_out, double *th_out)
{
    if (!(fabs(yy) <= ymax)) { // also catches NaN
        *m_out = 0;
        *th_out = 0.25;
        return false;
    }
    const GridUnits gu = grid_units(yy, c_hi, c_lo);
    double n = gu.n, th = gu.th;
    if (th > 0.5) {
        th -= 1.0;
        n += 1.0;
    } else if (th < -0.5) {
        th += 1.0;
        n -= 1.0;
    }
    if (fabs(th) < HIT_SNAP)
        th = 0.0;
    // m = n mod N in binary64: n and q N are integers below 2^53, so the
    // difference is exact; the quotient estimate is off by at most one
    const double dN = (double)N;
    double mr = n - floor(n * invN) * dN;
    if (mr < 0.0)
        mr += dN;
    else if (mr >= dN)
        mr -= dN;
    int64_t m = (int64_t)mr;
    if (m == 0 && th < 0.0)
        m = N;
    *m_out = m;
    *th_out = th;
    return true;
}

// Arguments of the counting sort of one point set into the leaves (all the
// passes share them).
struct SortArgs {
    int64_t n;              // points
    const double *y;        // radians
    double c_hi, c_lo;      // N / (2 pi) in double-double
    int64_t N;
    double invN;            // 1 / N
    int l, keyshift;        // key = level-(l - keyshift) box
    double ymax;
    int64_t chunk;          // points per histogram block
    int nbins, nblk;        // keys; histogram blocks
    int32_t *um;            // unsorted grid units and keys
    double *uth;
    int32_t *ukey;
    int32_t *H;             // nblk x nbins block histograms
    int32_t *tot;           // points per key
    int32_t *off;           // nbins + 1 offsets
    int32_t *cursor;        // (atomic path) placement cursors
    int32_t *sm;            // sorted m, th, perm, key
    double *sth;
    int32_t *sperm;
    int32_t *skey;
    SortedPt *spt;          // if set: sorted (m, perm, th) records instead
                            // of sm, sth, sperm, skey (forward targets)
    int32_t *hit;           // (optional) index of a point on x_m, per m
    int *flags;
    // k_hist also prepares the plan's device state (nothing of it is read
    // before k_place): init_flags clears the flags, and a non-zero nhit fills
    // hit[0 .. nhit) with -1 (no grid point is hit)
    int init_flags;
    int64_t nhit;
};

// Grid units and sort key (the level-(l - keyshift) box) of one point.  The
// histogram and placement passes each compute them from y: cheaper than
// writing them out once and reading them back.
__device__ __forceinline__ int32_t point_key(const SortArgs &a, double yy, int32_t *m_out,
                                             double *th_out, bool *ok)
{
    int64_t m;
    double th;
    *ok = reduce_point(yy, a.c_hi, a.c_lo, a.N, a.invN, a.ymax, &m, &th);
    *m_out = (int32_t)m;
    *th_out = th;
    return (int32_t)(box_of(m, th, a.l, a.N, a.invN) >> a.keyshift);
}

constexpr int SORT_BATCH = 8;     // points in flight per thread in the sort passes
constexpr int SORT_THREADS = 1024; // threads of a histogram / placement block

// Counting sort, pass 1: per-block histograms of the keys in LDS.  Block b
// takes points [b chunk, (b+1) chunk); H is block-major, H[b nbins + key].
// Runs of equal keys in consecutive lanes of a wavefront (nearly sorted
// input, e.g. a jittered grid, puts a wave's points into one or two keys):
// *start = first lane of my run, *len = its length where I am its first
// lane (0 elsewhere).  One LDS atomic per run then replaces one per lane.
__device__ __forceinline__ void key_runs(int32_t key, int *start, int *len)
{
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(key, 1);
    const bool head = lane == 0 || key != prev;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    *start = 63 - __clzll(heads & upto);
    const unsigned long long above = heads & ~upto;
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    *len = head ? next - lane : 0;
}

__device__ __forceinline__ void hist_body(const SortArgs &a, int blk)
{
    extern __shared__ int32_t hist[];
    const int nbins = a.nbins;
    if (a.init_flags && blk == 0 && threadIdx.x == 0)
        *a.flags = 0;
    for (int64_t i = (int64_t)blk * SORT_THREADS + threadIdx.x; i < a.nhit;
         i += (int64_t)a.nblk * SORT_THREADS)
        a.hit[i] = -1;
    for (int i = threadIdx.x; i < nbins; i += SORT_THREADS)
        hist[i] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blk * a.chunk;
    const int64_t j1 = j0 + a.chunk < a.n ? j0 + a.chunk : a.n;
    // every lane runs every iteration (key_runs works across the wavefront)
    for (int64_t jw = j0; jw < j1; jw += SORT_THREADS * SORT_BATCH) {
        const int64_t jb = jw + threadIdx.x;
        int32_t key[SORT_BATCH];
        double yv[SORT_BATCH];
#pragma unroll
        for (int u = 0; u < SORT_BATCH; ++u) { // loads clamped: all in flight
            const int64_t j = jb + u * SORT_THREADS;
            yv[u] = a.y[j < j1 ? j : j1 - 1];
        }
#pragma unroll
        for (int u = 0; u < SORT_BATCH; ++u) {
            const int64_t j = jb + u * SORT_THREADS;
            // (a slot past the chunk for every lane of the wave costs no
            // key computation: small chunks fill half the batch)
            key[u] = -1;
            if (j < j1) {
                int32_t mm;
                double tt;
                bool ok;
                key[u] = point_key(a, yv[u], &mm, &tt, &ok);
            }
        }
#pragma unroll
        for (int u = 0; u < SORT_BATCH; ++u) {
            int start, len;
            key_runs(key[u], &start, &len);
            if (len && key[u] >= 0)
                atomicAdd(&hist[key[u]], len);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += SORT_THREADS)
        a.H[(int64_t)blk * nbins + i] = hist[i];
}

__global__ void __launch_bounds__(SORT_THREADS) k_hist(SortArgs a) { hist_body(a, blockIdx.x); }

// A plan's device state before its sort, in one launch: the error flags
// (nflags words, when flags is given) to 0 and the hit table (nhit entries,
// when hit is given) to -1 (no grid point is hit).
__global__ void __launch_bounds__(256) k_init(int *flags, int nflags, int32_t *hit,
                                              int64_t nhit)
{
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (flags && i0 < nflags)
        flags[i0] = 0;
    if (hit)
        for (int64_t i = i0; i < nhit; i += (int64_t)gridDim.x * blockDim.x)
            hit[i] = -1;
}

// Copies the n error flags into host memory mapped into the device's address
// space (fine-grained pinned memory: the stores reach the host before the
// kernel ends), so that a synchronisation is the only host call needed to
// read them.
__global__ void k_flags_out(const int *flags, int n, int *host)
{
    const int i = threadIdx.x;
    if (i < n)
        __hip_atomic_store(host + i, flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
}



// Counting sort, between the passes: for every key, the exclusive prefix of
// its counts over the blocks (in place in H) and its total (tot[key]).  A
// workgroup of 256 threads takes CS_COLS consecutive keys; its threads split
// the blocks into CS_ROWG row groups, each scanning its rows of a key in
// registers (every load issued first), then the row groups' totals are
// scanned in LDS.  Column-parallel alone, a key's blocks would be one
// dependent chain.
constexpr int CS_COLS = 32, CS_ROWG = 8, CS_MAXR = 32; // nblk <= ROWG * MAXR
constexpr int CS_THREADS = CS_COLS * CS_ROWG;
__device__ __forceinline__ void colscan_body(const SortArgs &a, int blk)
{
    __shared__ int32_t part[CS_ROWG][CS_COLS];
    const int nbins = a.nbins, nblk = a.nblk;
    int32_t *H = a.H;
    const int c = threadIdx.x % CS_COLS, g = threadIdx.x / CS_COLS;
    const int64_t k = (int64_t)blk * CS_COLS + c;
    const int per = (nblk + CS_ROWG - 1) / CS_ROWG; // rows of one group
    const int r0 = g * per;
    const bool kv = k < nbins;
    // rows of this thread: r0 .. r0 + nr - 1, addressed by a running
    // pointer (per-row offsets held as scalars would spill)
    const int nr = kv ? max(0, min(per, nblk - r0)) : 0;
    int32_t *col = H + (int64_t)r0 * nbins + (kv ? k : 0);
    int32_t v[CS_MAXR];
    {
        const int32_t *q = col;
#pragma unroll
        for (int u = 0; u < CS_MAXR; ++u) {
            v[u] = u < nr ? *q : 0;
            q += nbins;
        }
    }
    int32_t run = 0;
#pragma unroll
    for (int u = 0; u < CS_MAXR; ++u) {
        const int32_t x = v[u];
        v[u] = run;
        run += x;
    }
    part[g][c] = run;
    __syncthreads();
    int32_t base = 0;
    for (int h = 0; h < g; ++h)
        base += part[h][c];
    if (kv) {
        int32_t *q = col;
#pragma unroll
        for (int u = 0; u < CS_MAXR; ++u) {
            if (u < nr)
                *q = base + v[u];
            q += nbins;
        }
        if (g == CS_ROWG - 1)
            a.tot[k] = base + run;
    }
}

__global__ void __launch_bounds__(CS_THREADS) k_colscan(SortArgs a) { colscan_body(a, blockIdx.x); }

// Counting sort, pass 2: block b places its points of every key at
// off[key] + (points of that key in blocks before b) + its LDS counter.
// off is the exclusive scan of the key totals.
__device__ __forceinline__ void place_body(const SortArgs &a, int blk)
{
    extern __shared__ int32_t cur[];
    const int nbins = a.nbins;
    // the cursors: every load of a batch in flight at once (indices clamped,
    // stores predicated)
    const int32_t *Hb = a.H + (int64_t)blk * nbins;
    for (int i0 = 0; i0 < nbins; i0 += 16 * SORT_THREADS) {
        int32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int i = i0 + (int)threadIdx.x + u * SORT_THREADS;
            i = i < nbins ? i : nbins - 1;
            v[u] = a.off[i] + Hb[i];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = i0 + (int)threadIdx.x + u * SORT_THREADS;
            if (i < nbins)
                cur[i] = v[u];
        }
    }
    __syncthreads();
    const int64_t j0 = (int64_t)blk * a.chunk;
    const int64_t j1 = j0 + a.chunk < a.n ? j0 + a.chunk : a.n;
    // every lane runs every iteration (key_runs works across the wavefront)
    for (int64_t jw = j0; jw < j1; jw += SORT_THREADS * SORT_BATCH) {
        const int64_t jb = jw + threadIdx.x;
        int32_t key[SORT_BATCH], mm[SORT_BATCH], pos[SORT_BATCH];
        double tt[SORT_BATCH], yv[SORT_BATCH];
#pragma unroll
        for (int u = 0; u < SORT_BATCH; ++u) { // loads clamped: all in flight
            const int64_t j = jb + u * SORT_THREADS;
            yv[u] = a.y[j < j1 ? j : j1 - 1];
        }
#pragma unroll
        for (int u = 0; u < SORT_BATCH; ++u) {
            const int64_t j = jb + u * SORT_THREADS;
            key[u] = -1;
            mm[u] = 0;
            tt[u] = 0.0;
            if (j < j1) {
                bool ok;
                key[u] = point_key(a, yv[u], &mm[u], &tt[u], &ok);
                if (!ok)
                    atomicOr(a.flags, FLAG_BAD_Y);
                if (a.hit && tt[u] == 0.0)
                    atomicExch(&a.hit[mm[u]], (int32_t)j);
            }
        }
#pragma unroll
        for (int u = 0; u < SORT_BATCH; ++u) {
            int start, len;
            key_runs(key[u], &start, &len);
            int32_t base = 0;
            if (len && key[u] >= 0)
                base = atomicAdd(&cur[key[u]], len);
            base = __shfl(base, start);
            pos[u] = base + ((int)(threadIdx.x & 63) - start);
        }
        if (a.spt) {
#pragma unroll
            for (int u = 0; u < SORT_BATCH; ++u)
                if (key[u] >= 0) {
                    a.spt[pos[u]] = {mm[u], (int32_t)(jb + u * SORT_THREADS), tt[u]};
                    if (a.skey)
                        a.skey[pos[u]] = key[u];
                }
        } else {
#pragma unroll
            for (int u = 0; u < SORT_BATCH; ++u)
                if (key[u] >= 0) {
                    a.sm[pos[u]] = mm[u];
                    a.sth[pos[u]] = tt[u];
                    a.sperm[pos[u]] = (int32_t)(jb + u * SORT_THREADS);
                    if (a.skey)
                        a.skey[pos[u]] = key[u];
                }
        }
    }
}

__global__ void __launch_bounds__(SORT_THREADS) k_place(SortArgs a) { place_body(a, blockIdx.x); }

// Counting sort with global atomics, for key ranges too large for LDS:
// pass 1 counts every key.
__global__ void k_reduce(int64_t M, const double *__restrict__ y, double c_hi,
                         double c_lo, int64_t N, int l, int keyshift, double ymax,
                         int32_t *um, double *uth, int32_t *ukey,
                         int32_t *count, int32_t *hit, int *flags)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < M;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t m;
        double th;
        const double invN = 1.0 / (double)N;
        if (!reduce_point(y[j], c_hi, c_lo, N, invN, ymax, &m, &th))
            atomicOr(flags, FLAG_BAD_Y);
        const int32_t key = (int32_t)(box_of(m, th, l, N, invN) >> keyshift);
        um[j] = (int32_t)m;
        uth[j] = th;
        ukey[j] = key;
        atomicAdd(&count[key], 1);
        if (hit && th == 0.0)
            atomicExch(&hit[m], (int32_t)j);
    }
}

// Exclusive scan of one value per thread over a workgroup of 1024 threads:
// wavefront scans by shuffles, then one scan of the 16 wavefront totals
// (ws: 16 words of LDS).  Two barriers instead of the twenty of a
// Hillis-Steele scan over LDS.  *total: the sum of all 1024 values.
__device__ __forceinline__ int32_t block_scan1024(int32_t x, int32_t *ws, int32_t *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(v, d);
        if (lane >= d)
            v += t;
    }
    if (lane == 63)
        ws[wv] = v;
    __syncthreads();
    if (wv == 0) {
        int32_t u = lane < 16 ? ws[lane] : 0;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const int32_t t = __shfl_up(u, d);
            if (lane >= d)
                u += t;
        }
        if (lane < 16)
            ws[16 + lane] = u; // inclusive scan of the wavefront totals
    }
    __syncthreads();
    *total = ws[31];
    return (wv ? ws[16 + wv - 1] : 0) + v - x;
}

// Placement of sorted records (the forward's targets) for small blocks:
// k_place with the block's records staged in LDS in their destination
// order before they are written.  A block's points of one key go to
// consecutive positions, so the write-out covers each run of positions
// with consecutive lanes instead of single 16-byte stores scattered over
// the output (which the memory system writes as whole sectors).  Needs the
// whole chunk in one pass (chunk <= PLACE_REC_MAX), nbins <= 4096 and no
// key array.
// LDS: cur, cur0, lbase (3 nbins words), 32 scan words, PLACE_REC_MAX
// records and their positions.
constexpr int PLACE_REC_MAX = 4096;

__device__ __forceinline__ void place_rec_body(const SortArgs &a, int blk)
{
    extern __shared__ __align__(16) int32_t lds_place[];
    const int nbins = a.nbins;
    SortedPt *rec = reinterpret_cast<SortedPt *>(lds_place); // PLACE_REC_MAX
    int32_t *gpos = lds_place + 4 * PLACE_REC_MAX;            // PLACE_REC_MAX
    int32_t *cur = gpos + PLACE_REC_MAX;                      // nbins
    int32_t *cur0 = cur + nbins;                              // nbins
    int32_t *lbase = cur0 + nbins;                            // nbins
    int32_t *ws = lbase + nbins;                              // 32
    const int32_t *Hb = a.H + (int64_t)blk * nbins;
    const bool last = blk + 1 == a.nblk;
    // cursors, and this block's count of every key: the next block's
    // exclusive prefix (or the key's total) minus this block's
    constexpr int KPT = 4; // keys per thread (nbins <= 4096)
    int32_t cnt[KPT], sum = 0;
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
        const int k = (int)threadIdx.x * KPT + u;
        cnt[u] = 0;
        if (k < nbins) {
            const int32_t c0 = a.off[k] + Hb[k];
            const int32_t c1 = last ? a.off[k + 1] : a.off[k] + Hb[nbins + k];
            cur[k] = c0;
            cur0[k] = c0;
            cnt[u] = c1 - c0;
        }
        sum += cnt[u];
    }
    int32_t total;
    int32_t run = block_scan1024(sum, ws, &total);
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
        const int k = (int)threadIdx.x * KPT + u;
        if (k < nbins)
            lbase[k] = run;
        run += cnt[u];
    }
    __syncthreads();
    const int64_t j0 = (int64_t)blk * a.chunk;
    const int64_t j1 = j0 + a.chunk < a.n ? j0 + a.chunk : a.n;
    const int64_t jb = j0 + threadIdx.x;
    int32_t key[SORT_BATCH], mm[SORT_BATCH];
    double tt[SORT_BATCH], yv[SORT_BATCH];
#pragma unroll
    for (int u = 0; u < SORT_BATCH; ++u) { // loads clamped: all in flight
        const int64_t j = jb + u * SORT_THREADS;
        yv[u] = a.y[j < j1 ? j : j1 - 1];
    }
#pragma unroll
    for (int u = 0; u < SORT_BATCH; ++u) {
        const int64_t j = jb + u * SORT_THREADS;
        key[u] = -1;
        mm[u] = 0;
        tt[u] = 0.0;
        if (j < j1) {
            bool ok;
            key[u] = point_key(a, yv[u], &mm[u], &tt[u], &ok);
            if (!ok)
                atomicOr(a.flags, FLAG_BAD_Y);
            if (a.hit && tt[u] == 0.0)
                atomicExch(&a.hit[mm[u]], (int32_t)j);
        }
    }
#pragma unroll
    for (int u = 0; u < SORT_BATCH; ++u) {
        int start, len;
        key_runs(key[u], &start, &len);
        int32_t base = 0;
        if (len && key[u] >= 0)
            base = atomicAdd(&cur[key[u]], len);
        base = __shfl(base, start);
        if (key[u] >= 0) {
            const int32_t pos = base + ((int)(threadIdx.x & 63) - start);
            const int32_t slot = lbase[key[u]] + (pos - cur0[key[u]]);
            rec[slot] = {mm[u], (int32_t)(jb + u * SORT_THREADS), tt[u]};
            gpos[slot] = pos;
        }
    }
    __syncthreads();
    for (int32_t q = threadIdx.x; q < total; q += SORT_THREADS)
        a.spt[gpos[q]] = rec[q];
}

__global__ void __launch_bounds__(SORT_THREADS) k_place_rec(SortArgs a)
{
    place_rec_body(a, blockIdx.x);
}

// Exclusive scan of up to SCAN1_MAX counts in one workgroup of 1024 threads:
// the counts are loaded coalesced into LDS (skewed by one word per 32, so
// that the per-thread runs below are free of bank conflicts), thread i scans
// the run [32 i, 32 i + 32), the 1024 run sums are scanned, and the results
// go out coalesced.  off[n] = total; cursor (optional) receives a copy.
constexpr int SCAN1_PER = 32;
constexpr int SCAN1_MAX = 1024 * SCAN1_PER;
__host__ __device__ __forceinline__ int scan1_slot(int i) { return i + (i >> 5); }

// The scan itself, with the counts staged in sv (scan1_slot(n) + 1 words of
// LDS) and part (64 words) for the block scan; thread i scans a run of
// ceil(n / 1024) consecutive counts.  part[63] receives the total.
__device__ __forceinline__ void scan_block(const int32_t *count, int n,
                                           int32_t *__restrict__ off,
                                           int32_t *__restrict__ cursor, int32_t *sv,
                                           int32_t *part)
{
    // 16 loads in flight per thread (indices clamped, values masked)
    for (int b = 0; b * 1024 < n; b += 16) {
        int32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = (int)threadIdx.x + (b + u) * 1024;
            v[u] = count[i < n ? i : n - 1];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = (int)threadIdx.x + (b + u) * 1024;
            if (i < n)
                sv[scan1_slot(i)] = v[u];
        }
    }
    __syncthreads();
    const int per = (n + 1023) / 1024;
    const int i0 = threadIdx.x * per;
    int32_t sum = 0;
    for (int u = 0; u < per; ++u)
        if (i0 + u < n)
            sum += sv[scan1_slot(i0 + u)];
    int32_t total;
    int32_t run = block_scan1024(sum, part, &total);
    for (int u = 0; u < per; ++u) {
        if (i0 + u < n) {
            const int k = scan1_slot(i0 + u);
            const int32_t c = sv[k];
            sv[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 1024) {
        const int32_t v = sv[scan1_slot(i)];
        off[i] = v;
        if (cursor)
            cursor[i] = v;
    }
    if (threadIdx.x == 1023) {
        off[n] = total;
        part[63] = total; // (after the block scan's 32 words) for callers that go on
    }
}

__device__ __forceinline__ void scan_one_body(const int32_t *__restrict__ count, int n,
                                              int32_t *__restrict__ off,
                                              int32_t *__restrict__ cursor)
{
    extern __shared__ int32_t sv[]; // scan1_slot(SCAN1_MAX) + 1024 words
    scan_block(count, n, off, cursor, sv, sv + scan1_slot(SCAN1_MAX));
}

// dynamic LDS of k_scan_one / kb_scan_one
constexpr size_t SCAN1_SMEM = (size_t)(SCAN1_MAX + SCAN1_MAX / 32 + 1024) * 4;

__global__ void __launch_bounds__(1024)
    k_scan_one(const int32_t *count, int n, int32_t *off, int32_t *cursor)
{
    scan_one_body(count, n, off, cursor);
}

// Exclusive scan of the leaf counts in three coalesced steps: sums of tiles
// of SCAN_TILE counts, a scan of the tile sums (one workgroup), and the scan
// inside every tile.
constexpr int SCAN_TILE = 4096;

__global__ void __launch_bounds__(256)
    k_scan_sums(const int32_t *count, int64_t n, int32_t *tsum)
{
    __shared__ int32_t red[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int32_t s = 0;
    for (int i = threadIdx.x; i < SCAN_TILE; i += 256)
        if (base + i < n)
            s += count[base + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d)
            red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        tsum[blockIdx.x] = red[0];
}

// In place: tsum[i] <- sum of tsum[0..i), for nt <= 4096 tiles; the total
// goes to *total.
__global__ void __launch_bounds__(1024)
    k_scan_top(int32_t *tsum, int nt, int32_t *total)
{
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (nt + 1023) / 1024;
    const int b0 = tid * per, b1 = b0 + per < nt ? b0 + per : nt;
    int32_t v[4];
    int32_t s = 0;
    for (int i = b0; i < b1; ++i) {
        v[i - b0] = tsum[i];
        s += v[i - b0];
    }
    int32_t all;
    int32_t run = block_scan1024(s, part, &all);
    for (int i = b0; i < b1; ++i) {
        tsum[i] = run;
        run += v[i - b0];
    }
    if (tid == 1023)
        *total = all;
}

__global__ void __launch_bounds__(256)
    k_scan_tiles(const int32_t *count, int64_t n, const int32_t *tsum,
                 int32_t *off, int32_t *cursor)
{
    __shared__ int32_t tile[SCAN_TILE];
    __shared__ int32_t part[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int i = tid; i < SCAN_TILE; i += 256)
        tile[i] = base + i < n ? count[base + i] : 0;
    __syncthreads();
    constexpr int per = SCAN_TILE / 256;
    int32_t s = 0;
    for (int i = 0; i < per; ++i)
        s += tile[tid * per + i];
    part[tid] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        int32_t x = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int32_t run = tsum[blockIdx.x] + (tid == 0 ? 0 : part[tid - 1]);
    for (int i = 0; i < per; ++i) {
        const int32_t c = tile[tid * per + i];
        tile[tid * per + i] = run;
        run += c;
    }
    __syncthreads();
    for (int i = tid; i < SCAN_TILE; i += 256)
        if (base + i < n) {
            off[base + i] = tile[i];
            if (cursor)
                cursor[base + i] = tile[i];
        }
}

// Counting-sort scatter: each point takes the next slot of its leaf.  The
// order inside a leaf is arbitrary (the forward results do not depend on it).
__global__ void k_scatter(int64_t M, const int32_t *um, const double *uth,
                          const int32_t *ukey, int32_t *cursor, int32_t *sm,
                          double *sth, int32_t *sperm, int32_t *skey, SortedPt *spt)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < M;
         j += (int64_t)gridDim.x * blockDim.x) {
        int32_t key = ukey[j];
        int32_t pos = atomicAdd(&cursor[key], 1);
        if (spt) {
            spt[pos] = {um[j], (int32_t)j, uth[j]};
            if (skey)
                skey[pos] = key;
            continue;
        }
        sm[pos] = um[j];
        sth[pos] = uth[j];
        sperm[pos] = (int32_t)j;
        if (skey)
            skey[pos] = key;
    }
}

// The order along the circle inside each leaf (the inverse): positions
// s = m + th are compared in the canonical form th in [-1/2, 1/2) (th = 1/2
// becomes m + 1, -1/2): the intervals [m - 1/2, m + 1/2) are disjoint, so
// s_u < s_t exactly when (m_u, th_u) < (m_t, th_t) lexicographically.  Two
// points at the same position raise FLAG_DUP.
__device__ __forceinline__ void canon_pos(int32_t &m, double &th)
{
    if (th == 0.5) {
        m += 1;
        th = -0.5;
    }
}

// Rank of point t (of the leaf [t0, t1)) among its leaf by position, from
// canonical grid units gm(u), gth(u); ties (duplicates) are ordered by index,
// so that the ranks stay a permutation of the leaf.  (Used where a key's
// points do not fit the counting sort by cell; a leaf of more than the
// dense limit is left unranked there: the point set is far too clustered
// for the inverse, which reports FLAG_DENSE.)
template <int UNROLL = 4, typename GetM, typename GetTh>
__device__ __forceinline__ int32_t leaf_rank(int32_t t, int32_t t0, int32_t t1, GetM gm,
                                             GetTh gth, int32_t mt, double tht, bool *dup)
{
    int32_t rank = 0;
    bool d = false;
#pragma unroll UNROLL
    for (int32_t u = t0; u < t1; ++u) {
        const int32_t mu = gm(u);
        const double tu = gth(u);
        const bool lt = mu < mt || (mu == mt && tu < tht);
        const bool eq = mu == mt && tu == tht;
        rank += (lt || (eq && u < t)) ? 1 : 0;
        d |= eq && u != t;
    }
    *dup |= d;
    return rank;
}

// Leaf order of the points of every key (a box of level l - ks, 2^ks
// leaves): the placement of the counting sort leaves the records of a key
// together in arbitrary order; one workgroup per key groups them by leaf,
// writes the leaves' offsets and, with RANK, orders every leaf along the
// circle (FLAG_DUP on two points at one position).  Outputs: sm, sth,
// sperm (grid units and input index as placed) and skey (the leaf) in the
// final order, and off[0 .. 2^l].
// A key of at most ORDER_CAP points is held in registers.  Its order along
// the circle is a counting sort by canonical grid cell m (at most
// ORDER_CELLS cells: a jittered grid puts about one point in each), then
// the order by th inside a cell; the leaves, whose boundaries are
// positions, come out contiguous in that order.  A key spanning more cells
// ranks each point against its leaf staged in LDS, and a key of more
// points (a clustered set) takes those steps through `tmp` in global
// memory.
constexpr int ORDER_THREADS = 512;
constexpr int ORDER_WAVES = ORDER_THREADS / 64;
constexpr int ORDER_PER = 4;                           // points per thread
constexpr int ORDER_CAP = ORDER_THREADS * ORDER_PER;   // points of a key in LDS
constexpr int ORDER_CELLS = 2048;                      // grid cells of a key in LDS
constexpr int ORDER_MAX_SHIFT = 6;                     // at most 64 leaves per key

struct OrderArgs {
    int64_t nkey;          // keys
    int ks;                // leaves per key: 2^ks (ks <= ORDER_MAX_SHIFT)
    int l;                 // leaves: 2^l = nkey 2^ks
    int64_t N;
    double invN;
    const SortedPt *rec;   // records grouped by key, as placed
    SortedPt *tmp;         // as many records of scratch (keys over ORDER_CAP)
    const int32_t *koff;   // nkey + 1 key offsets
    int32_t *off;          // out: 2^l + 1 leaf offsets
    int32_t dense_max;     // larger leaves raise FLAG_DENSE and stay unranked
    int32_t *sm;
    double *sth;
    int32_t *sperm;
    int32_t *skey;
    int *flags;
};

__device__ __forceinline__ int order_leaf(const OrderArgs &a, const SortedPt &q, int64_t leaf0)
{
    const int64_t b = box_of(q.m, q.th, a.l, a.N, a.invN) - leaf0;
    const int nl = 1 << a.ks;
    return b < 0 ? 0 : (b >= nl ? nl - 1 : (int)b); // (in range by construction)
}

// Exclusive scan of one value per thread over a workgroup of NW wavefronts
// (ws: 2 NW words of LDS); *total: the sum of all values.
template <int NW>
__device__ __forceinline__ int32_t block_scan_waves(int32_t x, int32_t *ws, int32_t *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(v, d);
        if (lane >= d)
            v += t;
    }
    if (lane == 63)
        ws[wv] = v;
    __syncthreads();
    if (wv == 0) {
        int32_t u = lane < NW ? ws[lane] : 0;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            const int32_t t = __shfl_up(u, d);
            if (lane >= d)
                u += t;
        }
        if (lane < NW)
            ws[NW + lane] = u;
    }
    __syncthreads();
    *total = ws[2 * NW - 1];
    return (wv ? ws[NW + wv - 1] : 0) + v - x;
}

template <bool RANK>
__global__ void __launch_bounds__(ORDER_THREADS) k_leaf_order(OrderArgs a)
{
    __shared__ int32_t lm[ORDER_CAP]; // canonical grid units (by leaf) or
    __shared__ double lth[ORDER_CAP]; // th (by cell) of the key's points
    __shared__ int32_t ccnt[ORDER_CELLS + 1]; // points per cell, then offsets
    __shared__ int32_t lcnt[1 << ORDER_MAX_SHIFT], lbase[1 << ORDER_MAX_SHIFT],
        lcur[1 << ORDER_MAX_SHIFT];
    __shared__ int32_t ws[2 * ORDER_WAVES], mrange[2];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t k = blockIdx.x;
    const int nl = 1 << a.ks;
    const int64_t leaf0 = k << a.ks;
    const int32_t S0 = a.koff[k], S1 = a.koff[k + 1], cnt = S1 - S0;
    const bool fast = cnt <= ORDER_CAP;
    if (tid < nl)
        lcnt[tid] = 0;
    if (RANK) {
        for (int i = tid; i <= ORDER_CELLS; i += ORDER_THREADS)
            ccnt[i] = 0;
        if (tid == 0) {
            mrange[0] = INT32_MAX;
            mrange[1] = INT32_MIN;
        }
    }
    __syncthreads();
    SortedPt q[ORDER_PER];
    int lf[ORDER_PER], c[ORDER_PER];
    if (fast) {
        // all loads in flight (indices clamped), then one LDS atomic per run
        // of equal leaves in consecutive lanes; c = place inside the leaf
#pragma unroll
        for (int u = 0; u < ORDER_PER; ++u) {
            const int i = tid + u * ORDER_THREADS;
            if (u * ORDER_THREADS < cnt)
                q[u] = a.rec[S0 + (i < cnt ? i : cnt - 1)];
        }
        int32_t mlo = INT32_MAX, mhi = INT32_MIN;
#pragma unroll
        for (int u = 0; u < ORDER_PER; ++u) {
            const int i = tid + u * ORDER_THREADS;
            lf[u] = -1;
            c[u] = 0;
            if (u * ORDER_THREADS < cnt) { // uniform over the workgroup
                lf[u] = i < cnt ? order_leaf(a, q[u], leaf0) : -1;
                int start, len;
                key_runs(lf[u], &start, &len);
                int32_t base = 0;
                if (len && lf[u] >= 0)
                    base = atomicAdd(&lcnt[lf[u]], len);
                base = __shfl(base, start);
                c[u] = base + (lane - start);
                if (RANK && lf[u] >= 0) {
                    int32_t m = q[u].m;
                    double th = q[u].th;
                    canon_pos(m, th);
                    mlo = m < mlo ? m : mlo;
                    mhi = m > mhi ? m : mhi;
                }
            }
        }
        if (RANK) { // the key's range of canonical cells
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                const int32_t lo = __shfl_xor(mlo, d), hi = __shfl_xor(mhi, d);
                mlo = lo < mlo ? lo : mlo;
                mhi = hi > mhi ? hi : mhi;
            }
            if (lane == 0 && mlo <= mhi) {
                atomicMin(&mrange[0], mlo);
                atomicMax(&mrange[1], mhi);
            }
        }
    } else {
        for (int32_t i = tid; i < cnt; i += ORDER_THREADS)
            atomicAdd(&lcnt[order_leaf(a, a.rec[S0 + i], leaf0)], 1);
    }
    __syncthreads();
    // leaf offsets: one wavefront scans the (at most 64) leaf counts
    if (tid < 64) {
        const int32_t v = tid < nl ? lcnt[tid] : 0;
        int32_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t t = __shfl_up(x, d);
            if (lane >= d)
                x += t;
        }
        if (tid < nl) {
            lbase[tid] = x - v;
            lcur[tid] = x - v;
            a.off[leaf0 + tid] = S0 + x - v;
            if (v > a.dense_max)
                atomicOr(a.flags, FLAG_DENSE);
        }
        if (tid == 0 && k == a.nkey - 1)
            a.off[(int64_t)a.nkey << a.ks] = S1;
    }
    const int32_t m0 = RANK ? mrange[0] : 0;
    const int64_t ncell = RANK ? (int64_t)mrange[1] - mrange[0] + 1 : 0;
    const bool cells = RANK && fast && cnt > 0 && ncell <= ORDER_CELLS;
    int cc[ORDER_PER];
    if (cells) {
#pragma unroll
        for (int u = 0; u < ORDER_PER; ++u)
            if (lf[u] >= 0) {
                int32_t m = q[u].m;
                double th = q[u].th;
                canon_pos(m, th);
                cc[u] = atomicAdd(&ccnt[m - m0], 1);
            }
    }
    __syncthreads();
    bool dup = false;
    auto emit = [&](const SortedPt &p, int32_t pos, int f) {
        a.sm[pos] = p.m;
        a.sth[pos] = p.th;
        a.sperm[pos] = p.perm;
        a.skey[pos] = (int32_t)(leaf0 + f);
    };
    if (cells) {
        // the cells' offsets (exclusive scan), the points' th staged by
        // cell, then each point's order inside its cell
        constexpr int CPT = (ORDER_CELLS + ORDER_THREADS - 1) / ORDER_THREADS;
        int32_t v[CPT], sum = 0;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int i = tid * CPT + e;
            v[e] = i < ncell ? ccnt[i] : 0;
            sum += v[e];
        }
        int32_t total;
        int32_t run = block_scan_waves<ORDER_WAVES>(sum, ws, &total);
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int i = tid * CPT + e;
            if (i < ncell)
                ccnt[i] = run;
            run += v[e];
        }
        if (tid == 0)
            ccnt[ncell] = total;
        __syncthreads();
        int32_t slot[ORDER_PER];
#pragma unroll
        for (int u = 0; u < ORDER_PER; ++u)
            if (lf[u] >= 0) {
                int32_t m = q[u].m;
                double th = q[u].th;
                canon_pos(m, th);
                slot[u] = ccnt[m - m0] + cc[u];
                lth[slot[u]] = th;
            }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < ORDER_PER; ++u)
            if (lf[u] >= 0) {
                int32_t m = q[u].m;
                double th = q[u].th;
                canon_pos(m, th);
                const int32_t b0 = ccnt[m - m0], b1 = ccnt[m - m0 + 1];
                int32_t rank = 0;
                for (int32_t s = b0; s < b1; ++s) {
                    const double ts = lth[s];
                    rank += (ts < th || (ts == th && s < slot[u])) ? 1 : 0;
                    dup |= ts == th && s != slot[u];
                }
                emit(q[u], S0 + b0 + rank, lf[u]);
            }
    } else if (fast) {
        if (RANK) {
#pragma unroll
            for (int u = 0; u < ORDER_PER; ++u)
                if (lf[u] >= 0) {
                    int32_t m = q[u].m;
                    double th = q[u].th;
                    canon_pos(m, th);
                    lm[lbase[lf[u]] + c[u]] = m;
                    lth[lbase[lf[u]] + c[u]] = th;
                }
            __syncthreads();
        }
        auto gm = [&](int32_t s) { return lm[s]; };
        auto gth = [&](int32_t s) { return lth[s]; };
#pragma unroll
        for (int u = 0; u < ORDER_PER; ++u)
            if (lf[u] >= 0) {
                const int32_t t0 = lbase[lf[u]], t1 = t0 + lcnt[lf[u]];
                int32_t rank = c[u];
                if (RANK && t1 - t0 <= a.dense_max) {
                    int32_t m = q[u].m;
                    double th = q[u].th;
                    canon_pos(m, th);
                    rank = leaf_rank(t0 + c[u], t0, t1, gm, gth, m, th, &dup);
                }
                emit(q[u], S0 + t0 + rank, lf[u]);
            }
    } else {
        // grouped by leaf into tmp (or straight to the output when no
        // ranking is asked for), then ranked from tmp
        for (int32_t i = tid; i < cnt; i += ORDER_THREADS) {
            const SortedPt p = a.rec[S0 + i];
            const int f = order_leaf(a, p, leaf0);
            const int32_t slot = atomicAdd(&lcur[f], 1);
            if (RANK)
                a.tmp[S0 + slot] = p;
            else
                emit(p, S0 + slot, f);
        }
        if (RANK) {
            __threadfence_block();
            __syncthreads();
            const SortedPt *g = a.tmp + S0;
            auto gm = [&](int32_t s) {
                SortedPt p = g[s];
                canon_pos(p.m, p.th);
                return p.m;
            };
            auto gth = [&](int32_t s) {
                SortedPt p = g[s];
                canon_pos(p.m, p.th);
                return p.th;
            };
            for (int32_t t = tid; t < cnt; t += ORDER_THREADS) {
                const SortedPt p = g[t];
                const int f = order_leaf(a, p, leaf0);
                const int32_t t0 = lbase[f], t1 = t0 + lcnt[f];
                int32_t rank = t - t0;
                if (t1 - t0 <= a.dense_max) {
                    int32_t m = p.m;
                    double th = p.th;
                    canon_pos(m, th);
                    rank = leaf_rank<1>(t, t0, t1, gm, gth, m, th, &dup);
                }
                emit(p, S0 + t0 + rank, f);
            }
        }
    }
    if (dup)
        atomicOr(a.flags, FLAG_DUP);
}

// Work list of the downward pass (one workgroup): for every subtree root R
// of level lr, its sorted targets [off[R << sh], off[(R+1) << sh]) cut into
// pieces of at most tmax (pieces = 0 for none), or one item carrying both
// the sorted range and the uniform targets of R when `uniform`.
struct WorkArgs {
    int64_t nroot;       // subtree roots (2^lr)
    int sh;              // off indexes level lr + sh
    const int32_t *off;
    int uniform;
    int64_t N;
    int lr;
    int32_t tmax;
    WorkItem *items;
    int32_t *nitems;
};

// offl(i) = off[i] for i <= nbins, from global memory or from LDS; part is
// 1024 words of LDS.  One workgroup of 1024 threads.
template <typename Off>
__device__ __forceinline__ void work_from(const WorkArgs &w, Off offl, int32_t *part)
{
    const int64_t nroot = w.nroot, N = w.N;
    const int sh = w.sh, lr = w.lr, uniform = w.uniform;
    const int32_t tmax = w.tmax;
    WorkItem *items = w.items;
    const int tid = threadIdx.x;
    const int64_t per = (nroot + 1023) / 1024;
    const int64_t r0 = tid * per, r1 = r0 + per < nroot ? r0 + per : nroot;
    auto pieces = [&](int64_t R) -> int32_t {
        const int32_t t0 = offl(R << sh), t1 = offl((R + 1) << sh);
        if (uniform)
            return 1;
        return (t1 - t0 + tmax - 1) / tmax;
    };
    int32_t s = 0;
    for (int64_t R = r0; R < r1; ++R)
        s += pieces(R);
    int32_t nall;
    int32_t pos = block_scan1024(s, part, &nall);
    for (int64_t R = r0; R < r1; ++R) {
        const int32_t t0 = offl(R << sh), t1 = offl((R + 1) << sh);
        if (uniform) {
            const int64_t nr = int64_t(1) << lr;
            const int32_t u0 = (int32_t)((R * N + nr - 1) >> lr);
            const int32_t u1 = (int32_t)(((R + 1) * N + nr - 1) >> lr);
            items[pos++] = {R, t0, t1, u0, u1, 1, 0};
        } else {
            for (int32_t a = t0; a < t1; a += tmax)
                items[pos++] = {R, a, a + tmax < t1 ? a + tmax : t1, 0, 0, a == t0 ? 1 : 0, 0};
        }
    }
    if (tid == 1023)
        *w.nitems = nall;
}

__device__ __forceinline__ void work_body(const WorkArgs &w)
{
    __shared__ int32_t part[1024];
    work_from(w, [&](int64_t i) { return w.off[i]; }, part);
}

__global__ void __launch_bounds__(1024) k_work(WorkArgs w) { work_body(w); }



// The one-block scan of the key totals followed by the work list, built from
// the offsets while they are still in LDS (one launch and no read-back).
// Dynamic LDS: SCAN1_SMEM + 1024 words.
__global__ void __launch_bounds__(1024) k_scan_work(const int32_t *count, int n, int32_t *off,
                                                    int32_t *cursor, WorkArgs w)
{
    extern __shared__ int32_t sv[];
    scan_one_body(count, n, off, cursor);
    __syncthreads();
    int32_t *part = sv + scan1_slot(SCAN1_MAX);
    const int32_t total = part[63];
    work_from(w, [&](int64_t i) { return i < n ? sv[scan1_slot((int)i)] : total; },
              part + 1024);
}

// Dhat in input order: out[perm[t]] = dhat[t].
__global__ void k_unsort_c128(int64_t n, const cx<double> *dhat, const int32_t *perm,
                              cx<double> *out)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        out[perm[t]] = dhat[t];
}

// ---- synthetic problems for the autotuner (never part of a transform)

// SplitMix64 (Steele, Lea and Flood, 2014): a counter-based hash.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ double unit_rand(uint64_t seed, uint64_t i)
{
    return (double)(splitmix64(seed ^ (i * 0x632be59bd9b4e019ull)) >> 11) * 0x1.0p-53;
}

// y_j uniform on [0, 2 pi) (jitter = 0) or the grid 2 pi (j + jitter (u - 1/2)) / N.
__global__ void k_synth_points(int64_t n, int64_t N, double jitter, uint64_t seed,
                               double *y)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double u = unit_rand(seed, (uint64_t)j);
        y[j] = jitter > 0.0 ? 6.283185307179586 * ((double)j + jitter * (u - 0.5)) / (double)N
                            : 6.283185307179586 * u;
    }
}

// Complex data with components uniform on [-1/2, 1/2).
template <typename R>
__global__ void k_synth_data(int64_t n, uint64_t seed, cx<R> *x)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        x[j] = {(R)(unit_rand(seed, 2 * (uint64_t)j) - 0.5),
                (R)(unit_rand(seed, 2 * (uint64_t)j + 1) - 0.5)};
}

// Per-block sums of |a - b|^2 and |b|^2 (part[2 blk], part[2 blk + 1]).
template <typename R>
__global__ void __launch_bounds__(256)
    k_diff2(int64_t n, const cx<R> *a, const cx<R> *b, double *part)
{
    __shared__ double sd[256], sb[256];
    double d = 0.0, r = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double dr = (double)a[j].re - (double)b[j].re;
        const double di = (double)a[j].im - (double)b[j].im;
        d += dr * dr + di * di;
        r += (double)b[j].re * (double)b[j].re + (double)b[j].im * (double)b[j].im;
    }
    sd[threadIdx.x] = d;
    sb[threadIdx.x] = r;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            sd[threadIdx.x] += sd[threadIdx.x + k];
            sb[threadIdx.x] += sb[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sd[0];
        part[2 * blockIdx.x + 1] = sb[0];
    }
}

// ---- the same passes over a batch of point sets: one launch each, block
// b working for problem bm_find(b) (see BlockMap)


__global__ void __launch_bounds__(SORT_THREADS) kb_hist(const SortArgs *aa, BlockMap bm)
{
    int blk, nblk;
    const int t = bm_find(bm, blockIdx.x, &blk, &nblk);
    hist_body(aa[t], blk);
}

__global__ void __launch_bounds__(CS_THREADS) kb_colscan(const SortArgs *aa, BlockMap bm)
{
    int blk, nblk;
    const int t = bm_find(bm, blockIdx.x, &blk, &nblk);
    colscan_body(aa[t], blk);
}

// one workgroup per problem
__global__ void __launch_bounds__(1024) kb_scan_one(const SortArgs *aa)
{
    const SortArgs &a = aa[blockIdx.x];
    scan_one_body(a.tot, a.nbins, a.off, a.cursor);
}

__global__ void __launch_bounds__(SORT_THREADS) kb_place(const SortArgs *aa, BlockMap bm)
{
    int blk, nblk;
    const int t = bm_find(bm, blockIdx.x, &blk, &nblk);
    place_body(aa[t], blk);
}

// one workgroup per problem
__global__ void __launch_bounds__(1024) kb_work(const WorkArgs *ww) { work_body(ww[blockIdx.x]); }

} // namespace fn
