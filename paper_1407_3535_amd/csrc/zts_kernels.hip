// HIP kernels for exhaustive ZNCC template search with transitive elimination
// (gfx950, wave64).  Launch wrappers at the end are what the host library
// calls; nothing here allocates.
#include "zts_kernels.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "zts_device.h"

namespace zts {

// ============================================================== block helpers

__device__ __forceinline__ int block_sum_int(int v, int *red)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    int s = 0;
    for (int k = 0; k < nw; k++)
        s += red[k];
    return s;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long *red)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off);
    __syncthreads();
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    unsigned long long s = 0;
    for (int k = 0; k < nw; k++)
        s += red[k];
    return s;
}

// Loads an m x n uint8 template into LDS as flipped int8 words, n4w words per
// row, rows [off, off+m) of rows_lds; everything else zero.  Returns sum(t')
// and sum(t'^2) to every thread.
// One template word (4 columns from 4j) flipped to int8, zero past column n;
// a whole-word load when the rows are word-aligned.
__device__ __forceinline__ uint32_t tpl_word(const uint8_t *__restrict__ tpl, int64_t ts, int n, int r, int j,
                                             bool words)
{
    if (4 * j >= n)
        return 0;
    const int nb = min(4, n - 4 * j);
    uint32_t w = 0;
    if (words) {
        w = flip4(*gptr((const uint32_t *)(tpl + (int64_t)r * ts + 4 * j)));
    } else {
        for (int b = 0; b < nb; b++)
            w |= ((uint32_t)gptr(tpl)[(int64_t)r * ts + 4 * j + b] ^ 0x80u) << (8 * b);
    }
    return nb < 4 ? (w & ((1u << (8 * nb)) - 1u)) : w;
}

// Word j of template row r as raw uint8 bytes (zero past column n) for
// word-aligned rows, with no branch around the load (the word index is
// clamped into the row), so that a caller's unrolled loads stay in flight
// together.  flip4 of it, masked the same way, is tpl_word's int8 view.
__device__ __forceinline__ uint32_t tpl_raw_word(const uint8_t *__restrict__ tpl, int64_t ts, int n, int r, int j)
{
    const int jj = min(j, (n - 1) >> 2);
    const uint32_t w = *gptr((const uint32_t *)(tpl + (int64_t)r * ts + 4 * jj));
    const int nb = n - 4 * j;
    return nb >= 4 ? w : nb <= 0 ? 0u : w & ((1u << (8 * nb)) - 1u);
}

// put(i, load(i)) for i = threadIdx.x + k blockDim.x < total, K at a time:
// each batch's K loads are issued (from clamped indices, without branches)
// before any of them is used, so they are in flight together instead of
// one round trip each.
template <int K, typename Load, typename Put>
__device__ __forceinline__ void batched_loads(int total, Load load, Put put)
{
    const int nt = blockDim.x;
    for (int base = threadIdx.x; base < total; base += K * nt) {
        uint32_t v[K];
#pragma unroll
        for (int k = 0; k < K; k++)
            v[k] = load(min(base + k * nt, total - 1));
#pragma unroll
        for (int k = 0; k < K; k++)
            if (base + k * nt < total)
                put(base + k * nt, v[k]);
    }
}

__device__ void load_template(const uint8_t *__restrict__ tpl, int64_t ts, int m, int n, int n4w, int off,
                              int rows_lds, uint32_t *lds, int *red, int64_t *st, int64_t *sq)
{
    const bool words = ((ts | (int64_t)(uintptr_t)tpl) & 3) == 0 && (n & 3) == 0;
    const uint32_t ones = 0x01010101u;
    int total = rows_lds * n4w;
    int s = 0, s2 = 0;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int r = idx / n4w - off, j = idx - (idx / n4w) * n4w;
        uint32_t w = 0;
        if (r >= 0 && r < m) {
            w = tpl_word(tpl, ts, n, r, j, words);
            s = dot4(w, ones, s);
            s2 = dot4(w, w, s2);
        }
        lds[idx] = w;
    }
    *st = block_sum_int(s, red);
    *sq = block_sum_int(s2, red);
    __syncthreads();
}

// Merges per-thread records of the block; thread 0 gets the result.
__device__ RecPod block_rec(RecPod r, RecPod *red)
{
    red[threadIdx.x] = r;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            rec_merge(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    RecPod out = red[0];
    __syncthreads();
    return out;
}

// Merges the records of a wave: a butterfly over the 64 lanes, after which
// every lane holds the merged record (the merge is commutative and
// associative: best by (rho, smallest index), max of r32max, sums of counts).
// With SPAN < 64, lanes merge within aligned groups of SPAN lanes.
template <int SPAN = 64>
__device__ RecPod wave_rec(RecPod r)
{
#pragma unroll
    for (int off = SPAN / 2; off > 0; off >>= 1) {
        RecPod b;
        b.rho = __shfl_xor(r.rho, off);
        b.l = (int64_t)__shfl_xor((long long)r.l, off);
        b.num = (int64_t)__shfl_xor((long long)r.num, off);
        b.dr = (int64_t)__shfl_xor((long long)r.dr, off);
        b.r32max = __shfl_xor(r.r32max, off);
        b.valid = __shfl_xor(r.valid, off);
        b.n_elim = __shfl_xor(r.n_elim, off);
        b.n_surv = __shfl_xor(r.n_surv, off);
        b.n_window = __shfl_xor(r.n_window, off);
        rec_merge(r, b);
    }
    return r;
}

// Block reduction through one record per wave; thread 0 gets the result.
__device__ RecPod block_rec4(RecPod r, RecPod *red)
{
    r = wave_rec(r);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = r;
    __syncthreads();
    RecPod out = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); k++)
        rec_merge(out, red[k]);
    __syncthreads();
    return out;
}

// Whole-block reduction of a record range (run by the last block only).
__device__ RecPod reduce_records(const RecPod *recs, int lo, int hi, RecPod *red)
{
    RecPod r = rec_empty();
    for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        RecPod b = recs[k];
        rec_merge(r, b);
    }
    return block_rec(r, red);
}

// Best (rho, l) of a record range, computed by every block that calls it
// (all threads call it; red holds one entry per wave).  The order is total
// (rho, then the smaller index), so every block gets the same answer, which
// is the best the one-block record reductions would find; an empty or
// all-invalid range gives rho = -2, l = INT64_MAX.
struct Best {
    double rho;
    int64_t l;
    int valid;
};

__device__ __forceinline__ void best_merge(Best &a, double rho, int64_t l, int valid)
{
    if (valid && (!a.valid || rec_better(rho, l, a.rho, a.l))) {
        a.rho = rho;
        a.l = l;
        a.valid = 1;
    }
}

// best_merge by selects: the record's flag and value are both loaded
// before the decision, so a caller's loads need no branch between them.
__device__ __forceinline__ void best_take(Best &a, double rho, int64_t l, int valid)
{
    const bool take = (valid != 0) & (!a.valid | rec_better(rho, l, a.rho, a.l));
    a.rho = take ? rho : a.rho;
    a.l = take ? l : a.l;
    a.valid = take ? 1 : a.valid;
}

__device__ Best reduce_best(const RecPod *recs, int lo, int hi, Best *red)
{
    Best b = {-2.0, INT64_MAX, 0};
    // four records per thread in flight at once (clamped, unconditional)
    constexpr int K = 4;
    const int nt = blockDim.x;
    for (int k0 = lo + (int)threadIdx.x; k0 < hi; k0 += K * nt) {
        double r[K];
        int64_t l[K];
        int v[K];
#pragma unroll
        for (int q = 0; q < K; q++) {
            const RecPod *p = recs + min(k0 + q * nt, hi - 1);
            r[q] = p->rho;
            l[q] = p->l;
            v[q] = p->valid;
        }
#pragma unroll
        for (int q = 0; q < K; q++)
            best_take(b, r[q], l[q], k0 + q * nt < hi ? v[q] : 0);
    }
    for (int off = 32; off > 0; off >>= 1) {
        double r = __shfl_xor(b.rho, off);
        long long l = __shfl_xor((long long)b.l, off);
        int v = __shfl_xor(b.valid, off);
        best_merge(b, r, (int64_t)l, v);
    }
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = b;
    __syncthreads();
    Best out = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); w++)
        best_merge(out, red[w].rho, red[w].l, red[w].valid);
    __syncthreads();
    return out;
}

// The scan-2 threshold computed inside the kernels that need it, from the
// per-block records of scan 1 [0, n1) and of the refinement window [n1, n1 +
// n2); with include_best0 the scan-1 best competes with the window's.
struct Thr {
    double best0;
    int64_t best0_l;
    double best;
    int64_t best_l;
    double thr64;
    float lo, hi;
};

// The threshold from the scan-1 best f0 and the window best fw (n2 window
// records; none: the scan-1 best alone).
__device__ Thr make_threshold(Best f0, Best fw, int n2, int include_best0, double delta, double floor)
{
    Thr r;
    r.best0 = f0.rho;
    r.best0_l = f0.l;
    if (n2 > 0) {
        if (include_best0)
            best_merge(fw, f0.rho, f0.l, 1);
    } else {
        fw = f0;
    }
    r.best = fw.rho;
    r.best_l = fw.l;
    r.thr64 = (floor > fw.rho ? floor : fw.rho) - delta;
    double c = r.thr64 > 1.0 ? 1.0 : (r.thr64 < -1.0 ? -1.0 : r.thr64);
    float th = (float)acos(c);
    r.lo = th - kEpsTheta;
    r.hi = th + kEpsTheta;
    return r;
}

__device__ Thr block_threshold(const RecPod *recs, int n1, int n2, int include_best0, double delta, double floor,
                               Best *red)
{
    // one pass over both record ranges: every load is issued before the
    // wave and block merges (red holds two entries per wave)
    Best b0 = {-2.0, INT64_MAX, 0}, bw = {-2.0, INT64_MAX, 0};
    // four records per thread in flight at once (clamped, unconditional
    // loads; the merges are selects)
    constexpr int K = 4;
    const int nt = blockDim.x, hi = n1 + n2;
    for (int k0 = (int)threadIdx.x; k0 < hi; k0 += K * nt) {
        double r[K];
        int64_t l[K];
        int v[K];
#pragma unroll
        for (int q = 0; q < K; q++) {
            const RecPod *p = recs + min(k0 + q * nt, hi - 1);
            r[q] = p->rho;
            l[q] = p->l;
            v[q] = p->valid;
        }
#pragma unroll
        for (int q = 0; q < K; q++) {
            const int k = k0 + q * nt;
            best_take(b0, r[q], l[q], k < n1 ? v[q] : 0);
            best_take(bw, r[q], l[q], k >= n1 && k < hi ? v[q] : 0);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        double r0 = __shfl_xor(b0.rho, off), r1 = __shfl_xor(bw.rho, off);
        long long l0 = __shfl_xor((long long)b0.l, off), l1 = __shfl_xor((long long)bw.l, off);
        int v0 = __shfl_xor(b0.valid, off), v1 = __shfl_xor(bw.valid, off);
        best_merge(b0, r0, (int64_t)l0, v0);
        best_merge(bw, r1, (int64_t)l1, v1);
    }
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = b0;
        red[nw + (threadIdx.x >> 6)] = bw;
    }
    __syncthreads();
    Best f0 = red[0], fw = red[nw];
    for (int w = 1; w < nw; w++) {
        best_merge(f0, red[w].rho, red[w].l, red[w].valid);
        best_merge(fw, red[nw + w].rho, red[nw + w].l, red[nw + w].valid);
    }
    __syncthreads();
    return make_threshold(f0, fw, n2, include_best0, delta, floor);
}

__device__ void store_threshold(QState *qs, const Thr &r)
{
    qs->best0 = r.best0;
    qs->best0_l = r.best0_l;
    qs->best = r.best;
    qs->best_l = r.best_l;
    qs->thr64 = r.thr64;
    qs->thr_lo = r.lo;
    qs->thr_hi = r.hi;
}

// The threshold from the scan-1 best that the window kernel wrote into the
// query state and the n2 window records, formed by each wave on its own
// (lanes over the records, then shuffles; no block barrier).
__device__ Thr wave_threshold(const QState *qs, const RecPod *wrecs, int n2, int include_best0, double delta,
                              double floor)
{
    const Best f0 = {qs->best0, qs->best0_l, 1};
    Best fw = {-2.0, INT64_MAX, 0};
    for (int k = threadIdx.x & 63; k < n2; k += 64) {
        // flag and value loaded together (a select, not a branch, takes the
        // record), so that one round trip brings both
        best_take(fw, wrecs[k].rho, wrecs[k].l, wrecs[k].valid);
    }
    for (int off = 32; off > 0; off >>= 1) {
        double r = __shfl_xor(fw.rho, off);
        long long l = __shfl_xor((long long)fw.l, off);
        int v = __shfl_xor(fw.valid, off);
        best_merge(fw, r, (int64_t)l, v);
    }
    return make_threshold(f0, fw, n2, include_best0, delta, floor);
}

__device__ __forceinline__ void group_geom(int g, int Gx, int Ly, int Lx, int h, int w, int &oy, int &ox, int &hh,
                                           int &ww, int &cy, int &cx)
{
    int gy = g / Gx, gx = g - (g / Gx) * Gx;
    oy = gy * h;
    ox = gx * w;
    hh = min(h, Ly - oy);
    ww = min(w, Lx - ox);
    cy = oy + (hh - 1) / 2;
    cx = ox + (ww - 1) / 2;
}

__device__ __forceinline__ int64_t centre_of(int y, int x, int Ly, int Lx, int h, int w)
{
    int oy = (y / h) * h, ox = (x / w) * w;
    int hh = min(h, Ly - oy), ww = min(w, Lx - ox);
    return (int64_t)(oy + (hh - 1) / 2) * Lx + (ox + (ww - 1) / 2);
}

// ============================================================== running sums

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t u = __shfl_up(v, off);
        if (lane >= off)
            v += u;
    }
    return v;
}

// Row pass: sat[(y+1)(q+1) + x+1] = sum over row y, columns <= x, of x' and
// x'^2 (uint32, modulo 2^32; box sums of fewer than 2^14 pixels are exact).
__global__ __launch_bounds__(256) void k_sat_rows(const uint8_t *__restrict__ img, int64_t pitch, int p, int q,
                                                  uint2 *__restrict__ sat)
{
    __shared__ uint32_t wa[4], wb[4];
    int y = blockIdx.x;
    int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint8_t *row = img + (int64_t)y * pitch;
    uint2 *out = sat + (int64_t)(y + 1) * (q + 1);
    if (t == 0)
        out[0] = make_uint2(0u, 0u);
    uint32_t ca = 0, cb = 0;
    for (int base = 0; base < q; base += 256) {
        int x = base + t;
        int v = x < q ? (int)row[x] - 128 : 0;
        uint32_t a = wave_incl_scan((uint32_t)v, lane);
        uint32_t b = wave_incl_scan((uint32_t)(v * v), lane);
        if (lane == 63) {
            wa[wv] = a;
            wb[wv] = b;
        }
        __syncthreads();
        uint32_t pa = ca, pb = cb;
        for (int k = 0; k < wv; k++) {
            pa += wa[k];
            pb += wb[k];
        }
        if (x < q)
            out[x + 1] = make_uint2(pa + a, pb + b);
        for (int k = 0; k < 4; k++) {
            ca += wa[k];
            cb += wb[k];
        }
        __syncthreads();
    }
}

// Row pass of the running sums of the product image J'(y, x) I'(y + dy,
// x + dx) (both shifted to int8, products up to 2^14; 0 where (y + dy,
// x + dx) leaves the image): row y + 1 of `sat` holds the prefix along x,
// modulo 2^32.  A box sum of the finished table is exact when the true sum
// fits in int32, which |sum| <= m n 2^14 <= 2^28 guarantees.
__global__ __launch_bounds__(256) void k_prod_rows(const uint8_t *__restrict__ J, const uint8_t *__restrict__ I,
                                                   int64_t pitch, int p, int q, int dy, int dx,
                                                   uint32_t *__restrict__ sat)
{
    // 2048 columns per step: a thread forms and scans 8 consecutive
    // products, the block scans the thread totals, and the row segment goes
    // out through LDS so that the stores are coalesced
    __shared__ uint32_t wa[4];
    __shared__ uint32_t seg[2048];
    int y = blockIdx.x;
    int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const bool rowok = y + dy >= 0 && y + dy < p;
    const uint8_t *rj = J + (int64_t)y * pitch, *ri = I + (int64_t)(rowok ? y + dy : y) * pitch;
    uint32_t *out = sat + (int64_t)(y + 1) * (q + 1);
    if (t == 0)
        out[0] = 0u;
    uint32_t ca = 0;
    for (int base = 0; base < q; base += 2048) {
        const int x0 = base + 8 * t;
        uint32_t v[8], s = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int x = x0 + k;
            const int pr = x < q && rowok && x + dx >= 0 && x + dx < q ? ((int)rj[x] - 128) * ((int)ri[x + dx] - 128)
                                                                       : 0;
            s += (uint32_t)pr;
            v[k] = s;
        }
        const uint32_t incl = wave_incl_scan(s, lane);
        if (lane == 63)
            wa[wv] = incl;
        __syncthreads();
        uint32_t pre = ca + incl - s;
        for (int k = 0; k < wv; k++)
            pre += wa[k];
#pragma unroll
        for (int k = 0; k < 8; k++)
            seg[8 * t + k] = pre + v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int x = base + t + 256 * k;
            if (x < q)
                out[x + 1] = seg[t + 256 * k];
        }
        ca += wa[0] + wa[1] + wa[2] + wa[3];
        __syncthreads();
    }
}

// Column pass of a running-sum table (rows 1..p, row 0 is zero), in two
// kernels over blocks of 64 columns x 64 rows so that the grid fills the
// chip: the first writes each block's column totals and the totals of its
// four 16-row parts, the second adds the totals of the chunks and parts
// above and scans its own rows, reading the table once.  A thread owns one
// column and 16 consecutive rows.
constexpr int kColChunk = 64;

__device__ __forceinline__ uint2 add_el(uint2 a, uint2 b) { return make_uint2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ uint32_t add_el(uint32_t a, uint32_t b) { return a + b; }
template <class T> __device__ __forceinline__ T zero_el();
template <> __device__ __forceinline__ uint2 zero_el<uint2>() { return make_uint2(0u, 0u); }
template <> __device__ __forceinline__ uint32_t zero_el<uint32_t>() { return 0u; }

template <class T>
__global__ __launch_bounds__(256) void k_cols_total(const T *__restrict__ sat, int p, int q, T *__restrict__ tot,
                                                    T *__restrict__ parts)
{
    __shared__ T part[4][64];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int c = blockIdx.x * 64 + tx, k = blockIdx.y;
    const int64_t W = q + 1;
    const int r0 = 1 + k * kColChunk + ty * 16, r1 = min(p + 1, r0 + 16);
    T acc = zero_el<T>();
    if (c <= q) {
#pragma unroll
        for (int j = 0; j < 16; j++)
            if (r0 + j < r1)
                acc = add_el(acc, sat[(int64_t)(r0 + j) * W + c]);
    }
    part[ty][tx] = acc;
    if (c <= q)
        parts[((int64_t)k * 4 + ty) * W + c] = acc;
    __syncthreads();
    if (ty == 0 && c <= q)
        tot[(int64_t)k * W + c] = add_el(add_el(part[0][tx], part[1][tx]), add_el(part[2][tx], part[3][tx]));
}

template <class T>
__global__ __launch_bounds__(256) void k_cols_apply(T *__restrict__ sat, int p, int q, const T *__restrict__ tot,
                                                    const T *__restrict__ parts)
{
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int c = blockIdx.x * 64 + tx, k = blockIdx.y;
    const int64_t W = q + 1;
    const int r0 = 1 + k * kColChunk + ty * 16, r1 = min(p + 1, r0 + 16);
    if (c > q)
        return;
    // this thread's 16 rows are loaded first, in flight with the totals above
    T v[16];
#pragma unroll
    for (int j = 0; j < 16; j++)
        if (r0 + j < r1)
            v[j] = sat[(int64_t)(r0 + j) * W + c];
    T run = zero_el<T>();
#pragma unroll 4
    for (int kk = 0; kk < k; kk++)
        run = add_el(run, tot[(int64_t)kk * W + c]);
    for (int j = 0; j < ty; j++)
        run = add_el(run, parts[((int64_t)k * 4 + j) * W + c]);
#pragma unroll
    for (int j = 0; j < 16; j++)
        if (r0 + j < r1) {
            run = add_el(run, v[j]);
            sat[(int64_t)(r0 + j) * W + c] = run;
        }
}

// Per-location box statistics for an m x n block from four table entries.
__global__ __launch_bounds__(256) void k_stats(const uint2 *__restrict__ sat, int q, int Ly, int Lx, int m, int n,
                                               int2 *__restrict__ stat)
{
    int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= (int64_t)Ly * Lx)
        return;
    int y = (int)(l / Lx), x = (int)(l - (l / Lx) * Lx);
    int64_t W = q + 1;
    uint2 a = sat[(int64_t)y * W + x], b = sat[(int64_t)y * W + x + n];
    uint2 c = sat[(int64_t)(y + m) * W + x], d = sat[(int64_t)(y + m) * W + x + n];
    uint32_t S = d.x - b.x - c.x + a.x;
    uint32_t Q = d.y - b.y - c.y + a.y;
    stat[l] = make_int2((int)S, (int)Q);
}

// ============================================================== dense search (every location)

// Tile: 64 lanes x 4 adjacent columns = 256 locations wide, 4 waves x R rows
// high.  The image tile (flipped to int8) and the template (padded with R-1
// zero rows above and below) sit in LDS.  For image row k of the wave's
// window and each 16-byte template chunk, a lane realigns its 5 image words
// into the 16 words its 4 columns need (v_alignbyte) and issues 16 v_dot4
// per output row.
template <int R>
__global__ __launch_bounds__(256) void k_full(FullArgs a)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        a.qs->t0 = __builtin_amdgcn_s_memrealtime();  // the query's first kernel
        a.qs->n_dense = 0;
        a.qs->n_sparse = 0;
    }
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[8];
    const int n4w = a.n4w;
    const int TR = 4 * R + a.m - 1;
    const int TWW = 64 + n4w;
    uint32_t *img_l = smem;
    uint32_t *tpl_l = smem + TR * TWW;
    int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int x0 = blockIdx.x * 256, y0 = blockIdx.y * (4 * R);

    int64_t st, sq;
    load_template(a.tpl, a.ts, a.m, a.n, n4w, R - 1, a.m + 2 * R - 2, tpl_l, red, &st, &sq);
    const int64_t mn = (int64_t)a.m * a.n;
    const int64_t dt = mn * sq - st * st;
    if (dt == 0) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0)
            a.qs->degenerate = 1;
        return;
    }
    for (int idx = t; idx < TR * TWW; idx += 256) {
        int r = idx / TWW, c = idx - (idx / TWW) * TWW;
        int gy = y0 + r;
        int64_t gx = (int64_t)x0 + 4 * c;
        uint32_t w = 0;
        if (gy < a.p && gx + 4 <= a.pitch)
            w = flip4(*(const uint32_t *)(a.img + (int64_t)gy * a.pitch + gx));
        img_l[idx] = w;
    }
    __syncthreads();

    int acc[R][4];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int s = 0; s < 4; s++)
            acc[r][s] = 0;

    for (int k = 0; k < R + a.m - 1; k++) {
        const uint32_t *irow = img_l + (wv * R + k) * TWW + lane;
        const uint32_t *tbase = tpl_l + (k + R - 1) * n4w;
        uint32_t w0 = irow[0];
        for (int jc = 0; jc < n4w; jc += 4) {
            uint32_t w1 = irow[jc + 1], w2 = irow[jc + 2], w3 = irow[jc + 3], w4 = irow[jc + 4];
            uint32_t sv[4][4];
            sv[0][0] = w0; sv[0][1] = bytes_at(w1, w0, 1); sv[0][2] = bytes_at(w1, w0, 2); sv[0][3] = bytes_at(w1, w0, 3);
            sv[1][0] = w1; sv[1][1] = bytes_at(w2, w1, 1); sv[1][2] = bytes_at(w2, w1, 2); sv[1][3] = bytes_at(w2, w1, 3);
            sv[2][0] = w2; sv[2][1] = bytes_at(w3, w2, 1); sv[2][2] = bytes_at(w3, w2, 2); sv[2][3] = bytes_at(w3, w2, 3);
            sv[3][0] = w3; sv[3][1] = bytes_at(w4, w3, 1); sv[3][2] = bytes_at(w4, w3, 2); sv[3][3] = bytes_at(w4, w3, 3);
#pragma unroll
            for (int r = 0; r < R; r++) {
                uint4 tw = *(const uint4 *)(tbase - r * n4w + jc);
#pragma unroll
                for (int s = 0; s < 4; s++) {
                    int v = acc[r][s];
                    v = dot4(sv[0][s], tw.x, v);
                    v = dot4(sv[1][s], tw.y, v);
                    v = dot4(sv[2][s], tw.z, v);
                    v = dot4(sv[3][s], tw.w, v);
                    acc[r][s] = v;
                }
            }
            w0 = w4;
        }
    }

    RecPod rec = rec_empty();
#pragma unroll
    for (int r = 0; r < R; r++) {
        int y = y0 + wv * R + r;
#pragma unroll
        for (int s = 0; s < 4; s++) {
            int x = x0 + 4 * lane + s;
            if (y < a.Ly && x < a.Lx) {
                int64_t l = (int64_t)y * a.Lx + x;
                int2 stl = a.stat[l];
                int64_t dr = var_num(mn, stl);
                int64_t num = mn * (int64_t)acc[r][s] - st * (int64_t)stl.x;
                float r32 = rho32(num, dt, dr);
                rec_offer(rec, r32, l, num, dt, dr);
                if (a.num_map)
                    a.num_map[l] = num;
                if (a.dr_map)
                    a.dr_map[l] = dr;
                if (a.rho_map)
                    a.rho_map[l] = r32;
                if (a.dec)
                    a.dec[l] = 2;
            }
        }
    }
    __syncthreads();
    __shared__ RecPod red4[4];
    RecPod b = block_rec4(rec, red4);
    int bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (t == 0) {
        a.recs[bid] = b;
        if (bid == 0) {  // the query state needs no fill before the scans
            a.qs->st = st;
            a.qs->dt = dt;
            a.qs->degenerate = 0;
        }
    }
}

// ============================================================== scan 1: group centres

// Strided tile: lane = one centre column, the wave holds R centre rows in
// registers and sweeps the image rows their windows cover once.  For each
// image row and 16-byte template chunk a lane loads 5 words at its centre's
// column, realigns them (v_alignbyte) and issues 4 v_dot4 for every centre
// row whose window contains that image row.  The waves of a block split the
// template chunks and sum their partial products through LDS.  Per group it
// keeps the exact N_tc and the binary32 angle A.
template <int R>
__global__ __launch_bounds__(256) void k_centres(ScanArgs a)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        a.qs->t0 = __builtin_amdgcn_s_memrealtime();  // the query's first kernel
        a.qs->n_dense = 0;
        a.qs->n_sparse = 0;
    }
    if (a.tile_cnt) {  // scan 2's survivor tile counts start from zero
        const int nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
        for (int i = b * (int)blockDim.x + (int)threadIdx.x; i < a.n_tiles; i += nb * (int)blockDim.x)
            a.tile_cnt[i] = 0;
    }
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[8];
    __shared__ RecPod rred[256];
    const int n4w = a.n4w;
    const int nw = blockDim.x >> 6;
    const int pad = a.pad;  // zero template rows above and below: >= cy[R-1] - cy[0]
    uint32_t *tpl = smem;
    int *xs = (int *)(smem + (a.m + 2 * pad) * n4w);  // [nw][R][64]
    int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int64_t st, sq;
    load_template(a.tpl, a.ts, a.m, a.n, n4w, pad, a.m + 2 * pad, tpl, red, &st, &sq);
    const int64_t mn = (int64_t)a.m * a.n;
    const int64_t dt = mn * sq - st * st;
    if (dt == 0) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0)
            a.qs->degenerate = 1;
        return;
    }
    const int gx = blockIdx.x * 64 + lane;
    const bool colok = gx < a.Gx;
    int cx = 0;
    if (colok) {
        int ox = gx * a.w;
        int ww = min(a.w, a.Lx - ox);
        cx = ox + (ww - 1) / 2;
    }
    const uint32_t sh = (uint32_t)(cx & 3);
    const int64_t pw = a.pitch >> 2;
    const uint32_t *colbase = (const uint32_t *)a.img + (cx >> 2);
    const int gy0 = blockIdx.y * R;
    const int nvalid = min(R, a.Gy - gy0);
    // centre rows of the wave; rows past the grid repeat the last one (their
    // results are discarded)
    int cy[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        int gy = min(gy0 + r, a.Gy - 1);
        int oy = gy * a.h;
        int hh = min(a.h, a.Ly - oy);
        cy[r] = oy + (hh - 1) / 2;
    }
    int acc[R];
#pragma unroll
    for (int r = 0; r < R; r++)
        acc[r] = 0;
    const int nch = n4w >> 2;
    const int ylo = cy[0], yhi = cy[R - 1] + a.m;
    for (int c = wv; c < nch; c += nw) {
        // padded template row of centre row r for image row yy + u is
        // pad + (yy + u) - cy[r]; tb points at row pad + (yy - ylo)
        const uint32_t *tb = tpl + pad * n4w + 4 * c;
        const uint32_t *pc = colbase + (int64_t)ylo * pw + 4 * c;
        for (int yy = ylo; yy < yhi; yy += 4, pc += 4 * pw, tb += 4 * n4w) {
            uint32_t W[4][5];
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (yy + u < yhi) {
#pragma unroll
                    for (int k = 0; k < 5; k++)
                        W[u][k] = pc[u * pw + k];
                }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (yy + u >= yhi)
                    break;
                uint32_t sv[4];
#pragma unroll
                for (int k = 0; k < 4; k++)
                    sv[k] = flip4(bytes_at(W[u][k + 1], W[u][k], sh));
                uint4 tw[R];
#pragma unroll
                for (int r = 0; r < R; r++)
                    tw[r] = *(const uint4 *)(tb + (u - (cy[r] - ylo)) * n4w);
#pragma unroll
                for (int r = 0; r < R; r++)
                    acc[r] = dot4(sv[0], tw[r].x, acc[r]);
#pragma unroll
                for (int r = 0; r < R; r++)
                    acc[r] = dot4(sv[1], tw[r].y, acc[r]);
#pragma unroll
                for (int r = 0; r < R; r++)
                    acc[r] = dot4(sv[2], tw[r].z, acc[r]);
#pragma unroll
                for (int r = 0; r < R; r++)
                    acc[r] = dot4(sv[3], tw[r].w, acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++)
        xs[(wv * R + r) * 64 + lane] = acc[r];
    __syncthreads();
    RecPod rec = rec_empty();
    for (int r = wv; r < nvalid; r += nw) {
        int X = 0;
        for (int k = 0; k < nw; k++)
            X += xs[(k * R + r) * 64 + lane];
        if (colok) {
            int g = (gy0 + r) * a.Gx + gx;
            int oy = (gy0 + r) * a.h;
            int hh = min(a.h, a.Ly - oy);
            int64_t l = (int64_t)(oy + (hh - 1) / 2) * a.Lx + cx;
            int2 sc = a.stat[l];
            int64_t dc = var_num(mn, sc);
            int64_t num = mn * (int64_t)X - st * (int64_t)sc.x;
            a.g_x[g] = X;
            a.g_theta[g] = theta32(num, dt, dc);
            rec_offer(rec, rho32(num, dt, dc), l, num, dt, dc);
            if (a.dec)
                a.dec[l] = 1;
        }
    }
    RecPod b = block_rec(rec, rred);
    int bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (t == 0) {
        a.recs[bid] = b;
        if (bid == 0) {  // the query state needs no fill before the scans
            a.qs->st = st;
            a.qs->dt = dt;
            a.qs->degenerate = 0;
        }
    }
}

// Scan 1 on int8 MFMA: M = 16 centre columns (stride w), N = 16 centre rows
// (stride h), K = 4 image rows x 16 columns.  A block holds 16 centre rows x
// 64 MTW centre columns: each of its four waves MTW M-tiles for every
// template of the launch (up to TM), all with their own accumulators.  The
// image region the block's windows cover streams through LDS in 4-row steps,
// each row staged as four byte-shifted copies so that every A lane reads
// whole words (lane j of an M-tile reads the copy shifted by its centre's
// byte offset mod 4); the fragments of the next column block are read before
// the current one's MFMAs, and the sequence of reads and MFMAs is the same in
// every step.  For image row y, lane (j, g) of the B fragment carries
// template row y - cy_j (the zero row outside the template, and for centre
// rows past the last).  Outputs equal k_centres'.
constexpr int kCmThreads = 256;
// staged words per thread and step, at most, for MTW M-tiles per wave
__host__ __device__ constexpr int cm_words_per_thread(int mtw) { return mtw == 1 ? 2 : mtw == 2 ? 3 : 4; }

// Template rows flipped to int8 at row stride tstr, then one zero row, and
// this thread's partial sums of t' and t'^2 (no barrier: the caller's next
// barrier publishes the rows, and the sums are reduced where they are
// needed).  Whole words are loaded when the rows are word-aligned (bytes
// past column n are masked to int8 zero).
__device__ __forceinline__ void load_template_rows(const uint8_t *__restrict__ tpl, int64_t ts, int m, int n,
                                                   int nw16, int tstr, uint32_t *lds, int *s, int *s2)
{
    const bool words = ((ts | (int64_t)(uintptr_t)tpl) & 3) == 0 && (n & 3) == 0;
    const uint32_t ones = 0x01010101u;
    int a = 0, a2 = 0;
    if (words) {
        batched_loads<8>(
            m * nw16,
            [&](int idx) {
                const int r = idx / nw16;
                return flip4(tpl_raw_word(tpl, ts, n, r, idx - r * nw16));
            },
            [&](int idx, uint32_t w) {
                const int r = idx / nw16, j = idx - r * nw16;
                const int nb = n - 4 * j;  // flip4 turned the zero bytes past column n into 0x80
                w = nb >= 4 ? w : nb <= 0 ? 0u : w & ((1u << (8 * nb)) - 1u);
                a = dot4(w, ones, a);
                a2 = dot4(w, w, a2);
                lds[r * tstr + j] = w;
            });
        for (int j = threadIdx.x; j < nw16; j += blockDim.x)
            lds[m * tstr + j] = 0u;
    } else {
        for (int idx = threadIdx.x; idx < (m + 1) * nw16; idx += blockDim.x) {
            int r = idx / nw16, j = idx - r * nw16;
            uint32_t w = 0;
            if (r < m) {
                w = tpl_word(tpl, ts, n, r, j, words);
                a = dot4(w, ones, a);
                a2 = dot4(w, w, a2);
            }
            lds[r * tstr + j] = w;
        }
    }
    *s = a;
    *s2 = a2;
}

// Per-template fields of a (batched) scan 1.
__device__ __forceinline__ ScanTpl scan_tpl(const ScanArgs &a, int i)
{
    if (i == 0)
        return ScanTpl{a.tpl, a.ts, a.g_x, a.g_theta, a.recs, a.qs, a.tile_cnt};
    return a.more[i - 1];
}

// TM: most templates per launch (a.ntpl of them run); NB: 16-byte column
// blocks of the template row (n16 = 16 NB); MTW: M-tiles per wave.
template <int NB, int TM, int MTW>
__global__ __launch_bounds__(kCmThreads) void k_centres_mfma(ScanArgs a)
{
    constexpr int KL = cm_words_per_thread(MTW);
    const int T = TM == 1 ? 1 : a.ntpl;
#pragma unroll
    for (int ti = 0; ti < TM; ti++) {
        if (ti >= T)
            break;
        const ScanTpl sp = scan_tpl(a, ti);
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            sp.qs->t0 = __builtin_amdgcn_s_memrealtime();  // the query's first kernel
            sp.qs->n_dense = 0;
            sp.qs->n_sparse = 0;
        }
        if (sp.tile_cnt) {  // scan 2's survivor tile counts start from zero
            const int nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
            for (int i = b * (int)blockDim.x + (int)threadIdx.x; i < a.n_tiles; i += nb * (int)blockDim.x)
                sp.tile_cnt[i] = 0;
        }
    }
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int red[2 * TM * 4];
    __shared__ RecPod rred[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int m = a.m, n = a.n;
    constexpr int nw16 = 4 * NB;
    const int tstr = batch_tstride(nw16), CS = a.cwd, CWn = a.cwn;
    const int twords = (m + 1) * tstr;       // one template's rows in LDS
    const int IMGW = 16 * CS;                // one step: 4 rows x 4 byte-shifted copies
    uint32_t *tpl_l = smem;                  // per template: m rows and the zero row m, stride tstr
    uint32_t *buf0 = smem + T * twords;      // two step buffers
    auto ccol = [&](int gx) { int ox = gx * a.w; return ox + (min(a.w, a.Lx - ox) - 1) / 2; };
    auto crow = [&](int gy) { int oy = gy * a.h; return oy + (min(a.h, a.Ly - oy) - 1) / 2; };
    // XCD-aware placement: the hardware deals workgroup ids round-robin over
    // the 8 XCDs; each XCD's ids are mapped to a contiguous run of blocks in
    // column-major order, so vertically adjacent regions (which overlap by
    // m - h image rows) are mostly read through the same L2
    int bxl, byl;
    {
        const int nb = gridDim.x * gridDim.y, hw = blockIdx.y * gridDim.x + blockIdx.x;
        const int q8 = nb >> 3, r8 = nb & 7, xcd = hw & 7;
        const int j = xcd * q8 + min(xcd, r8) + (hw >> 3);
        bxl = j / gridDim.y;
        byl = j - bxl * gridDim.y;
    }
    const int gx0 = bxl * 64 * MTW, gy0 = byl * 16;
    const int ny = min(16, a.Gy - gy0);
    const int xw0 = ccol(gx0) >> 2;                 // first staged word of the region's rows
    const int ylo = crow(gy0), yhi = crow(gy0 + ny - 1) + m;
    const int steps = (yhi - ylo + 3) >> 2;
    const uint8_t *img = a.img;
    // Staging: thread t takes words t, t + 256, ... of the step's 4 x CWn
    // words (row idx / CWn), each with the word after it, from clamped
    // in-image addresses without branches (a staged byte that is not a pixel
    // of a centre's window only ever meets a zero template byte: a column
    // past n, or the zero row), and writes the word's four byte-shifted
    // copies.  The host keeps 4 CWn <= 256 KL.
    uint32_t rA[KL][2], rB[KL][2], rC[KL][2];
    auto gload = [&](int s, uint32_t (&ri)[KL][2]) {
#pragma unroll
        for (int k = 0; k < KL; k++) {
            const int idx = min(t + 256 * k, 4 * CWn - 1);
            const int r = idx / CWn, wd = idx - r * CWn;
            const int y = min(ylo + 4 * s + r, yhi - 1);
            const int64_t x = min((int64_t)4 * (xw0 + wd), a.pitch - 8);
            const uint8_t *rp = img + (int64_t)y * a.pitch + x;
            ri[k][0] = *gptr((const uint32_t *)rp);
            ri[k][1] = *gptr((const uint32_t *)(rp + 4));
        }
    };
    auto lstore = [&](int s, const uint32_t (&ri)[KL][2]) {
        uint32_t *b = buf0 + (s & 1) * IMGW;
#pragma unroll
        for (int k = 0; k < KL; k++) {
            const int idx = t + 256 * k;
            if (idx < 4 * CWn) {
                const int r = idx / CWn, wd = idx - r * CWn;
                const uint32_t lo = flip4(ri[k][0]), hi = flip4(ri[k][1]);
                b[(r * 4 + 0) * CS + wd] = lo;
                b[(r * 4 + 1) * CS + wd] = bytes_at(hi, lo, 1);
                b[(r * 4 + 2) * CS + wd] = bytes_at(hi, lo, 2);
                b[(r * 4 + 3) * CS + wd] = bytes_at(hi, lo, 3);
            }
        }
    };
    gload(0, rA);
    // the template statistics are reduced after the main loop, which needs
    // only the rows (published by the first barrier)
    int ps[TM], ps2[TM];
#pragma unroll
    for (int ti = 0; ti < TM; ti++) {
        ps[ti] = ps2[ti] = 0;
        if (ti < T) {
            const ScanTpl sp = scan_tpl(a, ti);
            load_template_rows(sp.tpl, sp.ts, m, n, nw16, tstr, tpl_l + ti * twords, &ps[ti], &ps2[ti]);
        }
    }
    lstore(0, rA);
    __syncthreads();
    gload(1, rB);
    gload(2, rC);
    const int g = lane >> 4, jr = lane & 15;
    // A lane (jr, g) of M-tile mt: centre column gx0 + 16 (MTW wv + mt) + jr
    // (the last one for columns past Gx), byte offset o from the region's
    // first staged word: copy o & 3 of row g, word o >> 2
    int a_off[MTW];
#pragma unroll
    for (int mt = 0; mt < MTW; mt++) {
        const int o = ccol(min(gx0 + 16 * (MTW * wv + mt) + jr, a.Gx - 1)) - 4 * xw0;
        a_off[mt] = (g * 4 + (o & 3)) * CS + (o >> 2);
    }
    // B lane (jr, g): template row 4s + g - cy_jr of the step's image rows
    const bool jok = jr < ny;
    const int bsh = g - (crow(min(gy0 + jr, a.Gy - 1)) - ylo);
    v4i acc[TM][MTW];
#pragma unroll
    for (int ti = 0; ti < TM; ti++)
#pragma unroll
        for (int mt = 0; mt < MTW; mt++)
            acc[ti][mt] = v4i{0, 0, 0, 0};
    auto compute = [&](int s) {
        const uint32_t *pa = buf0 + (s & 1) * IMGW;
        const int tr = 4 * s + bsh;
        const uint32_t *pb = tpl_l + (jok && (unsigned)tr < (unsigned)m ? tr : m) * tstr;
        v4i A0[MTW], A1[MTW], B0[TM], B1[TM];
        auto frag = [&](v4i (&A)[MTW], v4i (&B)[TM], int cb) {
#pragma unroll
            for (int mt = 0; mt < MTW; mt++)
                __builtin_memcpy(&A[mt], pa + a_off[mt] + 4 * cb, 16);
#pragma unroll
            for (int ti = 0; ti < TM; ti++)
                if (ti < T)
                    B[ti] = *(const v4i *)(pb + ti * twords + 4 * cb);
        };
        auto mma = [&](const v4i (&A)[MTW], const v4i (&B)[TM]) {
#pragma unroll
            for (int ti = 0; ti < TM; ti++)
                if (ti < T)
#pragma unroll
                    for (int mt = 0; mt < MTW; mt++)
                        acc[ti][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], B[ti], acc[ti][mt], 0, 0, 0);
        };
        frag(A0, B0, 0);
#pragma unroll
        for (int cb = 0; cb < NB; cb += 2) {
            if (cb + 1 < NB) {
                frag(A1, B1, cb + 1);
                mma(A0, B0);
                if (cb + 2 < NB)
                    frag(A0, B0, cb + 2);
                mma(A1, B1);
            } else {
                mma(A0, B0);
            }
        }
    };
    // step s reads buffer s & 1; the data of step s + 1 (loaded three steps
    // ahead, into rA, rB, rC by turns) goes to the other buffer, free since
    // the last barrier.  Loads past the last step are issued too (clamped
    // rows, never stored), so that every wait counts the same loads in flight.
    for (int s = 0; s < steps; s += 3) {
        gload(s + 3, rA);
        compute(s);
        if (s + 1 < steps)
            lstore(s + 1, rB);
        __syncthreads();
        if (s + 1 >= steps)
            break;
        gload(s + 4, rB);
        compute(s + 1);
        if (s + 2 < steps)
            lstore(s + 2, rC);
        __syncthreads();
        if (s + 2 >= steps)
            break;
        gload(s + 5, rC);
        compute(s + 2);
        if (s + 3 < steps)
            lstore(s + 3, rA);
        __syncthreads();
    }
    // template statistics of every template at once
#pragma unroll
    for (int ti = 0; ti < TM; ti++) {
        const int s1 = wave_sum(ps[ti]), s2 = wave_sum(ps2[ti]);
        if (lane == 0 && ti < T) {
            red[(2 * ti) * 4 + wv] = s1;
            red[(2 * ti + 1) * 4 + wv] = s2;
        }
    }
    // accumulator lane: centre row gy0 + jr, centre columns
    // gx0 + 16 (MTW wv + mt) + 4 g + v; their statistics in one round trip
    const int gyy = gy0 + jr;
    int2 sc[MTW][4];
#pragma unroll
    for (int mt = 0; mt < MTW; mt++)
#pragma unroll
        for (int v = 0; v < 4; v++)
            sc[mt][v] = ld_int2(a.cstat + ((int64_t)min(gyy, a.Gy - 1) * a.Gx +
                                           min(gx0 + 16 * (MTW * wv + mt) + 4 * g + v, a.Gx - 1)));
    __syncthreads();
    const int64_t mn = (int64_t)m * n;
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
    for (int ti = 0; ti < TM; ti++) {
        if (ti >= T)
            break;
        const ScanTpl sp = scan_tpl(a, ti);
        const int64_t st = (int64_t)red[(2 * ti) * 4] + red[(2 * ti) * 4 + 1] + red[(2 * ti) * 4 + 2] +
                           red[(2 * ti) * 4 + 3];
        const int64_t sq2 = (int64_t)red[(2 * ti + 1) * 4] + red[(2 * ti + 1) * 4 + 1] +
                            red[(2 * ti + 1) * 4 + 2] + red[(2 * ti + 1) * 4 + 3];
        const int64_t dt = mn * sq2 - st * st;
        if (dt == 0) {  // uniform over the block
            if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0)
                sp.qs->degenerate = 1;
            continue;
        }
        // Only centres within kEpsRho of the wave's largest binary32 rho can be
        // the block's best: they alone are evaluated in binary64 (one at a
        // time per lane, usually one in the whole wave), and the wave's
        // record is picked among those lanes in lane order.
        // N and D_c formed in binary64, where they are exact (no int64
        // products or conversions per centre)
        float r32[MTW][4];
        float lmax = -2.0f;
        const double mnd = (double)mn, dtd = (double)dt, std_ = (double)st;
#pragma unroll
        for (int mt = 0; mt < MTW; mt++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int gxx = gx0 + 16 * (MTW * wv + mt) + 4 * g + v;
                const bool ok = gyy < a.Gy && gxx < a.Gx;
                const int x = acc[ti][mt][v];
                const double S = (double)sc[mt][v].x;
                const double dc = fma(mnd, (double)(uint32_t)sc[mt][v].y, -S * S);
                const double num = fma(mnd, (double)x, -std_ * S);
                r32[mt][v] = ok ? rho32_exact(num, dtd, dc) : -2.0f;
                if (ok) {
                    const int gi = gyy * a.Gx + gxx;
                    sp.g_x[gi] = x;
                    sp.g_theta[gi] = theta32_exact(num, dtd, dc);
                    lmax = fmaxf(lmax, r32[mt][v]);
                    if (ti == 0 && a.dec)
                        a.dec[(int64_t)crow(gyy) * a.Lx + ccol(gxx)] = 1;
                }
            }
        float wmax = lmax;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            wmax = fmaxf(wmax, __shfl_xor(wmax, off));
        uint32_t cmask = 0;
#pragma unroll
        for (int mt = 0; mt < MTW; mt++)
#pragma unroll
            for (int v = 0; v < 4; v++)
                if (r32[mt][v] > -2.0f && r32[mt][v] >= wmax - kEpsRho)
                    cmask |= 1u << (4 * mt + v);
        double brho = -2.0;
        int64_t bl = INT64_MAX, bnum = 0, bdr = 0;
        bool bv = false;
        while (cmask) {
            const int e = __ffs(cmask) - 1;
            cmask &= cmask - 1;
            int x = 0;
            int2 scv = make_int2(0, 0);
#pragma unroll
            for (int q = 0; q < 4 * MTW; q++)
                if (q == e) {
                    x = acc[ti][q >> 2][q & 3];
                    scv = sc[q >> 2][q & 3];
                }
            const int gxx = gx0 + 16 * (MTW * wv + (e >> 2)) + 4 * g + (e & 3);
            const int64_t l = (int64_t)crow(gyy) * a.Lx + ccol(gxx);
            const int64_t dc = var_num(mn, scv);
            const int64_t num = mn * (int64_t)x - st * (int64_t)scv.x;
            const double r = rho64(num, dt, dc);
            if (!bv || rec_better(r, l, brho, bl)) {
                brho = r;
                bl = l;
                bnum = num;
                bdr = dc;
                bv = true;
            }
        }
        RecPod rec = rec_empty();
        rec.r32max = wmax;
        for (uint64_t msk = __ballot(bv); msk; msk &= msk - 1) {
            const int src = __ffsll((unsigned long long)msk) - 1;
            const double r = __shfl(brho, src);
            const int64_t l = (int64_t)__shfl((long long)bl, src);
            if (!rec.valid || rec_better(r, l, rec.rho, rec.l)) {
                rec.rho = r;
                rec.l = l;
                rec.num = (int64_t)__shfl((long long)bnum, src);
                rec.dr = (int64_t)__shfl((long long)bdr, src);
                rec.valid = 1;
            }
        }
        if (lane == 0)
            rred[wv] = rec;
        __syncthreads();
        if (wv == 0) {  // the four wave records merged by shuffles in lanes 0..3
            RecPod bb = wave_rec<4>(lane < 4 ? rred[lane] : rec_empty());
            if (lane == 0) {
                sp.recs[bid] = bb;
                if (bid == 0) {  // the query state needs no fill before the scans
                    sp.qs->st = st;
                    sp.qs->dt = dt;
                    sp.qs->degenerate = 0;
                }
            }
        }
        __syncthreads();  // rred is rewritten by the next template
    }
}

// ============================================================== refinement window

// Matches the template on the original image at every location within
// `radius` of the best scan-1 centre (skipping locations scan 1 already
// matched when it ran on the same image), one block per location; scan 2
// forms its threshold from these records and, when thr_out is set, from the
// scan-1 best that block 0 writes into the query state (so that scan 2 does
// not reduce the scan-1 records again).
constexpr int kWinWords = 16;  // template words per thread read ahead (all of a 128 x 128 template)

__global__ __launch_bounds__(256) void k_window(WinArgs a)
{
    __shared__ int red[8];
    __shared__ Best bred[4];
    const int t = threadIdx.x;
    // The query state (template statistics from scan 1), this thread's
    // template words and the scan-1 records are read in one round trip; the
    // block's window location and its image words in a second one.
    const int degenerate = a.qs->degenerate;
    const int64_t st = a.qs->st, dt = a.qs->dt;
    const int n4 = (a.n + 3) >> 2, nwords = a.m * n4;
    const bool aligned = ((a.ts | (int64_t)(uintptr_t)a.tpl) & 3) == 0 && (a.n & 3) == 0;
    uint32_t tw[kWinWords];
    if (aligned) {  // clamped indices, no branch around a load: all in flight together
#pragma unroll
        for (int q = 0; q < kWinWords; q++) {
            const int idx = t + 256 * q, ci = min(idx, nwords - 1);
            const uint32_t w = flip4(tpl_raw_word(a.tpl, a.ts, a.n, ci / n4, ci % n4));
            const int nb = a.n - 4 * (ci % n4);
            tw[q] = idx < nwords ? (nb >= 4 ? w : w & ((1u << (8 * nb)) - 1u)) : 0u;
        }
    } else {
#pragma unroll
        for (int q = 0; q < kWinWords; q++) {
            const int idx = t + 256 * q;
            tw[q] = idx < nwords ? tpl_word(a.tpl, a.ts, a.n, idx / n4, idx % n4, aligned) : 0u;
        }
    }
    const Best b0 = reduce_best(a.recs, 0, a.rec_off, bred);  // best scan-1 centre (has barriers)
    if (degenerate)
        return;
    const int64_t c0 = b0.l;
    if (a.thr_out && blockIdx.x == 0 && t == 0) {  // scan 2 takes the scan-1 best from here
        a.qs->best0 = b0.rho;
        a.qs->best0_l = b0.l;
    }
    const int W = 2 * a.radius + 1, k = blockIdx.x;
    const int y = (int)(c0 / a.Lx) - a.radius + k / W, x = (int)(c0 % a.Lx) - a.radius + k % W;
    const int64_t l = (int64_t)y * a.Lx + x;
    const bool live = y >= 0 && y < a.Ly && x >= 0 && x < a.Lx &&
                      !(a.skip_centres && centre_of(y, x, a.Ly, a.Lx, a.h, a.w) == l);
    RecPod rec = rec_empty();
    if (live) {  // uniform over the block
        int2 so = make_int2(0, 0);
        if (t == 0)
            so = a.stat[l];
        const uint32_t sh = (uint32_t)(x & 3);
        const int64_t pw = a.pitch >> 2;
        const uint32_t *row0 = (const uint32_t *)(a.img + (((int64_t)y * a.pitch + x) & ~(int64_t)3));
        int acc = 0;
        // every word from a clamped index (tw is zero past the template), so
        // that the loads are in flight together
        uint32_t lo[kWinWords], hi[kWinWords];
#pragma unroll
        for (int q = 0; q < kWinWords; q++) {
            const int ci = min(t + 256 * q, nwords - 1);
            const int i = ci / n4, j = ci % n4;
            const uint32_t *pr = row0 + (int64_t)i * pw + j;  // rows carry >= 64 bytes of padding
            lo[q] = pr[0];
            hi[q] = pr[1];
        }
#pragma unroll
        for (int q = 0; q < kWinWords; q++)
            acc = dot4(flip4(bytes_at(hi[q], lo[q], sh)), tw[q], acc);
        for (int idx = t + 256 * kWinWords; idx < nwords; idx += 256) {  // tall, narrow templates
            const int i = idx / n4, j = idx % n4;
            const uint32_t *pr = row0 + (int64_t)i * pw + j;
            acc = dot4(flip4(bytes_at(pr[1], pr[0], sh)), tpl_word(a.tpl, a.ts, a.n, i, j, aligned), acc);
        }
        const int X = block_sum_int(acc, red);
        if (t == 0) {
            const int64_t mn = (int64_t)a.m * a.n;
            const int64_t dr = var_num(mn, so);
            const int64_t num = mn * (int64_t)X - st * (int64_t)so.x;
            rec_offer_inline(rec, rho32(num, dt, dr), l, num, dt, dr);
            rec.n_window = 1;
            if (a.dec)
                a.dec[l] = 3;
        }
    }
    if (t == 0)
        a.recs[a.rec_off + blockIdx.x] = rec;
}

// ============================================================== scan 2: members

constexpr int kMemGPT = 4;                 // groups per k_members thread
constexpr int kMemGroups = 256 * kMemGPT;  // groups per k_members block

__device__ __forceinline__ bool in_window(int y, int x, int wy, int wx, int radius)
{
    return radius >= 0 && abs(y - wy) <= radius && abs(x - wx) <= radius;
}

// Loads the template words only (statistics come from scan 1), as raw
// uint8 bytes with zeros past column n: survivors are matched with unsigned
// dot products, N being the same from unsigned sums (it is shift-invariant).
__device__ void load_template_words(const uint8_t *__restrict__ tpl, int64_t ts, int m, int n, int n4,
                                    uint32_t *lds)
{
    const bool words = ((ts | (int64_t)(uintptr_t)tpl) & 3) == 0 && (n & 3) == 0;
    if (words) {
        batched_loads<8>(
            m * n4,
            [&](int idx) {
                const int r = idx / n4;
                return tpl_raw_word(tpl, ts, n, r, idx - r * n4);
            },
            [&](int idx, uint32_t w) { lds[idx] = w; });
        return;
    }
    for (int idx = threadIdx.x; idx < m * n4; idx += blockDim.x) {
        int r = idx / n4, j = idx - (idx / n4) * n4;
        const uint32_t w = tpl_word(tpl, ts, n, r, j, words);  // int8 view, zero past column n
        const int nb = min(4, n - 4 * j);
        const uint32_t keep = nb < 4 ? (1u << (8 * nb)) - 1u : 0xffffffffu;
        lds[idx] = (w ^ 0x80808080u) & keep;
    }
}

// Canonical binary64 elimination test (the transitive bound of Eq. 2, or
// its angle-triangle form with the blur angle C when a.opta).  True: keep.
// o: location, s: its slot in the group-major tables, c: centre location.
__device__ bool keep_canonical(const MemArgs &a, int64_t o, int64_t s, int64_t c, int g, int64_t mn, int64_t st,
                               int64_t dt, double thr64)
{
    int2 sc = a.statS[c], so = a.statS[o];
    int64_t dc = var_num(mn, sc), dso = var_num(mn, so);
    int64_t dio = dso;
    int2 si = so;
    if (a.opta) {
        si = a.statI[o];
        dio = var_num(mn, si);
    }
    if (dc == 0 || dso == 0 || dio == 0)
        return true;
    int64_t ntc = mn * (int64_t)a.g_x[g] - st * (int64_t)sc.x;
    double ra = rho64(ntc, dt, dc), sa = sin64(ntc, dt, dc);
    int64_t nco = mn * (int64_t)a.x_b[s] - (int64_t)sc.x * (int64_t)so.x;
    double rb = rho64(nco, dc, dso), sb = sin64(nco, dc, dso);
    double rc = 1.0, sc2 = 0.0;
    if (a.opta) {
        int64_t noo = mn * (int64_t)a.x_c[s] - (int64_t)so.x * (int64_t)si.x;
        rc = rho64(noo, dso, dio);
        sc2 = sin64(noo, dso, dio);
    }
    double ub;
    if (ub_general(ra, sa, rb, sb, rc, sc2, &ub) && ub < thr64)
        return false;
    return true;
}

__device__ __forceinline__ int block_excl_scan(int v, int *tmp, int *total)
{
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(incl, off);
        if (lane >= off)
            incl += u;
    }
    if (lane == 63)
        tmp[wv] = incl;
    __syncthreads();
    int base = 0, tot = 0;
    for (int k = 0; k < 4; k++) {
        if (k < wv)
            base += tmp[k];
        tot += tmp[k];
    }
    *total = tot;
    return base + incl - v;  // tmp must not be written again before the caller's next barrier
}

// kMemGroups consecutive groups per block (kMemGPT per thread).  Phase 1: one thread
// per group drops the whole group when the interval of its member angles
// lies beyond the threshold angle from A.  Phase 2: the members of the
// remaining groups are tested one per thread slot, up to 4096 per pass, each
// slot finding its group in an owner map the group's thread wrote, reading
// the group-major angle tables contiguously (binary32 angles; canonical
// binary64 inside the guard band); survivors go to an LDS list and are binned
// by survivor tile.
// Bins one pass's survivors by tile: a tile's survivors take consecutive
// slots of its bin (the first tile_cap are kept; a fuller tile is matched
// whole).  The block's survivors are counted per tile in LDS first, so each
// (block, tile) pair takes one global atomic; blocks whose groups span more
// than kBinTiles tiles take one atomic per survivor.  All threads call it.
constexpr int kBinTiles = 256;
constexpr int kSurvList = 3072;  // survivors a k_members block collects before binning them

__device__ void bin_survivors(const MemArgs &a, const int *s_list, int ns, int tile_lo, int ntl, uint32_t *s_tc,
                              uint32_t *s_tb)
{
    const int t = threadIdx.x;
    const int cap = a.tile_cap;
    auto tile_of = [&](int o) {
        const int y = o / a.Lx, x = o - (o / a.Lx) * a.Lx;
        return (y / kTileRows) * a.tiles_x + x / kTileCols;
    };
    if (ntl > kBinTiles) {
        for (int k = t; k < ns; k += 256) {
            const int o = s_list[k], tile = tile_of(o);
            const uint32_t slot = atomicAdd(&a.tile_cnt[tile], 1u);
            if ((int)slot < cap)
                a.tile_bin[(int64_t)tile * cap + slot] = o;
        }
        return;
    }
    for (int i = t; i < ntl; i += 256)
        s_tc[i] = 0;
    __syncthreads();
    constexpr int PER = kSurvList / 256;  // survivors per thread
    int tl[PER], ps[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int k = t + 256 * q;
        tl[q] = -1;
        if (k < ns) {
            tl[q] = tile_of(s_list[k]) - tile_lo;
            ps[q] = (int)atomicAdd(&s_tc[tl[q]], 1u);
        }
    }
    __syncthreads();
    for (int i = t; i < ntl; i += 256) {
        const uint32_t c = s_tc[i];
        s_tb[i] = c ? atomicAdd(&a.tile_cnt[tile_lo + i], c) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
        if (tl[q] < 0)
            continue;
        const int slot = (int)s_tb[tl[q]] + ps[q];
        if (slot < cap)
            a.tile_bin[(int64_t)(tile_lo + tl[q]) * cap + slot] = s_list[t + 256 * q];
    }
}

// Five blocks per CU (96 VGPRs, 31 KB of LDS): the passes wait on their
// angle loads, so the resident waves set the time.
__global__ __launch_bounds__(256, 5) void k_members(MemArgs a)
{
    constexpr int CAP = 2048;  // members per pass: 8 per thread
    static_assert(CAP <= kSurvList, "a pass's survivors fit the list");
    constexpr int GB = kMemGroups;
    static_assert(GB <= 65536, "group slots fit 16 bits");
    __shared__ int s_pref[GB + 1];
    __shared__ uint16_t s_owner[CAP];  // the block group of each member slot of a pass
    __shared__ int s_tmp[4];
    __shared__ int s_geo[GB][2];  // packed (oy, ox), A bits (extents and centre follow from the origin)
    __shared__ int s_list[kSurvList];
    __shared__ int s_nsurv;
    __shared__ RecPod wrec[4];
    __shared__ Best bred[8];
    __shared__ uint32_t s_tc[kBinTiles], s_tb[kBinTiles];
    int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // This thread's groups (kMemGPT t .. of the block), the query state and
    // the earlier kernels' records are all read in the first round trip.
    const int G = a.Gy * a.Gx;
    const int g0 = blockIdx.x * GB;
    float A2[kMemGPT];
    GroupSum gs2[kMemGPT];
#pragma unroll
    for (int e = 0; e < kMemGPT; e++) {
        // clamped, unconditional loads: all of them in flight at once
        const int gc = min(g0 + kMemGPT * t + e, G - 1);
        A2[e] = a.g_theta[gc];
        gs2[e] = a.gsum[gc];
    }
    const int degenerate = a.qs->degenerate;
    const Thr thr = a.thr_ready
                        ? wave_threshold(a.qs, a.recs + a.n_best0, a.n_win, a.include_best0, a.delta, a.floor)
                        : block_threshold(a.recs, a.n_best0, a.n_win, a.include_best0, a.delta, a.floor, bred);
    if (degenerate)
        return;
    if (blockIdx.x == 0 && t == 0)
        store_threshold(a.qs, thr);
    const int64_t mn = (int64_t)a.m * a.n;
    const int64_t st = a.qs->st, dt = a.qs->dt;
    const float lo = thr.lo, hi = thr.hi;
    const double thr64 = thr.thr64;
    const int hw = a.h * a.w;
    int wy = -1, wx = -1;
    if (a.radius >= 0) {
        int64_t c0 = thr.best0_l;
        wy = (int)(c0 / a.Lx);
        wx = (int)(c0 - (c0 / a.Lx) * a.Lx);
    }
    unsigned long long n_elim = 0, n_surv = 0;
    // the survivor tiles this block's groups can touch: every tile column of
    // the tile rows its location rows span
    const int glast = min(G, g0 + GB) - 1;
    const int ty_lo = ((g0 / a.Gx) * a.h) / kTileRows;
    const int ty_hi = min(a.Ly - 1, (glast / a.Gx) * a.h + a.h - 1) / kTileRows;
    const int tile_lo = ty_lo * a.tiles_x, ntl = (ty_hi - ty_lo + 1) * a.tiles_x;

    int cnt2[kMemGPT];
#pragma unroll
    for (int e = 0; e < kMemGPT; e++) {
        cnt2[e] = 0;
        const int u = kMemGPT * t + e, g = g0 + u;
        const float A = A2[e];
        const GroupSum gs = gs2[e];
        int &cnt = cnt2[e];
        if (g < G) {
            int oy, ox, hh, ww, cy, cx;
            group_geom(g, a.Gx, a.Ly, a.Lx, a.h, a.w, oy, ox, hh, ww, cy, cx);
            s_geo[u][0] = (oy << 16) | ox;
            s_geo[u][1] = __float_as_int(A);
            bool drop = false;
            if (!(gs.flags & 1)) {
                float d = 0.0f;
                bool outside = true;
                if (A < gs.bmin)
                    d = gs.bmin - A;
                else if (A > gs.bmax)
                    d = A - gs.bmax;
                else
                    outside = false;
                if (outside && (d - gs.cmax) > hi)
                    drop = true;
            }
            if (drop) {
                int inter = 0, cin = 0;
                if (a.radius >= 0) {
                    int y0 = max(oy, wy - a.radius), y1 = min(oy + hh - 1, wy + a.radius);
                    int x0 = max(ox, wx - a.radius), x1 = min(ox + ww - 1, wx + a.radius);
                    if (y0 <= y1 && x0 <= x1)
                        inter = (y1 - y0 + 1) * (x1 - x0 + 1);
                    cin = in_window(cy, cx, wy, wx, a.radius) ? 1 : 0;
                }
                n_elim += a.opta ? (hh * ww - inter) : (hh * ww - 1 - (inter - cin));
                if (a.dec)
                    for (int yy = oy; yy < oy + hh; yy++)
                        for (int xx = ox; xx < ox + ww; xx++) {
                            if ((!a.opta && yy == cy && xx == cx) || in_window(yy, xx, wy, wx, a.radius))
                                continue;
                            a.dec[(int64_t)yy * a.Lx + xx] = 0;
                        }
            } else {
                cnt = hh * ww;
            }
        }
    }
    int total;
    int csum = 0;
#pragma unroll
    for (int e = 0; e < kMemGPT; e++)
        csum += cnt2[e];
    const int off = block_excl_scan(csum, s_tmp, &total);
    {
        int o = off;
#pragma unroll
        for (int e = 0; e < kMemGPT; e++) {
            s_pref[kMemGPT * t + e] = o;
            o += cnt2[e];
        }
    }
    if (t == 0) {
        s_pref[GB] = total;
        s_nsurv = 0;
    }
    __syncthreads();
    RecPod rec = rec_empty();
    for (int base = 0; base < total; base += CAP) {
        int end = min(total, base + CAP);
        // each thread marks the pass's slots of its groups with the group,
        // so that a member slot finds its group in one read (the previous
        // pass read s_owner before its last barrier)
#pragma unroll
        for (int e = 0, lo = off; e < kMemGPT; lo += cnt2[e], e++) {
            const int i0 = max(lo, base), i1 = min(lo + cnt2[e], end);
            for (int i = i0; i < i1; i++)
                s_owner[i - base] = (uint16_t)(kMemGPT * t + e);
        }
        __syncthreads();
        // locate this thread's (up to 16) members and load their angles first
        // (locations and slots fit 32 bits: image sides are at most 32767,
        // so the tables hold fewer than 2^31 entries); the locations are
        // found again from the owner map when the angles are tested, so that
        // only the angles stay in registers meanwhile
        auto centre = [&](int u, int &cy, int &cx) {
            const int oy = s_geo[u][0] >> 16, ox = s_geo[u][0] & 0xffff;
            cy = oy + (min(a.h, a.Ly - oy) - 1) / 2;
            cx = ox + (min(a.w, a.Lx - ox) - 1) / 2;
        };
        auto member = [&](int idx, int &u, int &o, int &sl) {
            u = s_owner[idx - base];
            const int k = idx - s_pref[u];
            const int oy = s_geo[u][0] >> 16, ox = s_geo[u][0] & 0xffff;
            const int ww = min(a.w, a.Lx - ox);
            int cy, cx;
            centre(u, cy, cx);
            const int my = k / ww, mx = k - my * ww;
            const int y = oy + my, x = ox + mx;
            sl = (g0 + u) * hw + my * a.w + mx;
            o = ((!a.opta && y == cy && x == cx) || in_window(y, x, wy, wx, a.radius)) ? -1 : y * a.Lx + x;
        };
        float B8[CAP / 256], C8[CAP / 256];
        uint32_t live = 0;
#pragma unroll
        for (int q = 0; q < CAP / 256; q++) {
            const int idx = base + t + 256 * q;
            B8[q] = C8[q] = 0.0f;
            if (idx >= end)
                continue;
            int u, o, sl;
            member(idx, u, o, sl);
            if (o < 0)
                continue;
            live |= 1u << q;
            B8[q] = a.theta_b[(uint32_t)sl];
            C8[q] = a.opta ? a.theta_c[(uint32_t)sl] : 0.0f;
        }
        // binary32 decisions; members inside the guard band are decided after
        // the loop by the canonical test, one at a time (they are rare; one
        // copy of that code keeps the loop small)
        uint32_t keepm = 0, band = 0;
#pragma unroll
        for (int q = 0; q < CAP / 256; q++) {
            if (!((live >> q) & 1))
                continue;
            int u, o32, sl32;
            member(base + t + 256 * q, u, o32, sl32);
            const float A = __int_as_float(s_geo[u][1]);
            const float e = fabsf(A - B8[q]) - C8[q];
            if (e > hi)
                continue;  // eliminated
            if (e < lo)
                keepm |= 1u << q;
            else
                band |= 1u << q;  // inside the guard band, or undefined (a flat block's angle)
        }
        while (band) {
            const int q = __ffs(band) - 1;
            band &= band - 1;
            int u, o32, sl32;
            member(base + t + 256 * q, u, o32, sl32);
            int cy, cx;
            centre(u, cy, cx);
            if (keep_canonical(a, o32, sl32, (int64_t)cy * a.Lx + cx, g0 + u, mn, st, dt, thr64))
                keepm |= 1u << q;
        }
#pragma unroll
        for (int q = 0; q < CAP / 256; q++) {
            const bool keep = (keepm >> q) & 1;
            int o32 = 0;
            if ((live >> q) & 1) {
                if (keep) {
                    int u, sl32;
                    member(base + t + 256 * q, u, o32, sl32);
                    n_surv++;
                } else {
                    n_elim++;
                }
                if (a.dec) {
                    int u, sl32;
                    member(base + t + 256 * q, u, o32, sl32);
                    a.dec[o32] = keep ? 2 : 0;
                }
            }
            // the wave's survivors take consecutive list slots: one LDS atomic
            // per wave, each lane's slot from the ballot
            const uint64_t km = __ballot(keep);
            if (km) {
                int wbase = 0;
                if (lane == 0)
                    wbase = atomicAdd(&s_nsurv, (int)__popcll(km));
                wbase = __shfl(wbase, 0);
                if (keep)
                    s_list[wbase + (int)__popcll(km & ((1ull << lane) - 1))] = o32;
            }
        }
        __syncthreads();
        // survivors collect over passes and are binned when the next pass
        // might not fit the list, and after the last pass
        const int ns = s_nsurv;
        const bool last = base + CAP >= total;
        if (last || ns + CAP > kSurvList) {
            if (ns > 0)
                bin_survivors(a, s_list, ns, tile_lo, ntl, s_tc, s_tb);
            if (!last) {
                __syncthreads();
                if (t == 0)
                    s_nsurv = 0;
                __syncthreads();
            }
        }
    }
    // the counts ride in the wave records (merging sums them): one barrier
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_elim += __shfl_xor(n_elim, off);
        n_surv += __shfl_xor(n_surv, off);
    }
    if (lane == 0) {
        rec.n_elim = n_elim;
        rec.n_surv = n_surv;
        wrec[wv] = rec;
    }
    __syncthreads();
    if (wv == 0) {  // the four wave records merged by shuffles in lanes 0..3
        RecPod b = wave_rec<4>(lane < 4 ? wrec[lane] : rec_empty());
        if (lane == 0)
            a.recs[a.rec_off + blockIdx.x] = b;
    }
}

// Copies a row-major per-location table into the group-major layout of
// group size (h, w): slot g*h*w + my*w + mx.
__global__ __launch_bounds__(256) void k_regroup(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int Ly,
                                                 int Lx, int h, int w)
{
    int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= (int64_t)Ly * Lx)
        return;
    int y = (int)(o / Lx), x = (int)(o - (o / Lx) * Lx);
    int gy = y / h, gx = x / w;
    int Gx = (Lx + w - 1) / w;
    int64_t sl = ((int64_t)gy * Gx + gx) * (h * w) + (y - gy * h) * w + (x - gx * w);
    out[sl] = in[o];
}

// ============================================================== Alg. 1: auto-correlation with the centre

// One wave per location: sum(r_c' r_o') over the m x n blocks of the
// location and its group centre, then per mode: exact integers out (debug),
// retained count (EGS, Eq. 15), or angle and exact sum (scan-2 tables).
// The per-location step of Alg. 1 once X = sum r_c' r_o' is known: exact
// integers out (debug), the angle and exact sum in the group-major tables
// (build), or the retained count of Eq. 15 (count; with the blur angle C
// added in the OptA form).  Returns the location's contribution to the count.
__device__ unsigned ac_finish(const AcArgs &a, int64_t o, int64_t c, int X)
{
    const int64_t mn = (int64_t)a.m * a.n;
    const int2 sc = a.statJ[c], so = a.statJ[o];
    const int64_t dc = var_num(mn, sc), dov = var_num(mn, so);
    const int64_t num = mn * (int64_t)X - (int64_t)sc.x * (int64_t)so.x;
    if (a.mode == AC_DEBUG) {
        a.num_out[o] = num;
        a.dc_out[o] = dc;
        a.do_out[o] = dov;
        return 0;
    }
    if (a.mode == AC_BUILD) {
        const int y = (int)o / a.Lx, x = (int)o - y * a.Lx;
        const int gy = y / a.h, gx = x / a.w;
        const int64_t sl = ((int64_t)gy * ((a.Lx + a.w - 1) / a.w) + gx) * (a.h * a.w) + (y - gy * a.h) * a.w +
                           (x - gx * a.w);
        a.theta_b[sl] = theta32(num, dc, dov);
        a.x_b[sl] = X;
        return 0;
    }
    if (a.mode == AC_COUNT31 || a.mode == AC_COUNT31_BLUR) {
        // Prop. 3.1: retained unless the bound through the centre, at the
        // assumed template-to-centre angle, is at most rho_th (binary64
        // throughout; preparation only)
        double rc = 1.0, sc2 = 0.0, ub;
        if (a.mode == AC_COUNT31) {
            if (c == o)
                return 0;
            if (dc == 0 || dov == 0)
                return 1;
        } else {
            const int2 si = a.statI[o];
            const int64_t di = var_num(mn, si);
            if (dc == 0 || dov == 0 || di == 0)
                return 1;
            const int64_t noo = mn * (int64_t)a.x_c[o] - (int64_t)so.x * (int64_t)si.x;
            rc = rho64(noo, dov, di);
            sc2 = sin64(noo, dov, di);
        }
        const double rb = rho64(num, dc, dov), sb = sin64(num, dc, dov);
        return !ub_general(a.ra, a.sa, rb, sb, rc, sc2, &ub) || ub > a.rho_th;
    }
    if (a.mode == AC_COUNT) {
        if (c == o)
            return 0;
        if (dc == 0 || dov == 0)
            return 1;
        const float r = rho32(num, dc, dov);
        if (r < a.thr_lo)
            return 1;
        if (r > a.thr_hi)
            return 0;
        return rho64(num, dc, dov) < a.thr;
    }
    // AC_COUNT_BLUR: every location, angle to the original added
    const int2 si = a.statI[o];
    const int64_t di = var_num(mn, si);
    if (dc == 0 || dov == 0 || di == 0)
        return 1;
    const float s = theta32(num, dc, dov) + a.theta_c[o];
    if (s > a.alo_hi && s < a.ahi_lo)
        return 1;
    if (s < a.alo_lo || s > a.ahi_hi)
        return 0;
    const int64_t noo = mn * (int64_t)a.x_c[o] - (int64_t)so.x * (int64_t)si.x;
    const double rb = rho64(num, dc, dov), sb = sin64(num, dc, dov);
    const double rc = rho64(noo, dov, di), sc2 = sin64(noo, dov, di);
    return (rb * rc - sb * sc2) < a.thr;
}

// Alg. 1 by direct dot products: one wave per location.
__global__ __launch_bounds__(256) void k_autocorr(AcArgs a)
{
    __shared__ unsigned long long ured[8];
    int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t L = (int64_t)a.Ly * a.Lx;
    unsigned long long cnt = 0;
    for (int k = 0; k < 16; k++) {
        int64_t o = (int64_t)blockIdx.x * 64 + wv * 16 + k;
        if (o >= L)
            break;
        int y = (int)o / a.Lx, x = (int)o - y * a.Lx;
        int64_t c = centre_of(y, x, a.Ly, a.Lx, a.h, a.w);
        int cy = (int)c / a.Lx, cx = (int)c - cy * a.Lx;
        int X;
        if (c == o)
            X = a.statJ[c].y;  // sum of squares of the centre block
        else
            X = wave_dot_img(a.J, a.pJ, cy, cx, a.J, a.pJ, y, x, a.m, a.n, lane);
        if (lane == 0)
            cnt += ac_finish(a, o, c, X);
    }
    if (a.mode == AC_COUNT || a.mode == AC_COUNT_BLUR || a.mode == AC_COUNT31 || a.mode == AC_COUNT31_BLUR) {
        unsigned long long s = block_sum_u64(cnt, ured);
        if (t == 0 && s)
            atomicAdd(a.counter, s);
    }
}

// Alg. 1 by running sums: for one offset (dy, dx) of a member from its group
// centre, X = the box sum at the centre of the product image
// r'(y, x) r'(y + dy, x + dx), read from its running sums (psat, row width
// q + 1).  One thread per group; the centre itself ((0, 0)) takes its sum of
// squares from the statistics.
__global__ __launch_bounds__(256) void k_ac_shift(AcArgs a, int dy, int dx, const uint32_t *__restrict__ psat, int q)
{
    __shared__ unsigned long long ured[8];
    const int g = blockIdx.x * 256 + threadIdx.x;
    const int Gx = (a.Lx + a.w - 1) / a.w, G = ((a.Ly + a.h - 1) / a.h) * Gx;
    unsigned long long cnt = 0;
    if (g < G) {
        int oy, ox, hh, ww, cy, cx;
        group_geom(g, Gx, a.Ly, a.Lx, a.h, a.w, oy, ox, hh, ww, cy, cx);
        const int y = cy + dy, x = cx + dx;
        if (y >= oy && y < oy + hh && x >= ox && x < ox + ww) {
            const int64_t c = (int64_t)cy * a.Lx + cx, o = (int64_t)y * a.Lx + x;
            int X;
            if (dy == 0 && dx == 0) {
                X = a.statJ[c].y;
            } else {
                const int64_t W = q + 1;
                const uint32_t *s0 = psat + (int64_t)cy * W + cx, *s1 = s0 + (int64_t)a.m * W;
                X = (int)(s1[a.n] - s1[0] - s0[a.n] + s0[0]);
            }
            cnt = ac_finish(a, o, c, X);
        }
    }
    if (a.mode == AC_COUNT || a.mode == AC_COUNT_BLUR || a.mode == AC_COUNT31 || a.mode == AC_COUNT31_BLUR) {
        unsigned long long s = block_sum_u64(cnt, ured);
        if (threadIdx.x == 0 && s)
            atomicAdd(a.counter, s);
    }
}

// Per-group range of member angles B (and largest C) for scan 2's group test.
__global__ __launch_bounds__(256) void k_gsum(GsumArgs a)
{
    int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= a.Gy * a.Gx)
        return;
    int oy, ox, hh, ww, cy, cx;
    group_geom(g, a.Gx, a.Ly, a.Lx, a.h, a.w, oy, ox, hh, ww, cy, cx);
    float bmin = __int_as_float(0x7f800000), bmax = -bmin, cmax = 0.0f;
    int flags = 0;
    for (int y = oy; y < oy + hh; y++)
        for (int x = ox; x < ox + ww; x++) {
            if (!a.opta && y == cy && x == cx)
                continue;
            int64_t sl = (int64_t)g * (a.h * a.w) + (y - oy) * a.w + (x - ox);
            float B = a.theta_b[sl];
            float C = a.opta ? a.theta_c[sl] : 0.0f;
            if (isnan(B) || isnan(C)) {
                flags |= 1;
                continue;
            }
            bmin = fminf(bmin, B);
            bmax = fmaxf(bmax, B);
            cmax = fmaxf(cmax, C);
        }
    GroupSum s;
    s.bmin = bmin;
    s.bmax = bmax;
    s.cmax = cmax;
    s.flags = flags;
    a.gsum[g] = s;
}

// ============================================================== blur (Eq. 18)

__global__ __launch_bounds__(256) void k_blur_h(const uint8_t *__restrict__ src, int64_t pitch, int p, int q, Taps tp,
                                                uint32_t *__restrict__ tmp)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)p * q)
        return;
    int y = (int)(i / q), x = (int)(i - (i / q) * q);
    const uint8_t *row = src + (int64_t)y * pitch;
    uint32_t v = 0;
    for (int j = -tp.d; j <= tp.d; j++) {
        int xx = min(max(x + j, 0), q - 1);
        v += (uint32_t)tp.w[j + tp.d] * row[xx];
    }
    tmp[i] = v;
}

__global__ __launch_bounds__(256) void k_blur_v(const uint32_t *__restrict__ tmp, int p, int q, Taps tp,
                                                uint32_t T, uint8_t *__restrict__ dst, int64_t pitch)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)p * q)
        return;
    int y = (int)(i / q), x = (int)(i - (i / q) * q);
    uint32_t v = 0;
    for (int j = -tp.d; j <= tp.d; j++) {
        int yy = min(max(y + j, 0), p - 1);
        v += (uint32_t)tp.w[j + tp.d] * tmp[(int64_t)yy * q + x];
    }
    dst[(int64_t)y * pitch + x] = (uint8_t)((v + T / 2) / T);
}

// ============================================================== blur correlation and revert (Alg. 3)

// One wave per location: the m x n block of J against the same block of I.
// Blur correlation of every block of J with the same block of I (Eq. 28's
// rho between a conditioned block and its original), one thread per
// location: the exact cross sum comes from the running sums of J' I' (four
// entries, modulo 2^32), the block statistics from the two images' tables.
__global__ __launch_bounds__(256) void k_blurcorr(BcArgs a)
{
    __shared__ unsigned long long ured[8];
    const int64_t L = (int64_t)a.Ly * a.Lx;
    const int64_t mn = (int64_t)a.m * a.n;
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long cnt = 0;
    if (o < L) {
        const int y = (int)o / a.Lx, x = (int)o - y * a.Lx;
        const int64_t W = a.q + 1;
        const uint32_t *s0 = a.psat + (int64_t)y * W + x, *s1 = s0 + (int64_t)a.m * W;
        const int X = (int)(s1[a.n] - s1[0] - s0[a.n] + s0[0]);
        const int2 sj = a.statJ[o], si = a.statI[o];
        const int64_t dj = var_num(mn, sj), di = var_num(mn, si);
        const int64_t num = mn * (int64_t)X - (int64_t)sj.x * (int64_t)si.x;
        if (a.mode == BC_VIOL) {
            bool v;
            if (dj == 0 || di == 0)
                v = true;
            else {
                float r = rho32(num, dj, di);
                if (r < a.lam_lo)
                    v = true;
                else if (r > a.lam_hi)
                    v = false;
                else
                    v = rho64(num, dj, di) < a.lambda;
            }
            a.viol[o] = v ? 1 : 0;
            cnt = v;
        } else if (a.mode == BC_BUILD) {
            a.theta_c[o] = theta32(num, dj, di);
            a.x_c[o] = X;
        } else {
            a.num_out[o] = num;
            a.dj_out[o] = dj;
            a.di_out[o] = di;
        }
    }
    if (a.mode == BC_VIOL) {
        unsigned long long s = block_sum_u64(cnt, ured);
        if (threadIdx.x == 0 && s)
            atomicAdd(a.counter, s);
    }
}

// colmask(y, lx) = 1 when a violating location in column lx covers pixel row y.
__global__ __launch_bounds__(256) void k_dilate_rows(const uint8_t *__restrict__ viol, int p, int Ly, int Lx, int m,
                                                     uint8_t *__restrict__ colmask)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)p * Lx)
        return;
    int y = (int)(i / Lx), lx = (int)(i - (i / Lx) * Lx);
    int lo = max(0, y - m + 1), hi = min(Ly - 1, y);
    uint8_t v = 0;
    for (int ly = lo; ly <= hi && !v; ly++)
        v = viol[(int64_t)ly * Lx + lx];
    colmask[i] = v;
}

// Copies I into J at every pixel covered by a violating block; counts the
// pixels that changed.
__global__ __launch_bounds__(256) void k_revert(const uint8_t *__restrict__ colmask, int p, int q, int Lx, int n,
                                                const uint8_t *__restrict__ I, uint8_t *__restrict__ J,
                                                int64_t pitch, unsigned long long *counter)
{
    __shared__ unsigned long long ured[8];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long changed = 0;
    if (i < (int64_t)p * q) {
        int y = (int)(i / q), x = (int)(i - (i / q) * q);
        int lo = max(0, x - n + 1), hi = min(Lx - 1, x);
        uint8_t v = 0;
        for (int lx = lo; lx <= hi && !v; lx++)
            v = colmask[(int64_t)y * Lx + lx];
        if (v) {
            int64_t a = (int64_t)y * pitch + x;
            uint8_t iv = I[a];
            if (J[a] != iv) {
                J[a] = iv;
                changed = 1;
            }
        }
    }
    unsigned long long s = block_sum_u64(changed, ured);
    if (threadIdx.x == 0 && s)
        atomicAdd(counter, s);
}

// ============================================================== batched templates on int8 MFMA


// Template statistics of a batch: one block per template (layout [T][m][n16],
// columns past n hold 0x80, i.e. int8 zero): tst[2t] = sum(t'), tst[2t+1] = D_t.
// Job of a flattened block index: the last job whose first index (block0,
// fold0 or tmpl0 by F) is <= idx.  The scan is uniform across the block.
template <int F> __device__ __forceinline__ int batch_job_of(const BatchJob *jobs, int njobs, int idx)
{
    int j = 0;
    while (j + 1 < njobs && (F == 0 ? jobs[j + 1].block0 : F == 1 ? jobs[j + 1].fold0 : jobs[j + 1].tmpl0) <= idx)
        j++;
    return j;
}

// Template statistics of a batch: one block per template (layout [T][m][n16],
// columns past n hold 0x80, i.e. int8 zero): tst[2t] = sum(t'), tst[2t+1] = D_t.
__global__ __launch_bounds__(256) void k_tstats(const BatchJob *__restrict__ jobs, int njobs)
{
    __shared__ int red[8];
    const BatchJob &a = jobs[batch_job_of<2>(jobs, njobs, blockIdx.x)];
    const int tt = blockIdx.x - a.tmpl0, m = a.m, n16 = a.n16;
    // m * n16 is a multiple of 16 and each template starts 16-byte aligned
    const uint4 *tp = (const uint4 *)(a.tpl + (int64_t)tt * m * n16);
    const uint32_t ones = 0x01010101u;
    int s = 0, s2 = 0;
    for (int idx = threadIdx.x; idx < (m * n16) >> 4; idx += 256) {
        uint4 v = tp[idx];
        uint32_t w[4] = {flip4(v.x), flip4(v.y), flip4(v.z), flip4(v.w)};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            s = dot4(w[k], ones, s);
            s2 = dot4(w[k], w[k], s2);
        }
    }
    int64_t S = block_sum_int(s, red), Q = block_sum_int(s2, red);
    if (threadIdx.x == 0) {
        a.tst[2 * tt] = S;
        a.tst[2 * tt + 1] = (int64_t)m * a.n * Q - S * S;
    }
}

// Cross-correlation of up to 16 templates of one size at every location as
// an implicit GEMM on v_mfma_i32_16x16x64_i8: M = 16 locations of one row,
// N = 16 templates, K = 64 = 4 consecutive image rows x 16 columns.  A wave
// keeps R output rows x 4 M-tiles (64 columns) of int32 accumulators; each
// realigned A fragment (image rows yy..yy+3) feeds the R output rows, each
// with the template rows that line up with it.  Per 4-row step the block
// stages the 4 image rows and the R+3 template rows they meet in LDS.  The
// epilogue forms N, rho32 and a per-template band-argmax record per block.
// Epilogue LDS (dwords): S' and 1/sqrt(D_r) per location of the block (R x
// 256 each), 64 block maxima, the candidate counter, then the candidate list
// (4 dwords each) and its binary64 results (6 dwords each).
constexpr int kBatchRows = 8;
constexpr int kBatchCandCap = 512;
constexpr int kBatchEpiList = 2 * kBatchRows * 256 + 68;
constexpr int kBatchEpiWords = kBatchEpiList + 4 * kBatchCandCap + 6 * kBatchCandCap;
static_assert(kBatchEpiList % 4 == 0, "candidate list is 16-byte aligned");


template <int R>
__global__ __launch_bounds__(256, 2) void k_batch(const BatchJob *__restrict__ jobs, int njobs)
{
    static_assert(R + 3 + 4 <= 16, "template ring holds 16 rows");
    static_assert(R == kBatchRows, "epilogue LDS layout is sized for kBatchRows");
    extern __shared__ __align__(16) uint32_t smem[];
    const BatchJob a = jobs[batch_job_of<0>(jobs, njobs, blockIdx.x)];
    const int lb = blockIdx.x - a.block0, bx = lb % a.gx, by = (lb / a.gx) % a.gy, bz = lb / (a.gx * a.gy);
    constexpr int TNEW = (4 * 16 * 32 + 255) / 256;  // new template words per thread and step, n16 <= 128
    const int n16 = a.n16, nb16 = n16 >> 4, nw16 = n16 >> 2;
    const int WW = (256 + n16 + 16) >> 2;  // dwords per staged image row
    const int CS = batch_copy_stride(WW);  // dwords per (row, byte shift) copy
    const int IMGW = 16 * CS;              // [4 rows][4 byte shifts][CS]
    const int tstr = batch_tstride(nw16);
    uint32_t *ring = smem + 2 * IMGW;      // 16 template rows x 16 templates x tstr; row ti in slot (ti + R - 1) & 15
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int x0 = bx * 256, y0 = by * R, tz = bz * 16;
    const int steps = (R + a.m - 1 + 3) >> 2;
    const uint32_t *tplg = (const uint32_t *)a.tpl;
    const int rowwords = 16 * nw16;      // words of one template row across the 16 templates (global)

    v4i acc[R][4];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
            acc[r][mt] = v4i{0, 0, 0, 0};

    // this thread's share of the 4 new template rows of a step: (row q, template tt, word c4)
    int tq[TNEW], toff[TNEW], tdst[TNEW];
#pragma unroll
    for (int k = 0; k < TNEW; k++) {
        int idx = t + 256 * k;
        tq[k] = -1;
        toff[k] = 0;
        tdst[k] = 0;
        if (idx < 4 * rowwords) {
            int q = idx / rowwords, rem = idx - q * rowwords;
            int tt = rem / nw16, c4 = rem - tt * nw16;
            tdst[k] = tt * tstr + c4;
            if (tz + tt < a.T) {
                tq[k] = q;
                toff[k] = (tz + tt) * a.m * nw16 + c4;
            }
        }
    }
    uint32_t ri[2][2];
    uint32_t rt[TNEW];
    auto gload = [&](int s) {
#pragma unroll
        for (int k = 0; k < 2; k++) {
            int idx = t + 256 * k;
            ri[k][0] = ri[k][1] = 0x80808080u;
            if (idx < 4 * WW) {
                int g = idx / WW, w = idx - g * WW;
                int gy = y0 + 4 * s + g;
                int64_t gx = (int64_t)x0 + 4 * w;
                if (gy < a.p) {
                    const uint8_t *rp = a.img + (int64_t)gy * a.pitch;
                    if (gx + 4 <= a.pitch)
                        ri[k][0] = *gptr((const uint32_t *)(rp + gx));
                    if (gx + 8 <= a.pitch)
                        ri[k][1] = *gptr((const uint32_t *)(rp + gx + 4));
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TNEW; k++) {
            rt[k] = 0;
            int ti = 4 * s + tq[k];
            if (tq[k] >= 0 && ti < a.m)
                rt[k] = flip4(gptr(tplg)[toff[k] + (int64_t)ti * nw16]);
        }
    };
    // image buffer of step s at smem + (s & 1) * IMGW (offsets, not a pointer
    // table, so the accesses stay LDS instructions)
    auto lstore = [&](int s) {
        uint32_t *b = smem + (s & 1) * IMGW;
#pragma unroll
        for (int k = 0; k < 2; k++) {
            int idx = t + 256 * k;
            if (idx < 4 * WW) {
                int g = idx / WW, w = idx - g * WW;
                uint32_t lo = flip4(ri[k][0]), hi = flip4(ri[k][1]);
                b[(g * 4 + 0) * CS + w] = lo;
                b[(g * 4 + 1) * CS + w] = bytes_at(hi, lo, 1);
                b[(g * 4 + 2) * CS + w] = bytes_at(hi, lo, 2);
                b[(g * 4 + 3) * CS + w] = bytes_at(hi, lo, 3);
            }
        }
#pragma unroll
        for (int k = 0; k < TNEW; k++) {
            int idx = t + 256 * k;
            if (idx < 4 * rowwords) {
                int q = idx / rowwords;
                int slot = (4 * s + q + R - 1) & 15;
                ring[slot * 16 * tstr + tdst[k]] = rt[k];
            }
        }
    };

    // template rows before row 0 read as zero
    for (int idx = t; idx < 16 * 16 * tstr; idx += 256)
        ring[idx] = 0;
    __syncthreads();
    gload(0);
    lstore(0);
    __syncthreads();
    const int g = lane >> 4, mrow = lane & 15;
    for (int s = 0; s < steps; s++) {
        const uint32_t *cur = smem + (s & 1) * IMGW;
        if (s + 1 < steps)
            gload(s + 1);
        const int slot0 = 4 * s + g + R - 1;  // slot of template row 4s + g - r is (slot0 - r) & 15
        for (int cb = 0; cb < nb16; cb++) {
            v4i A[4];
#pragma unroll
            for (int mt = 0; mt < 4; mt++) {
                // 16 image bytes at column c: copy (c & 3) holds them 4-byte aligned
                int c = 64 * wv + 16 * mt + mrow + 16 * cb;
                __builtin_memcpy(&A[mt], cur + (g * 4 + (c & 3)) * CS + (c >> 2), 16);
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                int slot = (slot0 - r) & 15;
                v4i B = *(const v4i *)((const uint8_t *)(ring + (slot * 16 + mrow) * tstr) + 16 * cb);
#pragma unroll
                for (int mt = 0; mt < 4; mt++)
                    acc[r][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], B, acc[r][mt], 0, 0, 0);
            }
        }
        if (s + 1 < steps)
            lstore(s + 1);
        __syncthreads();
    }

    // Epilogue.  Lane holds template tz + (lane & 15) at rows y0 + r and
    // columns x0 + 64 wv + 16 mt + 4 (lane >> 4) + v.
    //  pass 0: per location of the block, S' and 1 / sqrt(D_r) into LDS
    //          (NaN marks a location past the map, 0 a flat block);
    //  pass 1: est = N / sqrt(D_t D_r) in binary32 from the exact N (binary64
    //          fma of exact products, |N| < 2^44); block maximum per template;
    //  pass 2: pairs with est >= max - kEpsRho go to an LDS candidate list;
    //  then the candidates' canonical binary64 rho picks each template's best.
    // est is within 5e-7 of rho, so the exact best of the block is always a
    // candidate.  A list overflow (many near-equal values, e.g. flat images)
    // falls back to the streaming band selection over every pair.
    const int64_t mn = (int64_t)a.m * a.n;
    const int tn = tz + (lane & 15);
    int64_t St = 0, Dt = 0;
    if (tn < a.T) {
        St = gptr(a.tst)[2 * tn];
        Dt = gptr(a.tst)[2 * tn + 1];
    }
    const float qnan = __int_as_float(0x7fc00000);
    int *sxs = (int *)smem;                              // [R][256]
    float *irss = (float *)(smem + R * 256);             // [R][256]
    float *bmx = (float *)(smem + 2 * R * 256);          // [4 waves][16 templates]
    int *ccnt = (int *)(smem + 2 * R * 256 + 64);
    int4 *clist = (int4 *)(smem + kBatchEpiList);        // (template, location in block, acc, 0)
    {
        // every load unconditional (clamped to the map) so all R are in flight together
        int2 stv[R];
        const int xc = min(x0 + t, a.Lx - 1);
#pragma unroll
        for (int r = 0; r < R; r++)
            stv[r] = ld_int2(a.stat + ((int64_t)min(y0 + r, a.Ly - 1) * a.Lx + xc));
#pragma unroll
        for (int r = 0; r < R; r++) {
            bool in = y0 + r < a.Ly && x0 + t < a.Lx;
            int64_t dr = var_num(mn, stv[r]);
            sxs[r * 256 + t] = in ? stv[r].x : 0;
            irss[r * 256 + t] = !in ? qnan : dr > 0 ? 1.0f / sqrtf((float)dr) : 0.0f;
        }
    }
    if (t == 0)
        *ccnt = 0;
    __syncthreads();
    const bool tok = tn < a.T && Dt != 0;
    const double nst = -(double)St, mnd = (double)mn;
    const float irt = tok ? 1.0f / sqrtf((float)Dt) : qnan;
    auto est_of = [&](int accv, int sx, float ir) -> float {
        double nd = fma(mnd, (double)accv, nst * (double)sx);
        return (float)nd * ir * irt;
    };
    const int g4 = lane >> 4;
    float bm = -INFINITY;
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            int li = r * 256 + 64 * wv + 16 * mt + 4 * g4;
            int4 sx4 = *(const int4 *)(sxs + li);
            float4 ir4 = *(const float4 *)(irss + li);
            bm = fmaxf(bm, est_of(acc[r][mt][0], sx4.x, ir4.x));
            bm = fmaxf(bm, est_of(acc[r][mt][1], sx4.y, ir4.y));
            bm = fmaxf(bm, est_of(acc[r][mt][2], sx4.z, ir4.z));
            bm = fmaxf(bm, est_of(acc[r][mt][3], sx4.w, ir4.w));
        }
    bm = fmaxf(bm, __shfl_xor(bm, 16));
    bm = fmaxf(bm, __shfl_xor(bm, 32));
    if (lane < 16)
        bmx[wv * 16 + lane] = bm;
    __syncthreads();
    const int tl = lane & 15;
    const float thr = fmaxf(fmaxf(bmx[tl], bmx[16 + tl]), fmaxf(bmx[32 + tl], bmx[48 + tl])) - kEpsRho;
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            int li = r * 256 + 64 * wv + 16 * mt + 4 * g4;
            int4 sx4 = *(const int4 *)(sxs + li);
            float4 ir4 = *(const float4 *)(irss + li);
            int sxv[4] = {sx4.x, sx4.y, sx4.z, sx4.w};
            float irv[4] = {ir4.x, ir4.y, ir4.z, ir4.w};
#pragma unroll
            for (int v = 0; v < 4; v++)
                if (est_of(acc[r][mt][v], sxv[v], irv[v]) >= thr) {
                    int k = atomicAdd(ccnt, 1);
                    if (k < kBatchCandCap)
                        clist[k] = make_int4(tl, li + v, acc[r][mt][v], 0);
                }
        }
    __syncthreads();
    const int ncand = *ccnt;
    const int bid = lb;  // record index of this block within its job
    if (ncand <= kBatchCandCap) {
        double *crho = (double *)(smem + kBatchEpiList + 4 * kBatchCandCap);
        int64_t *cnum = (int64_t *)(crho + kBatchCandCap);
        int64_t *cdr = cnum + kBatchCandCap;
        for (int e = t; e < ncand; e += 256) {
            int4 c = clist[e];
            int tg = tz + c.x;
            int64_t l = (int64_t)(y0 + (c.y >> 8)) * a.Lx + x0 + (c.y & 255);
            int2 st = ld_int2(a.stat + (l));
            int64_t dr = var_num(mn, st);
            int64_t num = mn * (int64_t)c.z - gptr(a.tst)[2 * tg] * (int64_t)st.x;
            crho[e] = rho64(num, gptr(a.tst)[2 * tg + 1], dr);
            cnum[e] = num;
            cdr[e] = dr;
        }
        __syncthreads();
        if (t < 16) {
            RecPod b = rec_empty();
            for (int e = 0; e < ncand; e++) {
                int4 c = clist[e];
                if (c.x != t)
                    continue;
                int64_t l = (int64_t)(y0 + (c.y >> 8)) * a.Lx + x0 + (c.y & 255);
                if (!b.valid || rec_better(crho[e], l, b.rho, b.l)) {
                    b.rho = crho[e];
                    b.l = l;
                    b.num = cnum[e];
                    b.dr = cdr[e];
                    b.valid = 1;
                }
            }
            st_rec(a.recs + (int64_t)bid * 16 + t, b);
        }
        return;
    }

    // overflow: streaming band selection over every pair, one output row at a
    // time through this wave's LDS slice
    RecPod rec = rec_empty();
    int *slice = (int *)smem + wv * 16 * 64;  // 16 values x 64 lanes per wave
#pragma unroll
    for (int r = 0; r < R; r++) {
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int v = 0; v < 4; v++)
                slice[(mt * 4 + v) * 64 + lane] = acc[r][mt][v];
        int y = y0 + r;
#pragma unroll 1
        for (int e = 0; e < 16; e++) {
            int mt = e >> 2, v = e & 3;
            int x = x0 + 64 * wv + 16 * mt + 4 * g4 + v;
            if (tok && y < a.Ly && x < a.Lx) {
                int64_t l = (int64_t)y * a.Lx + x;
                int2 stl = ld_int2(a.stat + (l));
                int64_t dr = var_num(mn, stl);
                int64_t num = mn * (int64_t)slice[e * 64 + lane] - St * (int64_t)stl.x;
                rec_offer(rec, rho32(num, Dt, dr), l, num, Dt, dr);
            }
        }
    }
    __syncthreads();
    RecPod *wr = (RecPod *)smem;
    wr[t] = rec;
    __syncthreads();
    if (t < 16) {
        RecPod b = rec_empty();
        for (int w = 0; w < 4; w++)
            for (int gg = 0; gg < 4; gg++)
                rec_merge(b, wr[w * 64 + gg * 16 + t]);
        st_rec(a.recs + (int64_t)bid * 16 + t, b);
    }
}

// Cross-correlation of ONE template at every location as an implicit GEMM on
// v_mfma_i32_16x16x64_i8 with M = 16 locations of a row, N = 16 consecutive
// output rows and K = 4 image rows x 16 columns.  For image rows 4s..4s+3
// and output row y0 + 16 rg + j, lane (j, g) of the B fragment carries
// template row 4s + g - 16 rg - j (a Toeplitz arrangement; rows outside the
// template read zero rows), so one A fragment feeds every row group.  The
// template is staged whole in LDS once with zero rows around it; the image
// streams through LDS in 4-row steps (four byte-shifted copies of each row,
// so every A lane reads whole words).  A wave holds RG row groups x 4
// M-tiles; the block's four waves sit side by side: 16 RG rows x 256
// columns per block.  Every row group takes part in every step (a group that
// meets no template row multiplies zero rows): the MFMA sequence of a step
// is then the same for every step, so the fragment reads of the next column
// block are issued before the MFMAs of the current one and each MFMA waits
// only for its own operands.  With RG = 2 a block needs about 15 to 40 KB of
// LDS and under 128 VGPRs, so four blocks share a CU and hide each other's
// staging and epilogue latency.
constexpr int kSingleCap = 256;   // candidate list entries
// Epilogue LDS (dwords, reusing the image buffers): the candidate list, the
// four wave maxima, the candidate count and the four wave records.
constexpr int kSingleEpiMax = 4 * kSingleCap;
constexpr int kSingleEpiRed = kSingleEpiMax + 8;
constexpr int kSingleLdsWords = kSingleEpiRed + 4 * (int)(sizeof(RecPod) / 4);

// The staged template carries zero rows around it: B lane (j, g) of row group
// rg at step s reads template row d + g - j with d = 4s - 16 rg clamped to
// -4 (before the template) or m + 16 (after it) when the group meets no
// template row, so rows -19 .. m + 19 are read without a per-lane clamp.
constexpr int kSinglePadLo = 19, kSinglePadHi = 20;
__host__ __device__ inline int single_tpl_words(int m, int n16)
{
    // 8 words of slack: the pipelined reads of the column block after the
    // last one stay inside the allocation (their values are never used)
    return (m + kSinglePadLo + kSinglePadHi) * batch_tstride(n16 >> 2) + 8;
}

// Zeroes the pad rows of a staged single template (tpl_l: row -kSinglePadLo).
__device__ __forceinline__ void single_tpl_pads(uint32_t *tpl_l, int m, int nw16, int tstr)
{
    for (int idx = threadIdx.x; idx < (kSinglePadLo + kSinglePadHi) * nw16; idx += blockDim.x) {
        const int r = idx / nw16, c = idx - r * nw16;
        tpl_l[(r < kSinglePadLo ? r : r + m) * tstr + c] = 0;
    }
}

// Staged image rows of the single-template body: 256 + n16 + 16 bytes from
// the block's first column, as copies shifted by 0..CP-1 bytes, of
// single_copy_stride dwords each; two buffers of 4 rows.  Templates 48 or 64
// wide take 16 copies (every A lane reads its 16 bytes in one aligned read;
// the copy stride, 4 mod 8 dwords, puts the 64 lanes' rows on distinct
// banks), the others 8 copies (two 8-byte reads at 8-byte boundaries): for
// 16 or 32 columns the extra staging costs more than the aligned reads save
// (measured), and wider templates keep their LDS within three blocks per CU.
__host__ __device__ inline int single_copies(int n16) { return n16 == 48 || n16 == 64 ? 16 : 8; }
__host__ __device__ inline int single_copy_stride(int n16)
{
    const int ww = (256 + n16 + 16) >> 2;
    return single_copies(n16) == 16 ? (ww + 3) / 8 * 8 + 4 : (ww + 1) & ~1;
}
__host__ __device__ inline int single_tpl_offset(int n16) { return 2 * 4 * single_copies(n16) * single_copy_stride(n16); }

// One 16 RG x 256 block of locations of one template (the body of k_single
// and of k_dense_tiles).  The caller has staged the template at
// smem + single_tpl_offset(n16) in the int8 view, row r at (r + kSinglePadLo)
// strides of batch_tstride(n16 / 4) words (n16 / 4 of them), with the pad
// rows zeroed by single_tpl_pads, and checked that D_t > 0.
struct SingleTile {
    const uint8_t *img;
    int64_t pitch;
    int p;
    const int2 *stat;  // per-location statistics of img for (m, n)
    int Ly, Lx, m, n, n16;
    int64_t St, Dt;    // sum(t') and D_t
};

// Returns the block's best location (valid in thread 0; the block's LDS is
// reused; some threads may return before others).
template <int RG, int CP>
__device__ RecPod single_tile_body(const SingleTile &a, int x0, int y0, uint32_t *smem, int t)
{
    static_assert(RG >= 1 && RG <= 4, "row groups per block");
    static_assert(CP == 8 || CP == 16, "byte-shifted copies");
    constexpr int MT = 4, ROWS = 16 * RG;
    const int m = a.m, n16 = a.n16, nb16 = n16 >> 4;
    const int CS = single_copy_stride(n16);
    const int WP = ((256 + n16 + 16) / 4 + 1) >> 1;  // staged dword pairs per row
    const int IMGW = 4 * CP * CS;
    const int tstr = batch_tstride(n16 >> 2);
    const uint32_t *tpl_l = smem + 2 * IMGW;  // row -kSinglePadLo of the padded template
    const int lane = t & 63, wv = t >> 6;
    const int steps = (ROWS + m - 1 + 3) >> 2;

    // Image rows stream through two LDS buffers; their global loads are issued
    // two steps ahead into two register sets.  The loads are unconditional,
    // from addresses clamped into the image (row p - 1, the last 8 bytes of
    // the pitch): a staged byte that is not a pixel only meets locations past
    // the last one, or zero template columns, so its value does not matter;
    // and with no branch around them the compiler can wait for one register
    // set while the other is still in flight.
    // Thread t stages dword pair t of the step (row t / WP, bytes 8p .. 8p + 7
    // of each copy, from the CP / 4 + 2 row words at 8p; 4 WP <= 256).
    constexpr int NW = CP / 4 + 2;
    const int sidx = min(t, 4 * WP - 1), srow = sidx / WP, spair = sidx - srow * WP;
    uint32_t rA[NW], rB[NW];
    auto gload = [&](int s, uint32_t (&ri)[NW]) {
        const int gy = min(y0 + 4 * s + srow, a.p - 1);
        const int64_t gx = min((int64_t)x0 + 8 * spair, a.pitch - 4 * NW);
        const uint32_t *rp = (const uint32_t *)(a.img + (int64_t)gy * a.pitch + gx);
#pragma unroll
        for (int k = 0; k < NW; k++)
            ri[k] = *gptr(rp + k);
    };
    auto lstore = [&](int s, const uint32_t (&ri)[NW]) {
        if (t < 4 * WP) {
            uint32_t *b = smem + (s & 1) * IMGW + srow * CP * CS + 2 * spair;
            uint32_t w[NW];
#pragma unroll
            for (int k = 0; k < NW; k++)
                w[k] = flip4(ri[k]);
#pragma unroll
            for (int c = 0; c < CP; c++) {  // copy c: row bytes shifted by c
                const int q = c >> 2, r = c & 3;
                *(uint2 *)(b + c * CS) = r == 0 ? make_uint2(w[q], w[q + 1])
                                                : make_uint2(bytes_at(w[q + 1], w[q], r), bytes_at(w[q + 2], w[q + 1], r));
            }
        }
    };

    v4i acc[RG][MT];
#pragma unroll
    for (int r = 0; r < RG; r++)
#pragma unroll
        for (int mt = 0; mt < MT; mt++)
            acc[r][mt] = v4i{0, 0, 0, 0};
    gload(0, rA);
    lstore(0, rA);
    __syncthreads();
    gload(1, rB);
    const int g = lane >> 4, jr = lane & 15;
    // A lane (jr, g) reads location column c = 64 wv + 16 mt + jr + 16 cb of
    // image row g: the copy shifted by c mod CP bytes (jr, or jr & 7), from
    // byte c rounded down to CP (one 16-byte read, or two 8-byte reads).  B
    // lane (jr, g) of row group rg reads template row d + g - jr.
    const uint32_t *tpl_b = tpl_l + (g - jr + kSinglePadLo) * tstr;
    const int a_off = CP == 16 ? (g * 16 + jr) * CS + 16 * wv : (g * 8 + (jr & 7)) * CS + 16 * wv + 2 * (jr >> 3);
    auto compute = [&](int s) {
        const uint32_t *pa = smem + (s & 1) * IMGW + a_off;
        const uint32_t *pb[RG];
#pragma unroll
        for (int rg = 0; rg < RG; rg++) {
            const int d = 4 * s - 16 * rg;
            pb[rg] = tpl_b + (d < 0 ? -4 : d > m + 14 ? m + 16 : d) * tstr;
        }
        v4i A0[MT], A1[MT], B0[RG], B1[RG];
        auto frag = [&](v4i (&A)[MT], v4i (&B)[RG], int cb) {
#pragma unroll
            for (int mt = 0; mt < MT; mt++) {
                if constexpr (CP == 16) {
                    A[mt] = *(const v4i *)(pa + 4 * mt + 4 * cb);
                } else {
                    const uint64_t *q = (const uint64_t *)(pa + 4 * mt + 4 * cb);
                    const uint64_t lo = q[0], hi = q[1];
                    A[mt] = v4i{(int)(uint32_t)lo, (int)(uint32_t)(lo >> 32), (int)(uint32_t)hi,
                                (int)(uint32_t)(hi >> 32)};
                }
            }
#pragma unroll
            for (int rg = 0; rg < RG; rg++)
                B[rg] = *(const v4i *)(pb[rg] + 4 * cb);
        };
        auto mma = [&](const v4i (&A)[MT], const v4i (&B)[RG]) {
#pragma unroll
            for (int rg = 0; rg < RG; rg++)
#pragma unroll
                for (int mt = 0; mt < MT; mt++)
                    acc[rg][mt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], B[rg], acc[rg][mt], 0, 0, 0);
        };
        // two column blocks per iteration, the next one's reads issued before
        // the current one's MFMAs
        frag(A0, B0, 0);
        int cb = 0;
        for (; cb + 2 < nb16; cb += 2) {
            frag(A1, B1, cb + 1);
            mma(A0, B0);
            frag(A0, B0, cb + 2);
            mma(A1, B1);
        }
        if (cb + 1 < nb16) {
            frag(A1, B1, cb + 1);
            mma(A0, B0);
            mma(A1, B1);
        } else {
            mma(A0, B0);
        }
    };
    // step s reads buffer s & 1; the data of step s + 1 is in rB (s even) or
    // rA (s odd) and goes to the other buffer, free since the last barrier.
    // Loads past the last step are issued too (clamped rows, never stored),
    // so that every wait counts the same loads in flight.
    for (int s = 0; s < steps; s += 2) {
        gload(s + 2, rA);
        compute(s);
        if (s + 1 < steps)
            lstore(s + 1, rB);
        __syncthreads();
        if (s + 1 >= steps)
            break;
        gload(s + 3, rB);
        compute(s + 1);
        if (s + 2 < steps)
            lstore(s + 2, rA);
        __syncthreads();
    }

    // Epilogue.  Lane holds rows y0 + 16 rg + (lane & 15), columns
    // x0 + 64 wv + 16 mt + 4 (lane >> 4) + v.  est = N / sqrt(D_t D_r) in
    // binary32 from the exact N (as in k_batch), kept in registers; the block
    // maximum; the lanes holding values within kEpsRho of it list them; the
    // listed candidates' canonical binary64 rho gives the block's record.
    const int64_t mn = (int64_t)m * a.n;
    const int64_t St = a.St, Dt = a.Dt;
    int4 *clist = (int4 *)smem;  // (row in block << 16 | column, acc, S, Q)
    float *bmx = (float *)(smem + kSingleEpiMax);
    int *ccnt = (int *)(smem + kSingleEpiMax + 4);
    RecPod *red = (RecPod *)(smem + kSingleEpiRed);
    const double nst = -(double)St, mnd = (double)mn;
    const float irt = 1.0f / sqrtf((float)Dt);
    const float qnan = __int_as_float(0x7fc00000);
    // est from the exact integers: D_r = mn Q - S^2 and N = mn X - S_t S are
    // exact in binary64 (every term below 2^53), each rounded once to
    // binary32; 1/sqrt(D_r) by v_rsq_f32 (about 1 ulp), so est is within
    // 1e-6 of rho, far inside kEpsRho.  D_r = 0 (flat block) gives est = 0.
    auto est_one = [&](int y, int x, int2 st, int accv) -> float {
        const double S = (double)st.x;
        const float drf = (float)fma(mnd, (double)(uint32_t)st.y, -S * S);
        const float ir = drf > 0.0f ? __builtin_amdgcn_rsqf(drf) : 0.0f;
        const double nd = fma(mnd, (double)accv, nst * S);
        return (y < a.Ly && x < a.Lx) ? (float)nd * ir * irt : qnan;
    };
    // statistics: lane (j, g) loads its 16 locations' int2 (rows and columns
    // clamped into the map; the values at clamped positions are not used)
    const int rmax = a.Ly - 1 - y0, cmax = a.Lx - 1 - x0;
    const int2 *sbase = a.stat + ((int64_t)y0 * a.Lx + x0);
    auto stat_of = [&](int r, int c) { return ld_int2(sbase + ((int64_t)min(r, rmax) * a.Lx + min(c, cmax))); };
    if (t == 0)
        *ccnt = 0;
    // (all of the lane's loads are issued at once: one round trip)
    float est[RG][16];
    int2 sv[RG][16];
#pragma unroll
    for (int rg = 0; rg < RG; rg++)
#pragma unroll
        for (int q = 0; q < 16; q++)
            sv[rg][q] = stat_of(16 * rg + jr, 64 * wv + 16 * (q >> 2) + 4 * g + (q & 3));
    float wm = -INFINITY;
#pragma unroll
    for (int rg = 0; rg < RG; rg++)
#pragma unroll
        for (int q = 0; q < 16; q++) {
            est[rg][q] = est_one(y0 + 16 * rg + jr, x0 + 64 * wv + 16 * (q >> 2) + 4 * g + (q & 3), sv[rg][q],
                                 acc[rg][q >> 2][q & 3]);
            wm = fmaxf(wm, est[rg][q]);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        wm = fmaxf(wm, __shfl_xor(wm, o));
    if (lane == 0)
        bmx[wv] = wm;
    __syncthreads();
    const float thr = fmaxf(fmaxf(bmx[0], bmx[1]), fmaxf(bmx[2], bmx[3])) - kEpsRho;
    if (wm >= thr) {
#pragma unroll
        for (int rg = 0; rg < RG; rg++)
#pragma unroll
            for (int q = 0; q < 16; q++)
                if (est[rg][q] >= thr) {
                    const int k = atomicAdd(ccnt, 1);
                    if (k < kSingleCap)
                        clist[k] = make_int4(((16 * rg + jr) << 16) | (64 * wv + 16 * (q >> 2) + 4 * g + (q & 3)),
                                             acc[rg][q >> 2][q & 3], sv[rg][q].x, sv[rg][q].y);
                }
    }
    __syncthreads();
    const int ncand = *ccnt;
    RecPod r = rec_empty();
    if (ncand <= kSingleCap) {
        if (t < ncand) {
            const int4 c = clist[t];
            const int64_t l = (int64_t)(y0 + (c.x >> 16)) * a.Lx + x0 + (c.x & 0xffff);
            const int64_t dr = var_num(mn, make_int2(c.z, c.w));
            const int64_t num = mn * (int64_t)c.y - St * (int64_t)c.z;
            r.rho = rho64(num, Dt, dr);
            r.l = l;
            r.num = num;
            r.dr = dr;
            r.valid = 1;
        }
    } else {
        // overflow (more than kSingleCap near-equal values, e.g. a flat or
        // periodic image): streaming band selection over every value
#pragma unroll
        for (int rg = 0; rg < RG; rg++)
#pragma unroll 1
            for (int q = 0; q < 16; q++) {
                const int y = y0 + 16 * rg + jr, x = x0 + 64 * wv + 16 * (q >> 2) + 4 * g + (q & 3);
                if (y < a.Ly && x < a.Lx) {
                    int64_t l = (int64_t)y * a.Lx + x;
                    int2 st = ld_int2(a.stat + (l));
                    int64_t dr = var_num(mn, st);
                    int accv = 0;
#pragma unroll
                    for (int e = 0; e < 16; e++)
                        if (e == q)
                            accv = acc[rg][e >> 2][e & 3];
                    int64_t num = mn * (int64_t)accv - St * (int64_t)st.x;
                    rec_offer(r, rho32(num, Dt, dr), l, num, Dt, dr);
                }
            }
    }
    // the candidates sit in the first ncand lanes: one needs no merge, and up
    // to 64 are merged within wave 0 (thread 0 holds the result either way)
    if (ncand == 1)
        return r;
    if (ncand <= 64)
        return wv == 0 ? wave_rec(r) : r;
    return block_rec4(r, red);
}

// The body with the copy count of the template's width.
template <int RG>
__device__ RecPod single_tile(const SingleTile &a, int x0, int y0, uint32_t *smem)
{
    if (single_copies(a.n16) == 16)
        return single_tile_body<RG, 16>(a, x0, y0, smem, threadIdx.x);
    return single_tile_body<RG, 8>(a, x0, y0, smem, threadIdx.x);
}

template <int RG>
__global__ __launch_bounds__(256, 3) void k_single(const BatchJob *__restrict__ jobs, int njobs)
{
    extern __shared__ __align__(16) uint32_t smem[];
    const BatchJob a = jobs[batch_job_of<0>(jobs, njobs, blockIdx.x)];
    const int lb = blockIdx.x - a.block0, bx = lb % a.gx, by = lb / a.gx;
    const int t = threadIdx.x, m = a.m, nw16 = a.n16 >> 2;
    const int tstr = batch_tstride(nw16);
    uint32_t *tpl_l = smem + single_tpl_offset(a.n16);
    const uint32_t *tplg = (const uint32_t *)a.tpl;
    const int64_t St = gptr(a.tst)[0], Dt = gptr(a.tst)[1];
    RecPod *out = a.recs + (int64_t)lb * 16;
    if (Dt == 0) {  // degenerate template: the host reports it from tst
        if (t < 16)
            st_rec(out + t, rec_empty());
        return;
    }
    for (int idx = t; idx < m * nw16; idx += 256) {
        int r = idx / nw16, c = idx - r * nw16;
        tpl_l[(r + kSinglePadLo) * tstr + c] = flip4(gptr(tplg)[idx]);
    }
    single_tpl_pads(tpl_l, m, nw16, tstr);
    const SingleTile st{a.img, a.pitch, a.p, a.stat, a.Ly, a.Lx, m, a.n, a.n16, St, Dt};
    const RecPod best = single_tile<RG>(st, bx * 256, by * 16 * RG, smem);
    if (t < 16)
        st_rec(out + t, t == 0 ? best : rec_empty());
}

// ============================================================== survivor tiles

// The survivor sum of wave_dot_tpl_u8 with the tile's image region staged in
// LDS as raw words (rsw words per region row, the region starting at the
// tile's first location): (dy, dx) is the location within the tile.  rsw is
// odd, so the rows a wave reads at once start on different banks.
__device__ __forceinline__ uint32_t wave_dot_lds_u8(const uint32_t *__restrict__ tplw, int n4,
                                                    const uint32_t *__restrict__ reg, int rsw, int dy, int dx, int m,
                                                    int lane)
{
    uint32_t acc = 0;
    const uint32_t sh = (uint32_t)(dx & 3);
    if (n4 <= kWave) {
        const int rp = kWave / n4;
        const int r0 = lane / n4, j = lane - r0 * n4;
        if (r0 < rp) {
            const uint32_t *pr = reg + (dy + r0) * rsw + (dx >> 2) + j;
            const int step = rp * rsw;
            const uint32_t *tp = tplw + r0 * n4 + j;
            const int tstep = rp * n4;
            const int nit = max(0, (m - r0 + rp - 1) / rp);  // rows r0, r0 + rp, ... below m
            // eight rows' reads issued together (clamped), then their products
            for (int i0 = 0; i0 < nit; i0 += 8) {
                uint32_t lo[8], hi[8], tv[8];
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const int i = min(i0 + k, nit - 1);
                    lo[k] = pr[i * step];
                    hi[k] = pr[i * step + 1];
                    tv[k] = tp[i * tstep];
                }
#pragma unroll
                for (int k = 0; k < 8; k++)
                    if (i0 + k < nit)
                        acc = __builtin_amdgcn_udot4(bytes_at(hi[k], lo[k], sh), tv[k], acc, false);
            }
        }
    } else {
#pragma unroll 1
        for (int i = 0; i < m; i++) {
            const uint32_t *row = reg + (dy + i) * rsw + (dx >> 2);
            for (int j = lane; j < n4; j += kWave)
                acc = __builtin_amdgcn_udot4(bytes_at(row[j + 1], row[j], sh), tplw[i * n4 + j], acc, false);
        }
    }
    return (uint32_t)wave_sum((int)acc);
}

// Whether super-tile (sy, tx) -- the (up to) four tiles of tile column tx
// and tile rows 4 sy .. 4 sy + 3, 128 x 256 locations -- is matched whole by
// k_dense_tiles: its tiles hold at least 4 dense_min survivors together, or
// one of them holds at least dense_min (so every tile left to k_surv_tiles
// fits its bin of dense_min).
__device__ __forceinline__ bool super_dense(const TileArgs &a, int sy, int tx)
{
    if (a.dense_min <= 0)
        return false;
    int sum = 0, most = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int ty = 4 * sy + k;
        const int c = ty < a.tiles_y ? (int)a.tile_cnt[ty * a.tiles_x + tx] : 0;
        sum += c;
        most = max(most, c);
    }
    return sum >= 4 * a.dense_min || most >= a.dense_min;
}

// This block's place among the blocks its XCD holds: the hardware deals
// block ids round-robin over the 8 XCDs, and this index gives each XCD's
// blocks a contiguous run (a permutation of the block ids).
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, hw = blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = hw & 7;
    return xcd * q8 + min(xcd, r8) + (hw >> 3);
}

// Tile k of the column-major order (down each tile column in turn) as a
// row-major tile index.
__device__ __forceinline__ int tile_down_columns(int k, int tiles_x, int tiles_y)
{
    const int tx = k / tiles_y;
    return (k - tx * tiles_y) * tiles_x + tx;
}

// The items of a tile-kernel block: b, b + G, b + 2G, ... (G blocks, at
// most 256 items each, so that clustered work spreads over the blocks; b is
// the block id, or `base` when given).  One round trip: thread k asks `want`
// about item b + kG, and the items it accepts (value > 0) are listed in
// order with their values.  Returns how many; all threads call it (s_tv may
// be null).
template <typename F>
__device__ int block_tiles(int ntiles, F want, int *s_tl, int *s_tv, int *s_tmp, int base = -1)
{
    const int tile = (base < 0 ? (int)blockIdx.x : base) + (int)threadIdx.x * (int)gridDim.x;
    const int v = tile < ntiles ? want(tile) : 0;
    int total;
    const int off = block_excl_scan(v > 0 ? 1 : 0, s_tmp, &total);
    if (v > 0) {
        s_tl[off] = tile;
        if (s_tv)
            s_tv[off] = v;
    }
    __syncthreads();
    return total;
}

// Dense tiles (32 x 256 locations): a tile of a dense super-tile (super_dense:
// the decision is taken per 128 x 256 super-tile, so that scattered
// survivors do not split it) is matched whole on int8 MFMA with the k_single
// body: the locations scan 2 eliminated lie below the threshold, so they
// cannot be the answer, and the counts stay those of the decisions.  The
// grid has as many blocks as the device holds at once, and at least one per
// kDenseTilesPerBlock tiles: each block lists its dense tiles in one round
// trip, stages the template once and matches the tiles one after another,
// writing one record.
template <int CP>
__global__ __launch_bounds__(256, 3) void k_dense_tiles(TileArgs a)
{
    static_assert(kTileRows == 32, "a dense tile is one block of two row groups");
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int s_tl[256], s_tmp[4];
    const int t = threadIdx.x;
    const int degenerate = a.qs->degenerate;
    // Items run down the tile columns (item k: tile row k mod tiles_y of tile
    // column k / tiles_y), and the blocks an XCD holds (the hardware deals
    // block ids round-robin over the 8 XCDs) take consecutive items, so the
    // tiles in flight on one XCD are vertical neighbours whose image rows
    // overlap in its L2.
    auto tile_of = [&](int item) { return tile_down_columns(item, a.tiles_x, a.tiles_y); };
    const int nd = block_tiles(
        a.tiles_x * a.tiles_y,
        [&](int item) {
            const int tile = tile_of(item);
            const int ty = tile / a.tiles_x;
            return !degenerate && super_dense(a, ty >> 2, tile - ty * a.tiles_x) ? 1 : 0;
        },
        s_tl, (int *)nullptr, s_tmp, xcd_block());
    // the block's record and area stay in LDS, so that no register is live
    // across the tiles' main loops
    __shared__ RecPod s_best;
    if (t == 0)
        s_best = rec_empty();
    if (nd > 0) {
        const int nw16 = a.n16 >> 2, tstr = batch_tstride(nw16);
        uint32_t *tpl_l = smem + single_tpl_offset(a.n16);
        const bool words = ((a.ts | (int64_t)(uintptr_t)a.tpl) & 3) == 0 && (a.n & 3) == 0;
        if (words) {
            batched_loads<8>(
                a.m * nw16,
                [&](int idx) {
                    const int r = idx / nw16;
                    return tpl_raw_word(a.tpl, a.ts, a.n, r, idx - r * nw16);
                },
                [&](int idx, uint32_t w) {
                    const int r = idx / nw16, c = idx - r * nw16, nb = a.n - 4 * c;
                    w = flip4(w);  // int8 view; the bytes past column n back to zero
                    tpl_l[(r + kSinglePadLo) * tstr + c] = nb >= 4 ? w : nb <= 0 ? 0u : w & ((1u << (8 * nb)) - 1u);
                });
        } else {
            for (int idx = t; idx < a.m * nw16; idx += 256) {
                const int r = idx / nw16, c = idx - r * nw16;
                tpl_l[(r + kSinglePadLo) * tstr + c] = tpl_word(a.tpl, a.ts, a.n, r, c, words);
            }
        }
        single_tpl_pads(tpl_l, a.m, nw16, tstr);
        const SingleTile st{a.img, a.pitch, a.p, a.stat, a.Ly, a.Lx, a.m, a.n, a.n16, a.qs->st, a.qs->dt};
#pragma unroll 1
        for (int i = 0; i < nd; i++) {
            const int tile = tile_of(s_tl[i]);
            const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
            // the thread index passes through an empty asm, so that nothing
            // the body derives from it is hoisted out of this loop (it would
            // stay live across the main loop and spill)
            int tv = t;
            asm volatile("" : "+v"(tv));
            const RecPod r = single_tile_body<2, CP>(st, tx * kTileCols, ty * kTileRows, smem, tv);
            if (t == 0)
                rec_merge(s_best, r);  // thread 0 holds the tile's record
            __syncthreads();  // the next tile restages the LDS this one's epilogue read
        }
    }
    if (t == 0) {
        unsigned long long area = 0;
        for (int i = 0; i < nd; i++) {
            const int tile = tile_of(s_tl[i]);
            const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
            area += (unsigned long long)min(kTileRows, a.Ly - ty * kTileRows) * min(kTileCols, a.Lx - tx * kTileCols);
        }
        a.recs[a.rec_off + a.surv_blocks + blockIdx.x] = s_best;
        if (area)
            atomicAdd(&a.qs->n_dense, area);
    }
}

// Sparse tiles (after scan 2 has binned the survivors): a tile with
// survivors that is not part of a dense super-tile (fewer than dense_min
// survivors, all in its bin) has each listed survivor matched by one wave
// with unsigned dot products, from the tile's image region staged in LDS
// when it fits and the tile has more than kSparseDirect survivors, else from
// global memory.  As many blocks as the device holds at once, over (tile,
// part) items: for templates of at least kSurvSplitArea pixels a tile's survivors
// are split into up to kSurvParts parts of at least kSurvPartMin, each
// matched by the block that draws the item (so the survivors near the answer
// are not one block's serial work; for smaller templates the restaging
// costs more than the split saves); each block lists its items in one round
// trip (empty and dense tiles cost nothing more), stages the template once
// and writes one record.
constexpr int kSparseDirect = 16;  // survivors of a part matched without staging its region
constexpr int kSurvParts = 4;
constexpr int kSurvPartMin = 24;
constexpr int kSurvSplitArea = 64 * 64;

__host__ __device__ inline int surv_parts_of(int c, int parts)
{
    return min(parts, max(1, (c + kSurvPartMin - 1) / kSurvPartMin));
}

__global__ __launch_bounds__(256) void k_surv_tiles(TileArgs a)
{
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ RecPod red4[4];
    __shared__ int s_tl[256], s_tv[256], s_tmp[4];
    const int t = threadIdx.x;
    const int degenerate = a.qs->degenerate;
    const int P = a.surv_parts;
    const int ns = block_tiles(
        a.tiles_x * a.tiles_y * P,
        [&](int item) {
            const int tile = item / P, part = item - tile * P;
            const int ty = tile / a.tiles_x;
            const bool sd = super_dense(a, ty >> 2, tile - ty * a.tiles_x);
            const int cnt = min((int)a.tile_cnt[tile], a.tile_cap);
            // nothing here, k_dense_tiles' work, or a part the tile does not have
            return degenerate || sd || part >= surv_parts_of(cnt, P) ? 0 : cnt;
        },
        s_tl, s_tv, s_tmp);
    RecPod rec = rec_empty();
    unsigned long long matched = 0;
    if (ns > 0) {
        const int64_t St = a.qs->st, Dt = a.qs->dt;
        const int64_t mn = (int64_t)a.m * a.n;
        const int n4 = (a.n + 3) >> 2;
        const int rsw = a.region_words;
        uint32_t *tplw = smem;
        uint32_t *reg = smem + ((a.m * n4 + 3) & ~3);
        load_template_words(a.tpl, a.ts, a.m, a.n, n4, tplw);
        const int lane = t & 63, wv = t >> 6;
        for (int i = 0; i < ns; i++) {
            const int tile = s_tl[i] / P, part = s_tl[i] - tile * P, cnt = s_tv[i];
            const int np = surv_parts_of(cnt, P);
            const int k0 = (int)((int64_t)cnt * part / np), k1 = (int)((int64_t)cnt * (part + 1) / np);
            const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
            const int y0 = ty * kTileRows, x0 = tx * kTileCols;
            // a few survivors read their windows from global memory: staging
            // the whole region would cost more than it saves
            const bool staged = a.sparse_lds && k1 - k0 > kSparseDirect;
            if (staged) {
                // rows y0 .. y0 + 31 + m - 1 (clipped to the image), words from x0
                const int R = min(kTileRows + a.m - 1, a.p - y0);
                const uint8_t *base = a.img + (int64_t)y0 * a.pitch + x0;
                const int wmax = (int)min((int64_t)rsw, (a.pitch - x0) >> 2);
                batched_loads<8>(
                    R * rsw,
                    [&](int idx) {
                        const int r = idx / rsw, w = idx - r * rsw;
                        const uint32_t v =
                            *gptr((const uint32_t *)(base + (int64_t)r * a.pitch + 4 * max(0, min(w, wmax - 1))));
                        return w < wmax ? v : 0u;
                    },
                    [&](int idx, uint32_t v) { reg[idx] = v; });
            }
            __syncthreads();  // the template (first item) and the region are in LDS
            const int c = k1 - k0;  // this part's survivors: bin slots k0 .. k1 - 1
            const int32_t *bin = a.tile_bin + (int64_t)tile * a.tile_cap + k0;
            // this wave's survivors wv, wv + 4, ... in batches of 64: lane L reads
            // the location and statistics of the batch's survivor L in one round trip
            for (int kb = wv; kb < c; kb += 4 * 64) {
                const int ks = kb + 4 * lane;
                const int ol = ks < c ? bin[ks] : 0;
                const int2 sol = ks < c ? a.stat[ol] : make_int2(0, 0);
                const int nbat = min(64, (c - kb + 3) >> 2);
                // the wave's sums, one survivor after another; lane q keeps
                // survivor q's, and the batch's epilogues then run in parallel
                uint32_t mine = 0;
                for (int q = 0; q < nbat; q++) {
                    const int o32 = __shfl(ol, q);
                    const int y = o32 / a.Lx, x = o32 - y * a.Lx;
                    const uint32_t Xu = staged ? wave_dot_lds_u8(tplw, n4, reg, rsw, y - y0, x - x0, a.m, lane)
                                               : wave_dot_tpl_u8(tplw, n4, a.img, a.pitch, y, x, a.m, lane);
                    mine = lane == q ? Xu : mine;
                }
                if (lane < nbat) {
                    // N = mn sum(t r) - sum(t) sum(r) on unshifted values; the
                    // shifted sums S' become sum(x) = S' + 128 mn
                    const int64_t dr = var_num(mn, sol);
                    const int64_t num = mn * (int64_t)mine - (St + 128 * mn) * ((int64_t)sol.x + 128 * mn);
                    rec_offer_inline(rec, rho32(num, Dt, dr), ol, num, Dt, dr);
                }
            }
            matched += (unsigned long long)c;
            __syncthreads();  // the next item restages the region
        }
    }
    const RecPod best = block_rec4(rec, red4);
    if (t == 0) {
        a.recs[a.rec_off + blockIdx.x] = best;
        if (matched)
            atomicAdd(&a.qs->n_sparse, matched);
    }
}

// First fold of the per-block records: fold block c of tile z merges the
// records of blocks 64c .. 64c+63 of the tile for its 16 templates
// (coalesced: 16 consecutive records per block row) into part[z][c][16].
__global__ __launch_bounds__(256) void k_fold_batch(const BatchJob *__restrict__ jobs, int njobs)
{
    __shared__ RecPod red[256];
    const BatchJob &a = jobs[batch_job_of<1>(jobs, njobs, blockIdx.x)];
    const int lb = blockIdx.x - a.fold0, c = lb % a.chunks, z = lb / a.chunks;
    const int bpt = a.gx * a.gy;
    const RecPod *recs = a.recs;
    RecPod *part = a.recs + (size_t)a.gz * bpt * 16;
    const int t = threadIdx.x, col = t & 15;
    const int hi = min(bpt, 64 * c + 64);
    RecPod r = rec_empty();
    for (int b = 64 * c + (t >> 4); b < hi; b += 16)
        rec_merge(r, recs[((int64_t)z * bpt + b) * 16 + col]);
    red[t] = r;
    __syncthreads();
    if (t < 16) {
        RecPod f = red[t];
        for (int k = 1; k < 16; k++)
            rec_merge(f, red[t + 16 * k]);
        part[((int64_t)z * a.chunks + c) * 16 + t] = f;
    }
}

// One block per template: fold the template's partial records into its
// answer.  The answer's r32max field is replaced by the binary32 rho of the
// answer.
__global__ __launch_bounds__(256) void k_reduce_batch(const BatchJob *__restrict__ jobs, int njobs)
{
    __shared__ RecPod rred[256];
    const BatchJob &a = jobs[batch_job_of<2>(jobs, njobs, blockIdx.x)];
    const int tt = blockIdx.x - a.tmpl0, z = tt >> 4, col = tt & 15;
    const RecPod *part = a.recs + (size_t)a.gz * a.gx * a.gy * 16;
    RecPod r = rec_empty();
    for (int b = threadIdx.x; b < a.chunks; b += blockDim.x)
        rec_merge(r, part[((int64_t)z * a.chunks + b) * 16 + col]);
    RecPod f = block_rec(r, rred);
    if (threadIdx.x == 0) {
        f.r32max = f.valid ? rho32(f.num, a.tst[2 * tt + 1], f.dr) : 0.0f;
        a.out[tt] = f;
    }
}

// ============================================================== final reduction

// One block folds the per-block records of the final scan (and of the window
// when it counts) into the answer, after the kernels that wrote them have
// finished: the kernel boundary makes the records visible on every XCD
// without a device-scope fence in each writing block.  It then publishes the
// query state to its host mirror (pinned, coherent): every word but the
// sequence number, a system-scope fence, then the sequence number, so a host
// that sees the new number reads a complete state.  The state the earlier
// kernels wrote is loaded by thread 0 together with the records, and the
// mirror is written from registers.
constexpr int kRedThreads = 256;

// Records of [start, hi), start = min(lo, count_lo): the best over [lo, hi)
// and the counts over [count_lo, hi), merged into one record per thread
// (up to four records per thread loaded before they are merged).  With
// stride > 1 the records are the partial results k_reduce_part left at
// start, start + stride, ... (each already follows those rules).
__device__ RecPod reduce_range(const RecPod *__restrict__ recs, int lo, int hi, int count_lo, int stride)
{
    const int t = threadIdx.x;
    RecPod r = rec_empty();
    const int start = min(lo, count_lo);
    if (stride > 1) {
        for (int k = start + t * stride; k < hi; k += kRedThreads * stride)
            rec_merge(r, recs[k]);
        return r;
    }
    for (int k0 = start + t; k0 < hi; k0 += 4 * kRedThreads) {
        RecPod b[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = k0 + j * kRedThreads;
            b[j] = k < hi ? recs[k] : rec_empty();
            if (k < lo)
                b[j].valid = 0;
            if (k < count_lo)
                b[j].n_elim = b[j].n_surv = b[j].n_window = 0;
        }
#pragma unroll
        for (int j = 0; j < 4; j++)
            rec_merge(r, b[j]);
    }
    return r;
}

// First level of the final reduction over many records: block b merges the
// chunk [start + b chunk, start + (b + 1) chunk) and writes its partial
// record over the chunk's first record (read by then).
constexpr int kRedChunk = 2048;

__global__ __launch_bounds__(kRedThreads) void k_reduce_part(RecPod *__restrict__ recs, int lo, int hi, int count_lo)
{
    __shared__ RecPod red[kRedThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int start = min(lo, count_lo), c0 = start + blockIdx.x * kRedChunk, c1 = min(hi, c0 + kRedChunk);
    RecPod r = reduce_range(recs, max(lo, c0), c1, max(count_lo, c0), 1);
    r = wave_rec(r);
    if (lane == 0)
        red[wv] = r;
    __syncthreads();
    if (wv == 0) {
        const RecPod f = wave_rec<kRedThreads / 64>(lane < kRedThreads / 64 ? red[lane] : rec_empty());
        if (lane == 0)
            recs[c0] = f;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const RecPod *__restrict__ recs, int lo, int hi,
                                                        int count_lo, int stride, QState *qs, QState *host)
{
    __shared__ RecPod red[kRedThreads / 64];
    constexpr int kWords = (int)(sizeof(QState) / 8), kSeqWord = (int)(offsetof(QState, seq) / 8);
    static_assert(sizeof(QState) % 8 == 0 && offsetof(QState, seq) % 8 == 0, "8-byte words");
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint64_t w[kWords];
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < kWords; k++)
            w[k] = ((const uint64_t *)qs)[k];
    }
    RecPod r = reduce_range(recs, lo, hi, count_lo, stride);
    r = wave_rec(r);
    if (lane == 0)
        red[wv] = r;
    __syncthreads();
    if (wv != 0)
        return;
    const RecPod f = wave_rec<kRedThreads / 64>(lane < kRedThreads / 64 ? red[lane] : rec_empty());
    if (lane != 0)
        return;
    QState q;
    __builtin_memcpy(&q, w, sizeof q);
    if (!q.degenerate) {
        q.fin = f;
        q.fin_r32 = rho32(f.num, q.dt, f.dr);
        q.n_elim = f.n_elim;
        q.n_surv = f.n_surv;
        q.n_window = f.n_window;
    }
    q.t1 = __builtin_amdgcn_s_memrealtime();
    q.seq += 1;
    // the device copy keeps the answer and the sequence (the next query
    // continues from it)
    qs->fin = q.fin;
    qs->fin_r32 = q.fin_r32;
    qs->n_elim = q.n_elim;
    qs->n_surv = q.n_surv;
    qs->n_window = q.n_window;
    qs->t1 = q.t1;
    qs->seq = q.seq;
    __builtin_memcpy(w, &q, sizeof q);
    uint64_t *__restrict__ dst = (uint64_t *)host;
#pragma unroll
    for (int k = 0; k < kWords; k++)
        if (k != kSeqWord)
            dst[k] = w[k];
    __threadfence_system();
    __hip_atomic_store(&host->seq, q.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ============================================================== launch wrappers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

size_t sat_elems(int p, int q)
{
    return (size_t)(p + 1) * (q + 1) + (size_t)5 * blocks_for(p, kColChunk) * (q + 1);
}

template <class T> static void launch_cols(T *sat, int p, int q, hipStream_t s)
{
    T *tot = sat + (size_t)(p + 1) * (q + 1);                         // [chunks][q + 1]
    T *parts = tot + (size_t)blocks_for(p, kColChunk) * (q + 1);      // [chunks][4][q + 1]
    dim3 grid(blocks_for(q + 1, 64), blocks_for(p, kColChunk)), blk(64, 4);
    hipLaunchKernelGGL(k_cols_total<T>, grid, blk, 0, s, (const T *)sat, p, q, tot, parts);
    hipLaunchKernelGGL(k_cols_apply<T>, grid, blk, 0, s, sat, p, q, (const T *)tot, (const T *)parts);
}

hipError_t launch_sat(const uint8_t *img, int64_t pitch, int p, int q, uint2 *sat, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(sat, 0, sizeof(uint2) * (size_t)(q + 1), s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sat_rows, dim3(p), dim3(256), 0, s, img, pitch, p, q, sat);
    launch_cols(sat, p, q, s);
    return hipGetLastError();
}

hipError_t launch_stats(const uint2 *sat, int q, int Ly, int Lx, int m, int n, int2 *stat, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats, dim3(blocks_for((int64_t)Ly * Lx, 256)), dim3(256), 0, s, sat, q, Ly, Lx, m, n,
                       stat);
    return hipGetLastError();
}

static constexpr int kFullR = 8;

hipError_t launch_reduce(RecPod *recs, int lo, int hi, int count_lo, QState *qs, QState *host, hipStream_t s)
{
    const int start = std::min(lo, count_lo);
    const unsigned parts = blocks_for(std::max(hi - start, 0), kRedChunk);
    if (parts > 1) {  // many records: chunks merged in parallel first
        hipLaunchKernelGGL(k_reduce_part, dim3(parts), dim3(kRedThreads), 0, s, recs, lo, hi, count_lo);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, (const RecPod *)recs, lo, hi, count_lo,
                           kRedChunk, qs, host);
    } else {
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, (const RecPod *)recs, lo, hi, count_lo, 1,
                           qs, host);
    }
    return hipGetLastError();
}

// Zeroes a query state (a fill kernel rather than a memset node, so the
// launch behaves the same when a caller captures it into a graph).
__global__ __launch_bounds__(64) void k_qs_clear(QState *qs)
{
    constexpr int kWords = (int)(sizeof(QState) / 8);
    for (int k = threadIdx.x; k < kWords; k += 64)
        ((uint64_t *)qs)[k] = 0;
}

hipError_t launch_qs_clear(QState *qs, hipStream_t s)
{
    hipLaunchKernelGGL(k_qs_clear, dim3(1), dim3(64), 0, s, qs);
    return hipGetLastError();
}

int full_record_count(int Ly, int Lx) { return (int)(blocks_for(Lx, 256) * blocks_for(Ly, 4 * kFullR)); }

size_t full_lds_bytes(int m, int n)
{
    int n4w = (((n + 3) / 4) + 3) / 4 * 4;
    return (size_t)(4 * kFullR + m - 1) * (64 + n4w) * 4 + (size_t)(m + 2 * kFullR - 2) * n4w * 4;
}

// LDS of one workgroup on gfx950.  A kernel whose static LDS plus the
// dynamic LDS a template shape needs exceeds it cannot run that shape: the
// host rejects such shapes before launching (full_fits, scan_fits).
constexpr size_t kLdsMax = 160 * 1024;

// Set when a static-LDS query fails on this thread (read and cleared by
// lds_query_failed).
static thread_local bool t_lds_failed = false;

bool lds_query_failed()
{
    const bool f = t_lds_failed;
    t_lds_failed = false;
    return f;
}

// Static LDS of a kernel on the current device, cached per kernel and device
// once a query succeeds.  A failed query is not cached: it counts as the
// whole LDS (so nothing is launched) and flags lds_query_failed.
static size_t static_lds(const void *f)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> memo;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        t_lds_failed = true;
        return kLdsMax;
    }
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_pair(f, dev);
    auto it = memo.find(key);
    if (it != memo.end())
        return it->second;
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) {
        (void)hipGetLastError();
        t_lds_failed = true;
        return kLdsMax;
    }
    memo.emplace(key, at.sharedSizeBytes);
    return at.sharedSizeBytes;
}

// Raises a kernel's dynamic-LDS allowance to `bytes` on the current device
// when that is above 64 KB, once per (kernel, device, high-water mark), so a
// repeated launch (including one under graph capture) makes no further call.
static hipError_t allow_lds(const void *f, size_t bytes)
{
    if (bytes <= 64 * 1024)
        return hipSuccess;
    if (bytes + static_lds(f) > kLdsMax)
        return hipErrorInvalidValue;
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> raised;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(mu);
    size_t &hw = raised[std::make_pair(f, dev)];
    if (bytes <= hw)
        return hipSuccess;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        hw = bytes;
    return e;
}

bool full_fits(int m, int n)
{
    return full_lds_bytes(m, n) + static_lds((const void *)k_full<kFullR>) <= kLdsMax;
}

hipError_t launch_full(FullArgs a, hipStream_t s)
{
    a.n4w = (((a.n + 3) / 4) + 3) / 4 * 4;
    dim3 grid(blocks_for(a.Lx, 256), blocks_for(a.Ly, 4 * kFullR));
    size_t lds = full_lds_bytes(a.m, a.n);
    if (!full_fits(a.m, a.n))
        return hipErrorInvalidValue;
    hipError_t e = allow_lds((const void *)k_full<kFullR>, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_full<kFullR>, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

static int centre_waves(int n)
{
    int nch = ((((n + 3) / 4) + 3) / 4 * 4) / 4;
    return nch >= 4 ? 4 : (nch >= 2 ? 2 : 1);
}

// Dynamic LDS of k_centres: the template rows a block's R centre rows reach
// (pad rows above and below) and the per-wave partial sums.
static size_t centres_lds_bytes(int m, int n, int R, int pad)
{
    int n4w = (((n + 3) / 4) + 3) / 4 * 4;
    return (size_t)(m + 2 * pad) * n4w * 4 + (size_t)centre_waves(n) * R * 64 * 4;
}

// Centre rows per wave: the most (8, 4, 2 or 1) whose zero-padded template
// rows cost at most a third of the useful ones, (R-1) h <= m/3, and whose
// padded template fits 48 KB of LDS.
static int centre_rows(int m, int n, int h)
{
    int n4w = (((n + 3) / 4) + 3) / 4 * 4;
    for (int R = 8; R > 1; R >>= 1)
        if (3 * (R - 1) * h <= m && (size_t)(m + 2 * (R - 1) * h) * n4w * 4 <= 48 * 1024)
            return R;
    return 1;
}

// Dwords of a staged row of k_centres_mfma's region that the A reads can
// reach (64 MTW centre columns of stride w, the template width, realignment
// slack).
static int centres_mfma_cwn(int n, int w, int mtw)
{
    int n16 = (n + 15) / 16 * 16;
    return ((64 * mtw - 1) * w + w / 2 + n16 + 12) / 4 + 2;
}

// LDS bank cost of the A reads for a staged-copy stride of cs dwords: lane
// (j, g) of an M-tile reads dwords (4 g + (o & 3)) cs + (o >> 2) + {0, 1}
// and {2, 3} (two ds_read2_b32), o = r + 16 w (mt) + w j being its centre's
// byte offset from the region's first staged word.  The cost is the largest
// number of distinct dwords in one of 128 four-byte banks among the 32 lanes
// served together, summed over r, the first M-tiles, both reads and both
// halves of the wave.
static int centres_bank_cost(int cs, int w)
{
    int cost = 0;
    for (int r = 0; r < 4; r++)
        for (int mt = 0; mt < 4; mt++)
            for (int half = 0; half < 2; half++)
                for (int pr = 0; pr < 2; pr++) {
                    int words[64], nw = 0, cnt[128] = {0};
                    for (int l = 32 * half; l < 32 * half + 32; l++) {
                        const int g = l >> 4, j = l & 15, o = r + 16 * w * mt + w * j;
                        for (int e = 0; e < 2; e++) {
                            const int d = (4 * g + (o & 3)) * cs + (o >> 2) + 2 * pr + e;
                            bool dup = false;
                            for (int k = 0; k < nw; k++)
                                dup |= words[k] == d;
                            if (!dup) {
                                words[nw++] = d;
                                cnt[d & 127]++;
                            }
                        }
                    }
                    int worst = 0;
                    for (int b = 0; b < 128; b++)
                        worst = cnt[b] > worst ? cnt[b] : worst;
                    cost += worst;
                }
    return cost;
}

static size_t centres_mfma_lds(int m, int n, int cs, int ntpl = 1)
{
    int n16 = (n + 15) / 16 * 16;
    return ((size_t)ntpl * (m + 1) * batch_tstride(n16 / 4) + (size_t)2 * 16 * cs) * 4;
}

// Shape of k_centres_mfma for a centre grid: M-tiles per wave (4, 2 or 1:
// the most that leaves at least kCmMinBlocks blocks and whose staged width
// fits the per-thread staging, 4 cwn <= 256 cm_words_per_thread), the
// reachable width cwn and the copy stride cs (among cwn and up to 63 dwords
// more, the least bank cost within 60 KB of LDS).  cs = 0 when the MFMA form
// does not apply (n > 128, or no width fits).
struct CmShape {
    int cs, cwn, mtw;
};
constexpr int64_t kCmMinBlocks = 512;

static CmShape centres_mfma_shape_search(int Gy, int Gx, int m, int n, int w)
{
    const size_t kLds = 60 * 1024;
    int n16 = (n + 15) / 16 * 16;
    CmShape r = {0, 0, 0};
    if (n16 > 128)
        return r;
    for (int mtw = 4; mtw >= 1; mtw >>= 1) {
        const int cwn = centres_mfma_cwn(n, w, mtw);
        if (4 * cwn > 256 * cm_words_per_thread(mtw) || centres_mfma_lds(m, n, cwn) > kLds)
            continue;
        const int64_t nb = blocks_for(Gx, 64 * mtw) * blocks_for(Gy, 16);
        if (mtw > 1 && nb < kCmMinBlocks)
            continue;
        r.cwn = cwn;
        r.mtw = mtw;
        break;
    }
    if (!r.mtw)
        return r;
    int best = r.cwn, best_cost = centres_bank_cost(r.cwn, w);
    for (int cs = r.cwn + 1; cs < r.cwn + 64 && centres_mfma_lds(m, n, cs) <= kLds; cs++) {
        int c = centres_bank_cost(cs, w);
        if (c < best_cost) {
            best = cs;
            best_cost = c;
        }
    }
    r.cs = best;
    return r;
}

// The search above, memoised per (Gy, Gx, m, n, w): it runs once per shape,
// not per query (callers may be on several threads).
static CmShape centres_mfma_shape(int Gy, int Gx, int m, int n, int w)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int>, CmShape> memo;
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(Gy, Gx, m, n, w);
    auto it = memo.find(key);
    if (it != memo.end())
        return it->second;
    CmShape r = centres_mfma_shape_search(Gy, Gx, m, n, w);
    memo.emplace(key, r);
    return r;
}

int centres_record_count(int Gy, int Gx, int m, int n, int h, int w)
{
    const CmShape sh = centres_mfma_shape(Gy, Gx, m, n, w);
    if (sh.cs)
        return (int)(blocks_for(Gx, 64 * sh.mtw) * blocks_for(Gy, 16));
    return (int)(blocks_for(Gx, 64) * blocks_for(Gy, centre_rows(m, n, h)));
}

// LDS of several templates' rows beside the step buffers of the one-template
// shape.
constexpr size_t kCmBatchLds = 150 * 1024;

bool centres_mfma_batchable(int Gy, int Gx, int m, int n, int w, int ntpl)
{
    const CmShape sh = centres_mfma_shape(Gy, Gx, m, n, w);
    return sh.cs && ntpl >= 1 && ntpl <= kScanMaxT &&
           centres_mfma_lds(m, n, sh.cs, ntpl) + static_lds((const void *)k_centres_mfma<8, kScanMaxT, 4>) <=
               kCmBatchLds;
}

template <int NB, int TM> static const void *cm_kernel(int mtw)
{
    return mtw == 4 ? (const void *)k_centres_mfma<NB, TM, 4>
         : mtw == 2 ? (const void *)k_centres_mfma<NB, TM, 2> : (const void *)k_centres_mfma<NB, TM, 1>;
}

template <int NB> static const void *cm_kernel(int ntpl, int mtw)
{
    return ntpl <= 1 ? cm_kernel<NB, 1>(mtw) : cm_kernel<NB, kScanMaxT>(mtw);
}

hipError_t launch_centres(ScanArgs a, hipStream_t s)
{
    if (a.ntpl < 1)
        a.ntpl = 1;
    const CmShape sh = centres_mfma_shape(a.Gy, a.Gx, a.m, a.n, a.w);
    if (a.ntpl > 1 && !centres_mfma_batchable(a.Gy, a.Gx, a.m, a.n, a.w, a.ntpl))
        return hipErrorInvalidValue;
    if (sh.cs) {
        a.cwd = sh.cs;
        a.cwn = sh.cwn;
        a.crows_log2 = 2;
        const size_t lds = centres_mfma_lds(a.m, a.n, sh.cs, a.ntpl);
        const dim3 grid(blocks_for(a.Gx, 64 * sh.mtw), blocks_for(a.Gy, 16)), blk(kCmThreads);
        const int nb = (a.n + 15) / 16;
        const void *f = nb == 1 ? cm_kernel<1>(a.ntpl, sh.mtw) : nb == 2 ? cm_kernel<2>(a.ntpl, sh.mtw)
                      : nb == 3 ? cm_kernel<3>(a.ntpl, sh.mtw) : nb == 4 ? cm_kernel<4>(a.ntpl, sh.mtw)
                      : nb == 5 ? cm_kernel<5>(a.ntpl, sh.mtw) : nb == 6 ? cm_kernel<6>(a.ntpl, sh.mtw)
                      : nb == 7 ? cm_kernel<7>(a.ntpl, sh.mtw) : cm_kernel<8>(a.ntpl, sh.mtw);
        hipError_t e = allow_lds(f, lds);
        if (e != hipSuccess)
            return e;
        void *args[] = {&a};
        return hipLaunchKernel(f, grid, blk, args, lds, s);
    }
    a.n4w = (((a.n + 3) / 4) + 3) / 4 * 4;
    int nw = centre_waves(a.n);
    int R = centre_rows(a.m, a.n, a.h);
    a.pad = (R - 1) * a.h;
    size_t lds = centres_lds_bytes(a.m, a.n, R, a.pad);
    const void *f = R == 8 ? (const void *)k_centres<8>
                  : R == 4 ? (const void *)k_centres<4>
                  : R == 2 ? (const void *)k_centres<2> : (const void *)k_centres<1>;
    hipError_t e = allow_lds(f, lds);
    if (e != hipSuccess)
        return e;
    dim3 grid(blocks_for(a.Gx, 64), blocks_for(a.Gy, R));
    switch (R) {
    case 8: hipLaunchKernelGGL(k_centres<8>, grid, dim3(64 * nw), lds, s, a); break;
    case 4: hipLaunchKernelGGL(k_centres<4>, grid, dim3(64 * nw), lds, s, a); break;
    case 2: hipLaunchKernelGGL(k_centres<2>, grid, dim3(64 * nw), lds, s, a); break;
    default: hipLaunchKernelGGL(k_centres<1>, grid, dim3(64 * nw), lds, s, a); break;
    }
    return hipGetLastError();
}

int window_record_count(int radius)
{
    int W = 2 * radius + 1;
    return W * W;  // one block per location
}

hipError_t launch_window(WinArgs a, hipStream_t s)
{
    hipLaunchKernelGGL(k_window, dim3(window_record_count(a.radius)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int members_record_count(int Gy, int Gx) { return (int)blocks_for((int64_t)Gy * Gx, kMemGroups); }

hipError_t launch_members(MemArgs a, hipStream_t s)
{
    hipLaunchKernelGGL(k_members, dim3(members_record_count(a.Gy, a.Gx)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int tiles_x_of(int Lx) { return (int)blocks_for(Lx, kTileCols); }
int tiles_y_of(int Ly) { return (int)blocks_for(Ly, kTileRows); }

// LDS of k_surv_tiles' sparse path: the template's raw words, then (with
// sparse_lds) the tile's image region.
static size_t tiles_sparse_bytes(int m, int n, int sparse_lds, int rsw)
{
    const size_t tw = ((size_t)m * ((n + 3) / 4) + 3) & ~(size_t)3;
    return (tw + (sparse_lds ? (size_t)(kTileRows + m - 1) * rsw : 0)) * 4;
}

static size_t single_lds_bytes(int m, int n16);

// Blocks of a tile kernel that loops over its tiles: as many as the device holds at once
// (occupancy at this dynamic LDS times the CUs, cached per kernel, device
// and size once the queries succeed), at least one per 256 tiles and at
// most one per tile.  Without an answer, one block per tile.
static int tile_blocks(const void *f, size_t lds, int ntiles)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t>, int> memo;
    int dev = 0, g = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        auto key = std::make_tuple(f, dev, lds);
        auto it = memo.find(key);
        if (it != memo.end()) {
            g = it->second;
        } else {
            int per_cu = 0, cus = 0;
            if (allow_lds(f, lds) == hipSuccess &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, lds) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                per_cu > 0 && cus > 0) {
                g = per_cu * cus;
                memo.emplace(key, g);
            } else {
                (void)hipGetLastError();
            }
        }
    }
    if (g <= 0)
        g = ntiles;
    return std::max((ntiles + 255) / 256, std::min(g, ntiles));
}

constexpr int kDenseTilesPerBlock = 4;

// The dense-tile kernel with the single-template body's copy count for n16.
static const void *dense_tiles_kernel(int n16)
{
    return single_copies(n16) == 16 ? (const void *)k_dense_tiles<16> : (const void *)k_dense_tiles<8>;
}

// The staged region is kept to 96 KB so that most tiles' blocks can share a CU.
constexpr size_t kSparseRegionMax = 96 * 1024;

void tile_plan(TileArgs &a, int dense_min)
{
    a.n16 = (a.n + 15) / 16 * 16;
    a.tiles_x = tiles_x_of(a.Lx);
    a.tiles_y = tiles_y_of(a.Ly);
    const bool dense = dense_min > 0 && dense_min <= kTileRows * kTileCols && batch_single_fits(a.m, a.n);
    a.dense_min = dense ? dense_min : 0;
    a.tile_cap = dense ? dense_min : kTileRows * kTileCols;
    const int n4 = (a.n + 3) / 4;
    a.region_words = (64 + n4 + 1) | 1;
    a.sparse_lds = tiles_sparse_bytes(a.m, a.n, 1, a.region_words) <= kSparseRegionMax ? 1 : 0;
    const int nt = a.tiles_x * a.tiles_y;
    a.surv_parts = a.m * a.n >= kSurvSplitArea ? kSurvParts : 1;
    a.surv_blocks = tile_blocks((const void *)k_surv_tiles, tiles_sparse_bytes(a.m, a.n, a.sparse_lds, a.region_words),
                                nt * a.surv_parts);
    // at most kDenseTilesPerBlock tiles per block: beyond what the device
    // holds at once, the later blocks start as earlier ones finish, which
    // evens out the blocks' unequal work
    a.dense_blocks = a.dense_min > 0 ? std::max(tile_blocks(dense_tiles_kernel(a.n16), single_lds_bytes(a.m, a.n16), nt),
                                                std::min(nt, (nt + kDenseTilesPerBlock - 1) / kDenseTilesPerBlock))
                                     : 0;
}

static size_t tiles_lds_bytes(const TileArgs &a) { return tiles_sparse_bytes(a.m, a.n, a.sparse_lds, a.region_words); }

int tile_record_count(const TileArgs &a) { return a.surv_blocks + a.dense_blocks; }

hipError_t launch_dense_tiles(TileArgs a, hipStream_t s)
{
    if (a.dense_min <= 0)
        return hipSuccess;
    const size_t dl = single_lds_bytes(a.m, a.n16);
    const void *f = dense_tiles_kernel(a.n16);
    hipError_t e = allow_lds(f, dl);
    if (e != hipSuccess)
        return e;
    if (a.dense_blocks < 1 || (int64_t)a.dense_blocks * 256 < (int64_t)a.tiles_x * a.tiles_y)
        return hipErrorInvalidValue;
    void *args[] = {&a};
    return hipLaunchKernel(f, dim3((unsigned)a.dense_blocks), dim3(256), args, dl, s);
    return hipGetLastError();
}

hipError_t launch_surv_tiles(TileArgs a, hipStream_t s)
{
    const size_t lds = tiles_lds_bytes(a);
    const int64_t nt = (int64_t)a.tiles_x * a.tiles_y;
    if (nt < 1 || a.surv_parts < 1 || a.surv_parts > kSurvParts || nt * a.surv_parts > INT32_MAX ||
        a.surv_blocks < 1 || (int64_t)a.surv_blocks * 256 < nt * a.surv_parts)
        return hipErrorInvalidValue;
    hipError_t e = allow_lds((const void *)k_surv_tiles, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_surv_tiles, dim3((unsigned)a.surv_blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

bool scan_fits(int m, int n)
{
    // scan 2 stages nothing of the template; the survivor tiles need at
    // least the template's words (the region and the dense path are optional)
    if (tiles_sparse_bytes(m, n, 0, 0) + static_lds((const void *)k_surv_tiles) > kLdsMax)
        return false;
    if (static_lds((const void *)k_members) > kLdsMax)
        return false;
    // k_centres_mfma's shape search keeps within its own budget; the v_dot4
    // form takes R = 1 (no pad rows) whenever a taller block would need more
    // than 48 KB, so R = 1 bounds its need from above
    size_t cl = std::max(centres_lds_bytes(m, n, 1, 0), (size_t)48 * 1024 + centres_lds_bytes(0, n, 8, 0));
    return cl + static_lds((const void *)k_centres<1>) <= kLdsMax;
}

hipError_t launch_regroup(const void *in, void *out, int Ly, int Lx, int h, int w, hipStream_t s)
{
    hipLaunchKernelGGL(k_regroup, dim3(blocks_for((int64_t)Ly * Lx, 256)), dim3(256), 0, s, (const uint32_t *)in,
                       (uint32_t *)out, Ly, Lx, h, w);
    return hipGetLastError();
}

bool autocorr_by_shifts(int m, int n, int h, int w)
{
    // measured on MI355X: one offset's product running sums and gather cost
    // about as much per pixel as 46 multiply-adds of the direct form (2048 x
    // 2048, 64 x 64), whose one wave per location also has a fixed cost of
    // about 61 offsets' worth (8192 x 8192, 16 x 16: 36 ms against 0.59 ms
    // per offset)
    return (int64_t)(h * w - 1) * 46 < std::max<int64_t>(61 * 46, (int64_t)m * n);
}

hipError_t launch_autocorr(AcArgs a, uint32_t *psat, hipStream_t s)
{
    if (!autocorr_by_shifts(a.m, a.n, a.h, a.w)) {
        hipLaunchKernelGGL(k_autocorr, dim3(blocks_for((int64_t)a.Ly * a.Lx, 64)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const int p = a.Ly + a.m - 1, q = a.Lx + a.n - 1;
    const int64_t G = (int64_t)((a.Ly + a.h - 1) / a.h) * ((a.Lx + a.w - 1) / a.w);
    // every member offset of a full group (a partial group's are a subset)
    for (int dy = -(a.h - 1) / 2; dy <= a.h - 1 - (a.h - 1) / 2; dy++)
        for (int dx = -(a.w - 1) / 2; dx <= a.w - 1 - (a.w - 1) / 2; dx++) {
            if (dy != 0 || dx != 0) {
                hipError_t e = hipMemsetAsync(psat, 0, sizeof(uint32_t) * (size_t)(q + 1), s);
                if (e != hipSuccess)
                    return e;
                hipLaunchKernelGGL(k_prod_rows, dim3(p), dim3(256), 0, s, a.J, a.J, a.pJ, p, q, dy, dx, psat);
                launch_cols(psat, p, q, s);
            }
            hipLaunchKernelGGL(k_ac_shift, dim3(blocks_for(G, 256)), dim3(256), 0, s, a, dy, dx,
                               (const uint32_t *)psat, q);
        }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_centre_stats(const int2 *__restrict__ stat, int Ly, int Lx, int h, int w,
                                                      int Gy, int Gx, int2 *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)Gy * Gx)
        return;
    const int gy = (int)(g / Gx), gx = (int)(g - (g / Gx) * Gx);
    const int oy = gy * h, ox = gx * w;
    const int cy = oy + (min(h, Ly - oy) - 1) / 2, cx = ox + (min(w, Lx - ox) - 1) / 2;
    out[g] = stat[(int64_t)cy * Lx + cx];
}

hipError_t launch_centre_stats(const int2 *stat, int Ly, int Lx, int h, int w, int Gy, int Gx, int2 *out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_centre_stats, dim3(blocks_for((int64_t)Gy * Gx, 256)), dim3(256), 0, s, stat, Ly, Lx, h, w,
                       Gy, Gx, out);
    return hipGetLastError();
}

hipError_t launch_gsum(GsumArgs a, hipStream_t s)
{
    hipLaunchKernelGGL(k_gsum, dim3(blocks_for((int64_t)a.Gy * a.Gx, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_blur(const uint8_t *src, uint8_t *dst, int64_t pitch, int p, int q, const Taps &tp,
                       uint32_t *tmp, hipStream_t s)
{
    uint32_t tsum = 0;
    for (int j = 0; j <= 2 * tp.d; j++)
        tsum += (uint32_t)tp.w[j];
    uint32_t T = tsum * tsum;
    unsigned nb = blocks_for((int64_t)p * q, 256);
    hipLaunchKernelGGL(k_blur_h, dim3(nb), dim3(256), 0, s, src, pitch, p, q, tp, tmp);
    hipLaunchKernelGGL(k_blur_v, dim3(nb), dim3(256), 0, s, (const uint32_t *)tmp, p, q, tp, T, dst, pitch);
    return hipGetLastError();
}

hipError_t launch_blurcorr(BcArgs a, uint32_t *psat, hipStream_t s)
{
    const int p = a.Ly + a.m - 1, q = a.Lx + a.n - 1;
    hipError_t e = hipMemsetAsync(psat, 0, sizeof(uint32_t) * (size_t)(q + 1), s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_prod_rows, dim3(p), dim3(256), 0, s, a.J, a.I, a.pitch, p, q, 0, 0, psat);
    launch_cols(psat, p, q, s);
    a.psat = psat;
    a.q = q;
    hipLaunchKernelGGL(k_blurcorr, dim3(blocks_for((int64_t)a.Ly * a.Lx, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_revert(const uint8_t *viol, uint8_t *colmask, int p, int q, int Ly, int Lx, int m, int n,
                         const uint8_t *I, uint8_t *J, int64_t pitch, unsigned long long *counter, hipStream_t s)
{
    hipLaunchKernelGGL(k_dilate_rows, dim3(blocks_for((int64_t)p * Lx, 256)), dim3(256), 0, s, viol, p, Ly, Lx, m,
                       colmask);
    hipLaunchKernelGGL(k_revert, dim3(blocks_for((int64_t)p * q, 256)), dim3(256), 0, s,
                       (const uint8_t *)colmask, p, q, Lx, n, I, J, pitch, counter);
    return hipGetLastError();
}


static constexpr int kBatchR = kBatchRows;

bool batch_single_fits(int m, int n)
{
    int n16 = (n + 15) / 16 * 16;
    if (n16 > 128 || m < 1 || m > 2048)
        return false;
    size_t words = (size_t)single_tpl_offset(n16) + (size_t)single_tpl_words(m, n16);
    return words * 4 <= 64 * 1024;
}

bool batch_job_geometry(BatchJob &j)
{
    j.n16 = (j.n + 15) / 16 * 16;
    if (j.n16 > 128 || j.T < 1)
        return false;
    j.gx = (int)blocks_for(j.Lx, 256);
    if (j.kind == BATCH_SINGLE) {
        if (j.T != 1 || !batch_single_fits(j.m, j.n))
            return false;
        if (j.rg != 2)
            return false;
        j.gy = (int)blocks_for(j.Ly, 16 * j.rg);
        j.gz = 1;
    } else {
        j.gy = (int)blocks_for(j.Ly, kBatchR);
        j.gz = (int)blocks_for(j.T, 16);
    }
    j.chunks = (int)blocks_for((int64_t)j.gx * j.gy, 64);
    return true;
}

size_t batch_job_records(const BatchJob &j) { return (size_t)j.gz * 16 * ((size_t)j.gx * j.gy + (size_t)j.chunks); }

static size_t batch_lds_bytes(int n16)
{
    int WW = (256 + n16 + 16) / 4;
    size_t lds = ((size_t)2 * 16 * batch_copy_stride(WW) + (size_t)16 * 16 * batch_tstride(n16 / 4)) * 4;
    lds = std::max(lds, 256 * sizeof(RecPod));
    return std::max(lds, (size_t)kBatchEpiWords * 4);
}

static size_t single_lds_bytes(int m, int n16)
{
    size_t lds = ((size_t)single_tpl_offset(n16) + (size_t)single_tpl_words(m, n16)) * 4;
    return std::max(lds, (size_t)kSingleLdsWords * 4);
}

hipError_t launch_batch_jobs(const BatchJob *d_jobs, const BatchJob *h_jobs, int njobs, hipStream_t s)
{
    if (njobs < 1)
        return hipErrorInvalidValue;
    int nm = 0;
    while (nm < njobs && h_jobs[nm].kind == BATCH_MULTI)
        nm++;
    size_t lds_m = 0, lds_s = 0;
    const int rg = nm < njobs ? h_jobs[nm].rg : 0;
    int64_t blocks_m = 0, blocks_s = 0;
    for (int k = 0; k < njobs; k++) {
        const BatchJob &j = h_jobs[k];
        if (j.n16 > 128 || (k >= nm && (j.kind != BATCH_SINGLE || j.rg != rg)))
            return hipErrorInvalidValue;
        int64_t end = (int64_t)j.block0 + (int64_t)j.gx * j.gy * j.gz;
        if (k < nm) {
            lds_m = std::max(lds_m, batch_lds_bytes(j.n16));
            blocks_m = end;
        } else {
            lds_s = std::max(lds_s, single_lds_bytes(j.m, j.n16));
            blocks_s = end;
        }
    }
    const BatchJob &e = h_jobs[njobs - 1];
    const int ntpl = e.tmpl0 + e.T;
    const int64_t nfold = (int64_t)e.fold0 + (int64_t)e.gz * e.chunks;
    if (blocks_m > INT32_MAX || blocks_s > INT32_MAX || nfold > INT32_MAX || lds_m > 65536 || lds_s > 65536)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tstats, dim3(ntpl), dim3(256), 0, s, d_jobs, njobs);
    if (nm > 0)
        hipLaunchKernelGGL(k_batch<kBatchR>, dim3((unsigned)blocks_m), dim3(256), lds_m, s, d_jobs, nm);
    if (nm < njobs) {
        if (rg != 2)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_single<2>, dim3((unsigned)blocks_s), dim3(256), lds_s, s, d_jobs + nm, njobs - nm);
    }
    hipLaunchKernelGGL(k_fold_batch, dim3((unsigned)nfold), dim3(256), 0, s, d_jobs, njobs);
    hipLaunchKernelGGL(k_reduce_batch, dim3(ntpl), dim3(256), 0, s, d_jobs, njobs);
    return hipGetLastError();
}

}  // namespace zts
