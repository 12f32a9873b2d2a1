// Device helpers shared by the zts kernels (gfx950, wave64).
//
// Pixels are kept as uint8 and read as int8 after flipping the top bit
// (x' = x - 128 = x ^ 0x80).  For blocks a, b of mn pixels the integers
//   N = mn*sum(a'b') - sum(a')sum(b'),   D_a = mn*sum(a'^2) - sum(a')^2
// equal the same expressions on the unshifted pixels, so every decision is
// taken on exact integers.  sum(a'b') fits int32 for mn <= 2^14.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zts_shared.h"

namespace zts {

constexpr int kWave = 64;
constexpr float kEpsTheta = 1e-5f;  // guard band on binary32 angles (rad)
constexpr float kEpsRho = 1e-5f;    // guard band on binary32 correlations

// ---------------------------------------------------------------- int8 words

__device__ __forceinline__ uint32_t flip4(uint32_t w) { return w ^ 0x80808080u; }

__device__ __forceinline__ int dot4(uint32_t a, uint32_t b, int acc)
{
    return __builtin_amdgcn_sdot4((int)a, (int)b, acc, false);
}

// The 4 bytes starting `sh` bytes into `lo`, continuing into `hi`.
__device__ __forceinline__ uint32_t bytes_at(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbyte(hi, lo, sh);
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------- 128-bit integers

struct u128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ u128 mul_u64(uint64_t a, uint64_t b)
{
    u128 r;
    r.lo = a * b;
    r.hi = __umul64hi(a, b);
    return r;
}

// a - b, clamped at 0 when b > a.
__device__ __forceinline__ u128 sub_sat(u128 a, u128 b)
{
    if (a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo))
        return u128{0, 0};
    u128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1 : 0);
    return r;
}

// Round-to-nearest-even conversion: keep the top 64 significant bits, fold
// every dropped bit into a sticky bit 0, let the (correctly rounded) u64
// conversion round, then scale exactly.
__device__ __forceinline__ double u128_to_f64(u128 v)
{
    if (v.hi == 0)
        return (double)v.lo;
    int lz = __clzll(v.hi);
    int s = 64 - lz;
    uint64_t top, dropped;
    if (lz == 0) {
        top = v.hi;
        dropped = v.lo;
    } else {
        top = (v.hi << lz) | (v.lo >> s);
        dropped = v.lo & ((1ull << s) - 1ull);
    }
    top |= (dropped != 0) ? 1ull : 0ull;
    return ldexp((double)top, s);
}

// ---------------------------------------------------------------- canonical binary64

// rho = N / sqrt(D_a * D_b) (Eq. 1 with the 1/mn factors cancelled); a flat
// block has rho := 0.  Three correctly rounded operations in this order.
__device__ __forceinline__ double rho64(int64_t num, int64_t da, int64_t db)
{
    if (da == 0 || db == 0)
        return 0.0;
    double den = (double)da * (double)db;
    return (double)num / __builtin_sqrt(den);
}

// sqrt(1 - rho^2) as sqrt((D_a D_b - N^2) / (D_a D_b)) with the numerator
// exact in 128 bits; a flat block has s := 1.
__device__ __forceinline__ double sin64(int64_t num, int64_t da, int64_t db)
{
    if (da == 0 || db == 0)
        return 1.0;
    uint64_t an = num < 0 ? (uint64_t)(-num) : (uint64_t)num;
    u128 d = sub_sat(mul_u64((uint64_t)da, (uint64_t)db), mul_u64(an, an));
    double nd = u128_to_f64(d);
    return __builtin_sqrt(nd / ((double)da * (double)db));
}

// Upper bound of rho_to from the angle triangle |A - B| - C (cos/sin pairs);
// returns false when no bound below 1 exists.  With C = (1, 0) this is the
// transitive bound of Eq. 2, rho_a*rho_b + s_a*s_b.
__device__ __forceinline__ bool ub_general(double ra, double sa, double rb, double sb, double rc, double sc,
                                           double *ub)
{
    double rab = ra * rb + sa * sb;
    double sab = fabs(sa * rb - ra * sb);
    if (rab >= rc)
        return false;
    *ub = rab * rc + sab * sc;
    return true;
}

// ---------------------------------------------------------------- binary32 prefilter values

// rho in binary32: N (D_a D_b)^(-1/2) with v_rsq_f32 (1 ulp); the three
// conversions, the product and the final multiply round once each, so the
// absolute error is below 5e-7.  A flat block has rho := 0.
// The same from the integers held exactly in binary64 (every N and D of a
// template of at most 16384 pixels is below 2^53): rounding the binary64
// value to binary32 equals rounding the integer, so both forms agree bit for
// bit, and kernels that form N and D in binary64 skip the int64 products
// and conversions.
__device__ __forceinline__ float rho32_exact(double num, double da, double db)
{
    if (da == 0.0 || db == 0.0)
        return 0.0f;
    return (float)num * __builtin_amdgcn_rsqf((float)da * (float)db);
}

__device__ __forceinline__ float rho32(int64_t num, int64_t da, int64_t db)
{
    return rho32_exact((double)num, (double)da, (double)db);
}

// atan(z) for z in [0, 1]: z P(z^2) with P of degree 7, coefficients fitted
// to the smallest largest error on [0, 1] (4e-8; 1.1e-7 evaluated in
// binary32).
__device__ __forceinline__ float atan01(float z)
{
    const float z2 = z * z;
    float p = -0.00405456249f;
    p = fmaf(p, z2, 0.0218629432f);
    p = fmaf(p, z2, -0.0559123102f);
    p = fmaf(p, z2, 0.0964219657f);
    p = fmaf(p, z2, -0.139086295f);
    p = fmaf(p, z2, 0.199465657f);
    p = fmaf(p, z2, -0.333298608f);
    p = fmaf(p, z2, 0.999999336f);
    return p * z;
}

// Angle between two mean-centred blocks, atan2(s, rho) in binary32 from the
// exact integers; NaN for a flat block.  s^2 = (D_a D_b - N^2) / (D_a D_b)
// with the difference taken in binary64 (absolute error of s^2 below 5e-16,
// so below 3e-8 in s even where rho is near +-1), rho by v_rsq_f32, then one
// octant of atan2 by atan01 and its reflections.  Absolute error below 1e-6
// rad (4.5e-7 over 2e5 sampled integer triples, with 1-ulp approximate
// reciprocal, square root and rsqrt).
__device__ __forceinline__ float theta32_exact(double nd, double da, double db)
{
    if (da == 0.0 || db == 0.0)
        return __int_as_float(0x7fc00000);
    const double P = da * db;
    const double d = P - nd * nd;
    const float pf = (float)P;
    const float s = __builtin_amdgcn_sqrtf(fmaxf((float)d, 0.0f) * __builtin_amdgcn_rcpf(pf));
    const float r = (float)nd * __builtin_amdgcn_rsqf(pf);
    const float ar = fabsf(r), lo = fminf(s, ar), hi = fmaxf(s, ar);
    float t = hi > 0.0f ? atan01(lo * __builtin_amdgcn_rcpf(hi)) : 0.0f;
    if (s > ar)
        t = 1.57079633f - t;
    return r < 0.0f ? 3.14159265f - t : t;
}

__device__ __forceinline__ float theta32(int64_t num, int64_t da, int64_t db)
{
    return theta32_exact((double)num, (double)da, (double)db);
}

// ---------------------------------------------------------------- block statistics

// Per-location statistics for one block size: S' = sum(x') (int32) and
// Q' = sum(x'^2) (uint32 bits).  D = mn Q' - S'^2 is exact in int64.
__device__ __forceinline__ int64_t var_num(int64_t mn, int2 st)
{
    return mn * (int64_t)(uint32_t)st.y - (int64_t)st.x * (int64_t)st.x;
}

// ---------------------------------------------------------------- window dot products

// Window dot products, one wave per location.  Lane -> (row in pass, word):
// ceil(n/4) consecutive lanes read consecutive words of one image row
// (coalesced) and the matching template words (consecutive LDS banks);
// 64 / ceil(n/4) rows are covered per pass.  The byte misalignment of the
// block is the same for every lane and row (pitch is a multiple of 4), so
// one v_alignbyte per word realigns it.

// sum over the m x n block at (y, x) of t * r on the unshifted uint8 values
// (v_dot4_u32_u8, no byte flips); the template is in LDS as raw words,
// n4 = ceil(n/4) per row, zero past column n.  Exact in 32 bits for
// m n <= 65536 (255^2 m n < 2^32).  Every lane returns the full sum.
__device__ __forceinline__ uint32_t wave_dot_tpl_u8(const uint32_t *__restrict__ tplw, int n4,
                                                    const uint8_t *__restrict__ img, int64_t pitch, int y, int x,
                                                    int m, int lane)
{
    uint32_t acc = 0;
    const uint32_t sh = (uint32_t)(x & 3);
    if (n4 <= kWave) {
        const int rp = kWave / n4;
        const int r0 = lane / n4, j = lane - r0 * n4;
        if (r0 < rp) {
            // image and template pointers advance by rp rows per step (the
            // pitch is a multiple of 4, so the aligned row starts differ by
            // whole words)
            const uint32_t *pr = (const uint32_t *)(img + ((((int64_t)y + r0) * pitch + x + 4 * j) & ~(int64_t)3));
            const int64_t step = (int64_t)rp * (pitch >> 2);
            const uint32_t *tp = tplw + r0 * n4 + j;
            const int tstep = rp * n4;
            const int nit = max(0, (m - r0 + rp - 1) / rp);  // rows r0, r0 + rp, ... below m
            // eight rows' loads issued together (clamped rows, no branch
            // around a load), then their products: one round trip per eight
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
        // rows wider than 64 words: the lanes walk each row 64 words at a time
        const int64_t pw = pitch >> 2;
        const uint32_t *row = (const uint32_t *)(img + (((int64_t)y * pitch + x) & ~(int64_t)3));
#pragma unroll 1
        for (int i = 0; i < m; i++, row += pw)
            for (int j = lane; j < n4; j += kWave)
                acc = __builtin_amdgcn_udot4(bytes_at(row[j + 1], row[j], sh), tplw[i * n4 + j], acc, false);
    }
    return (uint32_t)wave_sum((int)acc);
}

// sum over m x n of a' * b' for the block of A at (ya, xa) and of B at
// (yb, xb); bytes past column n of the last word are masked off.
__device__ __forceinline__ int wave_dot_img(const uint8_t *__restrict__ A, int64_t pa, int ya, int xa,
                                            const uint8_t *__restrict__ B, int64_t pb, int yb, int xb, int m, int n,
                                            int lane)
{
    const int n4 = (n + 3) >> 2;
    int acc = 0;
    // rows wider than 64 words are taken 64 words at a time
    for (int c0 = 0; c0 < n4; c0 += kWave) {
        const int nc = min(kWave, n4 - c0);
        const int rp = kWave / nc;
        const int r0 = lane / nc, j = c0 + lane - r0 * nc;
        const uint32_t mask = (j == n4 - 1 && (n & 3)) ? ((1u << (8 * (n & 3))) - 1u) : 0xffffffffu;
        if (r0 < rp) {
            int64_t a0 = (int64_t)ya * pa + xa + 4 * j;
            int64_t b0 = (int64_t)yb * pb + xb + 4 * j;
            uint32_t sa = (uint32_t)(xa & 3), sb = (uint32_t)(xb & 3);
            const uint32_t *ba = (const uint32_t *)(A + (a0 & ~(int64_t)3));
            const uint32_t *bb = (const uint32_t *)(B + (b0 & ~(int64_t)3));
            int64_t pwa = pa >> 2, pwb = pb >> 2;
#pragma unroll 4
            for (int i = r0; i < m; i += rp) {
                const uint32_t *pA = ba + (int64_t)i * pwa;
                const uint32_t *pB = bb + (int64_t)i * pwb;
                uint32_t va = flip4(bytes_at(pA[1], pA[0], sa)) & mask;
                uint32_t vb = flip4(bytes_at(pB[1], pB[0], sb));
                acc = dot4(va, vb, acc);
            }
        }
    }
    return wave_sum(acc);
}

// ---------------------------------------------------------------- MFMA operands and LDS strides

typedef int v4i __attribute__((ext_vector_type(4)));  // one int8 MFMA operand or accumulator tile

// Dword stride of one template row in the LDS ring: an odd number of 16-byte
// units, so the 16 lanes of a B-fragment read (16 templates, one row) fall
// on distinct banks.
__host__ __device__ inline int batch_tstride(int nw16) { return ((nw16 >> 2) & 1) ? nw16 : nw16 + 4; }

// Dword stride of one byte-shifted image row copy: 8 mod 16, so the 16 lanes
// of an A-fragment read (4 copies x 4 consecutive words, 2 dwords each) and
// the next 16 lanes (next row, 4 strides on) fall on distinct banks.
__host__ __device__ inline int batch_copy_stride(int ww) { return ww + ((8 - ww) & 15); }

// ---------------------------------------------------------------- address spaces

// Pointers read from a device-side table are generic to the compiler, which
// then emits flat accesses; those count on the LDS counter too, so a wait for
// LDS data would also wait for outstanding global loads.  Casting to the
// global address space keeps them global_load / global_store.
template <class T> __device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// Global loads and stores of the vector and record types (the cast applies to
// scalar types only).
__device__ __forceinline__ int2 ld_int2(const int2 *p)
{
    uint64_t v = *gptr((const uint64_t *)p);
    return make_int2((int)(uint32_t)v, (int)(uint32_t)(v >> 32));
}

// ---------------------------------------------------------------- best-location records

__device__ __forceinline__ void st_rec(RecPod *p, const RecPod &r)
{
    static_assert(sizeof(RecPod) % 8 == 0, "records are stored as 8-byte words");
    const uint64_t *w = (const uint64_t *)&r;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(RecPod) / 8); k++)
        gptr((uint64_t *)p)[k] = w[k];
}

__device__ __forceinline__ bool rec_better(double r1, int64_t l1, double r2, int64_t l2)
{
    return r1 > r2 || (r1 == r2 && l1 < l2);
}

__device__ __forceinline__ RecPod rec_empty()
{
    RecPod r;
    r.rho = -2.0;
    r.l = INT64_MAX;
    r.num = 0;
    r.dr = 0;
    r.r32max = -2.0f;
    r.valid = 0;
    r.n_elim = r.n_surv = r.n_window = 0;
    return r;
}

__device__ __forceinline__ void rec_merge(RecPod &a, const RecPod &b)
{
    float m = fmaxf(a.r32max, b.r32max);
    unsigned long long e = a.n_elim + b.n_elim, s = a.n_surv + b.n_surv, w = a.n_window + b.n_window;
    if (b.valid && (!a.valid || rec_better(b.rho, b.l, a.rho, a.l)))
        a = b;
    a.r32max = m;
    a.n_elim = e;
    a.n_surv = s;
    a.n_window = w;
}

// Streaming band selection: a candidate is evaluated in binary64 when its
// binary32 rho is within kEpsRho of the largest binary32 rho seen so far by
// this owner.  The running maximum only grows, so every candidate within the
// band of the final maximum is evaluated.
__device__ __forceinline__ void rec_take(RecPod &r, int64_t l, int64_t num, int64_t dt, int64_t dr)
{
    double rho = rho64(num, dt, dr);
    if (!r.valid || rec_better(rho, l, r.rho, r.l)) {
        r.rho = rho;
        r.l = l;
        r.num = num;
        r.dr = dr;
        r.valid = 1;
    }
}

// Out of line for the kernels that offer many values per thread (the
// binary64 evaluation stays out of their register budget).  The record goes
// in and out by value, so the caller's copy can stay in registers.
__device__ __noinline__ RecPod rec_offer_band(RecPod r, int64_t l, int64_t num, int64_t dt, int64_t dr)
{
    rec_take(r, l, num, dt, dr);
    return r;
}

__device__ __forceinline__ void rec_offer(RecPod &r, float r32, int64_t l, int64_t num, int64_t dt, int64_t dr)
{
    if (r32 >= r.r32max - kEpsRho)
        r = rec_offer_band(r, l, num, dt, dr);
    r.r32max = fmaxf(r.r32max, r32);
}

// The same, inlined: for kernels that offer a value or two per thread, so
// that the record stays in registers instead of private memory.
__device__ __forceinline__ void rec_offer_inline(RecPod &r, float r32, int64_t l, int64_t num, int64_t dt,
                                                 int64_t dr)
{
    if (r32 >= r.r32max - kEpsRho)
        rec_take(r, l, num, dt, dr);
    r.r32max = fmaxf(r.r32max, r32);
}

}  // namespace zts
