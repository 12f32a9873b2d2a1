/*
 * CPU oracle for exhaustive zero-mean NCC template search with transitive
 * elimination, Efficient Group Size (EGS) and OptA blur conditioning
 * (Mahmood, Mian, Owens, "Optimizing Auto-correlation for Fast Target Search
 * in Large Search Space", arXiv 1407.3535).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file.  It is used by the tests, by the package's smoke check and
 * by the benchmark's CPU-baseline leg, and by nothing else.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * Plain, slow and written to be checked by eye against the paper:
 *   - every sum is an int64 loop over the raw uint8 pixels (no shift, no
 *     blocking), every ratio is binary64 evaluated in the stated order;
 *   - build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Conventions.  Image I is p rows by q columns, row stride in bytes.  A
 * template t is m by n.  Location (y, x) is the top-left corner of the block
 * I[y..y+m-1][x..x+n-1]; valid locations are Ly = p-m+1 by Lx = q-n+1 and
 * the linear index is l = y*Lx + x.
 *
 * Canonical numbers.  For blocks a, b of the same size (mn pixels):
 *   N  = mn*sum(ab) - sum(a)*sum(b)        D_a = mn*sum(a^2) - sum(a)^2
 *   rho = (double)N / sqrt((double)D_a * (double)D_b)          (Eq. 1)
 *   s   = sqrt((double)(D_a*D_b - N^2) / ((double)D_a*(double)D_b))
 * with D_a*D_b - N^2 formed exactly in 128-bit integers.  rho is Eq. 1 with
 * the 1/mn factors cancelled; s is sqrt(1 - rho^2) computed without the
 * cancellation near |rho| = 1.  A block with zero variance has rho := 0 and
 * s := 1 (Eq. 1 is undefined there).
 *
 * Pinned by the CPU tests against numpy/scipy, closed forms (Eq. 2-4,
 * Eq. 28, Prop. 3.2's sqrt(1 - rho_th^2)), the Fig. 2 worked example and brute
 * force on tiny inputs.  Parity unpinned against the paper: the EGS choice of
 * start size and step (Alg. 2 leaves h0, w0, dh, dw open) and the OptA blur
 * schedule and stop rule (Alg. 3, no worked example); these follow the
 * readings stated at each function.
 */

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_SIZE (-2)
#define ORC_E_DEGENERATE (-3)
#define ORC_E_NOMEM (-11)

/* ------------------------------------------------------------------ */
/* Canonical scalars                                                   */
/* ------------------------------------------------------------------ */

/* Correlation coefficient, Eq. 1, from exact integers. */
double orc_rho(int64_t num, int64_t da, int64_t db)
{
    if (da == 0 || db == 0)
        return 0.0;
    return (double)num / sqrt((double)da * (double)db);
}

/* sqrt(1 - rho^2) of the same pair, from the exact 128-bit numerator. */
double orc_sin(int64_t num, int64_t da, int64_t db)
{
    if (da == 0 || db == 0)
        return 1.0;
    i128 numer = (i128)da * (i128)db - (i128)num * (i128)num;
    if (numer < 0)
        numer = 0; /* cannot happen: Cauchy-Schwarz */
    return sqrt((double)numer / ((double)da * (double)db));
}

/* Literal two-pass Eq. 1: means first, then centred sums. */
double orc_rho_twopass(const uint8_t *a, int64_t sa, const uint8_t *b, int64_t sb, int m, int n)
{
    double mu_a = 0.0, mu_b = 0.0;
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) {
            mu_a += a[i * sa + j];
            mu_b += b[i * sb + j];
        }
    mu_a /= (double)m * n;
    mu_b /= (double)m * n;
    double sab = 0.0, saa = 0.0, sbb = 0.0;
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) {
            double da = a[i * sa + j] - mu_a;
            double db = b[i * sb + j] - mu_b;
            sab += da * db;
            saa += da * da;
            sbb += db * db;
        }
    if (saa == 0.0 || sbb == 0.0)
        return 0.0;
    return sab / (sqrt(saa) * sqrt(sbb));
}

/* Transitive bounds on rho_to from rho_tc and rho_co, Eq. 2 and Eq. 3. */
void orc_transitive_bounds(double rtc, double rco, double *lb, double *ub)
{
    double g = sqrt((1.0 - rtc * rtc) * (1.0 - rco * rco));
    *ub = rtc * rco + g;
    *lb = rtc * rco - g;
}

/* Transitive gap, Eq. 4. */
double orc_transitive_gap(double rtc, double rco)
{
    return 2.0 * sqrt(1.0 - rtc * rtc) * sqrt(1.0 - rco * rco);
}

/* Blur-correlation threshold lambda: Eq. 28 (Prop. 4.3 with rho_to = rho_max),
 * evaluated in the printed order. */
double orc_lambda(double rho_th, double rho_max)
{
    double r = 1.0 + rho_th * rho_th * rho_max * rho_max - (rho_th * rho_th + rho_max * rho_max);
    if (r < 0.0)
        r = 0.0;
    return rho_th * rho_max + sqrt(r);
}

/* Upper bound on rho_to from three angles between mean-centred unit blocks:
 * A = angle(t, c), B = angle(c, o'), C = angle(o', o).  By the triangle
 * inequality on the sphere angle(t, o) >= |A - B| - C, so
 * rho_to <= cos(|A - B| - C) when |A - B| > C.  Each angle is given by its
 * (cos, sin) pair.  With C = 0 (rc = 1, sc = 0) the bound is exactly Eq. 2,
 * rho_tc*rho_co + s_tc*s_co.  Returns 0 and leaves *ub alone when no bound
 * below 1 exists (|A - B| <= C). */
int orc_ub_general(double ra, double sa, double rb, double sb, double rc, double sc, double *ub)
{
    double rab = ra * rb + sa * sb;     /* cos(A - B) */
    double sab = fabs(sa * rb - ra * sb); /* sin|A - B| */
    if (rab >= rc)
        return 0;
    *ub = rab * rc + sab * sc;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Block sums by direct loops                                          */
/* ------------------------------------------------------------------ */

static void block_sums(const uint8_t *img, int64_t st, int y, int x, int m, int n, int64_t *s, int64_t *s2)
{
    int64_t a = 0, b = 0;
    for (int i = 0; i < m; i++) {
        const uint8_t *row = img + (int64_t)(y + i) * st + x;
        for (int j = 0; j < n; j++) {
            a += row[j];
            b += (int64_t)row[j] * row[j];
        }
    }
    *s = a;
    *s2 = b;
}

static int64_t block_cross(const uint8_t *a, int64_t sa, int ya, int xa, const uint8_t *b, int64_t sb, int yb,
                           int xb, int m, int n)
{
    int64_t acc = 0;
    for (int i = 0; i < m; i++) {
        const uint8_t *ra = a + (int64_t)(ya + i) * sa + xa;
        const uint8_t *rb = b + (int64_t)(yb + i) * sb + xb;
        for (int j = 0; j < n; j++)
            acc += (int64_t)ra[j] * rb[j];
    }
    return acc;
}

static int64_t var_num(int64_t mn, int64_t s, int64_t s2) { return mn * s2 - s * s; }

/* Per-location sum, sum of squares and D = mn*sum(r^2) - sum(r)^2, direct loops. */
int orc_location_stats(const uint8_t *img, int p, int q, int64_t st, int m, int n, int64_t *S, int64_t *S2,
                       int64_t *D)
{
    if (!img || m < 1 || n < 1 || m > p || n > q)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t mn = (int64_t)m * n;
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            int64_t s, s2, l = (int64_t)y * Lx + x;
            block_sums(img, st, y, x, m, n, &s, &s2);
            if (S)
                S[l] = s;
            if (S2)
                S2[l] = s2;
            if (D)
                D[l] = var_num(mn, s, s2);
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Running sums (the paper's Run-Sum, section III-A and Alg. 3)        */
/* ------------------------------------------------------------------ */

/* Summed-area table of a p x q int64 array: R[(y)*(q+1)+x] = sum over rows < y, cols < x. */
static void run_sum(const int64_t *P, int p, int q, int64_t *R)
{
    for (int x = 0; x <= q; x++)
        R[x] = 0;
    for (int y = 0; y < p; y++) {
        int64_t row = 0;
        R[(int64_t)(y + 1) * (q + 1)] = 0;
        for (int x = 0; x < q; x++) {
            row += P[(int64_t)y * q + x];
            R[(int64_t)(y + 1) * (q + 1) + x + 1] = R[(int64_t)y * (q + 1) + x + 1] + row;
        }
    }
}

/* Sum over the m x n block at (y, x) from four table entries. */
static int64_t box(const int64_t *R, int q, int y, int x, int m, int n)
{
    int64_t w = q + 1;
    return R[(int64_t)(y + m) * w + x + n] - R[(int64_t)y * w + x + n] - R[(int64_t)(y + m) * w + x] +
           R[(int64_t)y * w + x];
}

/* Same statistics as orc_location_stats, through running sums of I and I*I. */
int orc_location_stats_rs(const uint8_t *img, int p, int q, int64_t st, int m, int n, int64_t *S, int64_t *S2,
                          int64_t *D)
{
    if (!img || m < 1 || n < 1 || m > p || n > q)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t mn = (int64_t)m * n;
    int64_t *P = malloc(sizeof(int64_t) * p * q);
    int64_t *R1 = malloc(sizeof(int64_t) * (p + 1) * (q + 1));
    int64_t *R2 = malloc(sizeof(int64_t) * (p + 1) * (q + 1));
    if (!P || !R1 || !R2) {
        free(P); free(R1); free(R2);
        return ORC_E_NOMEM;
    }
    for (int y = 0; y < p; y++)
        for (int x = 0; x < q; x++)
            P[(int64_t)y * q + x] = img[(int64_t)y * st + x];
    run_sum(P, p, q, R1);
    for (int y = 0; y < p; y++)
        for (int x = 0; x < q; x++) {
            int64_t v = img[(int64_t)y * st + x];
            P[(int64_t)y * q + x] = v * v;
        }
    run_sum(P, p, q, R2);
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            int64_t l = (int64_t)y * Lx + x;
            int64_t s = box(R1, q, y, x, m, n), s2 = box(R2, q, y, x, m, n);
            if (S)
                S[l] = s;
            if (S2)
                S2[l] = s2;
            if (D)
                D[l] = var_num(mn, s, s2);
        }
    free(P); free(R1); free(R2);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* A small parallel-for over an index range (pthreads)                 */
/* ------------------------------------------------------------------ */

typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi, int tid);

typedef struct {
    range_fn fn;
    void *ctx;
    int64_t lo, hi;
    int tid;
} range_job;

static void *range_thread(void *arg)
{
    range_job *j = arg;
    j->fn(j->ctx, j->lo, j->hi, j->tid);
    return NULL;
}

/* Runs fn over [0, count) split into nthreads contiguous chunks, chunk k on thread k. */
static void parallel_for(int64_t count, int nthreads, range_fn fn, void *ctx)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    if (count < nthreads)
        nthreads = count > 0 ? (int)count : 1;
    pthread_t th[256];
    range_job jobs[256];
    for (int k = 0; k < nthreads; k++) {
        jobs[k].fn = fn;
        jobs[k].ctx = ctx;
        jobs[k].lo = count * k / nthreads;
        jobs[k].hi = count * (k + 1) / nthreads;
        jobs[k].tid = k;
    }
    for (int k = 1; k < nthreads; k++)
        pthread_create(&th[k], NULL, range_thread, &jobs[k]);
    range_thread(&jobs[0]);
    for (int k = 1; k < nthreads; k++)
        pthread_join(th[k], NULL);
}

/* ------------------------------------------------------------------ */
/* C1: plain full search (Eq. 1 at every location)                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t y, x;
    double rho;
    int64_t num, den_t, den_r;
    int64_t n_locations, n_centres, n_eliminated, n_survivors, n_computed;
    int32_t group_h, group_w;
    double best0;
    int32_t best0_y, best0_x;
} orc_result;

typedef struct {
    int64_t l;
    double rho;
} best_rec;

/* Larger rho wins; equal rho goes to the smaller linear index. */
static void best_update(best_rec *b, int64_t l, double rho)
{
    if (b->l < 0 || rho > b->rho || (rho == b->rho && l < b->l)) {
        b->l = l;
        b->rho = rho;
    }
}

typedef struct {
    const uint8_t *img, *tpl;
    int64_t is, ts;
    int m, n, Lx;
    int64_t mn, st, st2, dt;
    int64_t *xs_map, *num_map, *dr_map;
    double *rho_map;
    best_rec best[256];
} full_ctx;

static void full_rows(void *vctx, int64_t lo, int64_t hi, int tid)
{
    full_ctx *c = vctx;
    best_rec b = {-1, 0.0};
    for (int64_t y = lo; y < hi; y++)
        for (int x = 0; x < c->Lx; x++) {
            int64_t l = y * c->Lx + x, s, s2;
            block_sums(c->img, c->is, (int)y, x, c->m, c->n, &s, &s2);
            int64_t xs = block_cross(c->tpl, c->ts, 0, 0, c->img, c->is, (int)y, x, c->m, c->n);
            int64_t dr = var_num(c->mn, s, s2);
            int64_t num = c->mn * xs - c->st * s;
            double rho = orc_rho(num, c->dt, dr);
            if (c->xs_map)
                c->xs_map[l] = xs;
            if (c->num_map)
                c->num_map[l] = num;
            if (c->dr_map)
                c->dr_map[l] = dr;
            if (c->rho_map)
                c->rho_map[l] = rho;
            best_update(&b, l, rho);
        }
    c->best[tid] = b;
}

static int template_stats(const uint8_t *tpl, int64_t ts, int m, int n, int64_t *st, int64_t *st2, int64_t *dt)
{
    block_sums(tpl, ts, 0, 0, m, n, st, st2);
    *dt = var_num((int64_t)m * n, *st, *st2);
    return *dt == 0 ? ORC_E_DEGENERATE : ORC_OK;
}

static void fill_best(orc_result *out, int64_t l, int Lx, double rho, int64_t num, int64_t dt, int64_t dr)
{
    out->y = (int32_t)(l / Lx);
    out->x = (int32_t)(l % Lx);
    out->rho = rho;
    out->num = num;
    out->den_t = dt;
    out->den_r = dr;
}

int orc_full_search(const uint8_t *img, int p, int q, int64_t is, const uint8_t *tpl, int m, int n, int64_t ts,
                    int nthreads, int64_t *xs_map, int64_t *num_map, int64_t *dr_map, double *rho_map,
                    orc_result *out)
{
    if (!img || !tpl || !out || m < 1 || n < 1)
        return ORC_E_ARG;
    if (m > p || n > q)
        return ORC_E_SIZE;
    full_ctx c;
    memset(&c, 0, sizeof c);
    c.img = img; c.tpl = tpl; c.is = is; c.ts = ts; c.m = m; c.n = n;
    c.Lx = q - n + 1;
    c.mn = (int64_t)m * n;
    int rc = template_stats(tpl, ts, m, n, &c.st, &c.st2, &c.dt);
    if (rc)
        return rc;
    c.xs_map = xs_map; c.num_map = num_map; c.dr_map = dr_map; c.rho_map = rho_map;
    int Ly = p - m + 1;
    if (nthreads > 256)
        nthreads = 256;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > Ly)
        nthreads = Ly;
    for (int k = 0; k < 256; k++)
        c.best[k].l = -1;
    parallel_for(Ly, nthreads, full_rows, &c);
    best_rec b = {-1, 0.0};
    for (int k = 0; k < nthreads; k++)
        if (c.best[k].l >= 0)
            best_update(&b, c.best[k].l, c.best[k].rho);
    int y = (int)(b.l / c.Lx), x = (int)(b.l % c.Lx);
    int64_t s, s2;
    block_sums(img, is, y, x, m, n, &s, &s2);
    int64_t xs = block_cross(tpl, ts, 0, 0, img, is, y, x, m, n);
    memset(out, 0, sizeof *out);
    fill_best(out, b.l, c.Lx, b.rho, c.mn * xs - c.st * s, c.dt, var_num(c.mn, s, s2));
    out->n_locations = (int64_t)Ly * c.Lx;
    out->n_computed = out->n_locations;
    out->group_h = out->group_w = 1;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Group tiling (Fig. 1)                                                */
/* ------------------------------------------------------------------ */

/* Groups of h x w locations tile the Ly x Lx grid from (0,0), row-major; the
 * last row and column of groups may be cut short.  A group with origin
 * (gy, gx) and true extent (hh, ww) has its centre at
 * (gy + (hh-1)/2, gx + (ww-1)/2). */
static void group_of(int Ly, int Lx, int h, int w, int y, int x, int *cy, int *cx)
{
    int gy = (y / h) * h, gx = (x / w) * w;
    int hh = Ly - gy < h ? Ly - gy : h;
    int ww = Lx - gx < w ? Lx - gx : w;
    *cy = gy + (hh - 1) / 2;
    *cx = gx + (ww - 1) / 2;
}

int64_t orc_centre_of(int Ly, int Lx, int h, int w, int64_t l)
{
    int cy, cx;
    group_of(Ly, Lx, h, w, (int)(l / Lx), (int)(l % Lx), &cy, &cx);
    return (int64_t)cy * Lx + cx;
}

int64_t orc_group_count(int Ly, int Lx, int h, int w)
{
    return (int64_t)((Ly + h - 1) / h) * ((Lx + w - 1) / w);
}

/* ------------------------------------------------------------------ */
/* Local auto-correlation of every location with its group centre      */
/* ------------------------------------------------------------------ */

/* Definition: N_co = mn*sum(r_c r_o) - S_c S_o by direct loops.  Outputs per
 * location l: num[l] = N_co, dc[l] = D_c, dov[l] = D_o (a centre pairs with
 * itself). */
int orc_autocorr_direct(const uint8_t *img, int p, int q, int64_t st, int m, int n, int h, int w, int64_t *num,
                        int64_t *dc, int64_t *dov)
{
    if (!img || m < 1 || n < 1 || h < 1 || w < 1)
        return ORC_E_ARG;
    if (m > p || n > q)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t mn = (int64_t)m * n;
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            int cy, cx;
            group_of(Ly, Lx, h, w, y, x, &cy, &cx);
            int64_t sc, sc2, so, so2, l = (int64_t)y * Lx + x;
            block_sums(img, st, cy, cx, m, n, &sc, &sc2);
            block_sums(img, st, y, x, m, n, &so, &so2);
            int64_t xco = block_cross(img, st, cy, cx, img, st, y, x, m, n);
            num[l] = mn * xco - sc * so;
            dc[l] = var_num(mn, sc, sc2);
            dov[l] = var_num(mn, so, so2);
        }
    return ORC_OK;
}

/* Alg. 1 (local auto-correlation): for every shift (sy, sx) a group member
 * can have from its centre, form the product image P = I * I(shifted), take
 * its running sum, and read the m x n box sum at every centre whose member at
 * that shift exists.  Shifts are centred on the group centre (the printed
 * one-sided loop indexes the block's far corner).  The box sums are then
 * normalised with the running-sum statistics of the two blocks. */
typedef struct {
    const uint8_t *img;
    int64_t st;
    int p, q, m, n, h, w, Ly, Lx;
    int sy0, sx0, nsx;
    const int64_t *S, *D;
    int64_t *num, *dc, *dov;
    int64_t **P, **R;
} lsa_ctx;

static void lsa_shifts(void *vctx, int64_t lo, int64_t hi, int tid)
{
    lsa_ctx *c = vctx;
    int64_t *P = c->P[tid], *R = c->R[tid];
    int64_t mn = (int64_t)c->m * c->n;
    for (int64_t k = lo; k < hi; k++) {
        int sy = c->sy0 + (int)(k / c->nsx), sx = c->sx0 + (int)(k % c->nsx);
        for (int y = 0; y < c->p; y++)
            for (int x = 0; x < c->q; x++) {
                int y2 = y + sy, x2 = x + sx;
                int64_t v = 0;
                if (y2 >= 0 && y2 < c->p && x2 >= 0 && x2 < c->q)
                    v = (int64_t)c->img[(int64_t)y * c->st + x] * c->img[(int64_t)y2 * c->st + x2];
                P[(int64_t)y * c->q + x] = v;
            }
        run_sum(P, c->p, c->q, R);
        for (int gy = 0; gy < c->Ly; gy += c->h)
            for (int gx = 0; gx < c->Lx; gx += c->w) {
                int cy, cx;
                group_of(c->Ly, c->Lx, c->h, c->w, gy, gx, &cy, &cx);
                int oy = cy + sy, ox = cx + sx;
                int hh = c->Ly - gy < c->h ? c->Ly - gy : c->h;
                int ww = c->Lx - gx < c->w ? c->Lx - gx : c->w;
                if (oy < gy || oy >= gy + hh || ox < gx || ox >= gx + ww)
                    continue;
                int64_t xco = box(R, c->q, cy, cx, c->m, c->n);
                int64_t lc = (int64_t)cy * c->Lx + cx, lo_ = (int64_t)oy * c->Lx + ox;
                c->num[lo_] = mn * xco - c->S[lc] * c->S[lo_];
                c->dc[lo_] = c->D[lc];
                c->dov[lo_] = c->D[lo_];
            }
    }
}

int orc_autocorr_lsa(const uint8_t *img, int p, int q, int64_t st, int m, int n, int h, int w, int nthreads,
                     int64_t *num, int64_t *dc, int64_t *dov)
{
    if (!img || m < 1 || n < 1 || h < 1 || w < 1)
        return ORC_E_ARG;
    if (m > p || n > q)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx;
    int64_t *S = malloc(sizeof(int64_t) * L), *D = malloc(sizeof(int64_t) * L);
    if (!S || !D) {
        free(S); free(D);
        return ORC_E_NOMEM;
    }
    orc_location_stats_rs(img, p, q, st, m, n, S, NULL, D);
    lsa_ctx c;
    memset(&c, 0, sizeof c);
    c.img = img; c.st = st; c.p = p; c.q = q; c.m = m; c.n = n; c.h = h; c.w = w; c.Ly = Ly; c.Lx = Lx;
    /* member offsets from the centre of a full group span [-(h-1)/2, h-1-(h-1)/2] */
    c.sy0 = -((h - 1) / 2);
    c.sx0 = -((w - 1) / 2);
    c.nsx = w;
    c.S = S; c.D = D; c.num = num; c.dc = dc; c.dov = dov;
    int64_t nshift = (int64_t)h * w;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > nshift)
        nthreads = (int)nshift;
    if (nthreads > 64)
        nthreads = 64;
    int64_t *Pb[64], *Rb[64];
    c.P = Pb; c.R = Rb;
    int ok = 1;
    for (int k = 0; k < nthreads; k++) {
        Pb[k] = malloc(sizeof(int64_t) * p * q);
        Rb[k] = malloc(sizeof(int64_t) * (p + 1) * (q + 1));
        if (!Pb[k] || !Rb[k])
            ok = 0;
    }
    if (ok)
        parallel_for(nshift, nthreads, lsa_shifts, &c);
    for (int k = 0; k < nthreads; k++) {
        free(Pb[k]); free(Rb[k]);
    }
    free(S); free(D);
    return ok ? ORC_OK : ORC_E_NOMEM;
}

/* ------------------------------------------------------------------ */
/* Transitive elimination search, two scans (sections II and VI)       */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint8_t *img, *tpl;
    int64_t is, ts, mn, st, dt;
    int m, n, Lx;
    const int64_t *S, *D;
} corr_ctx;

/* Canonical rho(t, r_l) and its exact N, by direct loops. */
static double corr_at(const corr_ctx *c, int64_t l, int64_t *num_out)
{
    int y = (int)(l / c->Lx), x = (int)(l % c->Lx);
    int64_t xs = block_cross(c->tpl, c->ts, 0, 0, c->img, c->is, y, x, c->m, c->n);
    int64_t num = c->mn * xs - c->st * c->S[l];
    if (num_out)
        *num_out = num;
    return orc_rho(num, c->dt, c->D[l]);
}

typedef struct {
    corr_ctx *cc;
    const int8_t *need; /* 1: compute this location */
    double *rho;
    int64_t *num;
} eval_ctx;

static void eval_rows(void *vctx, int64_t lo, int64_t hi, int tid)
{
    (void)tid;
    eval_ctx *e = vctx;
    for (int64_t l = lo; l < hi; l++)
        if (e->need[l])
            e->rho[l] = corr_at(e->cc, l, &e->num[l]);
}

/* Scan 1 computes rho_tc at every group centre and takes best0 = their
 * maximum (early high threshold, section VI; a centre with a flat block
 * counts with rho := 0, which is an attained value).  Scan 2 applies the
 * sufficient elimination condition (Eq. 5) to every other member with the
 * bound of Eq. 2 in its canonical form rho_tc*rho_co + s_tc*s_co, eliminating
 * strictly: UB < best0 - delta.  Members whose own block or whose centre
 * block is flat are never eliminated.  The answer is the best of the centres
 * and the survivors (ties to the smallest linear index).
 *
 * radius > 0 adds a refinement between the scans: every location within
 * radius (Chebyshev distance) of the best centre is matched too, and best0
 * becomes the best of the centres and that window (the localisation idea of
 * section IV-C used to raise the threshold; radius 0 is section VI as
 * printed).  Window locations count as computed.
 *
 * floor_ (detection semantics, section VII's threshold; -2 = off): the
 * elimination threshold is max(best0, floor_) - delta.  When the true maximum
 * reaches the floor the answer is unchanged; otherwise every eliminated
 * location lies below the floor and the answer is the best computed one.
 *
 * ac_num/ac_dc/ac_do: auto-correlation of every location with its centre
 * (orc_autocorr_*).  decision (nullable, L entries): 1 centre, 3 window,
 * 2 survivor, 0 eliminated. */
int orc_te_search(const uint8_t *img, int p, int q, int64_t is, const uint8_t *tpl, int m, int n, int64_t ts, int h,
                  int w, double delta, double floor_, int radius, const int64_t *ac_num, const int64_t *ac_dc,
                  const int64_t *ac_do, int nthreads, int8_t *decision, orc_result *out)
{
    if (!img || !tpl || !out || !ac_num || !ac_dc || !ac_do || h < 1 || w < 1)
        return ORC_E_ARG;
    if (m > p || n > q || m < 1 || n < 1)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx;
    corr_ctx c;
    c.img = img; c.tpl = tpl; c.is = is; c.ts = ts; c.m = m; c.n = n; c.Lx = Lx;
    c.mn = (int64_t)m * n;
    int64_t st2;
    int rc = template_stats(tpl, ts, m, n, &c.st, &st2, &c.dt);
    if (rc)
        return rc;
    int64_t *S = malloc(sizeof(int64_t) * L), *D = malloc(sizeof(int64_t) * L);
    int64_t *num = malloc(sizeof(int64_t) * L);
    double *rho = malloc(sizeof(double) * L);
    int8_t *need = malloc(L), *dec = malloc(L);
    if (!S || !D || !num || !rho || !need || !dec) {
        free(S); free(D); free(num); free(rho); free(need); free(dec);
        return ORC_E_NOMEM;
    }
    orc_location_stats_rs(img, p, q, is, m, n, S, NULL, D);
    c.S = S; c.D = D;
    eval_ctx e = {&c, need, rho, num};

    /* scan 1: group centres */
    memset(need, 0, L);
    for (int64_t l = 0; l < L; l++)
        if (orc_centre_of(Ly, Lx, h, w, l) == l)
            need[l] = 1;
    parallel_for(L, nthreads, eval_rows, &e);
    best_rec b0 = {-1, 0.0};
    int64_t n_centres = 0;
    for (int64_t l = 0; l < L; l++)
        if (need[l]) {
            n_centres++;
            best_update(&b0, l, rho[l]);
        }
    /* scan 2: elimination test on the other members */
    memcpy(dec, need, L); /* centres: 1, others 0 for now */
    int64_t n_elim = 0, n_surv = 0, n_win = 0;
    best_rec bt = b0;
    if (radius > 0) {
        int cy = (int)(b0.l / Lx), cx = (int)(b0.l % Lx);
        for (int y = cy - radius; y <= cy + radius; y++)
            for (int x = cx - radius; x <= cx + radius; x++) {
                if (y < 0 || y >= Ly || x < 0 || x >= Lx)
                    continue;
                int64_t l = (int64_t)y * Lx + x;
                if (dec[l] == 1)
                    continue;
                rho[l] = corr_at(&c, l, &num[l]);
                dec[l] = 3;
                n_win++;
                best_update(&bt, l, rho[l]);
            }
    }
    double thr = (floor_ > bt.rho ? floor_ : bt.rho) - delta;
    for (int64_t l = 0; l < L; l++) {
        if (dec[l] == 1 || dec[l] == 3)
            continue;
        int64_t lc = orc_centre_of(Ly, Lx, h, w, l);
        int keep = 1;
        if (D[l] != 0 && D[lc] != 0) {
            double rtc = orc_rho(num[lc], c.dt, D[lc]), stc = orc_sin(num[lc], c.dt, D[lc]);
            double rco = orc_rho(ac_num[l], ac_dc[l], ac_do[l]), sco = orc_sin(ac_num[l], ac_dc[l], ac_do[l]);
            double ub;
            if (orc_ub_general(rtc, stc, rco, sco, 1.0, 0.0, &ub) && ub < thr)
                keep = 0;
        }
        if (keep) {
            dec[l] = 2;
            n_surv++;
        } else {
            n_elim++;
        }
    }
    /* survivors */
    for (int64_t l = 0; l < L; l++)
        need[l] = dec[l] == 2;
    parallel_for(L, nthreads, eval_rows, &e);
    best_rec b = {-1, 0.0};
    for (int64_t l = 0; l < L; l++)
        if (dec[l])
            best_update(&b, l, rho[l]);
    memset(out, 0, sizeof *out);
    fill_best(out, b.l, Lx, b.rho, num[b.l], c.dt, D[b.l]);
    out->n_locations = L;
    out->n_centres = n_centres;
    out->n_eliminated = n_elim;
    out->n_survivors = n_surv;
    out->n_computed = n_centres + n_win + n_surv;
    out->group_h = h;
    out->group_w = w;
    out->best0 = bt.rho;
    out->best0_y = (int32_t)(b0.l / Lx);
    out->best0_x = (int32_t)(b0.l % Lx);
    if (decision)
        memcpy(decision, dec, L);
    free(S); free(D); free(num); free(rho); free(need); free(dec);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Blur-correlation: every block of J against the same block of I      */
/* ------------------------------------------------------------------ */

/* Alg. 3's P = J*I, S_oo = Run-Sum(P), with J's and I's own running sums:
 * num[l] = mn*sum(J I) - sum(J) sum(I), dj[l] = D_J, di[l] = D_I. */
int orc_blurcorr(const uint8_t *I, const uint8_t *J, int p, int q, int64_t st, int m, int n, int64_t *num,
                 int64_t *dj, int64_t *di)
{
    if (!I || !J || m < 1 || n < 1)
        return ORC_E_ARG;
    if (m > p || n > q)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx, mn = (int64_t)m * n;
    int64_t *SI = malloc(sizeof(int64_t) * L), *SJ = malloc(sizeof(int64_t) * L);
    int64_t *P = malloc(sizeof(int64_t) * p * q), *R = malloc(sizeof(int64_t) * (p + 1) * (q + 1));
    if (!SI || !SJ || !P || !R) {
        free(SI); free(SJ); free(P); free(R);
        return ORC_E_NOMEM;
    }
    orc_location_stats_rs(I, p, q, st, m, n, SI, NULL, di);
    orc_location_stats_rs(J, p, q, st, m, n, SJ, NULL, dj);
    for (int y = 0; y < p; y++)
        for (int x = 0; x < q; x++)
            P[(int64_t)y * q + x] = (int64_t)J[(int64_t)y * st + x] * I[(int64_t)y * st + x];
    run_sum(P, p, q, R);
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            int64_t l = (int64_t)y * Lx + x;
            num[l] = mn * box(R, q, y, x, m, n) - SJ[l] * SI[l];
        }
    free(SI); free(SJ); free(P); free(R);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Blur (Eq. 18) with integer weights                                  */
/* ------------------------------------------------------------------ */

/* Gaussian weights (Eq. 19, read with the minus sign and sigma the standard
 * deviation) on support [-d, d] with d = ceil(3 sigma), quantised to integers
 * summing to 256: floor of 256*g_j/sum(g), then one unit to the centre when
 * the remainder is odd, then one unit to each pair (j, -j) in order of
 * decreasing fractional part (ties to the smaller |j|).  taps[0..2d]. */
int orc_gauss_taps(double sigma, int32_t *taps, int cap, int *d_out)
{
    if (!(sigma > 0.0)) {
        if (cap < 1)
            return ORC_E_ARG;
        taps[0] = 256;
        *d_out = 0;
        return ORC_OK;
    }
    int d = (int)ceil(3.0 * sigma);
    if (2 * d + 1 > cap || d > 64)
        return ORC_E_ARG;
    double g[65], a[65], frac[65];
    int f[65];
    double total = 0.0;
    for (int j = 0; j <= d; j++)
        g[j] = exp(-(double)(j * j) / (2.0 * sigma * sigma));
    total = g[0];
    for (int j = 1; j <= d; j++)
        total += 2.0 * g[j];
    int sum = 0;
    for (int j = 0; j <= d; j++) {
        a[j] = 256.0 * g[j] / total;
        f[j] = (int)floor(a[j]);
        frac[j] = a[j] - f[j];
        sum += j == 0 ? f[j] : 2 * f[j];
    }
    int rem = 256 - sum;
    if (rem % 2) {
        f[0] += 1;
        rem -= 1;
    }
    int used[65] = {0};
    while (rem >= 2) {
        int pick = -1;
        for (int j = 1; j <= d; j++)
            if (!used[j] && (pick < 0 || frac[j] > frac[pick]))
                pick = j;
        if (pick < 0)
            break;
        used[pick] = 1;
        f[pick] += 1;
        rem -= 2;
    }
    f[0] += rem;
    for (int j = -d; j <= d; j++)
        taps[j + d] = f[j < 0 ? -j : j];
    *d_out = d;
    return ORC_OK;
}

/* 2-D blur with the separable weights w_i * w_j on [-d, d]^2, borders clamped
 * to the nearest edge pixel, rounded half up:  out = (V + T/2) / T  with
 * T = (sum of taps)^2.  Written as the plain double sum over the support. */
int orc_blur(const uint8_t *src, int p, int q, int64_t st, const int32_t *taps, int d, uint8_t *dst, int64_t dst_st)
{
    if (!src || !dst || !taps || d < 0)
        return ORC_E_ARG;
    int64_t tsum = 0;
    for (int j = 0; j <= 2 * d; j++)
        tsum += taps[j];
    int64_t T = tsum * tsum;
    for (int y = 0; y < p; y++)
        for (int x = 0; x < q; x++) {
            int64_t V = 0;
            for (int i = -d; i <= d; i++) {
                int yy = y + i < 0 ? 0 : (y + i >= p ? p - 1 : y + i);
                for (int j = -d; j <= d; j++) {
                    int xx = x + j < 0 ? 0 : (x + j >= q ? q - 1 : x + j);
                    V += (int64_t)taps[i + d] * taps[j + d] * src[(int64_t)yy * st + xx];
                }
            }
            dst[(int64_t)y * dst_st + x] = (uint8_t)((V + T / 2) / T);
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Revert (Alg. 3 copy-back), repeated to a fixpoint                    */
/* ------------------------------------------------------------------ */

/* A location violates when its blocks in J and I are not both non-flat or
 * when R_oo = rho(J block, I block) < lambda (Eq. 28).  Every pixel covered
 * by a violating block is copied back from I.  Copying back can lower the
 * correlation of an overlapping block, so the test is repeated until no
 * covered pixel differs from I.  Returns the number of passes that changed
 * pixels and the number of pixels changed. */
int orc_revert(const uint8_t *I, uint8_t *J, int p, int q, int64_t st, int m, int n, double lambda, int *passes,
               int64_t *reverted)
{
    if (!I || !J)
        return ORC_E_ARG;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx;
    int64_t *num = malloc(sizeof(int64_t) * L), *dj = malloc(sizeof(int64_t) * L),
            *di = malloc(sizeof(int64_t) * L);
    uint8_t *viol = malloc(L), *mask = malloc((size_t)p * q);
    if (!num || !dj || !di || !viol || !mask) {
        free(num); free(dj); free(di); free(viol); free(mask);
        return ORC_E_NOMEM;
    }
    *passes = 0;
    *reverted = 0;
    for (;;) {
        orc_blurcorr(I, J, p, q, st, m, n, num, dj, di);
        for (int64_t l = 0; l < L; l++)
            viol[l] = (dj[l] == 0 || di[l] == 0) ? 1 : (orc_rho(num[l], dj[l], di[l]) < lambda);
        memset(mask, 0, (size_t)p * q);
        for (int y = 0; y < Ly; y++)
            for (int x = 0; x < Lx; x++)
                if (viol[(int64_t)y * Lx + x])
                    for (int i = 0; i < m; i++)
                        memset(mask + (int64_t)(y + i) * q + x, 1, n);
        int64_t changed = 0;
        for (int y = 0; y < p; y++)
            for (int x = 0; x < q; x++)
                if (mask[(int64_t)y * q + x] && J[(int64_t)y * st + x] != I[(int64_t)y * st + x]) {
                    J[(int64_t)y * st + x] = I[(int64_t)y * st + x];
                    changed++;
                }
        if (changed == 0)
            break;
        (*passes)++;
        *reverted += changed;
    }
    free(num); free(dj); free(di); free(viol); free(mask);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* EGS (Alg. 2, Eq. 15-17)                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t h, w;
    int64_t cc, cr, ct;
    int32_t accepted;
} orc_egs_step;

/* Retained-location count for group size (h, w).
 *
 * estimate 0 (Eq. 15 via Prop. 3.2): a member is retained when
 * rho_co < sqrt(1 - rho_th^2).  Members with a flat block or a flat centre
 * count as retained.  With the blur-correlation arrays (c_*) given, every
 * location o of the searched image J (centres included) is counted with the
 * angle to its original block added: retained when cos(B + C) < thr,
 * B = angle(centre, o in J), C = angle(o in J, o in I), i.e.
 * rho_B rho_C - s_B s_C < thr; flat blocks in J or I count as retained.
 *
 * estimate 1 (Prop. 3.1, Eq. 7, both roots of Eq. 8): the template is
 * assumed to correlate rho_tc with every group centre.  A member is
 * eliminated when the bound of Eq. 2 through that centre is at most the
 * threshold, rho_tc rho_co + s_tc s_co <= rho_th, which holds above the
 * upper root and below the lower root of Eq. 8; otherwise it is retained.
 * With blur arrays the angle C to the original block is added (every
 * location, centres included, with B = 0 at a centre): the bound is
 * cos(|A - B| - C), A = acos(rho_tc), and no bound (retained) when
 * |A - B| <= C.  Flat blocks count as retained. */
static int64_t retained_count(int Ly, int Lx, int h, int w, const int64_t *num, const int64_t *dc,
                              const int64_t *dov, const int64_t *c_num, const int64_t *c_dj, const int64_t *c_di,
                              double rho_th, int estimate, double rho_tc)
{
    int64_t L = (int64_t)Ly * Lx, cr = 0;
    double thr = sqrt(1.0 - rho_th * rho_th);
    double ra = rho_tc, sa = sqrt(1.0 - rho_tc * rho_tc);
    for (int64_t l = 0; l < L; l++) {
        int is_centre = orc_centre_of(Ly, Lx, h, w, l) == l;
        if (!c_num) {
            if (is_centre)
                continue;
            if (dc[l] == 0 || dov[l] == 0) {
                cr++;
                continue;
            }
            double rb = orc_rho(num[l], dc[l], dov[l]);
            if (estimate == 0) {
                if (rb < thr)
                    cr++;
            } else {
                double sb = orc_sin(num[l], dc[l], dov[l]), ub;
                if (!orc_ub_general(ra, sa, rb, sb, 1.0, 0.0, &ub) || ub > rho_th)
                    cr++;
            }
        } else {
            if (dc[l] == 0 || dov[l] == 0 || c_dj[l] == 0 || c_di[l] == 0) {
                cr++;
                continue;
            }
            double rb = orc_rho(num[l], dc[l], dov[l]), sb = orc_sin(num[l], dc[l], dov[l]);
            double rc = orc_rho(c_num[l], c_dj[l], c_di[l]), sc = orc_sin(c_num[l], c_dj[l], c_di[l]);
            if (estimate == 0) {
                if (rb * rc - sb * sc < thr)
                    cr++;
            } else {
                double ub;
                if (!orc_ub_general(ra, sa, rb, sb, rc, sc, &ub) || ub > rho_th)
                    cr++;
            }
        }
    }
    return cr;
}

/* Greedy descent of the total cost c_t = mn (c_c + c_r) of Eq. 16 over
 * group sizes (Alg. 2, objective Eq. 17), c_c the exact number of groups.
 * The start cost is mn*L (every location a centre, group size 1x1); the
 * first candidate is (h0, w0).
 *
 * shape 0 (Alg. 2 as printed): the next candidate is (h + dh, w + dw), tried
 * while the cost fell by more than xi times the previous cost.
 * shape 1 (groups need not be square): from the last accepted (h, w) the
 * candidates (h + dh, w), (h, w + dw) and (h + dh, w + dw) within the caps
 * are all evaluated and the cheapest (first listed on ties) is accepted when
 * it lowers the cost by more than xi times the previous cost.
 *
 * Sizes are capped at hmax and at the location grid.  Returns the last
 * accepted size (1x1 if none); the trace lists every evaluated candidate,
 * marking the ones accepted. */
int orc_egs(const uint8_t *img, int p, int q, int64_t st, int m, int n, int h0, int w0, int dh, int dw, int hmax,
            double rho_th, double xi, const int64_t *c_num, const int64_t *c_dj, const int64_t *c_di, int estimate,
            double rho_tc, int shape, int nthreads, orc_egs_step *trace, int trace_cap, int *ntrace, int *he,
            int *we, int64_t *cost)
{
    if (!img || m < 1 || n < 1 || h0 < 1 || w0 < 1 || dh < 0 || dw < 0 || (dh == 0 && dw == 0) ||
        estimate < 0 || estimate > 1 || shape < 0 || shape > 1 || !(rho_tc > -1.0 && rho_tc < 1.0))
        return ORC_E_ARG;
    if (m > p || n > q)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx, mn = (int64_t)m * n;
    int64_t *num = malloc(sizeof(int64_t) * L), *dc = malloc(sizeof(int64_t) * L),
            *dov = malloc(sizeof(int64_t) * L);
    if (!num || !dc || !dov) {
        free(num); free(dc); free(dov);
        return ORC_E_NOMEM;
    }
    int64_t prev = mn * L;
    int bh = 1, bw = 1, k = 0, rc = ORC_OK;
    for (int first = 1;; first = 0) {
        int ch[3], cw[3], nc = 0;
        if (first) {
            ch[0] = h0; cw[0] = w0; nc = 1;
        } else if (shape == 0) {
            ch[0] = bh + dh; cw[0] = bw + dw; nc = 1;
        } else {
            int cand[3][2] = {{bh + dh, bw}, {bh, bw + dw}, {bh + dh, bw + dw}};
            for (int i = 0; i < 3; i++) {
                int dup = cand[i][0] == bh && cand[i][1] == bw;
                for (int j = 0; j < nc; j++)
                    dup |= ch[j] == cand[i][0] && cw[j] == cand[i][1];
                if (!dup) {
                    ch[nc] = cand[i][0]; cw[nc] = cand[i][1]; nc++;
                }
            }
        }
        int best = -1, best_h = 0, best_w = 0;
        int64_t best_ct = 0;
        for (int i = 0; i < nc; i++) {
            int h = ch[i], w = cw[i];
            if (h > hmax || w > hmax || h > Ly || w > Lx)
                continue;
            rc = orc_autocorr_lsa(img, p, q, st, m, n, h, w, nthreads, num, dc, dov);
            if (rc)
                goto done;
            int64_t cc = orc_group_count(Ly, Lx, h, w);
            int64_t cr = retained_count(Ly, Lx, h, w, num, dc, dov, c_num, c_dj, c_di, rho_th, estimate, rho_tc);
            int64_t ct = mn * (cc + cr);
            if (trace && k < trace_cap) {
                trace[k].h = h; trace[k].w = w; trace[k].cc = cc; trace[k].cr = cr; trace[k].ct = ct;
                trace[k].accepted = 0;
            }
            if (best < 0 || ct < best_ct) {
                best = k;
                best_ct = ct;
                best_h = h;
                best_w = w;
            }
            k++;
        }
        if (best < 0)
            break;
        if (!((double)(prev - best_ct) > xi * (double)prev))
            break;
        if (trace && best < trace_cap)
            trace[best].accepted = 1;
        bh = best_h;
        bw = best_w;
        prev = best_ct;
    }
done:
    if (rc == ORC_OK) {
        if (ntrace)
            *ntrace = k;
        *he = bh;
        *we = bw;
        *cost = prev;
    }
    free(num); free(dc); free(dov);
    return rc;
}

/* ------------------------------------------------------------------ */
/* OptA (Alg. 3)                                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    double rho_th, rho_max, xi;
    int32_t h0, w0, dh, dw, hmax;
    int32_t blur_kind; /* 0: the paper's W = {1,4,10,4,1}/20 per axis; 1: Gaussian schedule */
    double sigma_step, sigma_max;
    int32_t max_iters;
    int32_t nthreads;
    int32_t paper;    /* 1: Alg. 3 as printed: EGS on each blurred image from its own
                         auto-correlation (Prop. 3.2, no angle to the original) */
    int32_t estimate; /* EGS retention estimate (orc_egs) */
    double rho_tc;
    int32_t shape;    /* EGS group-size ascent (orc_egs) */
    double accept_xi; /* Alg. 3's acceptance margin: an iterate is kept when the cost fell by
                         more than accept_xi times the new cost (0.005 in the paper; a negative
                         value keeps iterates whose cost rose by less than that fraction) */
} orc_opta_params;

typedef struct {
    int32_t k, d, passes, h, w, accepted;
    double sigma;
    int64_t reverted, cost;
} orc_opta_step;

/* Iterate: blur the last accepted image (Eq. 18), copy back every block
 * whose blur correlation falls below lambda (Eq. 28) until none does, and
 * re-run EGS warm-started at the current group size.  The iterate is
 * accepted when the estimated cost fell by more than accept_xi times the new
 * cost;
 * otherwise, or when the blur schedule ends, stop and return the last
 * accepted image.
 *
 * EGS counts: with paper = 0 (the exact search's conditioning) every
 * location is counted with the angle to its original block added (the
 * search bounds original locations through the blurred ones); with
 * paper = 1 each EGS call sees only the blurred image and its own
 * auto-correlation, as Alg. 3 prints it (the paper's search runs on the
 * blurred image).
 *
 * Blur schedule: kind 0 applies the paper's W every iteration; kind 1
 * applies a Gaussian of standard deviation sigma_step*sqrt(2k-1) at
 * iteration k, so unreverted pixels carry a total of sigma_step*k, up to
 * sigma_max.  *radius: sum of the supports d of the accepted iterations,
 * capped at 8 (the localisation window of section IV-C). */
int orc_opta(const uint8_t *I, int p, int q, int64_t st, int m, int n, const orc_opta_params *pr, uint8_t *out,
             orc_opta_step *trace, int cap, int *ntrace, int *he, int *we, int64_t *cost, int *radius)
{
    if (!I || !out || !pr)
        return ORC_E_ARG;
    if (m > p || n > q || m < 1 || n < 1)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx;
    double lambda = orc_lambda(pr->rho_th, pr->rho_max);
    uint8_t *cur = malloc((size_t)p * q), *J = malloc((size_t)p * q), *Ic = malloc((size_t)p * q);
    int64_t *cn = malloc(sizeof(int64_t) * L), *cj = malloc(sizeof(int64_t) * L), *ci = malloc(sizeof(int64_t) * L);
    if (!cur || !J || !Ic || !cn || !cj || !ci) {
        free(cur); free(J); free(Ic); free(cn); free(cj); free(ci);
        return ORC_E_NOMEM;
    }
    for (int y = 0; y < p; y++) {
        memcpy(Ic + (int64_t)y * q, I + (int64_t)y * st, q);
        memcpy(cur + (int64_t)y * q, I + (int64_t)y * st, q);
    }
    const int with_c = !pr->paper;
    if (with_c)
        orc_blurcorr(Ic, cur, p, q, q, m, n, cn, cj, ci);
    int h, w, nt, rad = 0;
    int64_t c_prev;
    int rc = orc_egs(cur, p, q, q, m, n, pr->h0, pr->w0, pr->dh, pr->dw, pr->hmax, pr->rho_th, pr->xi,
                     with_c ? cn : NULL, with_c ? cj : NULL, with_c ? ci : NULL, pr->estimate, pr->rho_tc,
                     pr->shape, pr->nthreads, NULL, 0, &nt, &h, &w, &c_prev);
    int k = 0;
    if (trace && cap > 0) {
        memset(&trace[0], 0, sizeof trace[0]);
        trace[0].h = h; trace[0].w = w; trace[0].cost = c_prev; trace[0].accepted = 1;
    }
    k = 1;
    for (int it = 1; rc == 0; it++) {
        int32_t taps[129];
        int d;
        double sigma;
        if (pr->blur_kind == 0) {
            if (it > pr->max_iters)
                break;
            static const int32_t W[5] = {1, 4, 10, 4, 1};
            memcpy(taps, W, sizeof W);
            d = 2;
            sigma = 0.0;
        } else {
            if (pr->sigma_step * it > pr->sigma_max + 1e-9 || it > pr->max_iters)
                break;
            sigma = pr->sigma_step * sqrt(2.0 * it - 1.0);
            rc = orc_gauss_taps(sigma, taps, 129, &d);
            if (rc)
                break;
        }
        orc_blur(cur, p, q, q, taps, d, J, q);
        int passes;
        int64_t reverted;
        rc = orc_revert(Ic, J, p, q, q, m, n, lambda, &passes, &reverted);
        if (rc)
            break;
        if (with_c) {
            rc = orc_blurcorr(Ic, J, p, q, q, m, n, cn, cj, ci);
            if (rc)
                break;
        }
        int h2, w2;
        int64_t c_new;
        rc = orc_egs(J, p, q, q, m, n, h, w, pr->dh, pr->dw, pr->hmax, pr->rho_th, pr->xi, with_c ? cn : NULL,
                     with_c ? cj : NULL, with_c ? ci : NULL, pr->estimate, pr->rho_tc, pr->shape, pr->nthreads,
                     NULL, 0, &nt, &h2, &w2, &c_new);
        if (rc)
            break;
        int accept = (double)(c_prev - c_new) > pr->accept_xi * (double)c_new;
        if (trace && k < cap) {
            trace[k].k = it; trace[k].d = d; trace[k].sigma = sigma; trace[k].passes = passes;
            trace[k].reverted = reverted; trace[k].h = h2; trace[k].w = w2; trace[k].cost = c_new;
            trace[k].accepted = accept;
        }
        k++;
        if (!accept)
            break;
        memcpy(cur, J, (size_t)p * q);
        h = h2;
        w = w2;
        c_prev = c_new;
        rad += d;
    }
    if (rc == 0) {
        for (int y = 0; y < p; y++)
            memcpy(out + (int64_t)y * q, cur + (int64_t)y * q, q);
        *he = h;
        *we = w;
        *cost = c_prev;
        *radius = rad > 8 ? 8 : rad;
        if (ntrace)
            *ntrace = k;
    }
    free(cur); free(J); free(Ic); free(cn); free(cj); free(ci);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Exact search through the conditioned image                          */
/* ------------------------------------------------------------------ */

/* Scan 1 matches the template against the group centres of the blurred
 * image J.  The best blurred centre is refined on the original image over a
 * (2r+1)^2 window around it (the localisation stage of section IV-C); the
 * best original rho found there is the threshold.  Every other original
 * location o is then bounded through its blurred centre and its own blurred
 * block: angle(t, o) >= |A - B| - C with A = angle(t, centre in J),
 * B = angle(centre in J, o in J), C = angle(o in J, o in I) (Eq. 2 and
 * Prop. 4.3 are the cosine forms of these angle inequalities).  Locations
 * whose bound falls strictly below threshold - delta are skipped; the rest
 * are matched on I, so the answer is the exact full-search answer.
 *
 * floor_: as in orc_te_search.
 * b_*: auto-correlation of J (every location with its J-group centre).
 * c_*: blur correlation (o in J vs o in I).  decision: 1 window, 2 survivor,
 * 0 eliminated.  n_centres counts the blurred centres matched. */
int orc_opta_search(const uint8_t *I, const uint8_t *J, int p, int q, int64_t st, const uint8_t *tpl, int m, int n,
                    int64_t ts, int h, int w, int radius, double delta, double floor_, const int64_t *b_num,
                    const int64_t *b_dc,
                    const int64_t *b_do, const int64_t *c_num, const int64_t *c_dj, const int64_t *c_di,
                    int nthreads, int8_t *decision, orc_result *out)
{
    if (!I || !J || !tpl || !out || !b_num || !b_dc || !b_do || !c_num || !c_dj || !c_di || h < 1 || w < 1 ||
        radius < 0)
        return ORC_E_ARG;
    if (m > p || n > q || m < 1 || n < 1)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    int64_t L = (int64_t)Ly * Lx;
    corr_ctx ci_, cj_;
    int64_t st2;
    ci_.img = I; ci_.tpl = tpl; ci_.is = st; ci_.ts = ts; ci_.m = m; ci_.n = n; ci_.Lx = Lx;
    ci_.mn = (int64_t)m * n;
    int rc = template_stats(tpl, ts, m, n, &ci_.st, &st2, &ci_.dt);
    if (rc)
        return rc;
    cj_ = ci_;
    cj_.img = J;
    int64_t *SI = malloc(sizeof(int64_t) * L), *DI = malloc(sizeof(int64_t) * L);
    int64_t *SJ = malloc(sizeof(int64_t) * L), *DJ = malloc(sizeof(int64_t) * L);
    int64_t *numJ = malloc(sizeof(int64_t) * L), *numI = malloc(sizeof(int64_t) * L);
    double *rhoJ = malloc(sizeof(double) * L), *rhoI = malloc(sizeof(double) * L);
    int8_t *need = malloc(L), *dec = malloc(L);
    if (!SI || !DI || !SJ || !DJ || !numJ || !numI || !rhoJ || !rhoI || !need || !dec) {
        free(SI); free(DI); free(SJ); free(DJ); free(numJ); free(numI); free(rhoJ); free(rhoI);
        free(need); free(dec);
        return ORC_E_NOMEM;
    }
    orc_location_stats_rs(I, p, q, st, m, n, SI, NULL, DI);
    orc_location_stats_rs(J, p, q, st, m, n, SJ, NULL, DJ);
    ci_.S = SI; ci_.D = DI;
    cj_.S = SJ; cj_.D = DJ;

    /* scan 1 on the blurred centres */
    memset(need, 0, L);
    int64_t n_centres = 0;
    for (int64_t l = 0; l < L; l++)
        if (orc_centre_of(Ly, Lx, h, w, l) == l) {
            need[l] = 1;
            n_centres++;
        }
    eval_ctx ej = {&cj_, need, rhoJ, numJ};
    parallel_for(L, nthreads, eval_rows, &ej);
    best_rec bj = {-1, 0.0};
    for (int64_t l = 0; l < L; l++)
        if (need[l])
            best_update(&bj, l, rhoJ[l]);

    /* localisation window on the original image */
    int cy = (int)(bj.l / Lx), cx = (int)(bj.l % Lx);
    memset(dec, 0, L);
    best_rec bw = {-1, 0.0};
    for (int y = cy - radius; y <= cy + radius; y++)
        for (int x = cx - radius; x <= cx + radius; x++) {
            if (y < 0 || y >= Ly || x < 0 || x >= Lx)
                continue;
            int64_t l = (int64_t)y * Lx + x;
            rhoI[l] = corr_at(&ci_, l, &numI[l]);
            dec[l] = 1;
            best_update(&bw, l, rhoI[l]);
        }
    double thr = (floor_ > bw.rho ? floor_ : bw.rho) - delta;

    /* scan 2 over every other original location */
    int64_t n_surv = 0, n_elim = 0, n_win = 0;
    for (int64_t l = 0; l < L; l++) {
        if (dec[l] == 1) {
            n_win++;
            continue;
        }
        int64_t lc = orc_centre_of(Ly, Lx, h, w, l);
        int keep = 1;
        if (DI[l] != 0 && b_dc[l] != 0 && b_do[l] != 0 && c_dj[l] != 0 && c_di[l] != 0) {
            double ra = orc_rho(numJ[lc], cj_.dt, DJ[lc]), sa = orc_sin(numJ[lc], cj_.dt, DJ[lc]);
            double rb = orc_rho(b_num[l], b_dc[l], b_do[l]), sb = orc_sin(b_num[l], b_dc[l], b_do[l]);
            double rcc = orc_rho(c_num[l], c_dj[l], c_di[l]), scc = orc_sin(c_num[l], c_dj[l], c_di[l]);
            double ub;
            if (orc_ub_general(ra, sa, rb, sb, rcc, scc, &ub) && ub < thr)
                keep = 0;
        }
        if (keep) {
            dec[l] = 2;
            n_surv++;
        } else {
            n_elim++;
        }
    }
    for (int64_t l = 0; l < L; l++)
        need[l] = dec[l] == 2;
    eval_ctx ei = {&ci_, need, rhoI, numI};
    parallel_for(L, nthreads, eval_rows, &ei);
    best_rec b = {-1, 0.0};
    for (int64_t l = 0; l < L; l++)
        if (dec[l])
            best_update(&b, l, rhoI[l]);
    memset(out, 0, sizeof *out);
    fill_best(out, b.l, Lx, b.rho, numI[b.l], ci_.dt, DI[b.l]);
    out->n_locations = L;
    out->n_centres = n_centres;
    out->n_eliminated = n_elim;
    out->n_survivors = n_surv;
    out->n_computed = n_win + n_surv;
    out->group_h = h;
    out->group_w = w;
    out->best0 = bw.rho;
    out->best0_y = (int32_t)(bj.l / Lx);
    out->best0_x = (int32_t)(bj.l % Lx);
    if (decision)
        memcpy(decision, dec, L);
    free(SI); free(DI); free(SJ); free(DJ); free(numJ); free(numI); free(rhoJ); free(rhoI);
    free(need); free(dec);
    return ORC_OK;
}

/* The localisation stage of section IV-C: the template is matched on `img`
 * at every location within Chebyshev distance `radius` of (cy, cx), clipped
 * to the location grid, by the plain definition (Eq. 1 through C1's exact
 * sums); the answer is the best of them, ties to the smaller linear index.
 * n_computed = the number of matched locations. */
int orc_window_search(const uint8_t *img, int p, int q, int64_t is, const uint8_t *tpl, int m, int n, int64_t ts,
                      int cy, int cx, int radius, orc_result *out)
{
    if (!img || !tpl || !out || radius < 0)
        return ORC_E_ARG;
    if (m > p || n > q || m < 1 || n < 1)
        return ORC_E_SIZE;
    int Ly = p - m + 1, Lx = q - n + 1;
    if (cy < 0 || cy >= Ly || cx < 0 || cx >= Lx)
        return ORC_E_ARG;
    int64_t st, st2, dt;
    int rc = template_stats(tpl, ts, m, n, &st, &st2, &dt);
    if (rc)
        return rc;
    const int64_t mn = (int64_t)m * n;
    memset(out, 0, sizeof *out);
    best_rec b = {-1, 0.0};
    int64_t bnum = 0, bdr = 0, cnt = 0;
    for (int y = cy - radius; y <= cy + radius; y++)
        for (int x = cx - radius; x <= cx + radius; x++) {
            if (y < 0 || y >= Ly || x < 0 || x >= Lx)
                continue;
            int64_t s, s2;
            block_sums(img, is, y, x, m, n, &s, &s2);
            int64_t dr = mn * s2 - s * s;
            int64_t num = mn * block_cross(tpl, ts, 0, 0, img, is, y, x, m, n) - st * s;
            double r = orc_rho(num, dt, dr);
            int64_t l = (int64_t)y * Lx + x;
            best_rec prev = b;
            best_update(&b, l, r);
            if (b.l != prev.l) {
                bnum = num;
                bdr = dr;
            }
            cnt++;
        }
    fill_best(out, b.l, Lx, b.rho, bnum, dt, bdr);
    out->n_locations = (int64_t)Ly * Lx;
    out->n_computed = cnt;
    out->group_h = out->group_w = 1;
    return ORC_OK;
}
