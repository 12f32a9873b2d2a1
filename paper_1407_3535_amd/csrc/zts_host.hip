// Host side of libzts: context, resident images, preparation (group size by
// EGS, OptA conditioning), query and batched-launch orchestration, and the
// synchronous entry points of zts.h.  The serving loop (submit / poll / wait)
// is in zts_serve.hip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "zts_runtime.h"

namespace zts {

// ------------------------------------------------------------------ errors and buffers

void hip_check_at(hipError_t e, const char *file, int line)
{
    if (e != hipSuccess) {
        if (std::getenv("ZTS_DEBUG"))
            std::fprintf(stderr, "zts: HIP error %d (%s) at %s:%d\n", (int)e, hipGetErrorString(e), file, line);
        throw ZtsError{ZTS_E_DEVICE};
    }
}

thread_local std::unique_lock<std::mutex> *t_ctx_lock = nullptr;

// Set while this thread builds preparation buffers that no other thread can
// reach yet (they enter the context's maps when the preparation ends): their
// device allocations are then made with the context lock released.
static thread_local bool t_alloc_unlocked = false;

struct AllocUnlockedScope {
    bool prev;
    AllocUnlockedScope() : prev(t_alloc_unlocked) { t_alloc_unlocked = true; }
    ~AllocUnlockedScope() { t_alloc_unlocked = prev; }
};

// Takes prep_mu for a thread that holds the context lock (through its
// CtxLockScope): the context lock is released first and taken again after,
// so the lock order is always prep_mu, then mu.
std::unique_lock<std::mutex> take_prep_lock(Ctx *c)
{
    std::unique_lock<std::mutex> *lk = t_ctx_lock;
    if (!lk || !lk->owns_lock())
        throw ZtsError{ZTS_E_DEVICE};  // every caller holds the context lock through a CtxLockScope
    std::unique_lock<std::mutex> plk(c->prep_mu, std::defer_lock);
    lk->unlock();
    try {
        plk.lock();
    } catch (...) {
        lk->lock();
        throw;
    }
    lk->lock();
    return plk;
}

void DBuf::reset()
{
    if (ptr) {
        if (ctx)
            ctx->free_blocks.emplace(bytes, ptr);  // stays charged to the budget until freed
        else
            (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
}

void release_free_blocks(Ctx *c)
{
    for (auto &kv : c->free_blocks) {
        (void)hipFree(kv.second);
        c->used -= kv.first;
    }
    c->free_blocks.clear();
}

void HostBuf::reset()
{
    if (ptr)
        (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

void HostBuf::grow(size_t n, unsigned flags)
{
    if (ptr && bytes >= n)
        return;
    reset();
    n = (std::max(n, (size_t)64) + 4095) & ~(size_t)4095;
    if (hipHostMalloc(&ptr, n, flags) != hipSuccess) {
        ptr = nullptr;
        throw ZtsError{ZTS_E_NOMEM};
    }
    bytes = n;
}

void Slot::init()
{
    hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    hip_check(hipEventCreate(&ev0));
    hip_check(hipEventCreate(&ev1));
    hip_check(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    for (auto &e : evp)
        hip_check(hipEventCreate(&e));
    h_qs.grow(sizeof(QState), hipHostMallocCoherent);  // written by the final reduction
    std::memset(h_qs.ptr, 0, sizeof(QState));
}

void Slot::drop_graphs()
{
    for (auto &g : graphs)
        if (g.exec)
            (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

void Slot::release_scratch()
{
    drop_graphs();
    qs.reset();
    recs.reset();
    gnum.reset();
    gtheta.reset();
    tcnt.reset();
    tbin.reset();
    tpl.reset();
    dec.reset();
    bdata.reset();
    bres.reset();
    brec.reset();
}

void Slot::destroy()
{
    if (stream)
        (void)hipStreamSynchronize(stream);
    release_scratch();
    h_qs.reset();
    h_stage.reset();
    h_out.reset();
    if (ev0)
        (void)hipEventDestroy(ev0);
    if (ev1)
        (void)hipEventDestroy(ev1);
    if (ev_in)
        (void)hipEventDestroy(ev_in);
    for (auto &e : evp)
        if (e)
            (void)hipEventDestroy(e);
    if (stream)
        (void)hipStreamDestroy(stream);
    stream = nullptr;
    ev0 = ev1 = ev_in = nullptr;
    for (auto &e : evp)
        e = nullptr;
}

Stats::~Stats()
{
    if (ready)
        (void)hipEventDestroy(ready);
}

namespace {

// Evicts the least recently used cached per-size table that no running work
// holds (its buffers go to the free list).  False when there is none.
bool evict_one(Ctx *c)
{
    Image *victim = nullptr;
    bool is_stats = false;
    uint64_t oldest = UINT64_MAX;
    std::pair<int, int> skey;
    std::tuple<int, int, int> pkey;
    for (auto &kv : c->images) {
        Image *im = kv.second.get();
        for (auto &s : im->stats)
            if (!s.second->pins && s.second->last_use < oldest) {
                oldest = s.second->last_use;
                victim = im;
                is_stats = true;
                skey = s.first;
            }
        for (auto &p : im->prep)
            if (!p.second->pins && p.second->last_use < oldest) {
                oldest = p.second->last_use;
                victim = im;
                is_stats = false;
                pkey = p.first;
            }
    }
    if (!victim)
        return false;
    if (is_stats)
        victim->stats.erase(skey);
    else
        victim->prep.erase(pkey);
    return true;
}

// A cached free block of `bytes` .. 2 `bytes`, removed from the list.
void *take_free_block(Ctx *c, size_t bytes, size_t *got)
{
    auto it = c->free_blocks.lower_bound(bytes);
    if (it == c->free_blocks.end() || it->first > 2 * bytes)
        return nullptr;
    void *p = it->second;
    *got = it->first;
    c->free_blocks.erase(it);
    return p;
}

}  // namespace

void dalloc(Ctx *c, DBuf &b, size_t bytes)
{
    if (b.ptr && b.bytes >= bytes)
        return;
    b.reset();
    if (bytes == 0)
        bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    size_t got = 0;
    void *p = take_free_block(c, bytes, &got);
    while (!p && c->budget && c->used + bytes > c->budget) {
        if (evict_one(c)) {
            p = take_free_block(c, bytes, &got);
            continue;
        }
        if (c->free_blocks.empty())
            throw ZtsError{ZTS_E_BUDGET};
        auto big = std::prev(c->free_blocks.end());  // give back the largest cached block
        (void)hipFree(big->second);
        c->used -= big->first;
        c->free_blocks.erase(big);
    }
    if (!p) {
        c->used += bytes;  // reserved before a possible unlock
        hipError_t e;
        std::unique_lock<std::mutex> *lk = t_alloc_unlocked ? t_ctx_lock : nullptr;
        if (lk && lk->owns_lock()) {
            lk->unlock();
            e = hipMalloc(&p, bytes);
            lk->lock();
        } else {
            e = hipMalloc(&p, bytes);
        }
        if (e != hipSuccess) {
            release_free_blocks(c);
            if (hipMalloc(&p, bytes) != hipSuccess) {
                c->used -= bytes;
                throw ZtsError{ZTS_E_NOMEM};
            }
        }
        got = bytes;
    }
    b.ctx = c;
    b.ptr = p;
    b.bytes = got;
}

zts_result error_result(zts_status st)
{
    zts_result r;
    std::memset(&r, 0, sizeof r);
    r.status = st;
    return r;
}

// ------------------------------------------------------------------ parameters and taps

void fill_default(zts_params *p)
{
    p->rho_th = 0.80;
    p->rho_max = 0.95;
    p->margin = 1e-9;
    p->xi = 0.005;
    p->group_h = 5;
    p->group_w = 5;
    p->h0 = 3;
    p->w0 = 3;
    p->dh = 2;
    p->dw = 2;
    p->h_max = 33;
    p->blur_kind = 1;
    p->sigma_step = 0.5;
    p->sigma_max = 3.0;
    p->max_iters = 6;
    p->refine_radius = 0;
    p->timing = 0;
    p->egs_estimate = 0;
    p->rho_tc = 0.0;
    p->egs_shape = 0;
    p->pad0 = 0;
    p->accept_xi = 0.005;
    p->rho_floor = -2.0;
    p->floor_prune = 0;
    p->pad1 = 0;
    p->tile_dense_min = 0;
    p->pad2 = 0;
}

zts_status params_status(const zts_params &p)
{
    auto fin = [](double v) { return std::isfinite(v); };
    auto in_dim = [](int v) { return v >= 1 && v <= 32767; };
    bool ok = fin(p.rho_th) && p.rho_th > -1.0 && p.rho_th < 1.0;
    ok = ok && fin(p.rho_max) && p.rho_max > -1.0 && p.rho_max <= 1.0;
    ok = ok && fin(p.margin) && p.margin >= 0.0;
    ok = ok && fin(p.xi) && p.xi >= 0.0;
    ok = ok && fin(p.accept_xi) && p.accept_xi > -1.0 && p.accept_xi < 1.0;
    ok = ok && in_dim(p.group_h) && in_dim(p.group_w) && in_dim(p.h0) && in_dim(p.w0) && in_dim(p.h_max);
    ok = ok && p.dh >= 0 && p.dw >= 0 && (p.dh > 0 || p.dw > 0) && p.dh <= 32767 && p.dw <= 32767;
    ok = ok && (p.blur_kind == 0 || p.blur_kind == 1);
    if (p.blur_kind == 1)
        ok = ok && fin(p.sigma_step) && p.sigma_step > 0.0 && fin(p.sigma_max) && p.sigma_max >= 0.0;
    ok = ok && p.max_iters >= 0 && p.max_iters <= 15;
    ok = ok && p.refine_radius >= 0 && p.refine_radius <= 255;
    ok = ok && (p.egs_estimate == 0 || p.egs_estimate == 1) && (p.egs_shape == 0 || p.egs_shape == 1);
    ok = ok && fin(p.rho_tc) && p.rho_tc > -1.0 && p.rho_tc < 1.0;
    ok = ok && fin(p.rho_floor) && (p.floor_prune == 0 || p.floor_prune == 1);
    ok = ok && p.tile_dense_min >= -1 && p.tile_dense_min <= kTileRows * kTileCols;
    return ok ? ZTS_OK : ZTS_E_ARG;
}

zts_params params_or_default(const zts_params *params)
{
    zts_params pr;
    if (params)
        pr = *params;
    else
        fill_default(&pr);
    if (params_status(pr) != ZTS_OK)
        throw ZtsError{ZTS_E_ARG};
    return pr;
}

// Gaussian weights on [-d, d], d = ceil(3 sigma), quantised to integers that
// sum to 256: floors of 256 g_j / sum g, one unit to the centre when the
// remainder is odd, then one unit per symmetric pair by decreasing
// fractional part (ties to the smaller offset).
bool gaussian_taps(double sigma, Taps &tp)
{
    std::memset(&tp, 0, sizeof tp);
    if (!(sigma > 0.0)) {
        tp.d = 0;
        tp.w[0] = 256;
        return true;
    }
    int d = (int)std::ceil(3.0 * sigma);
    if (d > 32)
        return false;
    std::vector<double> g(d + 1), frac(d + 1);
    std::vector<int> f(d + 1);
    for (int j = 0; j <= d; j++)
        g[j] = std::exp(-(double)(j * j) / (2.0 * sigma * sigma));
    double total = g[0];
    for (int j = 1; j <= d; j++)
        total += 2.0 * g[j];
    int sum = 0;
    for (int j = 0; j <= d; j++) {
        double a = 256.0 * g[j] / total;
        f[j] = (int)std::floor(a);
        frac[j] = a - f[j];
        sum += (j == 0) ? f[j] : 2 * f[j];
    }
    int rem = 256 - sum;
    if (rem % 2 != 0) {
        f[0] += 1;
        rem -= 1;
    }
    std::vector<int> order;
    for (int j = 1; j <= d; j++)
        order.push_back(j);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return frac[a] > frac[b]; });
    for (int k = 0; k < (int)order.size() && rem >= 2; k++) {
        f[order[k]] += 1;
        rem -= 2;
    }
    f[0] += rem;
    for (int j = -d; j <= d; j++)
        tp.w[j + d] = f[j < 0 ? -j : j];
    tp.d = d;
    return true;
}

void paper_taps(Taps &tp)
{
    std::memset(&tp, 0, sizeof tp);
    const int W[5] = {1, 4, 10, 4, 1};
    for (int j = 0; j < 5; j++)
        tp.w[j] = W[j];
    tp.d = 2;
}

double lambda_of(double rho_th, double rho_max)
{
    double r = 1.0 + rho_th * rho_th * rho_max * rho_max - (rho_th * rho_th + rho_max * rho_max);
    if (r < 0.0)
        r = 0.0;
    return rho_th * rho_max + std::sqrt(r);
}

// ------------------------------------------------------------------ images and statistics

Image *find_image(Ctx *c, int id)
{
    auto it = c->images.find(id);
    if (it == c->images.end())
        throw ZtsError{ZTS_E_NOIMAGE};
    return it->second.get();
}

int64_t pitch_for(int cols) { return ((int64_t)cols + 64 + 255) / 256 * 256; }

// Allocates a pitched image buffer filled with 0x80 (int8 zero after the flip).
void alloc_image(Ctx *c, DBuf &b, int rows, int64_t pitch)
{
    dalloc(c, b, (size_t)pitch * rows + 4096);
    hip_check(hipMemsetAsync(b.ptr, 0x80, b.bytes, c->stream));
}

void build_sat(Ctx *c, const uint8_t *img, int64_t pitch, int rows, int cols, DBuf &sat)
{
    dalloc(c, sat, sizeof(uint2) * sat_elems(rows, cols));
    hip_check(launch_sat(img, pitch, rows, cols, sat.as<uint2>(), c->stream));
}

// Preparation scratch for the running sums of a product image over the
// whole image of an (Ly + m - 1) x (Lx + n - 1) search.
uint32_t *psat_for(Ctx *c, int Ly, int Lx, int m, int n)
{
    dalloc(c, c->psat, sizeof(uint32_t) * sat_elems(Ly + m - 1, Lx + n - 1));
    return c->psat.as<uint32_t>();
}

Stats *stats_entry(Ctx *c, Image *im, int m, int n, hipStream_t s)
{
    auto key = std::make_pair(m, n);
    auto it = im->stats.find(key);
    if (it != im->stats.end()) {
        Stats *st = it->second.get();
        st->last_use = ++c->clock;
        hip_check(hipStreamWaitEvent(s, st->ready, 0));
        return st;
    }
    auto st = std::make_unique<Stats>();
    int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
    dalloc(c, st->stat, sizeof(int2) * (size_t)Ly * Lx);
    hip_check(launch_stats(im->sat.as<uint2>(), im->cols, Ly, Lx, m, n, st->stat.as<int2>(), s));
    hip_check(hipEventCreateWithFlags(&st->ready, hipEventDisableTiming));
    hip_check(hipEventRecord(st->ready, s));
    st->last_use = ++c->clock;
    Stats *p = st.get();
    im->stats[key] = std::move(st);
    return p;
}

// Statistics for work on the main stream (preparation).
const int2 *stats_for(Ctx *c, Image *im, int m, int n) { return stats_entry(c, im, m, n, c->stream)->stat.as<int2>(); }

// Waits for the main stream with the context lock released (preparation only:
// its buffers are not reachable from the context's maps until it ends, and it
// holds prep_mu and a pin on its image).
void sync_main_unlocked(Ctx *c)
{
    std::unique_lock<std::mutex> *lk = t_ctx_lock;
    if (!lk || !lk->owns_lock()) {
        hip_check(hipStreamSynchronize(c->stream));
        return;
    }
    lk->unlock();
    hipError_t e = hipStreamSynchronize(c->stream);
    lk->lock();
    hip_check(e);
}

unsigned long long read_counter(Ctx *c)
{
    c->h_cnt.grow(64);
    hip_check(hipMemcpyAsync(c->h_cnt.ptr, c->counter.ptr, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             c->stream));
    sync_main_unlocked(c);
    return *c->h_cnt.as<unsigned long long>();
}

void zero_counter(Ctx *c)
{
    dalloc(c, c->counter, 64);
    hip_check(hipMemsetAsync(c->counter.ptr, 0, sizeof(unsigned long long), c->stream));
}

// ------------------------------------------------------------------ preparation

// The image a group tiling is built on, with its statistics.
struct Searched {
    const uint8_t *px;
    int64_t pitch;
    const int2 *stat;
};

// Retained-member count of Alg. 2 for group size (h, w) on image S: Eq. 15
// (Prop. 3.2) or, with pr.egs_estimate = 1, Prop. 3.1 at the assumed rho_tc
// (both roots).  With blur data (theta_c, x_c, statI) every location counts
// with the angle to its original block added.
int64_t retained_count(Ctx *c, const Searched &S, int m, int n, int Ly, int Lx, int h, int w, const zts_params &pr,
                       const float *theta_c, const int32_t *x_c, const int2 *statI)
{
    AcArgs a;
    std::memset(&a, 0, sizeof a);
    a.J = S.px;
    a.pJ = S.pitch;
    a.statJ = S.stat;
    a.statI = statI;
    a.m = m;
    a.n = n;
    a.Ly = Ly;
    a.Lx = Lx;
    a.h = h;
    a.w = w;
    a.thr = std::sqrt(1.0 - pr.rho_th * pr.rho_th);
    const float eps = 1e-5f;
    a.thr_lo = (float)a.thr - eps;
    a.thr_hi = (float)a.thr + eps;
    float al = (float)std::acos(a.thr);
    float ah = (float)(2.0 * M_PI - std::acos(a.thr));
    a.alo_lo = al - eps;
    a.alo_hi = al + eps;
    a.ahi_lo = ah - eps;
    a.ahi_hi = ah + eps;
    a.theta_c = theta_c;
    a.x_c = x_c;
    a.rho_th = pr.rho_th;
    a.ra = pr.rho_tc;
    a.sa = std::sqrt(1.0 - pr.rho_tc * pr.rho_tc);
    if (pr.egs_estimate == 1)
        a.mode = theta_c ? AC_COUNT31_BLUR : AC_COUNT31;
    else
        a.mode = theta_c ? AC_COUNT_BLUR : AC_COUNT;
    zero_counter(c);
    a.counter = c->counter.as<unsigned long long>();
    hip_check(launch_autocorr(a, psat_for(c, Ly, Lx, m, n), c->stream));
    return (int64_t)read_counter(c);
}

// Alg. 2: greedy descent of the estimated cost over group sizes, starting at
// (h0, w0): square steps (egs_shape 0) or the cheapest of the three
// neighbouring sizes (egs_shape 1).  Fills trace/ntrace (up to 64 evaluated
// candidates).
void run_egs(Ctx *c, const Searched &S, int m, int n, int Ly, int Lx, const zts_params &pr, int h0, int w0,
             const float *theta_c, const int32_t *x_c, const int2 *statI, int &he, int &we, int64_t &cost,
             zts_egs_step *trace, int &ntrace)
{
    const int kTrace = 64;
    int64_t mn = (int64_t)m * n;
    int64_t prev = mn * (int64_t)Ly * Lx;
    int bh = 1, bw = 1, k = 0;
    if (pr.dh < 0 || pr.dw < 0 || (pr.dh == 0 && pr.dw == 0) || h0 < 1 || w0 < 1)
        throw ZtsError{ZTS_E_ARG};
    for (bool first = true;; first = false) {
        int ch[3], cw[3], nc = 0;
        if (first) {
            ch[0] = h0, cw[0] = w0, nc = 1;
        } else if (pr.egs_shape == 0) {
            ch[0] = bh + pr.dh, cw[0] = bw + pr.dw, nc = 1;
        } else {
            const int cand[3][2] = {{bh + pr.dh, bw}, {bh, bw + pr.dw}, {bh + pr.dh, bw + pr.dw}};
            for (int i = 0; i < 3; i++) {
                bool dup = cand[i][0] == bh && cand[i][1] == bw;
                for (int j = 0; j < nc; j++)
                    dup = dup || (ch[j] == cand[i][0] && cw[j] == cand[i][1]);
                if (!dup)
                    ch[nc] = cand[i][0], cw[nc] = cand[i][1], nc++;
            }
        }
        int best = -1, best_h = 0, best_w = 0;
        int64_t best_ct = 0;
        for (int i = 0; i < nc; i++) {
            const int h = ch[i], w = cw[i];
            if (h > pr.h_max || w > pr.h_max || h > Ly || w > Lx)
                continue;
            int64_t cc = (int64_t)((Ly + h - 1) / h) * ((Lx + w - 1) / w);
            int64_t cr = retained_count(c, S, m, n, Ly, Lx, h, w, pr, theta_c, x_c, statI);
            int64_t ct = mn * (cc + cr);
            if (trace && k < kTrace) {
                zts_egs_step &s = trace[k];
                std::memset(&s, 0, sizeof s);
                s.h = h;
                s.w = w;
                s.cc = cc;
                s.cr = cr;
                s.ct = ct;
            }
            if (best < 0 || ct < best_ct)
                best = k, best_ct = ct, best_h = h, best_w = w;
            k++;
        }
        if (best < 0 || !((double)(prev - best_ct) > pr.xi * (double)prev))
            break;
        if (trace && best < kTrace)
            trace[best].accepted = 1;
        prev = best_ct;
        bh = best_h;
        bw = best_w;
    }
    ntrace = std::min(k, kTrace);
    he = bh;
    we = bw;
    cost = prev;
}

// Angle tables of every location to its group centre on S, and group summaries.
void build_tables(Ctx *c, Prepared &P, const Searched &S, int Ly, int Lx)
{
    P.Gy = (Ly + P.h - 1) / P.h;
    P.Gx = (Lx + P.w - 1) / P.w;
    size_t slots = (size_t)P.Gy * P.Gx * P.h * P.w;  // group-major: slot g*h*w + my*w + mx
    dalloc(c, P.theta_b, sizeof(float) * slots);
    dalloc(c, P.x_b, sizeof(int32_t) * slots);
    if (P.mode == ZTS_OPTA) {
        dalloc(c, P.theta_cg, sizeof(float) * slots);
        dalloc(c, P.x_cg, sizeof(int32_t) * slots);
        hip_check(launch_regroup(P.theta_c.ptr, P.theta_cg.ptr, Ly, Lx, P.h, P.w, c->stream));
        hip_check(launch_regroup(P.x_c.ptr, P.x_cg.ptr, Ly, Lx, P.h, P.w, c->stream));
    }
    AcArgs a;
    std::memset(&a, 0, sizeof a);
    a.J = S.px;
    a.pJ = S.pitch;
    a.statJ = S.stat;
    a.m = P.m;
    a.n = P.n;
    a.Ly = Ly;
    a.Lx = Lx;
    a.h = P.h;
    a.w = P.w;
    a.mode = AC_BUILD;
    a.theta_b = P.theta_b.as<float>();
    a.x_b = P.x_b.as<int32_t>();
    hip_check(launch_autocorr(a, psat_for(c, Ly, Lx, P.m, P.n), c->stream));
    dalloc(c, P.cstat, sizeof(int2) * (size_t)P.Gy * P.Gx);
    hip_check(launch_centre_stats(S.stat, Ly, Lx, P.h, P.w, P.Gy, P.Gx, P.cstat.as<int2>(), c->stream));
    dalloc(c, P.gsum, sizeof(GroupSum) * (size_t)P.Gy * P.Gx);
    GsumArgs g;
    g.theta_b = P.theta_b.as<float>();
    g.theta_c = P.mode == ZTS_OPTA ? P.theta_cg.as<float>() : nullptr;
    g.Ly = Ly;
    g.Lx = Lx;
    g.h = P.h;
    g.w = P.w;
    g.Gy = P.Gy;
    g.Gx = P.Gx;
    g.opta = P.mode == ZTS_OPTA;
    g.gsum = P.gsum.as<GroupSum>();
    hip_check(launch_gsum(g, c->stream));
}

// Blur correlation of every block of J against the same block of I.
void blurcorr(Ctx *c, const uint8_t *J, const int2 *statJ, const uint8_t *I, const int2 *statI, int64_t pitch, int m,
              int n, int Ly, int Lx, int mode, double lambda, uint8_t *viol, float *theta_c, int32_t *x_c,
              int64_t *num_out, int64_t *dj_out, int64_t *di_out)
{
    BcArgs a;
    std::memset(&a, 0, sizeof a);
    a.J = J;
    a.I = I;
    a.pitch = pitch;
    a.statJ = statJ;
    a.statI = statI;
    a.m = m;
    a.n = n;
    a.Ly = Ly;
    a.Lx = Lx;
    a.mode = mode;
    a.viol = viol;
    a.lambda = lambda;
    a.lam_lo = (float)lambda - 1e-5f;
    a.lam_hi = (float)lambda + 1e-5f;
    a.theta_c = theta_c;
    a.x_c = x_c;
    a.num_out = num_out;
    a.dj_out = dj_out;
    a.di_out = di_out;
    if (mode == BC_VIOL) {
        zero_counter(c);
        a.counter = c->counter.as<unsigned long long>();
    }
    hip_check(launch_blurcorr(a, psat_for(c, Ly, Lx, m, n), c->stream));
}

// One OptA candidate image with its tables.
struct Cand {
    DBuf J, Jsat, Jstat, theta_c, x_c;
};

// Alg. 3.  The conditioned image ends in P.J (with its running sums and
// statistics), its blur angles in P.theta_c / P.x_c.  For ZTS_OPTA every EGS
// count adds each location's angle to its original block (the search bounds
// original locations through blurred ones); for ZTS_OPTA_PAPER each EGS run
// sees only the blurred image, as Alg. 3 prints it, and no blur angles are
// kept.
void run_opta(Ctx *c, Image *im, Prepared &P, const zts_params &pr, const int2 *statI)
{
    const bool with_c = P.mode == ZTS_OPTA;
    int p = im->rows, q = im->cols, m = P.m, n = P.n;
    int Ly = p - m + 1, Lx = q - n + 1;
    size_t L = (size_t)Ly * Lx;
    int64_t pitch = im->pitch;
    double lambda = lambda_of(pr.rho_th, pr.rho_max);
    Cand cur, nxt;
    auto setup = [&](Cand &k) {
        alloc_image(c, k.J, p, pitch);
        dalloc(c, k.Jstat, sizeof(int2) * L);
        if (with_c) {
            dalloc(c, k.theta_c, sizeof(float) * L);
            dalloc(c, k.x_c, sizeof(int32_t) * L);
        }
    };
    auto stats_of = [&](Cand &k) {
        build_sat(c, k.J.as<uint8_t>(), pitch, p, q, k.Jsat);
        hip_check(launch_stats(k.Jsat.as<uint2>(), q, Ly, Lx, m, n, k.Jstat.as<int2>(), c->stream));
    };
    auto build_c = [&](Cand &k) {
        if (with_c)
            blurcorr(c, k.J.as<uint8_t>(), k.Jstat.as<int2>(), im->img.as<uint8_t>(), statI, pitch, m, n, Ly, Lx,
                     BC_BUILD, lambda, nullptr, k.theta_c.as<float>(), k.x_c.as<int32_t>(), nullptr, nullptr,
                     nullptr);
    };
    setup(cur);
    setup(nxt);
    dalloc(c, c->tmp32, sizeof(uint32_t) * (size_t)p * q);
    dalloc(c, c->viol, L);
    dalloc(c, c->colmask, (size_t)p * Lx);
    hip_check(hipMemcpyAsync(cur.J.ptr, im->img.ptr, (size_t)pitch * p, hipMemcpyDeviceToDevice, c->stream));
    stats_of(cur);
    build_c(cur);
    int h, w, nt;
    int64_t cost;
    zts_egs_step tr[64];
    Searched S{cur.J.as<uint8_t>(), pitch, cur.Jstat.as<int2>()};
    run_egs(c, S, m, n, Ly, Lx, pr, pr.h0, pr.w0, cur.theta_c.as<float>(), cur.x_c.as<int32_t>(),
            with_c ? statI : nullptr, h, w, cost, tr, nt);
    zts_prep_info &info = P.info;
    info.n_opta = 1;
    std::memset(&info.opta[0], 0, sizeof info.opta[0]);
    info.opta[0].h = h;
    info.opta[0].w = w;
    info.opta[0].cost = cost;
    info.opta[0].accepted = 1;
    std::memcpy(info.egs, tr, sizeof(zts_egs_step) * nt);
    info.n_egs = nt;
    int radius = 0;
    for (int it = 1;; it++) {
        Taps tp;
        double sigma = 0.0;
        if (pr.blur_kind == 0) {
            if (it > pr.max_iters)
                break;
            paper_taps(tp);
        } else {
            if (pr.sigma_step * it > pr.sigma_max + 1e-9 || it > pr.max_iters)
                break;
            sigma = pr.sigma_step * std::sqrt(2.0 * it - 1.0);
            if (!gaussian_taps(sigma, tp))
                throw ZtsError{ZTS_E_ARG};
        }
        hip_check(launch_blur(cur.J.as<uint8_t>(), nxt.J.as<uint8_t>(), pitch, p, q, tp, c->tmp32.as<uint32_t>(),
                              c->stream));
        int passes = 0;
        int64_t reverted = 0;
        for (;;) {
            stats_of(nxt);
            blurcorr(c, nxt.J.as<uint8_t>(), nxt.Jstat.as<int2>(), im->img.as<uint8_t>(), statI, pitch, m, n, Ly,
                     Lx, BC_VIOL, lambda, c->viol.as<uint8_t>(), nullptr, nullptr, nullptr, nullptr, nullptr);
            zero_counter(c);
            hip_check(launch_revert(c->viol.as<uint8_t>(), c->colmask.as<uint8_t>(), p, q, Ly, Lx, m, n,
                                    im->img.as<uint8_t>(), nxt.J.as<uint8_t>(), pitch,
                                    c->counter.as<unsigned long long>(), c->stream));
            unsigned long long changed = read_counter(c);
            if (changed == 0)
                break;
            passes++;
            reverted += (int64_t)changed;
        }
        build_c(nxt);
        int h2, w2;
        int64_t c2;
        Searched S2{nxt.J.as<uint8_t>(), pitch, nxt.Jstat.as<int2>()};
        run_egs(c, S2, m, n, Ly, Lx, pr, h, w, nxt.theta_c.as<float>(), nxt.x_c.as<int32_t>(),
                with_c ? statI : nullptr, h2, w2, c2, tr, nt);
        bool accept = (double)(cost - c2) > pr.accept_xi * (double)c2;
        if (info.n_opta < 16) {
            zts_opta_step &s = info.opta[info.n_opta++];
            std::memset(&s, 0, sizeof s);
            s.k = it;
            s.d = tp.d;
            s.sigma = sigma;
            s.passes = passes;
            s.reverted = reverted;
            s.h = h2;
            s.w = w2;
            s.cost = c2;
            s.accepted = accept;
        }
        if (!accept)
            break;
        std::swap(cur.J.ptr, nxt.J.ptr);
        std::swap(cur.Jsat.ptr, nxt.Jsat.ptr);
        std::swap(cur.Jsat.bytes, nxt.Jsat.bytes);
        std::swap(cur.Jstat.ptr, nxt.Jstat.ptr);
        std::swap(cur.theta_c.ptr, nxt.theta_c.ptr);
        std::swap(cur.x_c.ptr, nxt.x_c.ptr);
        std::memcpy(info.egs, tr, sizeof(zts_egs_step) * nt);
        info.n_egs = nt;
        h = h2;
        w = w2;
        cost = c2;
        radius += tp.d;
    }
    P.h = h;
    P.w = w;
    P.radius = std::min(radius, 8);
    info.cost = cost;
    // keep the accepted candidate's buffers in P
    std::swap(P.J.ptr, cur.J.ptr), std::swap(P.J.bytes, cur.J.bytes), std::swap(P.J.ctx, cur.J.ctx);
    std::swap(P.Jsat.ptr, cur.Jsat.ptr), std::swap(P.Jsat.bytes, cur.Jsat.bytes), std::swap(P.Jsat.ctx, cur.Jsat.ctx);
    std::swap(P.Jstat.ptr, cur.Jstat.ptr), std::swap(P.Jstat.bytes, cur.Jstat.bytes),
        std::swap(P.Jstat.ctx, cur.Jstat.ctx);
    std::swap(P.theta_c.ptr, cur.theta_c.ptr), std::swap(P.theta_c.bytes, cur.theta_c.bytes),
        std::swap(P.theta_c.ctx, cur.theta_c.ctx);
    std::swap(P.x_c.ptr, cur.x_c.ptr), std::swap(P.x_c.bytes, cur.x_c.bytes), std::swap(P.x_c.ctx, cur.x_c.ctx);
}

bool same_prep_params(const Prepared &P, zts_mode mode, const zts_params &a)
{
    const zts_params &b = P.params;
    if (mode == ZTS_TE_FIXED)
        return a.group_h == b.group_h && a.group_w == b.group_w;
    bool egs = a.rho_th == b.rho_th && a.xi == b.xi && a.h0 == b.h0 && a.w0 == b.w0 && a.dh == b.dh &&
               a.dw == b.dw && a.h_max == b.h_max && a.egs_estimate == b.egs_estimate &&
               a.egs_shape == b.egs_shape && (a.egs_estimate == 0 || a.rho_tc == b.rho_tc);
    if (mode == ZTS_EGS)
        return egs;
    return egs && a.rho_max == b.rho_max && a.blur_kind == b.blur_kind && a.sigma_step == b.sigma_step &&
           a.sigma_max == b.sigma_max && a.max_iters == b.max_iters && a.accept_xi == b.accept_xi;
}

// Holds a pin for the lifetime of a scope.
struct PinGuard {
    int &pins;
    explicit PinGuard(int &p) : pins(p) { pins++; }
    ~PinGuard() { pins--; }
};

// The cached tables of (m, n, mode) when they were made with these
// parameters; drops tables made with others (ZTS_E_BUSY while pinned).
static Prepared *cached_prep(Ctx *c, Image *im, const std::tuple<int, int, int> &key, zts_mode mode,
                             const zts_params &pr)
{
    auto it = im->prep.find(key);
    if (it == im->prep.end())
        return nullptr;
    if (same_prep_params(*it->second, mode, pr)) {
        it->second->last_use = ++c->clock;
        return it->second.get();
    }
    if (it->second->pins)  // running work still reads the tables made with other parameters
        throw ZtsError{ZTS_E_BUSY};
    im->prep.erase(it);
    return nullptr;
}

static Prepared *build_prep(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr);

// Tables of (image, m, n, mode): cached, or built.  Building holds prep_mu
// (taken with the context lock released, then the lock again) and a pin on
// the image; it releases the context lock while it waits for the device.
Prepared *prepare(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr)
{
    auto key = std::make_tuple(m, n, (int)mode);
    if (Prepared *P = cached_prep(c, im, key, mode, pr))
        return P;
    im->busy++;  // zts_image_unload refuses while the lock is released below
    std::unique_lock<std::mutex> plk;
    try {
        plk = take_prep_lock(c);
    } catch (...) {
        im->busy--;
        throw;
    }
    im->busy--;
    // another thread may have built the same tables meanwhile
    if (Prepared *P = cached_prep(c, im, key, mode, pr))
        return P;
    im->busy++;
    try {
        Prepared *P = build_prep(c, im, m, n, mode, pr);
        im->busy--;
        return P;
    } catch (...) {
        im->busy--;
        throw;
    }
}

static Prepared *build_prep(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr)
{
    auto key = std::make_tuple(m, n, (int)mode);
    auto t0 = std::chrono::steady_clock::now();
    int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
    Stats *sI = stats_entry(c, im, m, n, c->stream);
    PinGuard pin(sI->pins);  // preparation's own allocations may evict cached tables, never these
    AllocUnlockedScope unlocked_allocs;  // from here on every buffer is the preparation's own
    const int2 *statI = sI->stat.as<int2>();
    auto P = std::make_unique<Prepared>();
    std::memset(&P->info, 0, sizeof P->info);
    P->mode = mode;
    P->m = m;
    P->n = n;
    P->params = pr;
    P->radius = 0;
    Searched SI{im->img.as<uint8_t>(), im->pitch, statI};
    if (mode == ZTS_TE_FIXED) {
        if (pr.group_h < 1 || pr.group_w < 1)
            throw ZtsError{ZTS_E_ARG};
        P->h = pr.group_h;
        P->w = pr.group_w;
        build_tables(c, *P, SI, Ly, Lx);
    } else if (mode == ZTS_EGS) {
        int nt;
        run_egs(c, SI, m, n, Ly, Lx, pr, pr.h0, pr.w0, nullptr, nullptr, nullptr, P->h, P->w, P->info.cost,
                P->info.egs, nt);
        P->info.n_egs = nt;
        build_tables(c, *P, SI, Ly, Lx);
    } else if (mode == ZTS_OPTA || mode == ZTS_OPTA_PAPER) {
        run_opta(c, im, *P, pr, statI);
        Searched SJ{P->J.as<uint8_t>(), im->pitch, P->Jstat.as<int2>()};
        build_tables(c, *P, SJ, Ly, Lx);
    } else {
        throw ZtsError{ZTS_E_ARG};
    }
    sync_main_unlocked(c);
    auto t1 = std::chrono::steady_clock::now();
    P->info.mode = mode;
    P->info.m = m;
    P->info.n = n;
    P->info.group_h = P->h;
    P->info.group_w = P->w;
    P->info.radius = P->radius;
    P->info.prepare_ms = (float)std::chrono::duration<double, std::milli>(t1 - t0).count();
    Prepared *raw = P.get();
    raw->last_use = ++c->clock;
    im->prep[key] = std::move(P);
    return raw;
}

void check_template_args(Image *im, const void *tpl, int m, int n, int64_t stride)
{
    if (!tpl || m < 1 || n < 1 || stride < n)
        throw ZtsError{ZTS_E_ARG};
    if (m > im->rows || n > im->cols)
        throw ZtsError{ZTS_E_SIZE};
    if ((int64_t)m * n > 16384)
        throw ZtsError{ZTS_E_SIZE};
}

void check_mode_shape(zts_mode mode, int m, int n)
{
    // The LDS needs grow with m and n, so when 128 x 128 fits every mode, so
    // does every shape within it: those skip the per-kernel queries below.
    // The answer is kept only once the queries behind it have succeeded; a
    // failed query is a device error, not a size refusal.
    static std::atomic<int> small_fit{-1};
    if (m <= 128 && n <= 128) {
        int sf = small_fit.load(std::memory_order_relaxed);
        if (sf < 0) {
            (void)lds_query_failed();
            const bool v = full_fits(128, 128) && scan_fits(128, 128);
            if (lds_query_failed())
                throw ZtsError{ZTS_E_DEVICE};
            sf = v ? 1 : 0;
            small_fit.store(sf, std::memory_order_relaxed);
        }
        if (sf == 1)
            return;
    }
    (void)lds_query_failed();
    const bool ok = mode == ZTS_FULL ? full_fits(m, n) : mode == ZTS_FULL_MFMA ? n <= 128 : scan_fits(m, n);
    if (lds_query_failed())
        throw ZtsError{ZTS_E_DEVICE};
    if (!ok)
        throw ZtsError{ZTS_E_SIZE};
}

// ------------------------------------------------------------------ one query

namespace {

int query_radius(const QueryPlan &q)
{
    if (q.mode == ZTS_OPTA || q.mode == ZTS_OPTA_PAPER)
        return std::max(q.P->radius, std::max(q.pr.refine_radius, 0));
    return q.pr.refine_radius > 0 ? q.pr.refine_radius : -1;
}

// Survivors of a tile from which it is matched whole on int8 MFMA (and four
// times that for a super-tile of four tiles): the built-in value, 128 of the
// tile's 8192 locations, is near the measured crossover on the 8192 x 8192
// workload (params.tile_dense_min overrides it; -1: never).
int tile_dense_min_of(const zts_params &pr)
{
    if (pr.tile_dense_min < 0)
        return 0;
    return pr.tile_dense_min > 0 ? pr.tile_dense_min : 128;
}

// Geometry of a query's survivor tiles (the fields tile_plan fills).
TileArgs tile_geometry(const QueryPlan &q)
{
    TileArgs t;
    std::memset(&t, 0, sizeof t);
    t.m = q.m;
    t.n = q.n;
    t.Ly = q.Ly;
    t.Lx = q.Lx;
    tile_plan(t, tile_dense_min_of(q.pr));
    return t;
}

}  // namespace

void unpin_query(QueryPlan &q)
{
    if (q.st)
        q.st->pins--;
    if (q.P)
        q.P->pins--;
    q.st = nullptr;
    q.P = nullptr;
}

QueryPlan plan_query(Ctx *c, Slot &S, Image *im, int m, int n, zts_mode mode, const zts_params &pr, bool want_dec)
{
    QueryPlan q;
    q.im = im;
    q.m = m;
    q.n = n;
    q.Ly = im->rows - m + 1;
    q.Lx = im->cols - n + 1;
    q.mode = mode;
    q.pr = pr;
    q.want_dec = want_dec;
    q.st = stats_entry(c, im, m, n, S.stream);
    q.st->pins++;
    try {
        if (mode != ZTS_FULL) {
            if (want_dec && mode == ZTS_OPTA_PAPER)  // no decision map for the paper's search
                throw ZtsError{ZTS_E_ARG};
            q.P = prepare(c, im, m, n, mode, pr);
            q.P->pins++;
            q.P->last_use = ++c->clock;
        }
        int64_t L = (int64_t)q.Ly * q.Lx;
        void *old_qs = S.qs.ptr;
        dalloc(c, S.qs, sizeof(QState));
        if (S.qs.ptr != old_qs) {  // a fresh state: both sequence numbers start at 0
            hip_check(hipMemsetAsync(S.qs.ptr, 0, sizeof(QState), S.stream));
            S.h_qs.as<QState>()->seq = 0;
            S.qseq = 0;
        }
        dalloc(c, S.tpl, (size_t)m * n);
        if (want_dec)
            dalloc(c, S.dec, (size_t)L);
        if (mode == ZTS_FULL) {
            dalloc(c, S.recs, sizeof(RecPod) * (size_t)full_record_count(q.Ly, q.Lx));
        } else {
            const Prepared *P = q.P;
            int radius = query_radius(q);
            int n1 = centres_record_count(P->Gy, P->Gx, m, n, P->h, P->w);
            int n2 = radius >= 0 ? window_record_count(radius) : 0;
            int n3 = members_record_count(P->Gy, P->Gx);
            const TileArgs tg = tile_geometry(q);
            const size_t ntile = (size_t)tg.tiles_x * tg.tiles_y;
            dalloc(c, S.recs, sizeof(RecPod) * ((size_t)n1 + n2 + n3 + (size_t)tile_record_count(tg)));
            dalloc(c, S.gnum, sizeof(int32_t) * (size_t)P->Gy * P->Gx);
            dalloc(c, S.gtheta, sizeof(float) * (size_t)P->Gy * P->Gx);
            dalloc(c, S.tcnt, sizeof(uint32_t) * ntile);
            dalloc(c, S.tbin, sizeof(int32_t) * ntile * (size_t)tg.tile_cap);
        }
    } catch (...) {
        unpin_query(q);
        throw;
    }
    return q;
}

void stage_template(Slot &S, const uint8_t *tpl, int m, int n, int64_t stride)
{
    size_t bytes = (size_t)m * n;
    S.h_stage.grow(bytes);
    uint8_t *h = S.h_stage.as<uint8_t>();
    for (int i = 0; i < m; i++)
        std::memcpy(h + (size_t)i * n, tpl + (size_t)i * stride, n);
    hip_check(hipMemcpyAsync(S.tpl.ptr, h, bytes, hipMemcpyHostToDevice, S.stream));
}

// Every argument of one query's launches.  The struct is zeroed before it is
// filled, so two launches with equal bytes enqueue identical work: the bytes
// are the key of the slot's graph cache.
struct QueryLaunch {
    int32_t full;
    int32_t radius, n1, n2, n3, n4, opta;
    int32_t paper;  // ZTS_OPTA_PAPER: scans on J, then the window on I after scan 2
    int32_t red_lo, red_hi, count_lo;  // final reduction: best over [lo, hi), counts over [count_lo, hi)
    FullArgs fa;
    ScanArgs sa;
    WinArgs wa;
    MemArgs ma;
    TileArgs ta;
    QState *qs;
    RecPod *recs;
    void *h_qs;
};

// Device scratch of one query (and the pinned host mirror of its state).
struct QueryBufs {
    QState *qs;
    RecPod *recs;
    int32_t *gnum;
    float *gtheta;
    uint32_t *tcnt;      // survivor tiles: counts
    int32_t *tbin;       // and bins
    const uint8_t *tpl;  // the staged template (pitch n) when the plan reads none in place
    void *h_qs;
};

static QueryBufs slot_bufs(Slot &S)
{
    return QueryBufs{S.qs.as<QState>(), S.recs.as<RecPod>(), S.gnum.as<int32_t>(), S.gtheta.as<float>(),
                     S.tcnt.as<uint32_t>(), S.tbin.as<int32_t>(), S.tpl.as<uint8_t>(), S.h_qs.ptr};
}

static void build_query_launch(const QueryPlan &q, const QueryBufs &B, int8_t *d_dec, QueryLaunch &Q)
{
    std::memset(&Q, 0, sizeof Q);
    Image *im = q.im;
    const int m = q.m, n = q.n, Ly = q.Ly, Lx = q.Lx;
    const zts_params &pr = q.pr;
    const Prepared *P = q.P;
    const int2 *statI = q.st->stat.as<int2>();
    QState *qs = B.qs;
    const uint8_t *tpl = q.tpl ? q.tpl : B.tpl;
    const int64_t ts = q.tpl ? q.ts : n;
    RecPod *recs = B.recs;
    Q.qs = qs;
    Q.recs = recs;
    Q.h_qs = B.h_qs;
    if (q.mode == ZTS_FULL) {
        Q.full = 1;
        FullArgs &a = Q.fa;
        a.img = im->img.as<uint8_t>();
        a.pitch = im->pitch;
        a.p = im->rows;
        a.q = im->cols;
        a.stat = statI;
        a.tpl = tpl;
        a.ts = ts;
        a.m = m;
        a.n = n;
        a.Ly = Ly;
        a.Lx = Lx;
        a.recs = recs;
        a.qs = qs;
        a.num_map = q.num_map;
        a.dr_map = q.dr_map;
        a.rho_map = q.rho_map;
        a.dec = d_dec;
        Q.n3 = full_record_count(Ly, Lx);
        Q.red_lo = Q.count_lo = 0;
        Q.red_hi = Q.n3;
        return;
    }
    const bool paper = q.mode == ZTS_OPTA_PAPER;
    const bool opta = q.mode == ZTS_OPTA;
    const bool onJ = opta || paper;  // the scans run on the conditioned image
    const int radius = query_radius(q);
    Q.opta = opta;
    Q.paper = paper;
    Q.radius = radius;
    TileArgs &ta = Q.ta;
    ta = tile_geometry(q);
    Q.n1 = centres_record_count(P->Gy, P->Gx, m, n, P->h, P->w);
    Q.n2 = radius >= 0 ? window_record_count(radius) : 0;
    Q.n3 = members_record_count(P->Gy, P->Gx);
    Q.n4 = tile_record_count(ta);
    // records: [0, n1) scan 1, then the window, scan 2 and the survivor tiles
    // (ZTS_OPTA_PAPER: scan 2 and the tiles, then the window on I, whose best
    // is the answer)
    const int win_off = paper ? Q.n1 + Q.n3 + Q.n4 : Q.n1, mem_off = paper ? Q.n1 : Q.n1 + Q.n2;
    Q.red_lo = paper ? win_off : (opta ? Q.n1 : 0);
    Q.red_hi = Q.n1 + Q.n2 + Q.n3 + Q.n4;
    Q.count_lo = paper ? Q.n1 : Q.red_lo;
    const uint8_t *spx = onJ ? P->J.as<uint8_t>() : im->img.as<uint8_t>();
    const int2 *sstat = onJ ? P->Jstat.as<int2>() : statI;
    ScanArgs &s = Q.sa;
    s.img = spx;
    s.pitch = im->pitch;
    s.stat = sstat;
    s.cstat = P->cstat.as<int2>();
    s.tpl = tpl;
    s.ts = ts;
    s.m = m;
    s.n = n;
    s.Ly = Ly;
    s.Lx = Lx;
    s.h = P->h;
    s.w = P->w;
    s.Gy = P->Gy;
    s.Gx = P->Gx;
    s.g_x = B.gnum;
    s.g_theta = B.gtheta;
    s.recs = recs;
    s.qs = qs;
    s.dec = onJ ? nullptr : d_dec;
    s.delta = pr.margin;
    s.tile_cnt = B.tcnt;
    s.n_tiles = ta.tiles_x * ta.tiles_y;
    if (radius >= 0) {
        WinArgs &wa = Q.wa;
        wa.img = im->img.as<uint8_t>();
        wa.pitch = im->pitch;
        wa.stat = statI;
        wa.tpl = tpl;
        wa.ts = ts;
        wa.m = m;
        wa.n = n;
        wa.Ly = Ly;
        wa.Lx = Lx;
        wa.h = P->h;
        wa.w = P->w;
        wa.radius = radius;
        wa.skip_centres = !onJ;
        wa.include_best0 = !onJ;
        wa.thr_out = !paper;  // scan 2 runs next and takes the scan-1 best from here
        wa.recs = recs;
        wa.rec_off = win_off;  // its centre: the best of the records before it
        wa.qs = qs;
        wa.dec = d_dec;
        wa.delta = pr.margin;
    }
    MemArgs &ma = Q.ma;
    ma.I = paper ? P->J.as<uint8_t>() : im->img.as<uint8_t>();  // where survivors are matched
    ma.pI = im->pitch;
    ma.statI = paper ? sstat : statI;
    ma.statS = sstat;
    ma.tpl = tpl;
    ma.ts = ts;
    ma.m = m;
    ma.n = n;
    ma.Ly = Ly;
    ma.Lx = Lx;
    ma.h = P->h;
    ma.w = P->w;
    ma.Gy = P->Gy;
    ma.Gx = P->Gx;
    ma.g_x = B.gnum;
    ma.g_theta = B.gtheta;
    ma.gsum = P->gsum.as<GroupSum>();
    ma.theta_b = P->theta_b.as<float>();
    ma.x_b = P->x_b.as<int32_t>();
    ma.theta_c = opta ? P->theta_cg.as<float>() : nullptr;
    ma.x_c = opta ? P->x_cg.as<int32_t>() : nullptr;
    ma.opta = opta;
    ma.radius = paper ? -1 : radius;  // the paper's search has no window before scan 2
    ma.recs = recs;
    ma.rec_off = mem_off;
    ma.final_from = opta ? Q.n1 : 0;
    ma.qs = qs;
    ma.dec = paper ? nullptr : d_dec;
    ma.n_best0 = Q.n1;
    ma.n_win = paper ? 0 : Q.n2;
    ma.include_best0 = !opta;
    ma.thr_ready = radius >= 0 && !paper;
    ma.delta = pr.margin;
    ma.floor = pr.floor_prune ? pr.rho_floor : -2.0;
    ma.tile_cnt = B.tcnt;
    ma.tile_bin = B.tbin;
    ma.tile_cap = ta.tile_cap;
    ma.tiles_x = ta.tiles_x;
    // survivors are matched where scan 2 says: on I, or on J for the paper's search
    ta.img = ma.I;
    ta.pitch = ma.pI;
    ta.p = im->rows;
    ta.q = im->cols;
    ta.stat = ma.statI;
    ta.tpl = tpl;
    ta.ts = ts;
    ta.tile_cnt = B.tcnt;
    ta.tile_bin = B.tbin;
    ta.qs = qs;
    ta.recs = recs;
    ta.rec_off = mem_off + Q.n3;
}

// The kernels of one query; the last one publishes the query state to the
// slot's pinned host mirror.
// The scan kernels initialise the query state themselves (no fill), so the
// sequence can be captured into a graph.  With `events`, an event follows
// each kernel (per-kernel times; never captured: event-record nodes made
// graph replays slower than eager launches).
static void enqueue_query(const QueryLaunch &Q, Slot &S, hipStream_t st, bool events)
{
    auto mark = [&](hipEvent_t e) {
        if (events)
            hip_check(hipEventRecord(e, st));
    };
    if (Q.full) {
        hip_check(launch_full(Q.fa, st));
        mark(S.evp[0]);
        hip_check(launch_reduce(Q.recs, Q.red_lo, Q.red_hi, Q.count_lo, Q.qs, (QState *)Q.h_qs, st));
        mark(S.evp[1]);
    } else {
        hip_check(launch_centres(Q.sa, st));
        mark(S.evp[0]);
        if (Q.radius >= 0 && !Q.paper) {
            hip_check(launch_window(Q.wa, st));
            mark(S.evp[1]);
        }
        hip_check(launch_members(Q.ma, st));
        mark(S.evp[2]);
        hip_check(launch_dense_tiles(Q.ta, st));
        mark(S.evp[4]);
        hip_check(launch_surv_tiles(Q.ta, st));
        mark(S.evp[5]);
        if (Q.paper) {  // localisation on I around the conditioned image's best
            hip_check(launch_window(Q.wa, st));
            mark(S.evp[1]);
        }
        hip_check(launch_reduce(Q.recs, Q.red_lo, Q.red_hi, Q.count_lo, Q.qs, (QState *)Q.h_qs, st));
        mark(S.evp[3]);
    }
}

// Graph cache of a slot: a launch sequence is run eagerly the first time its
// key is seen, captured the second time and replayed from then on (shapes
// that come once are never captured).  The key holds every argument of the
// sequence, so equal keys mean identical work.
static const int kGraphCache = 16;

static hipGraphExec_t graph_for(Slot &S, const std::string &key, bool *capture)
{
    *capture = false;
    S.graph_clock++;
    for (auto &g : S.graphs)
        if (g.key == key) {
            g.stamp = S.graph_clock;
            if (!g.exec)
                *capture = true;
            return g.exec;
        }
    if ((int)S.graphs.size() >= kGraphCache) {
        auto old = S.graphs.begin();
        for (auto it = S.graphs.begin(); it != S.graphs.end(); ++it)
            if (it->stamp < old->stamp)
                old = it;
        if (old->exec)
            (void)hipGraphExecDestroy(old->exec);
        S.graphs.erase(old);
    }
    S.graphs.push_back(SlotGraph{key, nullptr, S.graph_clock});
    return nullptr;
}

// Runs `enqueue` (work on st only, no fills) through the slot's graph cache.
template <class F> static void run_cached(Slot &S, const std::string &key, hipStream_t st, F &&enqueue)
{
    bool capture = false;
    hipGraphExec_t exec = graph_for(S, key, &capture);
    if (capture) {
        hipGraph_t g = nullptr;
        hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            enqueue();
        } catch (...) {
            (void)hipStreamEndCapture(st, &g);
            if (g)
                (void)hipGraphDestroy(g);
            throw;
        }
        hip_check(hipStreamEndCapture(st, &g));
        hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hip_check(e);
        for (auto &sg : S.graphs)
            if (sg.stamp == S.graph_clock)
                sg.exec = exec;
    }
    if (exec)
        hip_check(hipGraphLaunch(exec, st));
    else
        enqueue();
}

// Enqueues one query on S.stream: scan 1, the optional refinement window,
// scan 2 with survivors, the final reduction, and the copy of the query state
// to pinned host memory.  Repeated launch sequences run as a replayed graph.
void launch_query(const QueryPlan &q, Slot &S, int8_t *dec_host)
{
    const int64_t L = (int64_t)q.Ly * q.Lx;
    hipStream_t st = S.stream;
    int8_t *d_dec = nullptr;
    if (q.want_dec) {
        hip_check(hipMemsetAsync(S.dec.ptr, 0x7f, (size_t)L, st));
        d_dec = S.dec.as<int8_t>();
    }
    QueryLaunch Q;
    build_query_launch(q, slot_bufs(S), d_dec, Q);
    const bool timing = q.pr.timing != 0;
    const bool graphable = S.use_graphs && !timing && !q.want_dec && !q.num_map && !q.dr_map && !q.rho_map;
    S.timed = timing;
    S.qseq++;  // the sequence number this query's final reduction publishes
    if (timing)
        hip_check(hipEventRecord(S.ev0, st));
    if (graphable)
        run_cached(S, std::string((const char *)&Q, sizeof Q), st, [&] { enqueue_query(Q, S, st, false); });
    else
        enqueue_query(Q, S, st, timing);
    if (timing)
        hip_check(hipEventRecord(S.ev1, st));
    if (dec_host)
        hip_check(hipMemcpyAsync(dec_host, S.dec.ptr, (size_t)L, hipMemcpyDeviceToHost, st));
}

// Waits until the slot's host mirror carries the sequence number of the last
// launched query (the final reduction writes it after the rest of the state).
// The stream is polled every 50 us so that a failed launch ends the wait with
// its error.
static void wait_seq(const QState *mirror, unsigned long long want, hipStream_t stream)
{
    const volatile unsigned long long *seq = &mirror->seq;
    auto next = std::chrono::steady_clock::now() + std::chrono::microseconds(50);
    while (*seq != want) {
        if (std::chrono::steady_clock::now() < next)
            continue;
        hipError_t e = hipStreamQuery(stream);
        if (e == hipSuccess) {
            if (*seq == want)
                break;
            throw ZtsError{ZTS_E_DEVICE};  // the stream finished without publishing
        }
        if (e != hipErrorNotReady)
            hip_check(e);
        next = std::chrono::steady_clock::now() + std::chrono::microseconds(50);
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

static void wait_published(Slot &S) { wait_seq(S.h_qs.as<QState>(), S.qseq, S.stream); }

static zts_status assemble_result(const QueryPlan &q, const QState &h, Slot *timed, zts_result *out,
                                  double wall_khz);

// Waits for the query on S.stream and assembles its result.
zts_status finish_query(const QueryPlan &q, Slot &S, zts_result *out, double wall_khz)
{
    if (S.timed || q.want_dec)
        hip_check(hipStreamSynchronize(S.stream));  // events, or the decision map's copy
    wait_published(S);
    return assemble_result(q, *S.h_qs.as<QState>(), S.timed ? &S : nullptr, out, wall_khz);
}

// The result of a query from its published state (timed: the slot whose
// events timed its kernels, or NULL).
static zts_status assemble_result(const QueryPlan &q, const QState &h, Slot *timed, zts_result *out,
                                  double wall_khz)
{
    if (h.degenerate)
        return ZTS_E_DEGENERATE;
    const int Lx = q.Lx;
    const int64_t L = (int64_t)q.Ly * Lx;
    zts_result r;
    std::memset(&r, 0, sizeof r);
    r.y = (int32_t)(h.fin.l / Lx);
    r.x = (int32_t)(h.fin.l % Lx);
    r.rho = h.fin.rho;
    r.rho32 = h.fin_r32;
    r.num = h.fin.num;
    r.den_t = h.dt;
    r.den_r = h.fin.dr;
    r.n_locations = L;
    r.batch_size = 1;
    if (q.mode == ZTS_FULL) {
        r.n_computed = L;
        r.group_h = r.group_w = 1;
        r.best0 = h.fin.rho;
        r.best0_y = r.y;
        r.best0_x = r.x;
    } else {
        const Prepared *P = q.P;
        int64_t G = (int64_t)P->Gy * P->Gx;
        r.n_centres = G;
        r.n_eliminated = (int64_t)h.n_elim;
        r.n_survivors = (int64_t)h.n_surv;
        r.n_computed = (int64_t)h.n_window + (int64_t)h.n_surv + (q.mode == ZTS_OPTA ? 0 : G);
        r.group_h = P->h;
        r.group_w = P->w;
        r.best0 = h.best;
        r.best0_y = (int32_t)(h.best0_l / Lx);
        r.best0_x = (int32_t)(h.best0_l % Lx);
        // ZTS_OPTA_PAPER: the window's locations on I were also counted on J
        const int64_t expect = L + (q.mode == ZTS_OPTA_PAPER ? (int64_t)h.n_window : 0);
        if (r.n_computed + r.n_eliminated != expect)
            return ZTS_E_DEVICE;
    }
    // device time: HIP events when timed, else the device clock stamps of
    // the first kernel's start and the final reduction
    float ms = (float)((double)(h.t1 - h.t0) / wall_khz);
    if (timed)
        hip_check(hipEventElapsedTime(&ms, timed->ev0, timed->ev1));
    r.device_ms = ms;
    // per-kernel times, when the query was launched with its events
    auto span = [](float *out, hipEvent_t a, hipEvent_t b) { hip_check(hipEventElapsedTime(out, a, b)); };
    if (timed && q.mode == ZTS_FULL) {
        span(&r.phase_ms[0], timed->ev0, timed->evp[0]);
        span(&r.phase_ms[3], timed->evp[0], timed->evp[1]);
    } else if (timed) {
        // launch order: scan 1, [window], scan 2, dense tiles, sparse tiles, [window of the paper's
        // search], reduction
        hipEvent_t *e = timed->evp;
        const bool paper = q.mode == ZTS_OPTA_PAPER, win = query_radius(q) >= 0;
        span(&r.phase_ms[0], timed->ev0, e[0]);
        if (paper) {
            span(&r.phase_ms[2], e[0], e[2]);
            span(&r.phase_ms[4], e[2], e[4]);
            span(&r.phase_ms[5], e[4], e[5]);
            span(&r.phase_ms[1], e[5], e[1]);
            span(&r.phase_ms[3], e[1], e[3]);
        } else {
            if (win)
                span(&r.phase_ms[1], e[0], e[1]);
            span(&r.phase_ms[2], win ? e[1] : e[0], e[2]);
            span(&r.phase_ms[4], e[2], e[4]);
            span(&r.phase_ms[5], e[4], e[5]);
            span(&r.phase_ms[3], e[5], e[3]);
        }
    }
    r.above_floor = r.rho >= q.pr.rho_floor;
    r.n_dense = q.mode == ZTS_FULL ? 0 : (int64_t)h.n_dense;
    r.n_sparse = q.mode == ZTS_FULL ? 0 : (int64_t)h.n_sparse;
    r.status = ZTS_OK;
    *out = r;
    return ZTS_OK;
}

// ------------------------------------------------------------------ batched launches

void unpin_batch(BatchPlan &b)
{
    for (Stats *s : b.stats)
        if (s)
            s->pins--;
    b.stats.clear();
}

// Groups the items by (image, m, n) into jobs, pins their statistics, sizes
// the slot's batch buffers and fills the job table with device addresses.
// Device data layout of S.bdata: [job table][templates of every job][tst].
// Smallest group of one size that shares 16-template tiles.  Measured
// (zts_tune_batch): the least T >= 2 with ceil(T / 16) shared < T single.
// Otherwise a fit of such measurements on MI355X: a shared tile costs as much
// as 3 + 0.055 s single searches, s = sqrt(m n16) (square sizes 16..128 on a
// 4096x4096 image).
static int multi_min_of(const Ctx *c, int m, int n)
{
    auto it = c->tuned.find(std::make_pair(m, n));
    if (it != c->tuned.end())
        return it->second.multi_min;
    double sz = std::sqrt((double)m * ((n + 15) / 16 * 16));
    return std::max(2, (int)std::ceil(3.0 + 0.055 * sz));
}

static int multi_min_from(float single_ms, float shared_ms)
{
    if (!(single_ms > 0.0f))
        return 1;
    for (int T = 2; T <= 16; T++)
        if (shared_ms < T * single_ms)
            return T;
    return INT32_MAX;  // a tile of 16 costs more than 16 lone templates
}


BatchPlan plan_batch(Ctx *c, Slot &S, std::vector<BatchItem> items, int force)
{
    BatchPlan b;
    b.items = std::move(items);
    // buckets of (image, m, n) in first-appearance order
    std::map<std::tuple<Image *, int, int>, int> bid;
    std::vector<std::vector<int>> buckets;
    for (int k = 0; k < (int)b.items.size(); k++) {
        const BatchItem &it = b.items[k];
        auto key = std::make_tuple(it.im, it.m, it.n);
        auto f = bid.find(key);
        if (f == bid.end()) {
            bid[key] = (int)buckets.size();
            buckets.emplace_back();
            buckets.back().push_back(k);
        } else {
            buckets[f->second].push_back(k);
        }
    }
    // A bucket of enough templates shares 16-wide template tiles (k_batch);
    // smaller ones run each template on its own (k_single, no empty template
    // columns); multi_min_of gives the crossover.  BATCH_MULTI jobs come first
    // in the table.
    auto add_job = [&](const std::vector<int> &mem, int kind) {
        const BatchItem &it = b.items[mem[0]];
        BatchJob J;
        std::memset(&J, 0, sizeof J);
        J.img = it.im->img.as<uint8_t>();
        J.pitch = it.im->pitch;
        J.p = it.im->rows;
        J.q = it.im->cols;
        J.m = it.m;
        J.n = it.n;
        J.Ly = it.im->rows - it.m + 1;
        J.Lx = it.im->cols - it.n + 1;
        J.kind = kind;
        b.jobs.push_back(J);
        b.members.push_back(mem);
    };
    for (int pass = 0; pass < 2; pass++)
        for (auto &bk : buckets) {
            const BatchItem &it = b.items[bk[0]];
            bool multi = force == BATCH_MULTI || !batch_single_fits(it.m, it.n) ||
                         (force != BATCH_SINGLE && (int)bk.size() >= multi_min_of(c, it.m, it.n));
            if (pass == 0 && multi)
                add_job(bk, BATCH_MULTI);
            if (pass == 1 && !multi)
                for (int k : bk)
                    add_job(std::vector<int>{k}, BATCH_SINGLE);
        }
    // Two row groups (32 output rows) per k_single block: the body runs every
    // row group in every step, which keeps the rows of a block few.
    for (BatchJob &J : b.jobs)
        J.rg = J.kind == BATCH_SINGLE ? 2 : 0;
    const size_t njobs = b.jobs.size();
    b.table_bytes = (njobs * sizeof(BatchJob) + 255) & ~(size_t)255;
    size_t off = b.table_bytes;
    std::vector<size_t> tpl_off(njobs), rec_off(njobs);
    int block0 = 0, fold0 = 0, tmpl0 = 0;
    size_t nrec = 0;
    for (size_t j = 0; j < njobs; j++) {
        BatchJob &J = b.jobs[j];
        J.T = (int)b.members[j].size();
        if (!batch_job_geometry(J))
            throw ZtsError{ZTS_E_SIZE};
        if (j > 0 && J.kind != b.jobs[j - 1].kind)
            block0 = 0;  // each kernel numbers its own blocks
        int64_t nb = (int64_t)block0 + (int64_t)J.gx * J.gy * J.gz;
        if (nb > INT32_MAX)
            throw ZtsError{ZTS_E_SIZE};
        J.block0 = block0;
        block0 = (int)nb;
        J.fold0 = fold0;
        fold0 += J.gz * J.chunks;
        J.tmpl0 = tmpl0;
        tmpl0 += J.T;
        tpl_off[j] = off;
        off += ((size_t)J.T * J.m * J.n16 + 255) & ~(size_t)255;
        rec_off[j] = nrec;
        nrec += batch_job_records(J);
    }
    b.tpl_bytes = off;
    b.nrec = nrec;
    b.ntpl = tmpl0;
    try {
        for (size_t j = 0; j < njobs; j++) {
            const BatchItem &it = b.items[b.members[j][0]];
            Stats *st = stats_entry(c, it.im, it.m, it.n, S.stream);
            st->pins++;
            b.stats.push_back(st);
        }
        dalloc(c, S.bdata, b.tpl_bytes + sizeof(int64_t) * 2 * (size_t)b.ntpl);
        dalloc(c, S.bres, sizeof(RecPod) * (size_t)b.ntpl);
        dalloc(c, S.brec, sizeof(RecPod) * b.nrec);
        S.h_stage.grow(b.tpl_bytes);
        S.h_out.grow((sizeof(RecPod) + 2 * sizeof(int64_t)) * (size_t)b.ntpl);
    } catch (...) {
        unpin_batch(b);
        throw;
    }
    uint8_t *base = S.bdata.as<uint8_t>();
    int64_t *tst = (int64_t *)(base + b.tpl_bytes);
    for (size_t j = 0; j < njobs; j++) {
        BatchJob &J = b.jobs[j];
        J.stat = b.stats[j]->stat.as<int2>();
        J.tpl = base + tpl_off[j];
        J.tst = tst + 2 * (size_t)J.tmpl0;
        J.recs = S.brec.as<RecPod>() + rec_off[j];
        J.out = S.bres.as<RecPod>() + J.tmpl0;
    }
    return b;
}

// Stages the templates (0x80 past column n) and the job table in pinned
// memory, copies them in one transfer and enqueues the fused launch.
void launch_batch_plan(BatchPlan &b, Slot &S)
{
    uint8_t *h = S.h_stage.as<uint8_t>();
    std::memcpy(h, b.jobs.data(), b.jobs.size() * sizeof(BatchJob));
    const uint8_t *dbase = S.bdata.as<uint8_t>();
    for (size_t j = 0; j < b.jobs.size(); j++) {
        const BatchJob &J = b.jobs[j];
        uint8_t *dst0 = h + (J.tpl - dbase);
        for (int t = 0; t < J.T; t++) {
            const BatchItem &it = b.items[b.members[j][t]];
            uint8_t *dst = dst0 + (size_t)t * J.m * J.n16;
            if (it.device) {  // copied device to device below; columns past n stay 0x80
                std::memset(dst, 0x80, (size_t)J.m * J.n16);
                continue;
            }
            for (int r = 0; r < J.m; r++) {
                std::memcpy(dst + (size_t)r * J.n16, it.tpl + (size_t)r * it.stride, J.n);
                std::memset(dst + (size_t)r * J.n16 + J.n, 0x80, J.n16 - J.n);
            }
        }
    }
    hipStream_t st = S.stream;
    hip_check(hipMemcpyAsync(S.bdata.ptr, h, b.tpl_bytes, hipMemcpyHostToDevice, st));
    for (size_t j = 0; j < b.jobs.size(); j++) {
        const BatchJob &J = b.jobs[j];
        for (int t = 0; t < J.T; t++) {
            const BatchItem &it = b.items[b.members[j][t]];
            if (it.device)
                hip_check(hipMemcpy2DAsync((uint8_t *)J.tpl + (size_t)t * J.m * J.n16, J.n16, it.tpl, it.stride, J.n,
                                           J.m, hipMemcpyDeviceToDevice, st));
        }
    }
    hip_check(hipEventRecord(S.ev0, st));
    // the kernels of a repeated plan (same jobs, same buffers) replay a graph
    std::string key((const char *)b.jobs.data(), b.jobs.size() * sizeof(BatchJob));
    key.append((const char *)&S.bdata.ptr, sizeof S.bdata.ptr);
    key.append("batch");
    auto kernels = [&] { hip_check(launch_batch_jobs(S.bdata.as<BatchJob>(), b.jobs.data(), (int)b.jobs.size(), st)); };
    if (S.use_graphs)
        run_cached(S, key, st, kernels);
    else
        kernels();
    hip_check(hipEventRecord(S.ev1, st));
    uint8_t *ho = S.h_out.as<uint8_t>();
    hip_check(hipMemcpyAsync(ho, S.bres.ptr, sizeof(RecPod) * (size_t)b.ntpl, hipMemcpyDeviceToHost, st));
    hip_check(hipMemcpyAsync(ho + sizeof(RecPod) * (size_t)b.ntpl, S.bdata.as<uint8_t>() + b.tpl_bytes,
                             sizeof(int64_t) * 2 * (size_t)b.ntpl, hipMemcpyDeviceToHost, st));
}

void finish_batch(const BatchPlan &b, Slot &S, zts_result *out)
{
    hip_check(hipStreamSynchronize(S.stream));
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, S.ev0, S.ev1));
    const RecPod *res = S.h_out.as<RecPod>();
    const int64_t *tst = (const int64_t *)(S.h_out.as<uint8_t>() + sizeof(RecPod) * (size_t)b.ntpl);
    for (size_t j = 0; j < b.jobs.size(); j++) {
        const BatchJob &J = b.jobs[j];
        for (int t = 0; t < J.T; t++) {
            const RecPod &f = res[J.tmpl0 + t];
            int64_t D_t = tst[2 * (J.tmpl0 + t) + 1];
            zts_result r;
            std::memset(&r, 0, sizeof r);
            int64_t L = (int64_t)J.Ly * J.Lx;
            r.n_locations = L;
            r.device_ms = ms;
            r.phase_ms[0] = ms;
            r.batch_size = (int32_t)b.items.size();
            if (D_t == 0 || !f.valid) {
                r.status = D_t == 0 ? ZTS_E_DEGENERATE : ZTS_E_DEVICE;
            } else {
                r.y = (int32_t)(f.l / J.Lx);
                r.x = (int32_t)(f.l % J.Lx);
                r.rho = f.rho;
                r.rho32 = f.r32max;
                r.num = f.num;
                r.den_t = D_t;
                r.den_r = f.dr;
                r.n_computed = L;
                r.group_h = r.group_w = 1;
                r.best0 = f.rho;
                r.best0_y = r.y;
                r.best0_x = r.x;
                r.above_floor = 1;  // a batch has no floor (the defaults)
                r.status = ZTS_OK;
            }
            out[b.members[j][t]] = r;
        }
    }
}

// ------------------------------------------------------------------ allocation-free search

// Device scratch of zts_search_device_noalloc, one copy per GPU, held until
// the process ends: the query state, the per-block records, the per-group
// centre sums and angles, and the survivor tiles' counts and bins of one
// query.  In host code the name `scratch` is a host-side stand-in, never a
// device address: host code uses only the address hipGetSymbolAddress
// returned for each device (scratch_setup).
constexpr size_t kNoAllocScratchBytes = (size_t)96 << 20;

}  // namespace zts

static __device__ __align__(256) uint8_t scratch[zts::kNoAllocScratchBytes];

namespace zts {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_setup_mu;
void *g_scratch_ptr[kMaxDevices];      // device address of `scratch` on each GPU, looked up once
std::mutex g_scratch_mu[kMaxDevices];  // one allocation-free search at a time per GPU

}  // namespace

// Looks up the device address of `scratch` on device `dev`, which must be
// current, once per device (zts_create calls it).
void scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices)
        throw ZtsError{ZTS_E_DEVICE};
    std::lock_guard<std::mutex> lk(g_scratch_setup_mu);
    if (g_scratch_ptr[dev])
        return;
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr)
        throw ZtsError{ZTS_E_DEVICE};
    g_scratch_ptr[dev] = ptr;
}

static uint8_t *scratch_ptr(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_setup_mu);
    if (dev < 0 || dev >= kMaxDevices || !g_scratch_ptr[dev])
        throw ZtsError{ZTS_E_DEVICE};
    return (uint8_t *)g_scratch_ptr[dev];
}

// A query plan from what is already resident: the image's statistics for
// (m, n) and, for the eliminating modes, tables prepared with the same
// parameters.  Nothing is built or allocated; ZTS_E_NOTPREPARED otherwise.
static QueryPlan plan_resident(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr)
{
    QueryPlan q;
    q.im = im;
    q.m = m;
    q.n = n;
    q.Ly = im->rows - m + 1;
    q.Lx = im->cols - n + 1;
    q.mode = mode;
    q.pr = pr;
    auto st = im->stats.find(std::make_pair(m, n));
    if (st == im->stats.end())
        throw ZtsError{ZTS_E_NOTPREPARED};
    if (mode != ZTS_FULL) {
        auto it = im->prep.find(std::make_tuple(m, n, (int)mode));
        if (it == im->prep.end() || !same_prep_params(*it->second, mode, pr))
            throw ZtsError{ZTS_E_NOTPREPARED};
        q.P = it->second.get();
    }
    hip_check(hipStreamWaitEvent(c->stream, st->second->ready, 0));
    q.st = st->second.get();
    q.st->pins++;
    q.st->last_use = ++c->clock;
    if (q.P) {
        q.P->pins++;
        q.P->last_use = ++c->clock;
    }
    return q;
}

// One query with every buffer it needs taken from the device's `scratch`
// (context lock held).  ZTS_E_SIZE when the query's scratch exceeds it.
static void run_query_noalloc(Ctx *c, Image *im, const uint8_t *tpl, int m, int n, int64_t stride,
                              hipStream_t caller, zts_mode mode, const zts_params &pr, zts_result *out)
{
    // scratch layout, 256-byte aligned parts: query state, records, centre sums, centre angles
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return at;
    };
    const int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
    QueryPlan q = plan_resident(c, im, m, n, mode, pr);
    zts_status st = ZTS_OK;
    try {
        size_t nrec = 0, groups = 0, ntile = 0, cap = 0;
        if (mode == ZTS_FULL) {
            nrec = (size_t)full_record_count(Ly, Lx);
        } else {
            const Prepared *P = q.P;
            const int radius = query_radius(q);
            const TileArgs tg = tile_geometry(q);
            ntile = (size_t)tg.tiles_x * tg.tiles_y;
            cap = (size_t)tg.tile_cap;
            nrec = (size_t)centres_record_count(P->Gy, P->Gx, m, n, P->h, P->w) +
                   (size_t)(radius >= 0 ? window_record_count(radius) : 0) +
                   (size_t)members_record_count(P->Gy, P->Gx) + (size_t)tile_record_count(tg);
            groups = (size_t)P->Gy * P->Gx;
        }
        const size_t o_qs = take(sizeof(QState)), o_rec = take(sizeof(RecPod) * nrec);
        const size_t o_gx = take(sizeof(int32_t) * groups), o_gt = take(sizeof(float) * groups);
        const size_t o_tc = take(sizeof(uint32_t) * ntile), o_tb = take(sizeof(int32_t) * ntile * cap);
        if (off > kNoAllocScratchBytes)
            throw ZtsError{ZTS_E_SIZE};
        q.tpl = tpl;
        q.ts = stride;
        std::lock_guard<std::mutex> dl(g_scratch_mu[c->device]);
        uint8_t *base = scratch_ptr(c->device);
        QState *mirror = c->h_qs_noalloc.as<QState>();
        const QueryBufs B{(QState *)(base + o_qs), (RecPod *)(base + o_rec), (int32_t *)(base + o_gx),
                          (float *)(base + o_gt), (uint32_t *)(base + o_tc), (int32_t *)(base + o_tb), nullptr,
                          mirror};
        hipStream_t s = c->stream;
        // the kernels read the caller's template in place, after the caller's
        // stream has reached this call
        if (caller != s && hipStreamQuery(caller) != hipSuccess) {
            (void)hipGetLastError();  // hipErrorNotReady: work is pending
            hip_check(hipEventRecord(c->main.ev_in, caller));
            hip_check(hipStreamWaitEvent(s, c->main.ev_in, 0));
        }
        // the state keeps the previous call's contents (any context on this
        // GPU): it starts from zero, so the final reduction publishes 1
        *(volatile unsigned long long *)&mirror->seq = 0;
        hip_check(launch_qs_clear(B.qs, s));
        QueryLaunch Q;
        build_query_launch(q, B, nullptr, Q);
        enqueue_query(Q, c->main, s, false);
        wait_seq(mirror, 1, s);
        st = assemble_result(q, *mirror, nullptr, out, c->wall_khz);
    } catch (...) {
        unpin_query(q);
        throw;
    }
    unpin_query(q);
    if (st != ZTS_OK)
        throw ZtsError{st};
}

// ------------------------------------------------------------------ synchronous helpers

namespace {

template <class F> zts_status guarded(Ctx *c, F &&f)
{
    if (!c)
        return ZTS_E_ARG;
    std::unique_lock<std::mutex> lk(c->mu);
    CtxLockScope scope(lk);
    try {
        hip_check(hipSetDevice(c->device));
        f();
        return ZTS_OK;
    } catch (const ZtsError &e) {
        return e.st;
    } catch (const std::bad_alloc &) {
        return ZTS_E_NOMEM;
    }
}

// One query on the main slot (context lock held).
void run_query_main(Ctx *c, Image *im, const uint8_t *tpl, int m, int n, int64_t stride, bool device,
                    hipStream_t caller, zts_mode mode, const zts_params &pr, zts_result *out, int8_t *dec,
                    int64_t *num_map = nullptr, int64_t *dr_map = nullptr, float *rho_map = nullptr)
{
    QueryPlan q = plan_query(c, c->main, im, m, n, mode, pr, dec != nullptr);
    q.num_map = num_map;
    q.dr_map = dr_map;
    q.rho_map = rho_map;
    zts_status st;
    try {
        if (device) {
            // the kernels read the caller's template in place, after the
            // caller's stream has reached this call (nothing to wait for when
            // that stream is idle)
            q.tpl = tpl;
            q.ts = stride;
            if (caller != c->main.stream && hipStreamQuery(caller) != hipSuccess) {
                (void)hipGetLastError();  // hipErrorNotReady: work is pending
                hip_check(hipEventRecord(c->main.ev_in, caller));
                hip_check(hipStreamWaitEvent(c->main.stream, c->main.ev_in, 0));
            }
        } else {
            stage_template(c->main, tpl, m, n, stride);
        }
        launch_query(q, c->main, dec);
        st = finish_query(q, c->main, out, c->wall_khz);
    } catch (...) {
        unpin_query(q);
        throw;
    }
    unpin_query(q);
    if (st != ZTS_OK)
        throw ZtsError{st};
}

// A batch on the main slot (context lock held).
void run_batch_main(Ctx *c, std::vector<BatchItem> items, zts_result *out)
{
    BatchPlan b = plan_batch(c, c->main, std::move(items));
    try {
        launch_batch_plan(b, c->main);
        finish_batch(b, c->main, out);
    } catch (...) {
        unpin_batch(b);
        throw;
    }
    unpin_batch(b);
}

zts_status load_common(Ctx *c, const void *src, int rows, int cols, int64_t stride, bool device, hipStream_t caller,
                       int *id)
{
    if (!src || !id || rows < 1 || cols < 1 || stride < cols)
        return ZTS_E_ARG;
    if (rows > 32767 || cols > 32767)  // group geometry is packed in 16-bit fields
        return ZTS_E_SIZE;
    return guarded(c, [&] {
        auto im = std::make_unique<Image>();
        im->rows = rows;
        im->cols = cols;
        im->pitch = pitch_for(cols);
        alloc_image(c, im->img, rows, im->pitch);
        hipStream_t s = c->stream;
        if (device && caller && caller != c->stream) {
            hip_check(hipStreamSynchronize(c->stream));
            s = caller;
        }
        hip_check(hipMemcpy2DAsync(im->img.ptr, im->pitch, src, stride, cols, rows,
                                   device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        if (s != c->stream)
            hip_check(hipStreamSynchronize(s));
        build_sat(c, im->img.as<uint8_t>(), im->pitch, rows, cols, im->sat);
        hip_check(hipStreamSynchronize(c->stream));
        int nid = c->next_id++;
        c->images[nid] = std::move(im);
        *id = nid;
    });
}

bool valid_mode(zts_mode mode)
{
    return mode == ZTS_FULL || mode == ZTS_FULL_MFMA || mode == ZTS_TE_FIXED || mode == ZTS_EGS || mode == ZTS_OPTA ||
           mode == ZTS_OPTA_PAPER;
}

}  // namespace

// ------------------------------------------------------------------ batched pruned search

namespace {

// Every kernel of one query after scan 1 (the batched search runs scan 1 for
// several templates of one size in one launch).
void enqueue_after_scan1(const QueryLaunch &Q, hipStream_t st)
{
    if (Q.radius >= 0 && !Q.paper)
        hip_check(launch_window(Q.wa, st));
    hip_check(launch_members(Q.ma, st));
    hip_check(launch_dense_tiles(Q.ta, st));
    hip_check(launch_surv_tiles(Q.ta, st));
    if (Q.paper)  // localisation on I around the conditioned image's best
        hip_check(launch_window(Q.wa, st));
    hip_check(launch_reduce(Q.recs, Q.red_lo, Q.red_hi, Q.count_lo, Q.qs, (QState *)Q.h_qs, st));
}

// One template's device scratch in a batched search.
struct PrunedBufs {
    DBuf qs, recs, gnum, gtheta, tcnt, tbin;
};

// The batched pruned search on the main slot (context lock held): every size
// prepared and pinned first, then per size one scan-1 launch for up to
// kScanMaxT templates at a time (one per template when its shape has no MFMA
// form), each template's remaining kernels with its own scratch, one stream
// synchronisation at the end.
void run_pruned_batch(Ctx *c, Image *im, int count, const uint8_t *const *tpls, const int32_t *ms, const int32_t *ns,
                      const int64_t *strides, bool device, hipStream_t caller, zts_mode mode, const zts_params &pr,
                      zts_result *out)
{
    Slot &S = c->main;
    const hipStream_t st = S.stream;
    if (device && caller != st && hipStreamQuery(caller) != hipSuccess) {
        // the kernels read the caller's templates in place, after its stream
        (void)hipGetLastError();  // hipErrorNotReady: work is pending
        hip_check(hipEventRecord(S.ev_in, caller));
        hip_check(hipStreamWaitEvent(st, S.ev_in, 0));
    }
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int k = 0; k < count; k++)
        groups[std::make_pair(ms[k], ns[k])].push_back(k);
    std::vector<QueryPlan> plans(count);
    std::vector<PrunedBufs> bufs(count);
    std::vector<QueryLaunch> Q(count);
    DBuf dtpl;
    auto unpin_all = [&] {
        for (auto &q : plans)
            unpin_query(q);
    };
    try {
        // tables and statistics of every size, pinned for the whole call
        for (auto &gr : groups) {
            const int m = gr.first.first, n = gr.first.second;
            for (int k : gr.second) {
                QueryPlan &q = plans[k];
                q.im = im;
                q.m = m;
                q.n = n;
                q.Ly = im->rows - m + 1;
                q.Lx = im->cols - n + 1;
                q.mode = mode;
                q.pr = pr;
                q.st = stats_entry(c, im, m, n, st);
                q.st->pins++;
                q.P = prepare(c, im, m, n, mode, pr);
                q.P->pins++;
                q.P->last_use = ++c->clock;
            }
        }
        // host templates: packed at pitch n, through pinned staging in one copy
        std::vector<size_t> off(count);
        size_t total = 0;
        uint8_t *h = nullptr;
        if (!device) {
            for (int k = 0; k < count; k++) {
                off[k] = total;
                total += ((size_t)ms[k] * ns[k] + 255) & ~(size_t)255;
            }
            S.h_stage.grow(total);
            h = S.h_stage.as<uint8_t>();
            for (int k = 0; k < count; k++)
                for (int i = 0; i < ms[k]; i++)
                    std::memcpy(h + off[k] + (size_t)i * ns[k], tpls[k] + (size_t)i * strides[k], ns[k]);
            dalloc(c, dtpl, total);
        }
        c->h_batch_qs.grow(sizeof(QState) * (size_t)count, hipHostMallocCoherent);
        QState *mirror = c->h_batch_qs.as<QState>();
        for (int k = 0; k < count; k++) {
            QueryPlan &q = plans[k];
            const Prepared *P = q.P;
            q.tpl = device ? tpls[k] : dtpl.as<uint8_t>() + off[k];
            q.ts = device ? strides[k] : ns[k];
            const int radius = query_radius(q);
            const TileArgs tg = tile_geometry(q);
            const size_t ntile = (size_t)tg.tiles_x * tg.tiles_y;
            const size_t nrec = (size_t)centres_record_count(P->Gy, P->Gx, q.m, q.n, P->h, P->w) +
                                (size_t)(radius >= 0 ? window_record_count(radius) : 0) +
                                (size_t)members_record_count(P->Gy, P->Gx) + (size_t)tile_record_count(tg);
            PrunedBufs &b = bufs[k];
            dalloc(c, b.qs, sizeof(QState));
            dalloc(c, b.recs, sizeof(RecPod) * nrec);
            dalloc(c, b.gnum, sizeof(int32_t) * (size_t)P->Gy * P->Gx);
            dalloc(c, b.gtheta, sizeof(float) * (size_t)P->Gy * P->Gx);
            dalloc(c, b.tcnt, sizeof(uint32_t) * ntile);
            dalloc(c, b.tbin, sizeof(int32_t) * ntile * (size_t)tg.tile_cap);
            const QueryBufs B{b.qs.as<QState>(), b.recs.as<RecPod>(), b.gnum.as<int32_t>(), b.gtheta.as<float>(),
                              b.tcnt.as<uint32_t>(), b.tbin.as<int32_t>(), nullptr, mirror + k};
            build_query_launch(q, B, nullptr, Q[k]);
        }
        if (!device)
            hip_check(hipMemcpyAsync(dtpl.ptr, h, total, hipMemcpyHostToDevice, st));
        // The scan-1 launches go to the main stream, one after another; the
        // templates' own chains (window, scan 2, tiles, reduction) take the
        // auxiliary streams in turn, each after an event recorded behind its
        // scan 1, so that one chain's tail overlaps the next one's start.
        if (!c->aux[0]) {
            for (int k = 0; k < Ctx::kAuxStreams; k++)
                hip_check(hipStreamCreateWithFlags(&c->aux[k], hipStreamNonBlocking));
            for (hipEvent_t &e : c->aux_ev)
                hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        int next_lane = 0;
        bool used[Ctx::kAuxStreams] = {};
        // the largest templates first: their scan 1 is the longest, and the
        // smaller sizes' scans then overlap with the larger ones' chains
        for (auto git = groups.rbegin(); git != groups.rend(); ++git) {
            auto &gr = *git;
            const std::vector<int> &ks = gr.second;
            const Prepared *P = plans[ks[0]].P;
            const bool shared = ks.size() > 1 && centres_mfma_batchable(P->Gy, P->Gx, gr.first.first, gr.first.second, P->w, 2);
            size_t i = 0;
            while (i < ks.size()) {
                int T = 1;
                if (shared)
                    while (T < kScanMaxT && i + T < ks.size() &&
                           centres_mfma_batchable(P->Gy, P->Gx, gr.first.first, gr.first.second, P->w, T + 1))
                        T++;
                ScanArgs sa = Q[ks[i]].sa;
                sa.ntpl = T;
                for (int j = 1; j < T; j++) {
                    const ScanArgs &o = Q[ks[i + j]].sa;
                    sa.more[j - 1] = ScanTpl{o.tpl, o.ts, o.g_x, o.g_theta, o.recs, o.qs, o.tile_cnt};
                }
                hip_check(launch_centres(sa, st));
                // the scan-1 event of this launch (events are reused: a wait
                // takes the event's state at the time it is enqueued)
                hip_check(hipEventRecord(c->aux_ev[0], st));
                for (int j = 0; j < T; j++) {
                    const int ln = next_lane;
                    next_lane = (next_lane + 1) % Ctx::kAuxStreams;
                    hip_check(hipStreamWaitEvent(c->aux[ln], c->aux_ev[0], 0));
                    used[ln] = true;
                    enqueue_after_scan1(Q[ks[i + j]], c->aux[ln]);
                }
                i += T;
            }
        }
        for (int k = 0; k < Ctx::kAuxStreams; k++)
            if (used[k]) {
                hip_check(hipEventRecord(c->aux_ev[k + 1], c->aux[k]));
                hip_check(hipStreamWaitEvent(st, c->aux_ev[k + 1], 0));
            }
        hip_check(hipStreamSynchronize(st));
        std::atomic_thread_fence(std::memory_order_acquire);
        for (int k = 0; k < count; k++) {
            zts_result r;
            const zts_status s2 = assemble_result(plans[k], mirror[k], nullptr, &r, c->wall_khz);
            if (s2 == ZTS_E_DEVICE)
                throw ZtsError{ZTS_E_DEVICE};
            if (s2 != ZTS_OK)
                r = error_result(s2);
            r.batch_size = count;
            out[k] = r;
        }
    } catch (...) {
        unpin_all();
        throw;
    }
    unpin_all();
}

}  // namespace

}  // namespace zts

// ====================================================================== C ABI

using namespace zts;

extern "C" {

ZTS_API void zts_params_default(zts_params *p)
{
    if (p)
        fill_default(p);
}

ZTS_API zts_status zts_params_check(const zts_params *p)
{
    return p ? params_status(*p) : ZTS_E_ARG;
}

ZTS_API const char *zts_status_str(zts_status s)
{
    switch (s) {
    case ZTS_OK: return "ok";
    case ZTS_E_ARG: return "invalid argument";
    case ZTS_E_SIZE: return "template larger than the image or than 16384 pixels";
    case ZTS_E_DEGENERATE: return "template has zero variance";
    case ZTS_E_NOIMAGE: return "unknown image id";
    case ZTS_E_BUDGET: return "HBM budget exhausted";
    case ZTS_E_AGAIN: return "not ready";
    case ZTS_E_BUSY: return "busy";
    case ZTS_E_TIMEOUT: return "timed out";
    case ZTS_E_CANCELLED: return "cancelled";
    case ZTS_E_DEVICE: return "device error";
    case ZTS_E_NOMEM: return "out of memory";
    case ZTS_E_NOTPREPARED: return "not prepared";
    }
    return "unknown status";
}

static void load_tune_cache(Ctx *c);

ZTS_API zts_status zts_create(const zts_ctx_params *params, zts_ctx **out)
{
    if (!out)
        return ZTS_E_ARG;
    if (params && (params->max_inflight < 0 || params->max_inflight > 64 || params->max_queued < 0))
        return ZTS_E_ARG;
    zts_ctx *z = new (std::nothrow) zts_ctx;
    if (!z)
        return ZTS_E_NOMEM;
    Ctx &c = z->c;
    c.device = params ? params->device : 0;
    c.budget = params ? params->hbm_budget_bytes : 0;
    if (params && params->max_inflight > 0)
        c.max_inflight = params->max_inflight;
    if (params && params->max_queued > 0)
        c.max_queued = params->max_queued;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c.device < 0 || c.device >= ndev) {
        delete z;
        return ZTS_E_DEVICE;
    }
    try {
        hip_check(hipSetDevice(c.device));
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, c.device));
        int khz = 0;
        hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c.device));
        c.wall_khz = khz > 0 ? khz : 100000;
        c.arch = prop.gcnArchName;
        for (auto &ch : c.arch)
            if (ch == ' ')
                ch = '_';
        if (params && params->tune_cache)
            c.tune_cache = params->tune_cache;
        load_tune_cache(&c);
        c.main.init();
        c.stream = c.main.stream;
        c.h_cnt.grow(64);
        c.h_qs_noalloc.grow(sizeof(QState), hipHostMallocCoherent);  // written by the final reduction
        std::memset(c.h_qs_noalloc.ptr, 0, sizeof(QState));
        scratch_setup(c.device);
    } catch (const ZtsError &e) {
        c.main.destroy();
        delete z;
        return e.st;
    }
    *out = z;
    return ZTS_OK;
}

ZTS_API void zts_destroy(zts_ctx *z)
{
    if (!z)
        return;
    Ctx &c = z->c;
    server_shutdown(&c);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        (void)hipSetDevice(c.device);
        if (c.stream)
            (void)hipStreamSynchronize(c.stream);
        c.images.clear();
        c.counter.reset();
        c.tmp32.reset();
        c.viol.reset();
        c.colmask.reset();
        c.psat.reset();
        c.h_cnt.reset();
        c.h_qs_noalloc.reset();
        for (int k = 0; k < Ctx::kAuxStreams; k++)
            if (c.aux[k]) {
                (void)hipStreamSynchronize(c.aux[k]);
                (void)hipStreamDestroy(c.aux[k]);
            }
        for (hipEvent_t e : c.aux_ev)
            if (e)
                (void)hipEventDestroy(e);
        c.main.destroy();
        release_free_blocks(&c);
    }
    delete z;
}

ZTS_API zts_status zts_image_load(zts_ctx *z, const uint8_t *host, int32_t rows, int32_t cols, int64_t stride,
                                  int32_t *id)
{
    if (!z)
        return ZTS_E_ARG;
    return load_common(&z->c, host, rows, cols, stride, false, nullptr, id);
}

ZTS_API zts_status zts_image_load_device(zts_ctx *z, const void *dev, int32_t rows, int32_t cols, int64_t stride,
                                         void *stream, int32_t *id)
{
    if (!z)
        return ZTS_E_ARG;
    return load_common(&z->c, dev, rows, cols, stride, true, (hipStream_t)stream, id);
}

ZTS_API zts_status zts_image_unload(zts_ctx *z, int32_t id)
{
    if (!z)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, id);
        if (im->busy)
            throw ZtsError{ZTS_E_BUSY};
        hip_check(hipStreamSynchronize(c->stream));
        c->images.erase(id);
        release_free_blocks(c);  // give the image's memory back now
    });
}

ZTS_API zts_status zts_prepare(zts_ctx *z, int32_t image, int32_t m, int32_t n, zts_mode mode,
                               const zts_params *params, void *stream)
{
    if (!z || !valid_mode(mode))
        return ZTS_E_ARG;
    (void)stream;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        if (m < 1 || n < 1)
            throw ZtsError{ZTS_E_ARG};
        if (m > im->rows || n > im->cols || (int64_t)m * n > 16384)
            throw ZtsError{ZTS_E_SIZE};
        check_mode_shape(mode, m, n);
        const zts_params pr = params_or_default(params);
        if (mode == ZTS_FULL || mode == ZTS_FULL_MFMA) {
            stats_entry(c, im, m, n, c->stream);
            hip_check(hipStreamSynchronize(c->stream));
            return;
        }
        prepare(c, im, m, n, mode, pr);
    });
}

ZTS_API zts_status zts_prep_query(zts_ctx *z, int32_t image, int32_t m, int32_t n, zts_mode mode,
                                  zts_prep_info *out)
{
    if (!z || !out)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Image *im = find_image(&z->c, image);
        auto it = im->prep.find(std::make_tuple(m, n, (int)mode));
        if (it == im->prep.end())
            throw ZtsError{ZTS_E_NOTPREPARED};
        *out = it->second->info;
    });
}

ZTS_API zts_status zts_prep_image(zts_ctx *z, int32_t image, int32_t m, int32_t n, zts_mode mode,
                                  uint8_t *host_out)
{
    if (!z || !host_out || (mode != ZTS_OPTA && mode != ZTS_OPTA_PAPER))
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        auto it = im->prep.find(std::make_tuple(m, n, (int)mode));
        if (it == im->prep.end())
            throw ZtsError{ZTS_E_NOTPREPARED};
        hip_check(hipMemcpy2DAsync(host_out, im->cols, it->second->J.ptr, im->pitch, im->cols, im->rows,
                                   hipMemcpyDeviceToHost, c->stream));
        hip_check(hipStreamSynchronize(c->stream));
    });
}

ZTS_API zts_status zts_search(zts_ctx *z, int32_t image, const uint8_t *tpl, int32_t m, int32_t n, int64_t stride,
                              zts_mode mode, const zts_params *params, zts_result *out, int8_t *decision)
{
    if (!z || !out || !valid_mode(mode))
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl, m, n, stride);
        check_mode_shape(mode, m, n);
        const zts_params pr = params_or_default(params);
        if (mode == ZTS_FULL_MFMA) {
            if (n > 128)
                throw ZtsError{ZTS_E_SIZE};
            zts_result r;
            run_batch_main(c, {BatchItem{im, tpl, m, n, stride}}, &r);
            if (r.status != ZTS_OK)
                throw ZtsError{r.status};
            r.above_floor = r.rho >= pr.rho_floor;
            if (decision)
                std::memset(decision, 2, (size_t)(im->rows - m + 1) * (im->cols - n + 1));
            *out = r;
            return;
        }
        run_query_main(c, im, tpl, m, n, stride, false, nullptr, mode, pr, out, decision);
    });
}

ZTS_API zts_status zts_search_device(zts_ctx *z, int32_t image, const void *tpl_dev, int32_t m, int32_t n,
                                     int64_t stride, zts_mode mode, const zts_params *params, void *stream,
                                     zts_result *out)
{
    if (!z || !out || !valid_mode(mode))
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl_dev, m, n, stride);
        check_mode_shape(mode, m, n);
        const zts_params pr = params_or_default(params);
        if (mode == ZTS_FULL_MFMA) {
            if (n > 128)
                throw ZtsError{ZTS_E_SIZE};
            if (stream && (hipStream_t)stream != c->stream)  // the template is ready on the caller's stream
                hip_check(hipStreamSynchronize((hipStream_t)stream));
            BatchItem it{im, (const uint8_t *)tpl_dev, m, n, stride};
            it.device = true;
            zts_result r;
            run_batch_main(c, {it}, &r);
            if (r.status != ZTS_OK)
                throw ZtsError{r.status};
            r.above_floor = r.rho >= pr.rho_floor;
            *out = r;
            return;
        }
        run_query_main(c, im, (const uint8_t *)tpl_dev, m, n, stride, true, (hipStream_t)stream, mode, pr, out,
                       nullptr);
    });
}

ZTS_API zts_status zts_search_device_noalloc(zts_ctx *z, int32_t image, const void *tpl_dev, int32_t m, int32_t n,
                                             int64_t stride, zts_mode mode, const zts_params *params, void *stream,
                                             zts_result *out)
{
    if (!z || !out || !valid_mode(mode) || mode == ZTS_FULL_MFMA)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl_dev, m, n, stride);
        check_mode_shape(mode, m, n);
        const zts_params pr = params_or_default(params);
        hipStream_t caller = stream ? (hipStream_t)stream : c->stream;
        run_query_noalloc(c, im, (const uint8_t *)tpl_dev, m, n, stride, caller, mode, pr, out);
    });
}

ZTS_API zts_status zts_search_batch(zts_ctx *z, int32_t image, int32_t count, const uint8_t *const *tpls,
                                    const int32_t *m, const int32_t *n, const int64_t *strides, zts_result *out)
{
    if (!z || !tpls || !m || !n || !strides || !out || count < 1)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        std::vector<BatchItem> items;
        for (int k = 0; k < count; k++) {
            check_template_args(im, tpls[k], m[k], n[k], strides[k]);
            if (n[k] > 128)
                throw ZtsError{ZTS_E_SIZE};
            items.push_back(BatchItem{im, tpls[k], m[k], n[k], strides[k]});
        }
        std::vector<zts_result> res(count);
        run_batch_main(c, std::move(items), res.data());
        for (auto &r : res)
            if (r.status == ZTS_E_DEVICE)
                throw ZtsError{ZTS_E_DEVICE};
        std::copy(res.begin(), res.end(), out);
    });
}

ZTS_API zts_status zts_search_batch_pruned(zts_ctx *z, int32_t image, int32_t count, const uint8_t *const *tpls,
                                           const int32_t *m, const int32_t *n, const int64_t *strides, zts_mode mode,
                                           const zts_params *params, zts_result *out)
{
    if (!z || !tpls || !m || !n || !strides || !out || count < 1)
        return ZTS_E_ARG;
    if (mode != ZTS_TE_FIXED && mode != ZTS_EGS && mode != ZTS_OPTA && mode != ZTS_OPTA_PAPER)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        for (int k = 0; k < count; k++) {
            check_template_args(im, tpls[k], m[k], n[k], strides[k]);
            check_mode_shape(mode, m[k], n[k]);
        }
        const zts_params pr = params_or_default(params);
        std::vector<zts_result> res(count);
        run_pruned_batch(c, im, count, tpls, m, n, strides, false, nullptr, mode, pr, res.data());
        std::copy(res.begin(), res.end(), out);
    });
}

ZTS_API zts_status zts_search_batch_pruned_device(zts_ctx *z, int32_t image, int32_t count,
                                                  const void *const *tpls_dev, const int32_t *m, const int32_t *n,
                                                  const int64_t *strides, zts_mode mode, const zts_params *params,
                                                  void *stream, zts_result *out)
{
    if (!z || !tpls_dev || !m || !n || !strides || !out || count < 1)
        return ZTS_E_ARG;
    if (mode != ZTS_TE_FIXED && mode != ZTS_EGS && mode != ZTS_OPTA && mode != ZTS_OPTA_PAPER)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        for (int k = 0; k < count; k++) {
            check_template_args(im, tpls_dev[k], m[k], n[k], strides[k]);
            check_mode_shape(mode, m[k], n[k]);
        }
        const zts_params pr = params_or_default(params);
        std::vector<zts_result> res(count);
        run_pruned_batch(c, im, count, (const uint8_t *const *)tpls_dev, m, n, strides, true,
                         stream ? (hipStream_t)stream : c->stream, mode, pr, res.data());
        std::copy(res.begin(), res.end(), out);
    });
}

// ------------------------------------------------------------------ autotuner

// tune_cache lines: "<arch> <m> <n> <single_ms> <shared_ms>".
static void load_tune_cache(Ctx *c)
{
    if (c->tune_cache.empty())
        return;
    FILE *f = std::fopen(c->tune_cache.c_str(), "r");
    if (!f)
        return;
    char arch[128];
    int m, n;
    float s1, s16;
    while (std::fscanf(f, "%127s %d %d %f %f", arch, &m, &n, &s1, &s16) == 5)
        if (c->arch == arch && m > 0 && n > 0) {
            zts_tune_entry e;
            std::memset(&e, 0, sizeof e);
            e.m = m;
            e.n = n;
            e.single_ms = s1;
            e.shared_ms = s16;
            e.multi_min = multi_min_from(s1, s16);
            c->tuned[std::make_pair(m, n)] = e;
        }
    std::fclose(f);
}

// Rewrites the file: other architectures' lines are kept, this one's are the
// context's table.  Written to a temporary file and renamed.
static void save_tune_cache(Ctx *c)
{
    if (c->tune_cache.empty())
        return;
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(c->tune_cache.c_str(), "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, f)) {
            char arch[128];
            if (std::sscanf(line, "%127s", arch) == 1 && c->arch != arch)
                keep.push_back(line);
        }
        std::fclose(f);
    }
    std::string tmp = c->tune_cache + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f)
        return;
    for (auto &l : keep)
        std::fputs(l.c_str(), f);
    for (auto &kv : c->tuned)
        std::fprintf(f, "%s %d %d %.6g %.6g\n", c->arch.c_str(), kv.second.m, kv.second.n, kv.second.single_ms,
                     kv.second.shared_ms);
    bool ok = std::fclose(f) == 0;
    if (ok)
        std::rename(tmp.c_str(), c->tune_cache.c_str());
}

// Median device time of a batch plan's kernels over three launches after a
// warm-up (context lock held, main slot).
static float time_batch(Ctx *c, const std::vector<BatchItem> &items, int force)
{
    float ms[3];
    for (int rep = 0; rep < 4; rep++) {
        BatchPlan b = plan_batch(c, c->main, items, force);
        try {
            launch_batch_plan(b, c->main);
            hip_check(hipStreamSynchronize(c->main.stream));
        } catch (...) {
            unpin_batch(b);
            throw;
        }
        unpin_batch(b);
        float t = 0.0f;
        hip_check(hipEventElapsedTime(&t, c->main.ev0, c->main.ev1));
        if (rep > 0)
            ms[rep - 1] = t;
    }
    std::sort(ms, ms + 3);
    return ms[1];
}

ZTS_API zts_status zts_tune_batch(zts_ctx *z, int32_t image, int32_t count, const int32_t *m, const int32_t *n,
                                  zts_tune_entry *out)
{
    if (!z || !m || !n || count < 1)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        for (int k = 0; k < count; k++)
            if (m[k] < 1 || n[k] < 1 || m[k] > im->rows || n[k] > im->cols || n[k] > 128 ||
                (int64_t)m[k] * n[k] > 16384)
                throw ZtsError{ZTS_E_SIZE};
        for (int k = 0; k < count; k++) {
            // 16 templates cut from the image at spread offsets, read in place
            const int Ly = im->rows - m[k] + 1, Lx = im->cols - n[k] + 1;
            std::vector<BatchItem> items;
            for (int t = 0; t < 16; t++) {
                int64_t y = (int64_t)t * 7919 % Ly, x = (int64_t)t * 104729 % Lx;
                items.push_back(BatchItem{im, im->img.as<uint8_t>() + y * im->pitch + x, m[k], n[k], im->pitch, true});
            }
            zts_tune_entry e;
            std::memset(&e, 0, sizeof e);
            e.m = m[k];
            e.n = n[k];
            e.shared_ms = time_batch(c, items, BATCH_MULTI);
            if (batch_single_fits(m[k], n[k]))
                e.single_ms = time_batch(c, std::vector<BatchItem>{items[0]}, BATCH_SINGLE);
            e.multi_min = multi_min_from(e.single_ms, e.shared_ms);
            c->tuned[std::make_pair(m[k], n[k])] = e;
            if (out)
                out[k] = e;
        }
        save_tune_cache(c);
    });
}

ZTS_API zts_status zts_debug_full_map(zts_ctx *z, int32_t image, const uint8_t *tpl, int32_t m, int32_t n,
                                      int64_t stride, int64_t *num_out, int64_t *den_r_out, float *rho_out)
{
    if (!z)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl, m, n, stride);
        check_mode_shape(ZTS_FULL, m, n);
        size_t L = (size_t)(im->rows - m + 1) * (im->cols - n + 1);
        DBuf dn, dd, dr;
        if (num_out)
            dalloc(c, dn, L * 8);
        if (den_r_out)
            dalloc(c, dd, L * 8);
        if (rho_out)
            dalloc(c, dr, L * 4);
        zts_params pr;
        fill_default(&pr);
        zts_result res;
        run_query_main(c, im, tpl, m, n, stride, false, nullptr, ZTS_FULL, pr, &res, nullptr, dn.as<int64_t>(),
                       dd.as<int64_t>(), dr.as<float>());
        if (num_out)
            hip_check(hipMemcpy(num_out, dn.ptr, L * 8, hipMemcpyDeviceToHost));
        if (den_r_out)
            hip_check(hipMemcpy(den_r_out, dd.ptr, L * 8, hipMemcpyDeviceToHost));
        if (rho_out)
            hip_check(hipMemcpy(rho_out, dr.ptr, L * 4, hipMemcpyDeviceToHost));
    });
}

ZTS_API zts_status zts_debug_autocorr(zts_ctx *z, int32_t image, int32_t m, int32_t n, int32_t h, int32_t w,
                                      int64_t *num_out, int64_t *dc_out, int64_t *do_out)
{
    if (!z || !num_out || !dc_out || !do_out || h < 1 || w < 1)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        std::unique_lock<std::mutex> plk = take_prep_lock(c);  // it uses the preparation scratch
        Image *im = find_image(c, image);
        if (m < 1 || n < 1)
            throw ZtsError{ZTS_E_ARG};
        if (m > im->rows || n > im->cols || (int64_t)m * n > 16384)
            throw ZtsError{ZTS_E_SIZE};
        int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
        size_t L = (size_t)Ly * Lx;
        Stats *st = stats_entry(c, im, m, n, c->stream);
        PinGuard pin(st->pins);
        DBuf a1, a2, a3;
        dalloc(c, a1, L * 8);
        dalloc(c, a2, L * 8);
        dalloc(c, a3, L * 8);
        AcArgs a;
        std::memset(&a, 0, sizeof a);
        a.J = im->img.as<uint8_t>();
        a.pJ = im->pitch;
        a.statJ = st->stat.as<int2>();
        a.m = m;
        a.n = n;
        a.Ly = Ly;
        a.Lx = Lx;
        a.h = h;
        a.w = w;
        a.mode = AC_DEBUG;
        a.num_out = a1.as<int64_t>();
        a.dc_out = a2.as<int64_t>();
        a.do_out = a3.as<int64_t>();
        hip_check(launch_autocorr(a, psat_for(c, Ly, Lx, m, n), c->stream));
        hip_check(hipStreamSynchronize(c->stream));
        hip_check(hipMemcpy(num_out, a1.ptr, L * 8, hipMemcpyDeviceToHost));
        hip_check(hipMemcpy(dc_out, a2.ptr, L * 8, hipMemcpyDeviceToHost));
        hip_check(hipMemcpy(do_out, a3.ptr, L * 8, hipMemcpyDeviceToHost));
    });
}

ZTS_API zts_status zts_debug_blur(zts_ctx *z, const uint8_t *host_in, int32_t rows, int32_t cols,
                                  const int32_t *taps, int32_t d, uint8_t *host_out)
{
    if (!z || !host_in || !taps || !host_out || rows < 1 || cols < 1 || d < 0 || d > 32)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        int64_t pitch = pitch_for(cols);
        DBuf src, dst, tmp;
        alloc_image(c, src, rows, pitch);
        alloc_image(c, dst, rows, pitch);
        dalloc(c, tmp, sizeof(uint32_t) * (size_t)rows * cols);
        Taps tp;
        std::memset(&tp, 0, sizeof tp);
        for (int j = 0; j <= 2 * d; j++)
            tp.w[j] = taps[j];
        tp.d = d;
        hip_check(hipMemcpy2DAsync(src.ptr, pitch, host_in, cols, cols, rows, hipMemcpyHostToDevice, c->stream));
        hip_check(launch_blur(src.as<uint8_t>(), dst.as<uint8_t>(), pitch, rows, cols, tp, tmp.as<uint32_t>(),
                              c->stream));
        hip_check(hipMemcpy2DAsync(host_out, cols, dst.ptr, pitch, cols, rows, hipMemcpyDeviceToHost, c->stream));
        hip_check(hipStreamSynchronize(c->stream));
    });
}

}  // extern "C"
