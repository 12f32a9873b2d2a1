// Host side of libzts: context, resident images, preparation (group size by
// EGS, OptA conditioning) and query orchestration behind the C ABI of zts.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/zts.h"
#include "zts_kernels.h"

using namespace zts;

namespace {

// ------------------------------------------------------------------ errors

struct ZtsError {
    zts_status st;
};

inline void hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        if (std::getenv("ZTS_DEBUG"))
            std::fprintf(stderr, "zts: HIP error %d: %s\n", (int)e, hipGetErrorString(e));
        throw ZtsError{ZTS_E_DEVICE};
    }
}

// ------------------------------------------------------------------ device buffers

struct Ctx;

// A device allocation charged against the context's HBM budget.
struct DBuf {
    Ctx *ctx = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { reset(); }
    void reset();
    template <class T> T *as() const { return (T *)ptr; }
};

struct Stats {
    DBuf stat;  // int2 per location
};

struct Prepared {
    zts_mode mode;
    int m, n, h, w, Gy, Gx, radius;
    zts_params params;
    DBuf theta_b, x_b, gsum;       // member vs centre on the searched image
    DBuf J, Jsat, Jstat;           // OptA: conditioned image and its statistics
    DBuf theta_c, x_c;             // OptA: conditioned block vs original block (row-major)
    DBuf theta_cg, x_cg;           // the same in the group-major layout of (h, w)
    zts_prep_info info;
};

struct Image {
    int rows, cols;
    int64_t pitch;
    DBuf img, sat;
    std::map<std::pair<int, int>, std::unique_ptr<Stats>> stats;
    std::map<std::tuple<int, int, int>, std::unique_ptr<Prepared>> prep;
};

struct Ctx {
    std::mutex mu;
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evp[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int next_id = 1;
    std::map<int, std::unique_ptr<Image>> images;
    // per-query scratch, grown on demand
    DBuf qs, recs, gnum, gtheta, tpl, dec, counter, tmp32, viol, colmask;
    QState *h_qs = nullptr;
    uint8_t *h_tpl = nullptr;
    size_t h_tpl_bytes = 0;
    unsigned long long *h_cnt = nullptr;
};

void DBuf::reset()
{
    if (ptr) {
        (void)hipFree(ptr);
        if (ctx)
            ctx->used -= bytes;
    }
    ptr = nullptr;
    bytes = 0;
}

void dalloc(Ctx *c, DBuf &b, size_t bytes)
{
    if (b.ptr && b.bytes >= bytes)
        return;
    b.reset();
    if (bytes == 0)
        bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (c->budget && c->used + bytes > c->budget)
        throw ZtsError{ZTS_E_BUDGET};
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        throw ZtsError{ZTS_E_NOMEM};
    b.ctx = c;
    b.ptr = p;
    b.bytes = bytes;
    c->used += bytes;
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

// ------------------------------------------------------------------ helpers

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
    dalloc(c, sat, sizeof(uint2) * (size_t)(rows + 1) * (cols + 1));
    hip_check(launch_sat(img, pitch, rows, cols, sat.as<uint2>(), c->stream));
}

const int2 *stats_for(Ctx *c, Image *im, int m, int n)
{
    auto key = std::make_pair(m, n);
    auto it = im->stats.find(key);
    if (it != im->stats.end())
        return it->second->stat.as<int2>();
    auto st = std::make_unique<Stats>();
    int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
    dalloc(c, st->stat, sizeof(int2) * (size_t)Ly * Lx);
    hip_check(launch_stats(im->sat.as<uint2>(), im->cols, Ly, Lx, m, n, st->stat.as<int2>(), c->stream));
    const int2 *p = st->stat.as<int2>();
    im->stats[key] = std::move(st);
    return p;
}

unsigned long long read_counter(Ctx *c)
{
    hip_check(hipMemcpyAsync(c->h_cnt, c->counter.ptr, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    hip_check(hipStreamSynchronize(c->stream));
    return *c->h_cnt;
}

void zero_counter(Ctx *c)
{
    dalloc(c, c->counter, 64);
    hip_check(hipMemsetAsync(c->counter.ptr, 0, sizeof(unsigned long long), c->stream));
}

// The image a group tiling is built on, with its statistics.
struct Searched {
    const uint8_t *px;
    int64_t pitch;
    const int2 *stat;
};

// Retained-member count of Alg. 2 / Eq. 15 for group size (h, w) on image S.
// With blur data (theta_c, x_c, statI) every location counts with the angle
// to its original block added.
int64_t retained_count(Ctx *c, const Searched &S, int m, int n, int Ly, int Lx, int h, int w, double rho_th,
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
    a.thr = std::sqrt(1.0 - rho_th * rho_th);
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
    a.mode = theta_c ? AC_COUNT_BLUR : AC_COUNT;
    zero_counter(c);
    a.counter = c->counter.as<unsigned long long>();
    hip_check(launch_autocorr(a, c->stream));
    return (int64_t)read_counter(c);
}

// Alg. 2: greedy ascent over group sizes.  Fills trace/ntrace (up to 32).
void run_egs(Ctx *c, const Searched &S, int m, int n, int Ly, int Lx, const zts_params &pr, int h0, int w0,
             const float *theta_c, const int32_t *x_c, const int2 *statI, int &he, int &we, int64_t &cost,
             zts_egs_step *trace, int &ntrace)
{
    int64_t mn = (int64_t)m * n;
    int64_t prev = mn * (int64_t)Ly * Lx;
    int bh = 1, bw = 1, k = 0;
    if (pr.dh < 0 || pr.dw < 0 || (pr.dh == 0 && pr.dw == 0) || h0 < 1 || w0 < 1)
        throw ZtsError{ZTS_E_ARG};
    for (int h = h0, w = w0; h <= pr.h_max && w <= pr.h_max && h <= Ly && w <= Lx; h += pr.dh, w += pr.dw) {
        int64_t cc = (int64_t)((Ly + h - 1) / h) * ((Lx + w - 1) / w);
        int64_t cr = retained_count(c, S, m, n, Ly, Lx, h, w, pr.rho_th, theta_c, x_c, statI);
        int64_t ct = mn * (cc + cr);
        bool accept = (double)(prev - ct) > pr.xi * (double)prev;
        if (trace && k < 32) {
            zts_egs_step &s = trace[k];
            std::memset(&s, 0, sizeof s);
            s.h = h;
            s.w = w;
            s.cc = cc;
            s.cr = cr;
            s.ct = ct;
            s.accepted = accept;
        }
        k++;
        if (!accept)
            break;
        prev = ct;
        bh = h;
        bw = w;
    }
    ntrace = std::min(k, 32);
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
    hip_check(launch_autocorr(a, c->stream));
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
    hip_check(launch_blurcorr(a, c->stream));
}

// One OptA candidate image with its tables.
struct Cand {
    DBuf J, Jsat, Jstat, theta_c, x_c;
};

// Alg. 3.  The conditioned image ends in P.J (with its running sums and
// statistics), its blur angles in P.theta_c / P.x_c.
void run_opta(Ctx *c, Image *im, Prepared &P, const zts_params &pr, const int2 *statI)
{
    int p = im->rows, q = im->cols, m = P.m, n = P.n;
    int Ly = p - m + 1, Lx = q - n + 1;
    size_t L = (size_t)Ly * Lx;
    int64_t pitch = im->pitch;
    double lambda = lambda_of(pr.rho_th, pr.rho_max);
    Cand cur, nxt;
    auto setup = [&](Cand &k) {
        alloc_image(c, k.J, p, pitch);
        dalloc(c, k.Jstat, sizeof(int2) * L);
        dalloc(c, k.theta_c, sizeof(float) * L);
        dalloc(c, k.x_c, sizeof(int32_t) * L);
    };
    auto stats_of = [&](Cand &k) {
        build_sat(c, k.J.as<uint8_t>(), pitch, p, q, k.Jsat);
        hip_check(launch_stats(k.Jsat.as<uint2>(), q, Ly, Lx, m, n, k.Jstat.as<int2>(), c->stream));
    };
    auto build_c = [&](Cand &k) {
        blurcorr(c, k.J.as<uint8_t>(), k.Jstat.as<int2>(), im->img.as<uint8_t>(), statI, pitch, m, n, Ly, Lx,
                 BC_BUILD, lambda, nullptr, k.theta_c.as<float>(), k.x_c.as<int32_t>(), nullptr, nullptr, nullptr);
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
    zts_egs_step tr[32];
    Searched S{cur.J.as<uint8_t>(), pitch, cur.Jstat.as<int2>()};
    run_egs(c, S, m, n, Ly, Lx, pr, pr.h0, pr.w0, cur.theta_c.as<float>(), cur.x_c.as<int32_t>(), statI, h, w, cost,
            tr, nt);
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
        run_egs(c, S2, m, n, Ly, Lx, pr, h, w, nxt.theta_c.as<float>(), nxt.x_c.as<int32_t>(), statI, h2, w2, c2, tr,
                nt);
        bool accept = (double)(cost - c2) > pr.xi * (double)c2;
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
               a.dw == b.dw && a.h_max == b.h_max;
    if (mode == ZTS_EGS)
        return egs;
    return egs && a.rho_max == b.rho_max && a.blur_kind == b.blur_kind && a.sigma_step == b.sigma_step &&
           a.sigma_max == b.sigma_max && a.max_iters == b.max_iters;
}

Prepared *prepare(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr)
{
    auto key = std::make_tuple(m, n, (int)mode);
    auto it = im->prep.find(key);
    if (it != im->prep.end()) {
        if (same_prep_params(*it->second, mode, pr))
            return it->second.get();
        im->prep.erase(it);
    }
    auto t0 = std::chrono::steady_clock::now();
    int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
    const int2 *statI = stats_for(c, im, m, n);
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
    } else if (mode == ZTS_OPTA) {
        run_opta(c, im, *P, pr, statI);
        Searched SJ{P->J.as<uint8_t>(), im->pitch, P->Jstat.as<int2>()};
        build_tables(c, *P, SJ, Ly, Lx);
    } else {
        throw ZtsError{ZTS_E_ARG};
    }
    hip_check(hipStreamSynchronize(c->stream));
    auto t1 = std::chrono::steady_clock::now();
    P->info.mode = mode;
    P->info.m = m;
    P->info.n = n;
    P->info.group_h = P->h;
    P->info.group_w = P->w;
    P->info.radius = P->radius;
    P->info.prepare_ms = (float)std::chrono::duration<double, std::milli>(t1 - t0).count();
    Prepared *raw = P.get();
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

// Runs one query with the template already at c->tpl (m x n, pitch n).
void run_query(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr, zts_result *out, int8_t *dec,
               int64_t *num_map, int64_t *dr_map, float *rho_map)
{
    int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
    int64_t L = (int64_t)Ly * Lx;
    const int2 *statI = stats_for(c, im, m, n);
    Prepared *P = nullptr;
    if (mode != ZTS_FULL)
        P = prepare(c, im, m, n, mode, pr);
    dalloc(c, c->qs, sizeof(QState));
    hip_check(hipMemsetAsync(c->qs.ptr, 0, sizeof(QState), c->stream));
    int8_t *d_dec = nullptr;
    if (dec) {
        dalloc(c, c->dec, (size_t)L);
        hip_check(hipMemsetAsync(c->dec.ptr, 0x7f, (size_t)L, c->stream));
        d_dec = c->dec.as<int8_t>();
    }
    QState *qs = c->qs.as<QState>();
    const uint8_t *tpl = c->tpl.as<uint8_t>();
    hip_check(hipEventRecord(c->ev0, c->stream));
    int G = 0, radius = -1;
    if (mode == ZTS_FULL) {
        dalloc(c, c->recs, sizeof(RecPod) * (size_t)full_record_count(Ly, Lx));
        FullArgs a;
        std::memset(&a, 0, sizeof a);
        a.img = im->img.as<uint8_t>();
        a.pitch = im->pitch;
        a.p = im->rows;
        a.q = im->cols;
        a.stat = statI;
        a.tpl = tpl;
        a.ts = n;
        a.m = m;
        a.n = n;
        a.Ly = Ly;
        a.Lx = Lx;
        a.recs = c->recs.as<RecPod>();
        a.qs = qs;
        a.num_map = num_map;
        a.dr_map = dr_map;
        a.rho_map = rho_map;
        a.dec = d_dec;
        hip_check(launch_full(a, c->stream));
        hip_check(hipEventRecord(c->evp[0], c->stream));
        hip_check(launch_reduce(c->recs.as<RecPod>(), 0, full_record_count(Ly, Lx), qs, RD_FINAL, 0, pr.margin,
                                c->stream));
        hip_check(hipEventRecord(c->evp[1], c->stream));
    } else {
        bool opta = mode == ZTS_OPTA;
        G = P->Gy * P->Gx;
        int n1 = centres_record_count(P->Gy, P->Gx, m, n, P->h);
        if (opta)
            radius = std::max(P->radius, std::max(pr.refine_radius, 0));
        else
            radius = pr.refine_radius > 0 ? pr.refine_radius : -1;
        int n2 = radius >= 0 ? window_record_count(radius) : 0;
        int n3 = members_record_count(P->Gy, P->Gx);
        dalloc(c, c->recs, sizeof(RecPod) * (size_t)(n1 + n2 + n3));
        dalloc(c, c->gnum, sizeof(int64_t) * (size_t)G);
        dalloc(c, c->gtheta, sizeof(float) * (size_t)G);
        Searched S = opta ? Searched{P->J.as<uint8_t>(), im->pitch, P->Jstat.as<int2>()}
                          : Searched{im->img.as<uint8_t>(), im->pitch, statI};
        ScanArgs s;
        std::memset(&s, 0, sizeof s);
        s.img = S.px;
        s.pitch = S.pitch;
        s.stat = S.stat;
        s.tpl = tpl;
        s.ts = n;
        s.m = m;
        s.n = n;
        s.Ly = Ly;
        s.Lx = Lx;
        s.h = P->h;
        s.w = P->w;
        s.Gy = P->Gy;
        s.Gx = P->Gx;
        s.g_num = c->gnum.as<int64_t>();
        s.g_theta = c->gtheta.as<float>();
        s.recs = c->recs.as<RecPod>();
        s.qs = qs;
        s.dec = opta ? nullptr : d_dec;
        s.delta = pr.margin;
        s.set_thr = radius < 0;
        hip_check(launch_centres(s, c->stream));
        hip_check(hipEventRecord(c->evp[0], c->stream));
        hip_check(launch_reduce(c->recs.as<RecPod>(), 0, n1, qs, RD_BEST0, radius < 0, pr.margin, c->stream));
        hip_check(hipEventRecord(c->evp[1], c->stream));
        if (radius >= 0) {
            WinArgs wa;
            std::memset(&wa, 0, sizeof wa);
            wa.img = im->img.as<uint8_t>();
            wa.pitch = im->pitch;
            wa.stat = statI;
            wa.tpl = tpl;
            wa.ts = n;
            wa.m = m;
            wa.n = n;
            wa.Ly = Ly;
            wa.Lx = Lx;
            wa.h = P->h;
            wa.w = P->w;
            wa.radius = radius;
            wa.skip_centres = !opta;
            wa.include_best0 = !opta;
            wa.recs = c->recs.as<RecPod>();
            wa.rec_off = n1;
            wa.qs = qs;
            wa.dec = d_dec;
            wa.delta = pr.margin;
            hip_check(launch_window(wa, c->stream));
        }
        hip_check(hipEventRecord(c->evp[2], c->stream));
        if (radius >= 0)
            hip_check(launch_reduce(c->recs.as<RecPod>(), n1, n1 + n2, qs, RD_WINDOW, !opta, pr.margin, c->stream));
        hip_check(hipEventRecord(c->evp[3], c->stream));
        MemArgs ma;
        std::memset(&ma, 0, sizeof ma);
        ma.I = im->img.as<uint8_t>();
        ma.pI = im->pitch;
        ma.statI = statI;
        ma.statS = S.stat;
        ma.tpl = tpl;
        ma.ts = n;
        ma.m = m;
        ma.n = n;
        ma.Ly = Ly;
        ma.Lx = Lx;
        ma.h = P->h;
        ma.w = P->w;
        ma.Gy = P->Gy;
        ma.Gx = P->Gx;
        ma.g_num = c->gnum.as<int64_t>();
        ma.g_theta = c->gtheta.as<float>();
        ma.gsum = P->gsum.as<GroupSum>();
        ma.theta_b = P->theta_b.as<float>();
        ma.x_b = P->x_b.as<int32_t>();
        ma.theta_c = opta ? P->theta_cg.as<float>() : nullptr;
        ma.x_c = opta ? P->x_cg.as<int32_t>() : nullptr;
        ma.opta = opta;
        ma.radius = radius;
        ma.recs = c->recs.as<RecPod>();
        ma.rec_off = n1 + n2;
        ma.final_from = opta ? n1 : 0;
        ma.qs = qs;
        ma.dec = d_dec;
        hip_check(launch_members(ma, c->stream));
        hip_check(hipEventRecord(c->evp[4], c->stream));
        hip_check(launch_reduce(c->recs.as<RecPod>(), opta ? n1 : 0, n1 + n2 + n3, qs, RD_FINAL, 0, pr.margin,
                                c->stream));
        hip_check(hipEventRecord(c->evp[5], c->stream));
    }
    hip_check(hipEventRecord(c->ev1, c->stream));
    hip_check(hipMemcpyAsync(c->h_qs, c->qs.ptr, sizeof(QState), hipMemcpyDeviceToHost, c->stream));
    if (dec)
        hip_check(hipMemcpyAsync(dec, c->dec.ptr, (size_t)L, hipMemcpyDeviceToHost, c->stream));
    hip_check(hipStreamSynchronize(c->stream));
    const QState &h = *c->h_qs;
    if (h.degenerate)
        throw ZtsError{ZTS_E_DEGENERATE};
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
    if (mode == ZTS_FULL) {
        r.n_computed = L;
        r.group_h = r.group_w = 1;
        r.best0 = h.fin.rho;
        r.best0_y = r.y;
        r.best0_x = r.x;
    } else {
        r.n_centres = G;
        r.n_eliminated = (int64_t)h.n_elim;
        r.n_survivors = (int64_t)h.n_surv;
        r.n_computed = (int64_t)h.n_window + (int64_t)h.n_surv + (mode == ZTS_OPTA ? 0 : G);
        r.group_h = P->h;
        r.group_w = P->w;
        r.best0 = h.best;
        r.best0_y = (int32_t)(h.best0_l / Lx);
        r.best0_x = (int32_t)(h.best0_l % Lx);
        if (r.n_computed + r.n_eliminated != L)
            throw ZtsError{ZTS_E_DEVICE};
    }
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    r.device_ms = ms;
    if (mode == ZTS_FULL) {
        hip_check(hipEventElapsedTime(&r.phase_ms[0], c->ev0, c->evp[0]));
        hip_check(hipEventElapsedTime(&r.phase_ms[3], c->evp[0], c->evp[1]));
    } else {
        float r1, r2, r3;
        hip_check(hipEventElapsedTime(&r.phase_ms[0], c->ev0, c->evp[0]));
        hip_check(hipEventElapsedTime(&r1, c->evp[0], c->evp[1]));
        hip_check(hipEventElapsedTime(&r.phase_ms[1], c->evp[1], c->evp[2]));
        hip_check(hipEventElapsedTime(&r2, c->evp[2], c->evp[3]));
        hip_check(hipEventElapsedTime(&r.phase_ms[2], c->evp[3], c->evp[4]));
        hip_check(hipEventElapsedTime(&r3, c->evp[4], c->evp[5]));
        r.phase_ms[3] = r1 + r2 + r3;
    }
    r.status = ZTS_OK;
    *out = r;
}

void stage_template(Ctx *c, const uint8_t *tpl, int m, int n, int64_t stride, bool device, hipStream_t caller)
{
    size_t bytes = (size_t)m * n;
    dalloc(c, c->tpl, bytes);
    if (device) {
        hip_check(hipMemcpy2DAsync(c->tpl.ptr, n, tpl, stride, n, m, hipMemcpyDeviceToDevice,
                                   caller ? caller : c->stream));
        if (caller && caller != c->stream)
            hip_check(hipStreamSynchronize(caller));
        return;
    }
    if (c->h_tpl_bytes < bytes) {
        if (c->h_tpl)
            (void)hipHostFree(c->h_tpl);
        c->h_tpl = nullptr;
        hip_check(hipHostMalloc((void **)&c->h_tpl, bytes, hipHostMallocDefault));
        c->h_tpl_bytes = bytes;
    }
    for (int i = 0; i < m; i++)
        std::memcpy(c->h_tpl + (size_t)i * n, tpl + (size_t)i * stride, n);
    hip_check(hipMemcpyAsync(c->tpl.ptr, c->h_tpl, bytes, hipMemcpyHostToDevice, c->stream));
}

template <class F> zts_status guarded(Ctx *c, F &&f)
{
    if (!c)
        return ZTS_E_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
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

}  // namespace

// ====================================================================== C ABI

struct zts_ctx {
    Ctx c;
};

extern "C" {

void zts_params_default(zts_params *p)
{
    if (p)
        fill_default(p);
}

const char *zts_status_str(zts_status s)
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

zts_status zts_create(const zts_ctx_params *params, zts_ctx **out)
{
    if (!out)
        return ZTS_E_ARG;
    zts_ctx *z = new (std::nothrow) zts_ctx;
    if (!z)
        return ZTS_E_NOMEM;
    Ctx &c = z->c;
    c.device = params ? params->device : 0;
    c.budget = params ? params->hbm_budget_bytes : 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c.device < 0 || c.device >= ndev) {
        delete z;
        return ZTS_E_DEVICE;
    }
    if (hipSetDevice(c.device) != hipSuccess || hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&c.ev0) != hipSuccess || hipEventCreate(&c.ev1) != hipSuccess ||
        hipEventCreate(&c.evp[0]) != hipSuccess || hipEventCreate(&c.evp[1]) != hipSuccess ||
        hipEventCreate(&c.evp[2]) != hipSuccess || hipEventCreate(&c.evp[3]) != hipSuccess ||
        hipEventCreate(&c.evp[4]) != hipSuccess || hipEventCreate(&c.evp[5]) != hipSuccess ||
        hipEventCreate(&c.evp[6]) != hipSuccess || hipEventCreate(&c.evp[7]) != hipSuccess ||
        hipHostMalloc((void **)&c.h_qs, sizeof(QState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c.h_cnt, 64, hipHostMallocDefault) != hipSuccess) {
        delete z;
        return ZTS_E_DEVICE;
    }
    *out = z;
    return ZTS_OK;
}

void zts_destroy(zts_ctx *z)
{
    if (!z)
        return;
    Ctx &c = z->c;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        (void)hipSetDevice(c.device);
        if (c.stream)
            (void)hipStreamSynchronize(c.stream);
        c.images.clear();
        c.qs.reset(); c.recs.reset(); c.gnum.reset(); c.gtheta.reset(); c.tpl.reset(); c.dec.reset();
        c.counter.reset(); c.tmp32.reset(); c.viol.reset(); c.colmask.reset();
        if (c.h_qs) (void)hipHostFree(c.h_qs);
        if (c.h_tpl) (void)hipHostFree(c.h_tpl);
        if (c.h_cnt) (void)hipHostFree(c.h_cnt);
        if (c.ev0) (void)hipEventDestroy(c.ev0);
        if (c.ev1) (void)hipEventDestroy(c.ev1);
        for (int k = 0; k < 8; k++)
            if (c.evp[k]) (void)hipEventDestroy(c.evp[k]);
        if (c.stream) (void)hipStreamDestroy(c.stream);
    }
    delete z;
}

zts_status zts_image_load(zts_ctx *z, const uint8_t *host, int32_t rows, int32_t cols, int64_t stride, int32_t *id)
{
    if (!z)
        return ZTS_E_ARG;
    return load_common(&z->c, host, rows, cols, stride, false, nullptr, id);
}

zts_status zts_image_load_device(zts_ctx *z, const void *dev, int32_t rows, int32_t cols, int64_t stride,
                                 void *stream, int32_t *id)
{
    if (!z)
        return ZTS_E_ARG;
    return load_common(&z->c, dev, rows, cols, stride, true, (hipStream_t)stream, id);
}

zts_status zts_image_unload(zts_ctx *z, int32_t id)
{
    if (!z)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        find_image(c, id);
        hip_check(hipStreamSynchronize(c->stream));
        c->images.erase(id);
    });
}

zts_status zts_prepare(zts_ctx *z, int32_t image, int32_t m, int32_t n, zts_mode mode, const zts_params *params,
                       void *stream)
{
    if (!z)
        return ZTS_E_ARG;
    (void)stream;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        if (m < 1 || n < 1)
            throw ZtsError{ZTS_E_ARG};
        if (m > im->rows || n > im->cols || (int64_t)m * n > 16384)
            throw ZtsError{ZTS_E_SIZE};
        zts_params pr;
        if (params)
            pr = *params;
        else
            fill_default(&pr);
        if (mode == ZTS_FULL) {
            stats_for(c, im, m, n);
            hip_check(hipStreamSynchronize(c->stream));
            return;
        }
        prepare(c, im, m, n, mode, pr);
    });
}

zts_status zts_prep_query(zts_ctx *z, int32_t image, int32_t m, int32_t n, zts_mode mode, zts_prep_info *out)
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

zts_status zts_prep_image(zts_ctx *z, int32_t image, int32_t m, int32_t n, uint8_t *host_out)
{
    if (!z || !host_out)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        auto it = im->prep.find(std::make_tuple(m, n, (int)ZTS_OPTA));
        if (it == im->prep.end())
            throw ZtsError{ZTS_E_NOTPREPARED};
        hip_check(hipMemcpy2DAsync(host_out, im->cols, it->second->J.ptr, im->pitch, im->cols, im->rows,
                                   hipMemcpyDeviceToHost, c->stream));
        hip_check(hipStreamSynchronize(c->stream));
    });
}

zts_status zts_search(zts_ctx *z, int32_t image, const uint8_t *tpl, int32_t m, int32_t n, int64_t stride,
                      zts_mode mode, const zts_params *params, zts_result *out, int8_t *decision)
{
    if (!z || !out)
        return ZTS_E_ARG;
    if (mode != ZTS_FULL && mode != ZTS_TE_FIXED && mode != ZTS_EGS && mode != ZTS_OPTA)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl, m, n, stride);
        zts_params pr;
        if (params)
            pr = *params;
        else
            fill_default(&pr);
        stage_template(c, tpl, m, n, stride, false, nullptr);
        run_query(c, im, m, n, mode, pr, out, decision, nullptr, nullptr, nullptr);
    });
}

zts_status zts_search_device(zts_ctx *z, int32_t image, const void *tpl_dev, int32_t m, int32_t n, int64_t stride,
                             zts_mode mode, const zts_params *params, void *stream, zts_result *out)
{
    if (!z || !out)
        return ZTS_E_ARG;
    if (mode != ZTS_FULL && mode != ZTS_TE_FIXED && mode != ZTS_EGS && mode != ZTS_OPTA)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl_dev, m, n, stride);
        zts_params pr;
        if (params)
            pr = *params;
        else
            fill_default(&pr);
        stage_template(c, (const uint8_t *)tpl_dev, m, n, stride, true, (hipStream_t)stream);
        run_query(c, im, m, n, mode, pr, out, nullptr, nullptr, nullptr, nullptr);
    });
}

zts_status zts_search_batch(zts_ctx *z, int32_t image, int32_t count, const uint8_t *const *tpls, const int32_t *m,
                            const int32_t *n, const int64_t *strides, zts_result *out)
{
    if (!z || !tpls || !m || !n || !strides || !out || count < 1)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        std::map<std::pair<int, int>, std::vector<int>> buckets;
        for (int k = 0; k < count; k++) {
            check_template_args(im, tpls[k], m[k], n[k], strides[k]);
            buckets[std::make_pair(m[k], n[k])].push_back(k);
        }
        // stage every bucket's templates: [T][m][n16] with 0x80 past column n
        struct Job {
            int m, n, n16, T, Ly, Lx;
            size_t off, tst_off, res_off, rec_off;
            std::vector<int> idx;
        };
        std::vector<Job> jobs;
        size_t tbytes = 0, nres = 0, nrec = 0;
        for (auto &kv : buckets) {
            Job j;
            j.m = kv.first.first;
            j.n = kv.first.second;
            j.n16 = (j.n + 15) / 16 * 16;
            j.T = (int)kv.second.size();
            j.Ly = im->rows - j.m + 1;
            j.Lx = im->cols - j.n + 1;
            j.idx = kv.second;
            j.off = tbytes;
            tbytes += ((size_t)j.T * j.m * j.n16 + 255) / 256 * 256;
            j.res_off = nres;
            nres += j.T;
            j.rec_off = nrec;
            nrec += (size_t)((j.T + 15) / 16) * batch_blocks_per_tile(j.Ly, j.Lx) * 16;
            jobs.push_back(j);
        }
        if (c->h_tpl_bytes < tbytes) {
            if (c->h_tpl)
                (void)hipHostFree(c->h_tpl);
            c->h_tpl = nullptr;
            hip_check(hipHostMalloc((void **)&c->h_tpl, tbytes, hipHostMallocDefault));
            c->h_tpl_bytes = tbytes;
        }
        for (auto &j : jobs)
            for (int t = 0; t < j.T; t++) {
                int k = j.idx[t];
                uint8_t *dst = c->h_tpl + j.off + (size_t)t * j.m * j.n16;
                for (int r = 0; r < j.m; r++) {
                    std::memcpy(dst + (size_t)r * j.n16, tpls[k] + (size_t)r * strides[k], j.n);
                    std::memset(dst + (size_t)r * j.n16 + j.n, 0x80, j.n16 - j.n);
                }
            }
        DBuf dt, dtst, dres, drec;
        dalloc(c, dt, tbytes);
        dalloc(c, dtst, sizeof(int64_t) * 2 * nres);
        dalloc(c, dres, sizeof(RecPod) * nres);
        dalloc(c, drec, sizeof(RecPod) * nrec);
        hip_check(hipMemcpyAsync(dt.ptr, c->h_tpl, tbytes, hipMemcpyHostToDevice, c->stream));
        std::vector<const int2 *> stats;
        for (auto &j : jobs)
            stats.push_back(stats_for(c, im, j.m, j.n));
        hip_check(hipEventRecord(c->ev0, c->stream));
        for (size_t q = 0; q < jobs.size(); q++) {
            Job &j = jobs[q];
            BatchArgs a;
            std::memset(&a, 0, sizeof a);
            a.img = im->img.as<uint8_t>();
            a.pitch = im->pitch;
            a.p = im->rows;
            a.q = im->cols;
            a.stat = stats[q];
            a.tpl = dt.as<uint8_t>() + j.off;
            a.tst = dtst.as<int64_t>() + 2 * j.res_off;
            a.T = j.T;
            a.m = j.m;
            a.n = j.n;
            a.Ly = j.Ly;
            a.Lx = j.Lx;
            a.recs = drec.as<RecPod>() + j.rec_off;
            hip_check(launch_batch(a, dres.as<RecPod>() + j.res_off, c->stream));
        }
        hip_check(hipEventRecord(c->ev1, c->stream));
        std::vector<RecPod> res(nres);
        std::vector<int64_t> tst(2 * nres);
        hip_check(hipMemcpyAsync(res.data(), dres.ptr, sizeof(RecPod) * nres, hipMemcpyDeviceToHost, c->stream));
        hip_check(hipMemcpyAsync(tst.data(), dtst.ptr, sizeof(int64_t) * 2 * nres, hipMemcpyDeviceToHost, c->stream));
        hip_check(hipStreamSynchronize(c->stream));
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        for (auto &j : jobs)
            for (int t = 0; t < j.T; t++) {
                const RecPod &f = res[j.res_off + t];
                int64_t D_t = tst[2 * (j.res_off + t) + 1];
                zts_result r;
                std::memset(&r, 0, sizeof r);
                int64_t L = (int64_t)j.Ly * j.Lx;
                r.n_locations = L;
                r.device_ms = ms;
                r.phase_ms[0] = ms;
                if (D_t == 0) {
                    r.status = ZTS_E_DEGENERATE;
                } else {
                    r.y = (int32_t)(f.l / j.Lx);
                    r.x = (int32_t)(f.l % j.Lx);
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
                    r.status = ZTS_OK;
                }
                out[j.idx[t]] = r;
            }
    });
}

zts_status zts_debug_full_map(zts_ctx *z, int32_t image, const uint8_t *tpl, int32_t m, int32_t n, int64_t stride,
                              int64_t *num_out, int64_t *den_r_out, float *rho_out)
{
    if (!z)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        check_template_args(im, tpl, m, n, stride);
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
        stage_template(c, tpl, m, n, stride, false, nullptr);
        zts_result res;
        run_query(c, im, m, n, ZTS_FULL, pr, &res, nullptr, dn.as<int64_t>(), dd.as<int64_t>(), dr.as<float>());
        if (num_out)
            hip_check(hipMemcpy(num_out, dn.ptr, L * 8, hipMemcpyDeviceToHost));
        if (den_r_out)
            hip_check(hipMemcpy(den_r_out, dd.ptr, L * 8, hipMemcpyDeviceToHost));
        if (rho_out)
            hip_check(hipMemcpy(rho_out, dr.ptr, L * 4, hipMemcpyDeviceToHost));
    });
}

zts_status zts_debug_autocorr(zts_ctx *z, int32_t image, int32_t m, int32_t n, int32_t h, int32_t w,
                              int64_t *num_out, int64_t *dc_out, int64_t *do_out)
{
    if (!z || !num_out || !dc_out || !do_out || h < 1 || w < 1)
        return ZTS_E_ARG;
    return guarded(&z->c, [&] {
        Ctx *c = &z->c;
        Image *im = find_image(c, image);
        if (m < 1 || n < 1)
            throw ZtsError{ZTS_E_ARG};
        if (m > im->rows || n > im->cols || (int64_t)m * n > 16384)
            throw ZtsError{ZTS_E_SIZE};
        int Ly = im->rows - m + 1, Lx = im->cols - n + 1;
        size_t L = (size_t)Ly * Lx;
        const int2 *st = stats_for(c, im, m, n);
        DBuf a1, a2, a3;
        dalloc(c, a1, L * 8);
        dalloc(c, a2, L * 8);
        dalloc(c, a3, L * 8);
        AcArgs a;
        std::memset(&a, 0, sizeof a);
        a.J = im->img.as<uint8_t>();
        a.pJ = im->pitch;
        a.statJ = st;
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
        hip_check(launch_autocorr(a, c->stream));
        hip_check(hipStreamSynchronize(c->stream));
        hip_check(hipMemcpy(num_out, a1.ptr, L * 8, hipMemcpyDeviceToHost));
        hip_check(hipMemcpy(dc_out, a2.ptr, L * 8, hipMemcpyDeviceToHost));
        hip_check(hipMemcpy(do_out, a3.ptr, L * 8, hipMemcpyDeviceToHost));
    });
}

zts_status zts_debug_blur(zts_ctx *z, const uint8_t *host_in, int32_t rows, int32_t cols, const int32_t *taps,
                          int32_t d, uint8_t *host_out)
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
