// Serving loop of libzts: asynchronous requests (zts_submit / zts_poll /
// zts_wait) on a pool of worker slots, each with its own HIP stream.  Work
// that arrives while other work is on the device is admitted as soon as a
// slot is free and its memory fits; exhaustive int8-MFMA requests that are
// queued together run as one fused batched launch.
#include <algorithm>
#include <cstring>

#include "zts_runtime.h"

namespace zts {

namespace {

constexpr int kMaxBatchTemplates = 64;

using Clock = std::chrono::steady_clock;

float ms_between(Clock::time_point a, Clock::time_point b)
{
    return (float)std::chrono::duration<double, std::milli>(b - a).count();
}

// Records a request's result (context lock held).
void finish_request(Request *r, const zts_result &res)
{
    Clock::time_point now = Clock::now();
    r->res = res;
    r->res.latency_ms = ms_between(r->t_submit, now);
    r->res.queue_ms = ms_between(r->t_submit, r->state == RQ_RUNNING ? r->t_start : now);
    if (r->res.status == ZTS_OK)
        r->res.above_floor = r->res.rho >= r->pr.rho_floor;
    r->state = RQ_DONE;
    r->im->busy--;
}

// Takes the next unit of work from the queue: the oldest request, and when it
// is an exhaustive MFMA search, every other queued MFMA search (any image and
// size) up to kMaxBatchTemplates.
std::vector<Request *> take_work(Server &sv)
{
    std::vector<Request *> work;
    Request *r0 = sv.queue.front();
    sv.queue.pop_front();
    work.push_back(r0);
    if (r0->mode == ZTS_FULL_MFMA) {
        for (auto it = sv.queue.begin(); it != sv.queue.end() && (int)work.size() < kMaxBatchTemplates;) {
            if ((*it)->mode == ZTS_FULL_MFMA) {
                work.push_back(*it);
                it = sv.queue.erase(it);
            } else {
                ++it;
            }
        }
    }
    return work;
}

// Plans (lock held), runs on the slot's stream (lock released) and finishes
// one unit of work.  Throws ZtsError with the lock held again.
void execute(Ctx *c, Slot &S, std::unique_lock<std::mutex> &lk, const std::vector<Request *> &work,
             std::vector<zts_result> &res)
{
    Request *r0 = work[0];
    if (r0->mode == ZTS_FULL_MFMA) {
        std::vector<BatchItem> items;
        for (Request *r : work)
            items.push_back(BatchItem{r->im, r->tpl.data(), r->m, r->n, r->n});
        BatchPlan b = plan_batch(c, S, std::move(items));
        lk.unlock();
        try {
            launch_batch_plan(b, S);
            finish_batch(b, S, res.data());
        } catch (...) {
            lk.lock();
            unpin_batch(b);
            throw;
        }
        lk.lock();
        unpin_batch(b);
        return;
    }
    QueryPlan q = plan_query(c, S, r0->im, r0->m, r0->n, r0->mode, r0->pr, false);
    zts_status st;
    lk.unlock();
    try {
        stage_template(S, r0->tpl.data(), r0->m, r0->n, r0->n);
        launch_query(q, S, nullptr);
        st = finish_query(q, S, &res[0], c->wall_khz);
    } catch (...) {
        lk.lock();
        unpin_query(q);
        throw;
    }
    lk.lock();
    unpin_query(q);
    if (st != ZTS_OK)
        res[0] = error_result(st);
}

void worker_main(Ctx *c, Slot *S)
{
    (void)hipSetDevice(c->device);
    Server &sv = *c->srv;
    std::unique_lock<std::mutex> lk(c->mu);
    CtxLockScope scope(lk);
    for (;;) {
        sv.cv_work.wait(lk, [&] { return sv.stop || !sv.queue.empty(); });
        if (sv.stop)
            break;
        std::vector<Request *> work = take_work(sv);
        Clock::time_point now = Clock::now();
        for (Request *r : work) {
            r->state = RQ_RUNNING;
            r->t_start = now;
        }
        sv.running++;
        std::vector<zts_result> res(work.size());
        zts_status fail = ZTS_OK;
        try {
            execute(c, *S, lk, work, res);
        } catch (const ZtsError &e) {
            fail = e.st;
        } catch (const std::bad_alloc &) {
            fail = ZTS_E_NOMEM;
        }
        sv.running--;
        if (fail == ZTS_E_BUDGET && sv.running > 0 && !sv.stop) {
            // Device memory is held by running work: give this slot's scratch
            // back, return the requests to the front of the queue and wait
            // until some work completes (finishing workers then release theirs).
            for (auto it = work.rbegin(); it != work.rend(); ++it) {
                (*it)->state = RQ_QUEUED;
                sv.queue.push_front(*it);
            }
            S->release_scratch();
            sv.need_memory++;
            uint64_t seen = sv.completions;
            sv.cv_done.wait(lk, [&] { return sv.stop || sv.completions != seen; });
            sv.need_memory--;
            sv.cv_work.notify_one();
            continue;
        }
        for (size_t k = 0; k < work.size(); k++)
            finish_request(work[k], fail != ZTS_OK ? error_result(fail) : res[k]);
        if (sv.need_memory)
            S->release_scratch();
        sv.completions++;
        sv.cv_done.notify_all();
    }
}

void start_server(Ctx *c)
{
    if (c->srv)
        return;
    auto srv = std::make_unique<Server>();
    try {
        for (int k = 0; k < c->max_inflight; k++) {
            srv->slots.push_back(std::make_unique<Slot>());
            srv->slots.back()->init();
        }
    } catch (...) {
        for (auto &s : srv->slots)
            s->destroy();
        throw;
    }
    c->srv = std::move(srv);
    for (auto &s : c->srv->slots)
        c->srv->workers.emplace_back(worker_main, c, s.get());
}

// Validates and copies one template into a new request (lock held).
std::unique_ptr<Request> make_request(Ctx *c, int image, const uint8_t *tpl, int m, int n, int64_t stride,
                                      zts_mode mode, const zts_params *params)
{
    Image *im = find_image(c, image);
    check_template_args(im, tpl, m, n, stride);
    check_mode_shape(mode, m, n);
    auto r = std::make_unique<Request>();
    r->image = image;
    r->im = im;
    r->m = m;
    r->n = n;
    r->mode = mode;
    r->pr = params_or_default(params);
    r->tpl.resize((size_t)m * n);
    for (int i = 0; i < m; i++)
        std::memcpy(r->tpl.data() + (size_t)i * n, tpl + (size_t)i * stride, n);
    std::memset(&r->res, 0, sizeof r->res);
    return r;
}

bool serve_mode(zts_mode mode)
{
    return mode == ZTS_FULL || mode == ZTS_FULL_MFMA || mode == ZTS_TE_FIXED || mode == ZTS_EGS || mode == ZTS_OPTA ||
           mode == ZTS_OPTA_PAPER;
}

template <class F> zts_status locked(zts_ctx *z, F &&f)
{
    if (!z)
        return ZTS_E_ARG;
    Ctx *c = &z->c;
    std::unique_lock<std::mutex> lk(c->mu);
    try {
        return f(c, lk);
    } catch (const ZtsError &e) {
        return e.st;
    } catch (const std::bad_alloc &) {
        return ZTS_E_NOMEM;
    } catch (const std::system_error &) {
        return ZTS_E_NOMEM;
    }
}

// Hands a finished request's result to the caller and forgets the ticket.
zts_status collect(Server &sv, uint64_t ticket, zts_result *out)
{
    auto it = sv.reqs.find(ticket);
    zts_status st = it->second->res.status;
    *out = it->second->res;
    sv.reqs.erase(it);
    return st;
}

}  // namespace

void server_shutdown(Ctx *c)
{
    std::unique_lock<std::mutex> lk(c->mu);
    if (!c->srv)
        return;
    Server &sv = *c->srv;
    sv.stop = true;
    for (Request *r : sv.queue)
        finish_request(r, error_result(ZTS_E_CANCELLED));
    sv.queue.clear();
    sv.cv_work.notify_all();
    sv.cv_done.notify_all();
    lk.unlock();
    for (auto &t : sv.workers)
        t.join();
    lk.lock();
    // requests a worker returned to the queue after the cancellation above
    for (Request *r : sv.queue)
        finish_request(r, error_result(ZTS_E_CANCELLED));
    sv.queue.clear();
    (void)hipSetDevice(c->device);
    for (auto &s : sv.slots)
        s->destroy();
    c->srv.reset();
}

}  // namespace zts

using namespace zts;

extern "C" {

ZTS_API zts_status zts_submit(zts_ctx *z, int32_t image, const uint8_t *tpl, int32_t m, int32_t n, int64_t stride,
                              zts_mode mode, const zts_params *params, uint64_t *ticket)
{
    if (!ticket || !serve_mode(mode))
        return ZTS_E_ARG;
    return locked(z, [&](Ctx *c, std::unique_lock<std::mutex> &) {
        hip_check(hipSetDevice(c->device));
        start_server(c);
        Server &sv = *c->srv;
        if ((int)sv.queue.size() >= c->max_queued)
            return ZTS_E_AGAIN;
        auto r = make_request(c, image, tpl, m, n, stride, mode, params);
        r->ticket = sv.next_ticket++;
        r->t_submit = std::chrono::steady_clock::now();
        r->im->busy++;
        *ticket = r->ticket;
        sv.queue.push_back(r.get());
        sv.reqs[r->ticket] = std::move(r);
        sv.cv_work.notify_one();
        return ZTS_OK;
    });
}

ZTS_API zts_status zts_submit_batch(zts_ctx *z, int32_t image, int32_t count, const uint8_t *const *tpls,
                                    const int32_t *m, const int32_t *n, const int64_t *strides, zts_mode mode,
                                    const zts_params *params, uint64_t *first_ticket)
{
    if (!tpls || !m || !n || !strides || !first_ticket || count < 1 || !serve_mode(mode))
        return ZTS_E_ARG;
    return locked(z, [&](Ctx *c, std::unique_lock<std::mutex> &) {
        hip_check(hipSetDevice(c->device));
        start_server(c);
        Server &sv = *c->srv;
        if ((int64_t)sv.queue.size() + count > c->max_queued)
            return ZTS_E_AGAIN;
        std::vector<std::unique_ptr<Request>> rs;
        for (int k = 0; k < count; k++)
            rs.push_back(make_request(c, image, tpls[k], m[k], n[k], strides[k], mode, params));
        auto now = std::chrono::steady_clock::now();
        *first_ticket = sv.next_ticket;
        for (auto &r : rs) {
            r->ticket = sv.next_ticket++;
            r->t_submit = now;
            r->im->busy++;
            sv.queue.push_back(r.get());
            sv.reqs[r->ticket] = std::move(r);
        }
        sv.cv_work.notify_all();
        return ZTS_OK;
    });
}

ZTS_API zts_status zts_poll(zts_ctx *z, uint64_t ticket, zts_result *out)
{
    if (!out)
        return ZTS_E_ARG;
    return locked(z, [&](Ctx *c, std::unique_lock<std::mutex> &) {
        if (!c->srv)
            return ZTS_E_ARG;
        auto it = c->srv->reqs.find(ticket);
        if (it == c->srv->reqs.end())
            return ZTS_E_ARG;
        if (it->second->state != RQ_DONE)
            return ZTS_E_AGAIN;
        return collect(*c->srv, ticket, out);
    });
}

ZTS_API zts_status zts_wait(zts_ctx *z, uint64_t ticket, int64_t timeout_ns, zts_result *out)
{
    if (!out)
        return ZTS_E_ARG;
    return locked(z, [&](Ctx *c, std::unique_lock<std::mutex> &lk) {
        if (!c->srv)
            return ZTS_E_ARG;
        Server &sv = *c->srv;
        auto ready = [&] {
            auto it = sv.reqs.find(ticket);
            return it == sv.reqs.end() || it->second->state == RQ_DONE;
        };
        if (timeout_ns < 0) {
            sv.cv_done.wait(lk, ready);
        } else if (!sv.cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
            return ZTS_E_TIMEOUT;
        }
        if (sv.reqs.find(ticket) == sv.reqs.end())
            return ZTS_E_ARG;
        return collect(sv, ticket, out);
    });
}

ZTS_API zts_status zts_cancel(zts_ctx *z, uint64_t ticket)
{
    return locked(z, [&](Ctx *c, std::unique_lock<std::mutex> &) {
        if (!c->srv)
            return ZTS_E_ARG;
        Server &sv = *c->srv;
        auto it = sv.reqs.find(ticket);
        if (it == sv.reqs.end())
            return ZTS_E_ARG;
        Request *r = it->second.get();
        if (r->state != RQ_QUEUED)
            return ZTS_E_BUSY;
        sv.queue.erase(std::find(sv.queue.begin(), sv.queue.end(), r));
        finish_request(r, error_result(ZTS_E_CANCELLED));
        sv.cv_done.notify_all();
        return ZTS_OK;
    });
}

ZTS_API zts_status zts_pending(zts_ctx *z, int32_t *queued, int32_t *running)
{
    if (!queued || !running)
        return ZTS_E_ARG;
    return locked(z, [&](Ctx *c, std::unique_lock<std::mutex> &) {
        *queued = c->srv ? (int32_t)c->srv->queue.size() : 0;
        *running = c->srv ? (int32_t)c->srv->running : 0;
        return ZTS_OK;
    });
}

}  // extern "C"
