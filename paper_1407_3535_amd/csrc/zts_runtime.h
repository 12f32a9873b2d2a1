// Host runtime shared by the library's translation units (not part of the C
// ABI): errors, budgeted device buffers, execution slots, resident images with
// their cached per-size tables, and the request queue of the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/zts.h"
#include "zts_kernels.h"

namespace zts {

struct ZtsError {
    zts_status st;
};

void hip_check_at(hipError_t e, const char *file, int line);
// Throws ZTS_E_DEVICE on a HIP error (printed with its call site when the
// environment sets ZTS_DEBUG).
#define hip_check(e) ::zts::hip_check_at((e), __FILE__, __LINE__)

struct Ctx;

// A device allocation charged against the context's HBM budget.  Allocation,
// release and the budget counter are guarded by the context mutex.
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

// Grows b to at least `bytes`: a cached free block of at most twice the size
// if there is one, else a new allocation.  Over the budget it evicts cached
// tables that no running work holds (least recently used first), then frees
// cached blocks; ZTS_E_BUDGET if that is not enough.
void dalloc(Ctx *c, DBuf &b, size_t bytes);
void release_free_blocks(Ctx *c);

// Pinned host staging that grows on demand.
struct HostBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { reset(); }
    void reset();
    void grow(size_t n, unsigned flags = hipHostMallocDefault);
    template <class T> T *as() const { return (T *)ptr; }
};

// Everything one in-flight search needs of its own: a stream (default
// priority, non-blocking), its timing events, device scratch grown on demand
// and pinned host staging.  The synchronous entry points use the context's
// main slot; every serving worker owns one.
// A captured query launch sequence (see launch_query).
struct SlotGraph {
    std::string key;
    hipGraphExec_t exec = nullptr;
    uint64_t stamp = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_in = nullptr;  // orders the slot's stream after a caller's stream
    hipEvent_t evp[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    DBuf qs, recs, gnum, gtheta, tpl, dec;       // one query
    DBuf tcnt, tbin;                             // one query's survivor tiles: counts and bins
    DBuf bdata, bres, brec;                      // one batched launch
    HostBuf h_qs, h_stage, h_out;
    bool use_graphs = true;
    bool timed = false;             // the last query recorded its per-kernel events
    unsigned long long qseq = 0;    // queries launched on this slot's state (published sequence)
    std::vector<SlotGraph> graphs;  // keyed by the launch arguments
    uint64_t graph_clock = 0;
    void init();      // throws ZTS_E_DEVICE
    void destroy();   // waits for the stream first
    void release_scratch();
    void drop_graphs();
};

struct Stats {
    DBuf stat;                    // int2 per location: (sum x', sum x'^2)
    hipEvent_t ready = nullptr;   // recorded after the kernel that builds it
    int pins = 0;
    uint64_t last_use = 0;
    ~Stats();
};

struct Prepared {
    zts_mode mode;
    int m, n, h, w, Gy, Gx, radius;
    zts_params params;
    DBuf theta_b, x_b, gsum;       // member vs centre on the searched image
    DBuf cstat;                    // statistics of each group centre's block on the searched image
    DBuf J, Jsat, Jstat;           // OptA (both forms): conditioned image and its statistics
    DBuf theta_c, x_c;             // ZTS_OPTA: conditioned block vs original block (row-major)
    DBuf theta_cg, x_cg;           // the same in the group-major layout of (h, w)
    zts_prep_info info;
    int pins = 0;
    uint64_t last_use = 0;
};

struct Image {
    int rows, cols;
    int64_t pitch;
    DBuf img, sat;
    int busy = 0;  // submitted requests not yet finished
    std::map<std::pair<int, int>, std::unique_ptr<Stats>> stats;
    std::map<std::tuple<int, int, int>, std::unique_ptr<Prepared>> prep;
};

// ------------------------------------------------------------------ serving

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Request {
    uint64_t ticket;
    int image;
    Image *im;
    std::vector<uint8_t> tpl;  // m x n, pitch n
    int m, n;
    zts_mode mode;
    zts_params pr;
    int state = RQ_QUEUED;
    zts_result res;
    std::chrono::steady_clock::time_point t_submit, t_start;
};

struct Server {
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<std::thread> workers;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::condition_variable cv_work, cv_done;
    uint64_t next_ticket = 1;
    uint64_t completions = 0;  // units of work finished
    int running = 0;           // workers executing a unit of work
    int need_memory = 0;       // workers waiting for device memory
    bool stop = false;
};

// ------------------------------------------------------------------ context

struct Ctx {
    std::mutex mu;
    // Serialises preparations (they share the preparation scratch below and
    // the main stream).  Taken without mu held (order: prep_mu, then mu); a
    // preparation releases mu while it waits for the device, so requests whose
    // tables are ready keep being planned and launched meanwhile.
    std::mutex prep_mu;
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;            // live buffers and cached free blocks
    // Released device blocks kept for reuse (size -> pointer): hipFree waits
    // for the whole device, so blocks are recycled instead and only freed when
    // the budget needs the room.
    std::multimap<size_t, void *> free_blocks;
    uint64_t clock = 0;           // LRU stamps
    Slot main;
    hipStream_t stream = nullptr; // main.stream: loads, preparation, synchronous searches
    DBuf counter, tmp32, viol, colmask, psat;  // preparation scratch
    HostBuf h_cnt;
    HostBuf h_qs_noalloc;         // host mirror of zts_search_device_noalloc's query state
    HostBuf h_batch_qs;           // host mirrors of zts_search_batch_pruned's query states
    int next_id = 1;
    std::map<int, std::unique_ptr<Image>> images;
    int max_inflight = 4;
    int max_queued = 4096;
    std::unique_ptr<Server> srv;
    // batch routes measured by zts_tune_batch, by (m, n); the device's
    // architecture name keys the tune_cache file
    std::map<std::pair<int, int>, zts_tune_entry> tuned;
    std::string tune_cache, arch;
    double wall_khz = 100000.0;   // device realtime clock (hipDeviceAttributeWallClockRate)
    // Streams beside the main one (default priority, non-blocking) for the
    // batched pruned search, whose templates' kernel chains are independent:
    // spread over them, one chain's tail overlaps the next chain's start.
    // Created on first use; events order them against the main stream.
    static constexpr int kAuxStreams = 8;
    hipStream_t aux[kAuxStreams] = {};
    hipEvent_t aux_ev[kAuxStreams + 1] = {};
};

// The context lock held by the calling thread (a synchronous entry point's or
// a serving worker's), so that preparation can release it while it waits for
// the device.  Every path that may prepare sets it (CtxLockScope).
extern thread_local std::unique_lock<std::mutex> *t_ctx_lock;
struct CtxLockScope {
    std::unique_lock<std::mutex> *prev;
    explicit CtxLockScope(std::unique_lock<std::mutex> &lk) : prev(t_ctx_lock) { t_ctx_lock = &lk; }
    ~CtxLockScope() { t_ctx_lock = prev; }
};

Image *find_image(Ctx *c, int id);
void fill_default(zts_params *p);
// ZTS_OK when every parameter is in range (the checks listed at zts_params_check).
zts_status params_status(const zts_params &p);
// *params (or the defaults when NULL), checked; throws ZTS_E_ARG when out of range.
zts_params params_or_default(const zts_params *params);
void check_template_args(Image *im, const void *tpl, int m, int n, int64_t stride);
// ZTS_E_SIZE when a mode's kernels cannot stage an m x n template in the LDS
// of one workgroup (ZTS_FULL: k_full's rows; ZTS_FULL_MFMA: n <= 128; the
// eliminating modes: scan 1 and scan 2).  Needs the context's device current.
void check_mode_shape(zts_mode mode, int m, int n);

// Per-(m, n) statistics of an image, built on `s` if missing (stream `s` is
// then ordered after the build; other streams wait on st->ready).
Stats *stats_entry(Ctx *c, Image *im, int m, int n, hipStream_t s);
Prepared *prepare(Ctx *c, Image *im, int m, int n, zts_mode mode, const zts_params &pr);

// One query, split so that only planning and finishing hold the context lock.
struct QueryPlan {
    Image *im = nullptr;
    Stats *st = nullptr;
    Prepared *P = nullptr;
    int m = 0, n = 0, Ly = 0, Lx = 0;
    zts_mode mode = ZTS_FULL;
    zts_params pr;
    bool want_dec = false;
    const uint8_t *tpl = nullptr;   // template read in place (device memory), else the slot's copy
    int64_t ts = 0;                 // its row stride
    int64_t *num_map = nullptr, *dr_map = nullptr;
    float *rho_map = nullptr;
};
QueryPlan plan_query(Ctx *c, Slot &S, Image *im, int m, int n, zts_mode mode, const zts_params &pr, bool want_dec);
// Copies a host template into the slot's device buffer (pitch n) through its
// pinned staging, on the slot's stream.
void stage_template(Slot &S, const uint8_t *tpl, int m, int n, int64_t stride);
void launch_query(const QueryPlan &q, Slot &S, int8_t *dec_host);
// Waits for the query (its state published to the slot's host mirror) and
// assembles the result; wall_khz: the device clock rate for device_ms.
zts_status finish_query(const QueryPlan &q, Slot &S, zts_result *out, double wall_khz);
void unpin_query(QueryPlan &q);

// Many templates, possibly of several sizes and images, in one fused launch
// of the batched MFMA kernels.
struct BatchItem {
    Image *im;
    const uint8_t *tpl;  // host memory, or device memory when `device`
    int m, n;
    int64_t stride;
    bool device = false;
};
struct BatchPlan {
    std::vector<BatchItem> items;
    std::vector<BatchJob> jobs;
    std::vector<std::vector<int>> members;  // item indices of each job, in template order
    std::vector<Stats *> stats;
    size_t table_bytes = 0, tpl_bytes = 0, nrec = 0;
    int ntpl = 0;
};
// force: -1 routes every size group by the tuned measurements (or the
// built-in estimate); BATCH_MULTI or BATCH_SINGLE puts every group on that
// kernel (the autotuner's timing runs).
BatchPlan plan_batch(Ctx *c, Slot &S, std::vector<BatchItem> items, int force = -1);
void launch_batch_plan(BatchPlan &b, Slot &S);
void finish_batch(const BatchPlan &b, Slot &S, zts_result *out);  // out[k] for items[k]
void unpin_batch(BatchPlan &b);

zts_result error_result(zts_status st);

// Stops the serving workers: queued requests end as ZTS_E_CANCELLED, running
// ones finish.  Called by zts_destroy before anything is freed.
void server_shutdown(Ctx *c);

}  // namespace zts

struct zts_ctx {
    zts::Ctx c;
};
