/*
 * zts.h - exhaustive zero-mean NCC template search on one MI355X (gfx950).
 *
 * The library finds, for a uint8 template t (m x n) and a resident uint8
 * search image I (p x q), the location maximising the correlation coefficient
 * rho(t, r) of Eq. 1 over all (p-m+1)(q-n+1) valid blocks r, and reports how
 * many locations were computed and how many were skipped.  Methods follow
 * Mahmood, Mian, Owens, "Optimizing Auto-correlation for Fast Target Search in
 * Large Search Space" (arXiv 1407.3535):
 *   - transitive elimination of group members (section II, Eq. 2 and Eq. 5)
 *     with the two-scan early threshold (section VI);
 *   - Efficient Group Size (section III-D, Alg. 2, Eq. 15-17);
 *   - OptA conditioning by controlled non-uniform blur (sections IV-V,
 *     Alg. 3, Prop. 4.3, Eq. 28).
 * Every mode returns the answer of an exhaustive search: the same location,
 * the same exact integers and the same binary64 rho.
 *
 * Pure C.  No C++ types, exceptions or globals cross this interface.
 *
 * Conventions (all entry points):
 *   - Pixels are row-major uint8; `stride` is the row pitch in bytes (>= cols).
 *   - Coordinates are 0-based (row y, column x) of the top-left corner of a
 *     block.  The linear location index is y*(q-n+1) + x.
 *   - Host pointers are read (or written) before the call returns; the caller
 *     keeps ownership.  Device pointers are borrowed for the duration of the
 *     call only.  The library owns every device buffer it allocates and frees
 *     them in zts_destroy / zts_image_unload.
 *   - NULL or out-of-range arguments return ZTS_E_ARG; a template with zero
 *     variance returns ZTS_E_DEGENERATE.  ZTS_E_SIZE: an image with more than
 *     32767 rows or columns; a template with m > rows, n > cols or m*n > 16384;
 *     or a template shape the chosen mode's kernels cannot stage in the
 *     160 KB of LDS of one workgroup, refused before anything is launched:
 *     ZTS_FULL stages (31 + m) * (256 + w) + (m + 14) * w bytes with
 *     w = 16*ceil(n/16) (so m <= 537 for n <= 16, m <= 481 for n <= 32, and
 *     n <= 2048 or so: 512x32 and 1x16384 are refused); ZTS_FULL_MFMA needs
 *     n <= 128; the eliminating modes stage m * w bytes plus about 17 KB,
 *     which refuses only single-column templates taller than 9198 rows.
 *     Every shape up to 128x128 is accepted by every mode.
 *     Nothing is written to outputs on error.
 *   - A `void* stream` is a hipStream_t (NULL = the context's own stream).
 *   - Every entry point is thread safe.  Synchronous calls on one context are
 *     serialised; submitted requests run concurrently on the context's worker
 *     slots (see "serving" below).
 */
#ifndef ZTS_H
#define ZTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define ZTS_API __attribute__((visibility("default")))
#else
#define ZTS_API
#endif

typedef struct zts_ctx zts_ctx;

typedef enum {
    ZTS_OK = 0,
    ZTS_E_ARG = -1,
    ZTS_E_SIZE = -2,
    ZTS_E_DEGENERATE = -3,
    ZTS_E_NOIMAGE = -4,
    ZTS_E_BUDGET = -5,
    ZTS_E_AGAIN = -6,
    ZTS_E_BUSY = -7,
    ZTS_E_TIMEOUT = -8,
    ZTS_E_CANCELLED = -9,
    ZTS_E_DEVICE = -10,
    ZTS_E_NOMEM = -11,
    ZTS_E_NOTPREPARED = -12
} zts_status;

/* Search modes.
 *   ZTS_FULL      every location computed (Eq. 1 everywhere); the plain
 *                 baseline (one template per launch, v_dot4 on the VALU).
 *   ZTS_FULL_MFMA every location computed, as an implicit GEMM on int8 MFMA
 *                 (v_mfma_i32_16x16x64_i8, int32 accumulation); templates
 *                 submitted together share launches.  n <= 128.
 *   ZTS_TE_FIXED  transitive elimination with a caller-given group size
 *                 (section II; the earlier algorithm's user parameter).
 *   ZTS_EGS       transitive elimination with the group size chosen by
 *                 Alg. 2 on the image.
 *   ZTS_OPTA      Alg. 3 conditions a blurred copy of the image; the search
 *                 scans the blurred group centres, refines on the original
 *                 image around the best one (section IV-C) and bounds every
 *                 original location through the triangle inequality on
 *                 angles (Eq. 2 with Prop. 4.3's blur correlation added), so
 *                 the result is still exact.
 *   ZTS_OPTA_PAPER the paper's own OptA (sections IV-C, V, VI): the image is
 *                 conditioned by Alg. 3 as printed (each EGS run sees only
 *                 the blurred image and its own auto-correlation, Prop. 3.2);
 *                 transitive elimination on the conditioned image finds its
 *                 best location, then the template is matched on the
 *                 original image within the cumulative blur radius (capped
 *                 at 8, or refine_radius when larger) of it.  Not exact: the
 *                 answer is the window's best.  n_centres, n_eliminated and
 *                 n_survivors are those of the search on the conditioned
 *                 image; n_computed adds the window's matches. */
typedef enum { ZTS_FULL = 0, ZTS_FULL_MFMA = 1, ZTS_TE_FIXED = 2, ZTS_EGS = 3, ZTS_OPTA = 4,
               ZTS_OPTA_PAPER = 5 } zts_mode;

typedef struct {
    int32_t device;            /* HIP device ordinal */
    uint64_t hbm_budget_bytes; /* cap on the library's device allocations, 0 = none */
    int32_t max_inflight;      /* serving: worker slots, i.e. launches on the device at once (one
                                  stream each), 0 = 4, at most 64 */
    int32_t max_queued;        /* serving: submitted requests not yet started beyond which
                                  zts_submit returns ZTS_E_AGAIN, 0 = 4096 */
    const char *tune_cache;    /* file of measured batch routes (zts_tune_batch) for this GPU
                                  model: read at creation, rewritten after each tuning; NULL =
                                  none.  The string is copied. */
} zts_ctx_params;

/* Method parameters; zts_params_default fills the paper's values. */
typedef struct {
    double rho_th;          /* initial threshold used by the estimates, 0.80 (section VII) */
    double rho_max;         /* assumed peak for Prop. 4.3, 0.95 (section VII) */
    double margin;          /* strict elimination margin delta, 1e-9 */
    double xi;              /* relative cost decrement to continue, 0.005 (section III-D) */
    int32_t group_h, group_w;               /* ZTS_TE_FIXED group size, 5x5 (section VII) */
    int32_t h0, w0, dh, dw, h_max;          /* EGS start, step and cap: 3, 3, 2, 2, 33 */
    int32_t blur_kind;      /* 0: the paper's W = {1,4,10,4,1}/20 each iteration;
                               1: Gaussian with total sigma = sigma_step * k at iteration k */
    double sigma_step;      /* 0.5 */
    double sigma_max;       /* 3.0 */
    int32_t max_iters;      /* OptA iteration cap, 6 */
    int32_t refine_radius;  /* >0: also match every location within this Chebyshev
                               distance of the best centre before scan 2 (raises the
                               threshold; exactness unaffected).  0: section VI as printed.
                               In ZTS_OPTA the window radius is max(this, cumulative blur
                               radius, capped at 8). */
    int32_t timing;         /* 1: run the query's kernels one by one with an event after
                               each, filling zts_result.phase_ms.  0 (default): a launch
                               sequence met before on the same slot replays a captured
                               HIP graph and phase_ms stays 0. */
    int32_t egs_estimate;   /* retained-location estimate of Alg. 2:
                               0 (default): Prop. 3.2 / Eq. 15, a member is retained when its
                               auto-correlation is below sqrt(1 - rho_th^2);
                               1: Prop. 3.1 / Eq. 7 with both roots of Eq. 8 at an assumed
                               template-to-centre correlation rho_tc: retained unless the
                               bound of Eq. 2 through the centre is at most rho_th */
    double rho_tc;          /* the assumed rho_tc of egs_estimate 1, in (-1, 1), default 0 */
    int32_t egs_shape;      /* group-size ascent of Alg. 2: 0 (default) square steps
                               (h + dh, w + dw) as printed; 1: from the last accepted size the
                               cheapest of (h + dh, w), (h, w + dw), (h + dh, w + dw) */
    int32_t pad0;
    double accept_xi;       /* Alg. 3's acceptance margin: a blurred iterate is kept when the
                               estimated cost fell by more than accept_xi times its new cost
                               (0.005, section V); in (-1, 1): a negative value keeps iterates
                               whose cost rose by less than that fraction */
    double rho_floor;       /* detection floor of the result (section VII's threshold):
                               zts_result.above_floor reports rho >= rho_floor.  Default -2
                               (off). */
    int32_t floor_prune;    /* 1: the floor also prunes: scan 2 eliminates against
                               max(best0, rho_floor).  The answer stays exact whenever the
                               true maximum reaches the floor; otherwise above_floor = 0 and
                               the answer is the best location matched (at least as good as
                               the best group centre and survivor; no exactness claim).
                               0 (default): the floor only labels the result. */
    int32_t pad1;
    int32_t tile_dense_min; /* scan 2 bins its survivors by tile of 32 x 256 locations; four
                               stacked tiles holding at least 4x this many survivors together,
                               or one of them at least this many, are matched whole on int8
                               MFMA (every location; n <= 128), the others survivor by survivor.
                               0 (default): the library's value (128); -1: never whole; at
                               most 8192.  Counts and answers do not depend on it. */
    int32_t pad2;
} zts_params;

/* Result of one search.  Valid only when status == ZTS_OK. */
typedef struct {
    int32_t y, x;            /* best location (ties: smallest linear index) */
    double rho;              /* canonical binary64 rho at (y, x) */
    float rho32;             /* binary32 rho from the same exact integers */
    int32_t pad0;
    int64_t num, den_t, den_r; /* exact N = mn*sum(t r) - sum(t) sum(r), D_t, D_r at (y, x) */
    int64_t n_locations;     /* (p-m+1)(q-n+1) */
    int64_t n_centres;       /* group centres matched in scan 1 */
    int64_t n_eliminated;    /* locations skipped by the bound */
    int64_t n_survivors;     /* members that failed the elimination test and were matched */
    int64_t n_computed;      /* locations of I whose rho was computed */
    int32_t group_h, group_w;
    double best0;            /* threshold used by scan 2 (an attained rho) */
    int32_t best0_y, best0_x;/* best group centre of scan 1 */
    float device_ms;         /* device time of the search: the device clock from the start of its
                                first kernel to the end of its last one (HIP events around the
                                launches when params.timing = 1; batches: events around the
                                batched kernels) */
    zts_status status;
    float phase_ms[6];       /* device time per kernel, HIP events on the library's stream
                                (params.timing = 1):
                                ZTS_FULL: [0] dense kernel; ZTS_FULL_MFMA: [0] the batched launch;
                                other modes: [0] scan 1 (centres), [1] refinement window,
                                [2] scan 2 (group and member tests, survivors binned by tile;
                                each block derives the threshold from the earlier kernels'
                                records), [4] dense survivor tiles on int8 MFMA, [5] the other
                                tiles' survivors one by one; [3] the one-block reduction to
                                the answer (ZTS_FULL too) */
    float latency_ms;        /* submitted requests: submission to result ready (host clock) */
    float queue_ms;          /* submitted requests: submission to the start of its launch */
    int32_t batch_size;      /* templates in the launch that produced this result */
    int32_t above_floor;     /* 1 when rho >= params.rho_floor (always 1 with the floor off) */
    int64_t n_dense;         /* locations matched whole in dense survivor tiles (every location
                                of a tile holding many survivors; they include eliminated
                                locations, which are not in n_computed); 0 for ZTS_FULL and
                                ZTS_FULL_MFMA */
    int64_t n_sparse;        /* survivors matched one by one (those outside dense tiles) */
} zts_result;

typedef struct {
    int32_t h, w;
    int64_t cc, cr, ct;      /* groups, retained members, estimated cost mn*(cc+cr) */
    int32_t accepted;
    int32_t pad0;
} zts_egs_step;

typedef struct {
    int32_t k, d, passes, h, w, accepted;
    double sigma;
    int64_t reverted, cost;
} zts_opta_step;

/* What zts_prepare decided for one (image, m, n, mode). */
typedef struct {
    int32_t mode, m, n, group_h, group_w, radius;
    int64_t cost;
    int32_t n_egs;           /* trace of the final EGS run (every evaluated candidate) */
    int32_t n_opta;          /* OptA iterations (entry 0 = the unblurred image) */
    zts_egs_step egs[64];
    zts_opta_step opta[16];
    float prepare_ms;        /* wall time of zts_prepare */
    int32_t pad0;
} zts_prep_info;

/* ---- context ----------------------------------------------------------- */

/* Fills *p with the paper's parameters. */
ZTS_API void zts_params_default(zts_params *p);

/* ZTS_OK when every field of *p is in range, else ZTS_E_ARG (host only, no
 * device use).  Every entry point that takes parameters applies this check
 * first: rho_th and rho_tc in (-1, 1); rho_max in (-1, 1]; margin finite and
 * >= 0 (a negative margin could eliminate the true maximum); xi finite and
 * >= 0; accept_xi in (-1, 1); group_h, group_w, h0, w0, h_max in
 * [1, 32767]; dh, dw >= 0 and not both 0; blur_kind 0 or 1; sigma_step
 * finite and > 0, sigma_max finite and >= 0 (blur_kind 1); max_iters in
 * [0, 15]; refine_radius in [0, 255]; egs_estimate and egs_shape 0 or 1;
 * rho_floor finite; floor_prune 0 or 1; tile_dense_min in [-1, 8192]. */
ZTS_API zts_status zts_params_check(const zts_params *p);

/* Creates a context on params->device (NULL params: device 0, no budget). */
ZTS_API zts_status zts_create(const zts_ctx_params *params, zts_ctx **out);

/* Waits for outstanding work and frees every device buffer of the context. */
ZTS_API void zts_destroy(zts_ctx *ctx);

/* Static text for a status code. */
ZTS_API const char *zts_status_str(zts_status s);

/* ---- images ------------------------------------------------------------ */

/* Copies a host image to the device and builds its running sums (the
 * Run-Sum of section III-A / Alg. 3) of x-128 and (x-128)^2.  *id receives
 * a handle.  ZTS_E_BUDGET when the copy would exceed the HBM budget. */
ZTS_API zts_status zts_image_load(zts_ctx *ctx, const uint8_t *host, int32_t rows, int32_t cols, int64_t stride,
                          int32_t *id);

/* Same from device memory (copied device-to-device on `stream`). */
ZTS_API zts_status zts_image_load_device(zts_ctx *ctx, const void *dev, int32_t rows, int32_t cols, int64_t stride,
                                 void *stream, int32_t *id);

/* Frees an image and everything prepared for it. */
ZTS_API zts_status zts_image_unload(zts_ctx *ctx, int32_t id);

/* ---- preparation ------------------------------------------------------- */

/* Builds and keeps the per-(image, m, n, mode) tables that searches of that
 * template size use: the group size (given, or chosen by Alg. 2), the angle
 * of every location to its group centre (Alg. 1, stored as binary32 angles
 * plus the exact integer sums), per-group angle ranges, and for ZTS_OPTA the
 * conditioned image of Alg. 3 with the angle of every blurred block to its
 * original.  ZTS_FULL needs no preparation.  Searches prepare on demand;
 * calling this first keeps preparation out of the search time. */
ZTS_API zts_status zts_prepare(zts_ctx *ctx, int32_t image, int32_t m, int32_t n, zts_mode mode, const zts_params *params,
                       void *stream);

/* Reports what zts_prepare decided (group size, EGS and OptA traces). */
ZTS_API zts_status zts_prep_query(zts_ctx *ctx, int32_t image, int32_t m, int32_t n, zts_mode mode, zts_prep_info *out);

/* Copies the conditioned image of a ZTS_OPTA or ZTS_OPTA_PAPER preparation
 * to host memory (rows*cols bytes, pitch cols). */
ZTS_API zts_status zts_prep_image(zts_ctx *ctx, int32_t image, int32_t m, int32_t n, zts_mode mode,
                                  uint8_t *host_out);

/* ---- search ------------------------------------------------------------ */

/* Synchronous search of one host template.  `decision` (nullable, one byte
 * per location) receives 1 for a scan-1 centre, 3 for a refinement-window
 * location, 2 for a survivor, 0 for an eliminated location (ZTS_FULL: all 2). */
ZTS_API zts_status zts_search(zts_ctx *ctx, int32_t image, const uint8_t *tpl, int32_t m, int32_t n, int64_t stride,
                      zts_mode mode, const zts_params *params, zts_result *out, int8_t *decision);

/* Same with the template already in device memory; work is enqueued on
 * `stream` and the call returns when the result is on the host. */
ZTS_API zts_status zts_search_device(zts_ctx *ctx, int32_t image, const void *tpl_dev, int32_t m, int32_t n,
                             int64_t stride, zts_mode mode, const zts_params *params, void *stream,
                             zts_result *out);

/* zts_search_device for callers that cannot allocate device memory (code
 * that runs while a caller captures a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc): the same search, the same kernels and the
 * same result, but the call allocates nothing (no hipMalloc, hipFree or
 * other allocating routine, host or device).  Its query state, per-block
 * records, per-group centre sums and angles and survivor-tile bins live in a
 * static device array of 96 MiB that each GPU the library runs on holds until
 * the process ends.
 *   - Everything else must already be resident: the image's statistics for
 *     (m, n) (zts_prepare with any mode, or an earlier search of that size)
 *     and, for ZTS_TE_FIXED, ZTS_EGS, ZTS_OPTA and ZTS_OPTA_PAPER, tables
 *     prepared for (m, n, mode) with the same preparation parameters;
 *     otherwise ZTS_E_NOTPREPARED.
 *   - ZTS_E_SIZE when the query needs more than 96 MiB of scratch: 8 bytes
 *     per group, 64 bytes per block record and, per survivor tile of
 *     32 x 256 locations, 4 bytes times the tile's bin size (tile_dense_min,
 *     or 8192 when tiles are never matched whole); a 3 x 3 tiling of a
 *     8192 x 8192 image with the default bins takes about 65 MB.
 *   - ZTS_FULL_MFMA is not offered (ZTS_E_ARG); params->timing is ignored
 *     (phase_ms stays 0, device_ms comes from the device clock).
 *   - The template is read in place after `stream` (NULL: the context's
 *     stream) has reached the call; the call returns with the result.
 *   - Every call on one GPU uses that GPU's one array, which keeps the last
 *     call's contents (the call clears what must start at zero).  Calls on
 *     one GPU, from any context, are serialised by the library; device work
 *     that another process or a graph replay puts on the same GPU while a call
 *     runs does not touch the array. */
ZTS_API zts_status zts_search_device_noalloc(zts_ctx *ctx, int32_t image, const void *tpl_dev, int32_t m, int32_t n,
                                             int64_t stride, zts_mode mode, const zts_params *params, void *stream,
                                             zts_result *out);

/* Exhaustive search (ZTS_FULL semantics, Eq. 1 at every location) of `count`
 * host templates against one image in one fused launch on int8 MFMA
 * (v_mfma_i32_16x16x64_i8, int32 accumulation).  Templates are grouped by
 * size.  A group large enough shares 16-template tiles (M = 16 locations of a
 * row, N = 16 templates, K = 4 image rows x 16 columns); a smaller one runs
 * each template on its own (N = 16 output rows).  The route of a size comes
 * from zts_tune_batch's measurements when the context has them, else from a
 * built-in estimate.  tpls[k] points to an m[k] x n[k] template with row pitch
 * strides[k] bytes.  out[k] receives template k's answer; a template with
 * zero variance gets out[k].status = ZTS_E_DEGENERATE while the call returns
 * ZTS_OK.  Counts: every location computed.  device_ms of every entry is the
 * device time of the whole call. */
ZTS_API zts_status zts_search_batch(zts_ctx *ctx, int32_t image, int32_t count, const uint8_t *const *tpls, const int32_t *m,
                            const int32_t *n, const int64_t *strides, zts_result *out);

/* Transitive-elimination search (ZTS_TE_FIXED, ZTS_EGS, ZTS_OPTA or
 * ZTS_OPTA_PAPER) of `count` host templates against one image in one call:
 * the paper's amortisation over the templates matched against one image
 * (section III-D, Eq. 16, the auto-correlation cost shared by n_t templates).
 * Templates are grouped by size; each size is prepared once (the tables are
 * shared, as for single searches), and scan 1 runs for up to 4 templates of a
 * size in one int8-MFMA launch (the staged, realigned image fragments feed
 * every template's MFMAs; a size whose scan 1 has no MFMA form, n > 128, runs
 * one template per launch).  Each template then gets its own scan 2, survivor
 * tiles and final reduction.  out[k] receives exactly what zts_search with the
 * same mode and parameters returns for template k (location, integers,
 * binary64 rho and counts); a template with zero variance gets
 * out[k].status = ZTS_E_DEGENERATE while the call returns ZTS_OK.
 * batch_size = count; device_ms is each template's own device-clock span.
 * Argument and size errors as for zts_search; ZTS_E_ARG for other modes. */
ZTS_API zts_status zts_search_batch_pruned(zts_ctx *ctx, int32_t image, int32_t count, const uint8_t *const *tpls,
                                           const int32_t *m, const int32_t *n, const int64_t *strides,
                                           zts_mode mode, const zts_params *params, zts_result *out);

/* The same with the templates in device memory (tpls_dev[k] with row pitch
 * strides[k] bytes), read in place after `stream` (NULL: the context's
 * stream) has reached the call; returns when the results are on the host. */
ZTS_API zts_status zts_search_batch_pruned_device(zts_ctx *ctx, int32_t image, int32_t count,
                                                  const void *const *tpls_dev, const int32_t *m, const int32_t *n,
                                                  const int64_t *strides, zts_mode mode, const zts_params *params,
                                                  void *stream, zts_result *out);

/* Measured cost of one template size on the two batched MFMA kernels. */
typedef struct {
    int32_t m, n;
    float single_ms;   /* one template on its own (0 when the size only runs on shared tiles) */
    float shared_ms;   /* one shared 16-template tile */
    int32_t multi_min; /* smallest group of this size that shares tiles: the least T with
                          ceil(T / 16) * shared_ms < T * single_ms (at least 2; INT32_MAX
                          when sharing never wins, 1 when the size only runs shared) */
    int32_t pad;
} zts_tune_entry;

/* Autotuner of the batched search: for each size (m[k], n[k]) times a shared
 * 16-template tile and a lone template on image `image` (templates cut from
 * the image itself; median of three launches after a warm-up) and keeps the
 * result in the context, where it routes later batches and served requests of
 * that size.  The measurements are written to the context's tune_cache file
 * when one was given.  out[k] receives size k's entry when out is not NULL.
 * ZTS_E_SIZE when a size exceeds the image. */
ZTS_API zts_status zts_tune_batch(zts_ctx *ctx, int32_t image, int32_t count, const int32_t *m, const int32_t *n,
                                  zts_tune_entry *out);

/* ---- serving ------------------------------------------------------------ */

/* Asynchronous requests.  The context runs max_inflight worker slots, each
 * with its own HIP stream and scratch; requests start in submission order as
 * slots become free, so work admitted while other work runs overlaps with it
 * on the device.  A worker that starts a ZTS_FULL_MFMA request also takes
 * every other queued ZTS_FULL_MFMA request (any image, any size, up to 64
 * templates) into the same fused batched launch.  Other modes run one request
 * per launch and prepare on demand (ZTS_TE_FIXED, ZTS_EGS, ZTS_OPTA).
 *
 * Device memory: a launch's scratch and the per-size tables it needs are
 * charged against hbm_budget_bytes.  When they do not fit, cached tables that
 * no running work holds are freed, least recently used first; if that is not
 * enough the request goes back to the head of the queue and starts when
 * running work completes and releases memory.  It fails with ZTS_E_BUDGET
 * only when nothing else runs.
 *
 * Each result equals that of the synchronous call with the same inputs (same
 * location, integers and binary64 rho), alone or in any mix. */

/* Copies the template, queues the request and returns its ticket.
 * ZTS_E_AGAIN when max_queued requests wait already; argument errors as for
 * zts_search (ZTS_FULL_MFMA also needs n <= 128). */
ZTS_API zts_status zts_submit(zts_ctx *ctx, int32_t image, const uint8_t *tpl, int32_t m, int32_t n, int64_t stride,
                      zts_mode mode, const zts_params *params, uint64_t *ticket);

/* Queues `count` templates (all or none); tickets first_ticket ..
 * first_ticket + count - 1 in order. */
ZTS_API zts_status zts_submit_batch(zts_ctx *ctx, int32_t image, int32_t count, const uint8_t *const *tpls,
                            const int32_t *m, const int32_t *n, const int64_t *strides, zts_mode mode,
                            const zts_params *params, uint64_t *first_ticket);

/* ZTS_E_AGAIN while the request is queued or running.  Once it has ended,
 * writes its result to *out, forgets the ticket and returns the request's
 * status (ZTS_OK, or e.g. ZTS_E_DEGENERATE, ZTS_E_CANCELLED, ZTS_E_BUDGET).
 * An unknown or already collected ticket gives ZTS_E_ARG. */
ZTS_API zts_status zts_poll(zts_ctx *ctx, uint64_t ticket, zts_result *out);

/* As zts_poll, blocking up to timeout_ns (negative: no limit);
 * ZTS_E_TIMEOUT leaves the ticket valid. */
ZTS_API zts_status zts_wait(zts_ctx *ctx, uint64_t ticket, int64_t timeout_ns, zts_result *out);

/* Cancels a request that has not started: it ends with ZTS_E_CANCELLED (still
 * to be collected).  ZTS_E_BUSY once it has started or ended. */
ZTS_API zts_status zts_cancel(zts_ctx *ctx, uint64_t ticket);

/* Requests waiting in the queue and worker slots executing work right now. */
ZTS_API zts_status zts_pending(zts_ctx *ctx, int32_t *queued, int32_t *running);

/* ---- parity helpers ------------------------------------------------------ */

/* Every location's exact N and D_r and binary32 rho for one template
 * (ZTS_FULL kernel with its maps written out).  Any output may be NULL. */
ZTS_API zts_status zts_debug_full_map(zts_ctx *ctx, int32_t image, const uint8_t *tpl, int32_t m, int32_t n,
                              int64_t stride, int64_t *num_out, int64_t *den_r_out, float *rho_out);

/* Alg. 1 on the device: for group size (h, w), every location's exact
 * N_co, D_c and D_o against its group centre (int64 arrays of L entries). */
ZTS_API zts_status zts_debug_autocorr(zts_ctx *ctx, int32_t image, int32_t m, int32_t n, int32_t h, int32_t w,
                              int64_t *num_out, int64_t *dc_out, int64_t *do_out);

/* Eq. 18 on the device: blurs a host image with separable integer taps
 * (2d+1 of them), clamp-to-edge borders, rounded half up. */
ZTS_API zts_status zts_debug_blur(zts_ctx *ctx, const uint8_t *host_in, int32_t rows, int32_t cols, const int32_t *taps,
                          int32_t d, uint8_t *host_out);

#ifdef __cplusplus
}
#endif

#endif /* ZTS_H */
