// Kernel argument blocks and launch wrappers (host side of zts_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zts_shared.h"

namespace zts {

// Dense search: every location of the image.
struct FullArgs {
    const uint8_t *img;
    int64_t pitch;
    int p, q;
    const int2 *stat;  // per-location (sum x', sum x'^2) for (m, n)
    const uint8_t *tpl;
    int64_t ts;
    int m, n, n4w;
    int Ly, Lx;
    RecPod *recs;
    QState *qs;
    int64_t *num_map;  // optional outputs (parity checks)
    int64_t *dr_map;
    float *rho_map;
    int8_t *dec;
};

// Per-template outputs of a batched scan 1 (templates 1 .. ntpl - 1; template
// 0 uses the scalar fields of ScanArgs).
constexpr int kScanMaxT = 4;
struct ScanTpl {
    const uint8_t *tpl;
    int64_t ts;
    int32_t *g_x;
    float *g_theta;
    RecPod *recs;
    QState *qs;
    uint32_t *tile_cnt;
};

// Scan 1: group centres of the searched image.
struct ScanArgs {
    const uint8_t *img;
    int64_t pitch;
    const int2 *stat;
    const int2 *cstat;  // MFMA form: statistics of each group centre's block, [Gy][Gx]
    const uint8_t *tpl;
    int64_t ts;
    int m, n, n4w, pad, Ly, Lx, h, w, Gy, Gx;
    int32_t *g_x;  // per group: the centre's exact sum of t' r' (N_tc = mn X - S_t S_c)
    float *g_theta;
    RecPod *recs;
    QState *qs;
    int8_t *dec;
    double delta;
    uint32_t *tile_cnt;  // survivor counts of scan 2's tiles, zeroed here (n_tiles entries)
    int n_tiles;
    int cwd;      // MFMA form: dword stride of the byte-shifted copies of a staged image row
    int cwn;      // MFMA form: dwords of each staged row that are read
    int crows_log2;  // unused (the MFMA form stages 4-row steps)
    // MFMA form, batched: ntpl templates of the same size matched in one launch
    // (each staged image fragment feeds all of them); 1 for a single query
    int ntpl;
    ScanTpl more[kScanMaxT - 1];
};

// Refinement window on the original image.
struct WinArgs {
    const uint8_t *img;
    int64_t pitch;
    const int2 *stat;
    const uint8_t *tpl;
    int64_t ts;
    int m, n, Ly, Lx, h, w;
    int radius;
    int skip_centres;   // scan 1 ran on this image: its centres are already matched
    int include_best0;  // the scan-1 best is an original-image rho
    int thr_out;        // scan 2 runs next: block 0 writes the scan-1 best into the query state
    RecPod *recs;       // scan-1 records [0, rec_off), then this kernel's
    int rec_off;
    QState *qs;
    int8_t *dec;
    double delta;
};

// Scan 2: group and member tests, survivors matched on the original image.
struct MemArgs {
    const uint8_t *I;
    int64_t pI;
    const int2 *statI;  // original image statistics
    const int2 *statS;  // statistics of the image scan 1 searched (I, or the blurred J)
    const uint8_t *tpl;
    int64_t ts;
    int m, n, Ly, Lx, h, w, Gy, Gx;
    const int32_t *g_x;
    const float *g_theta;
    const GroupSum *gsum;
    const float *theta_b;   // member vs its centre on the searched image (group-major)
    const int32_t *x_b;
    const float *theta_c;   // searched-image block vs original block (opta, group-major)
    const int32_t *x_c;
    int opta;
    int radius;  // window radius, -1 when there is none
    RecPod *recs;
    int rec_off;
    int final_from;
    QState *qs;
    int8_t *dec;
    // the threshold comes from the records of scan 1 [0, n_best0) and of the
    // window [n_best0, n_best0 + n_win); include_best0: the scan-1 best is an
    // original-image rho and competes with the window's
    int n_best0, n_win, include_best0;
    int thr_ready;  // the window kernel wrote the scan-1 best into the query state: only the window
                    // records are reduced, by each wave
    double delta;
    double floor;   // eliminate against max(best, floor) (-2: the attained best alone)
    // survivors are binned by tile of kTileRows x kTileCols locations (row-major tiles_x per row):
    // tile_cnt counts them, tile_bin holds each tile's first tile_cap
    uint32_t *tile_cnt;
    int32_t *tile_bin;
    int tile_cap, tiles_x;
};

// Survivor tiles: kTileRows x kTileCols locations (the footprint of one
// two-row-group block of the single-template MFMA kernel).
constexpr int kTileRows = 32, kTileCols = 256;

// Matching of scan 2's survivors.  Super-tiles of four stacked tiles that
// hold many survivors are matched whole on int8 MFMA (k_dense_tiles; every
// location, the extra ones were eliminated so they cannot be the answer);
// the other tiles' listed survivors are matched one wave each (k_surv_tiles),
// from the tile's image region staged in LDS when it fits (sparse_lds) or
// from global memory.
struct TileArgs {
    const uint8_t *img;  // the image survivors are matched on
    int64_t pitch;
    int p, q;
    const int2 *stat;    // its statistics for (m, n)
    const uint8_t *tpl;
    int64_t ts;
    int m, n, n16, Ly, Lx;
    int tiles_x, tiles_y;
    const uint32_t *tile_cnt;
    const int32_t *tile_bin;
    int tile_cap;
    int dense_min;       // 0: never dense
    int sparse_lds;      // 1: stage the tile's image region in LDS
    int region_words;    // words per staged region row
    int surv_blocks;     // the tile kernels' grids (blocks loop over tiles): k_surv_tiles' records first,
    int dense_blocks;    // then k_dense_tiles' (0 without a dense path)
    int surv_parts;      // parts a sparse tile's survivors may be split into
    QState *qs;
    RecPod *recs;
    int rec_off;
};

// AC_COUNT / AC_COUNT_BLUR: Eq. 15 (Prop. 3.2) retained count, without and
// with the angle to the original block; AC_COUNT31 / AC_COUNT31_BLUR: the
// same with Prop. 3.1's bound at an assumed template-to-centre correlation.
enum { AC_DEBUG = 0, AC_COUNT = 1, AC_COUNT_BLUR = 2, AC_BUILD = 3, AC_COUNT31 = 4, AC_COUNT31_BLUR = 5 };

struct AcArgs {
    const uint8_t *J;
    int64_t pJ;
    const int2 *statJ;
    const int2 *statI;
    int m, n, Ly, Lx, h, w;
    int mode;
    int64_t *num_out, *dc_out, *do_out;
    float *theta_b;
    int32_t *x_b;
    const float *theta_c;
    const int32_t *x_c;
    double thr;                  // sqrt(1 - rho_th^2)
    float thr_lo, thr_hi;        // thr -/+ guard band
    float alo_lo, alo_hi;        // acos(thr) -/+ guard band
    float ahi_lo, ahi_hi;        // 2 pi - acos(thr) -/+ guard band
    double rho_th;               // AC_COUNT31*: the threshold of Prop. 3.1
    double ra, sa;               // AC_COUNT31*: assumed rho_tc and sqrt(1 - rho_tc^2)
    unsigned long long *counter;
};

struct GsumArgs {
    const float *theta_b;
    const float *theta_c;
    int Ly, Lx, h, w, Gy, Gx;
    int opta;
    GroupSum *gsum;
};

enum { BC_VIOL = 0, BC_BUILD = 1, BC_DEBUG = 2 };

struct BcArgs {
    const uint8_t *J;
    const uint8_t *I;
    int64_t pitch;
    const int2 *statJ;
    const int2 *statI;
    int m, n, Ly, Lx;
    int mode;
    uint8_t *viol;
    unsigned long long *counter;
    double lambda;
    float lam_lo, lam_hi;
    float *theta_c;
    int32_t *x_c;
    int64_t *num_out, *dj_out, *di_out;
    const uint32_t *psat;  // running sums of J' I' ((p+1) x (q+1)), set by launch_blurcorr
    int q;
};

// One bucket of a batched launch: the templates of one size searched in one
// image.  A launch takes a device table of jobs; each kernel's flattened
// block index selects its job (block0 / fold0 / tmpl0 are the job's first
// block of k_batch, of the first fold and its first template).
struct BatchJob {
    const uint8_t *img;
    int64_t pitch;
    int p, q;
    const int2 *stat;     // per-location statistics of img for (m, n)
    const uint8_t *tpl;   // uint8 templates, [T][m][n16], 0x80 past column n
    int64_t *tst;         // per template: sum(t'), D_t (written by the launch)
    int T, m, n, n16, Ly, Lx;
    int gx, gy, gz;       // blocks: 256-column strips, row strips, tiles of 16 templates
    int chunks;           // first-fold blocks per tile
    int block0, fold0, tmpl0;  // block0 counts within the kernel that runs the job
    int kind;             // BATCH_MULTI: up to 16 templates of one size per tile (N = templates);
                          // BATCH_SINGLE: one template (N = 16 output rows)
    int rg;               // BATCH_SINGLE: 16-row groups per block (8, 4 or 2; one value per table)
    RecPod *recs;         // batch_job_records(job) records: [gz][gy*gx][16], then [gz][chunks][16]
    RecPod *out;          // [T] answers
};

enum { BATCH_MULTI = 0, BATCH_SINGLE = 1 };

// Fills n16, gx, gy, gz and chunks from kind, T, m, n, Ly, Lx (and rg for
// BATCH_SINGLE); false when n > 128 (or, for BATCH_SINGLE, T != 1, rg not
// 8, 4 or 2, or the template does not fit LDS).
bool batch_job_geometry(BatchJob &j);
// Whether one m x n template fits the single-template kernel's LDS.
bool batch_single_fits(int m, int n);
size_t batch_job_records(const BatchJob &j);
// Runs template statistics, the MFMA search, and the two record folds for
// every job of the table (d_jobs on the device, h_jobs its host copy).  The
// table lists the BATCH_MULTI jobs first, then the BATCH_SINGLE ones.
hipError_t launch_batch_jobs(const BatchJob *d_jobs, const BatchJob *h_jobs, int njobs, hipStream_t s);

// Running-sum tables are allocated with sat_elems(p, q) elements: the
// (p+1) x (q+1) table followed by the column pass's per-chunk totals and
// per-part (16-row) totals.
size_t sat_elems(int p, int q);
hipError_t launch_sat(const uint8_t *img, int64_t pitch, int p, int q, uint2 *sat, hipStream_t s);
hipError_t launch_stats(const uint2 *sat, int q, int Ly, int Lx, int m, int n, int2 *stat, hipStream_t s);

int full_record_count(int Ly, int Lx);
size_t full_lds_bytes(int m, int n);
// Whether k_full can stage a template of m x n (LDS of one workgroup).
bool full_fits(int m, int n);
hipError_t launch_full(FullArgs a, hipStream_t s);

// Scan 1 runs on int8 MFMA (k_centres_mfma) when the region a block's windows
// cover fits its LDS budget, else on v_dot4 (k_centres); both write one
// record per block.
int centres_record_count(int Gy, int Gx, int m, int n, int h, int w);
// The best record of [lo, hi) and the counts summed over [count_lo, hi) into
// the query state, then copies the state to its pinned host mirror `host` and
// bumps qs->seq there last.  Over more than 2048 records, chunks are merged
// by a first launch that overwrites each chunk's first record.
hipError_t launch_reduce(RecPod *recs, int lo, int hi, int count_lo, QState *qs, QState *host, hipStream_t s);
// Zeroes *qs (every word, the sequence number included) with a fill kernel.
hipError_t launch_qs_clear(QState *qs, hipStream_t s);
hipError_t launch_centres(ScanArgs a, hipStream_t s);
// Whether scan 1 of an m x n template with group width w over a Gy x Gx
// centre grid runs on int8 MFMA (then a.ntpl templates can share one launch
// of launch_centres).
bool centres_mfma_batchable(int Gy, int Gx, int m, int n, int w, int ntpl);
int window_record_count(int radius);
hipError_t launch_window(WinArgs a, hipStream_t s);
int members_record_count(int Gy, int Gx);
hipError_t launch_members(MemArgs a, hipStream_t s);
// Tiles of scan 2 over an Ly x Lx location grid.
int tiles_x_of(int Lx);
int tiles_y_of(int Ly);
// Fills the geometry fields of a (n16, dense_min, tile_cap, sparse_lds,
// region_words, the tile kernels' grids) for its m, n and the wanted dense
// threshold (0: never), on the current device.
void tile_plan(TileArgs &a, int dense_min);
// Records of the two tile kernels from rec_off: one per k_surv_tiles block,
// then one per k_dense_tiles block (whether a tile is matched whole is
// decided per super-tile of 4 stacked tiles, 128 x 256 locations).
int tile_record_count(const TileArgs &a);
// k_dense_tiles (nothing when a.dense_min is 0), then k_surv_tiles.
hipError_t launch_dense_tiles(TileArgs a, hipStream_t s);
hipError_t launch_surv_tiles(TileArgs a, hipStream_t s);
// Whether scan 1 (either form) and scan 2 can stage a template of m x n.
bool scan_fits(int m, int n);
// Whether a static-LDS query behind full_fits / scan_fits failed on this
// thread since the last call (a failed query answers "does not fit" and is not
// cached); clears the flag.
bool lds_query_failed();
hipError_t launch_regroup(const void *in, void *out, int Ly, int Lx, int h, int w, hipStream_t s);

// Alg. 1: direct dot products per location, or, when cheaper
// (autocorr_by_shifts), running sums of one product image per member offset
// (psat: scratch of sat_elems(p, q) uint32).
bool autocorr_by_shifts(int m, int n, int h, int w);
hipError_t launch_autocorr(AcArgs a, uint32_t *psat, hipStream_t s);
hipError_t launch_gsum(GsumArgs a, hipStream_t s);
// Statistics of every group centre's block, gathered from the per-location
// map into [Gy][Gx] (centres as scan 1 places them).
hipError_t launch_centre_stats(const int2 *stat, int Ly, int Lx, int h, int w, int Gy, int Gx, int2 *out,
                               hipStream_t s);
hipError_t launch_blur(const uint8_t *src, uint8_t *dst, int64_t pitch, int p, int q, const Taps &tp,
                       uint32_t *tmp, hipStream_t s);
// psat: scratch of sat_elems(p, q) uint32 for the running sums of J' I'.
hipError_t launch_blurcorr(BcArgs a, uint32_t *psat, hipStream_t s);
hipError_t launch_revert(const uint8_t *viol, uint8_t *colmask, int p, int q, int Ly, int Lx, int m, int n,
                         const uint8_t *I, uint8_t *J, int64_t pitch, unsigned long long *counter, hipStream_t s);

}  // namespace zts
