// Plain structs shared by the host library and the kernels.
#pragma once

#include <stdint.h>

namespace zts {

// Best-location record of one block (or of a whole query after reduction).
struct RecPod {
    double rho;    // canonical binary64 rho of the best candidate
    int64_t l;     // its linear location index (INT64_MAX when empty)
    int64_t num;   // exact N at l
    int64_t dr;    // exact D_r at l
    float r32max;  // largest binary32 rho among the candidates of the block
    int32_t valid;
    // location counts of the block, summed when records are merged
    unsigned long long n_elim, n_surv, n_window;
};

// Per-query state in device memory; the host reads it back once at the end.
struct QState {
    // template statistics (every block recomputes them; one writes)
    int64_t st;  // sum(t')
    int64_t dt;  // D_t
    int32_t degenerate;
    int32_t pad0;
    // scan 1 result
    double best0;
    int64_t best0_l;
    // threshold used by scan 2
    double best;
    int64_t best_l;
    double thr64;  // best - delta
    float thr_lo, thr_hi;  // acos(thr64) -/+ guard band, binary32
    // counters
    unsigned long long n_centres, n_window, n_elim, n_surv;
    // answer
    RecPod fin;
    float fin_r32;
    int32_t pad1;
    // device realtime clock at the first kernel's start and the last one's end
    unsigned long long t0, t1;
    // locations matched whole in dense survivor tiles, and survivors matched
    // one by one in the other tiles (scan 1 zeroes both)
    unsigned long long n_dense, n_sparse;
    // completed queries of this state; the final reduction copies the state
    // to the host mirror and writes this last
    unsigned long long seq;
};

// Taps of one separable integer blur pass.
struct Taps {
    int32_t w[65];
    int32_t d;
};

// Per-group summary for scan 2: range of member angles to the centre and
// largest angle of a member to its original block (0 without blur).
struct GroupSum {
    float bmin, bmax, cmax;
    int32_t flags;  // 1: some member angle is undefined (flat block)
};

}  // namespace zts
