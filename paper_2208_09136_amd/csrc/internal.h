// internal.h -- device data layout shared by the kernels and the host code of
// the averaged-RQA library.  Not part of the public C ABI (see include/rqa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rqa.h"

namespace rqa {

// One wavefront walks a band of TILE_W consecutive diagonals; lane L owns
// diagonal d0 + L and steps along it.
constexpr int TILE_W = 64;

// Radix split of the 31 significant bits of a key (the sign bit is always 0):
// pass 1 histograms the top SEL_B1 bits for every pair; pass 2 the next SEL_B2
// bits of keys whose pass-1 prefix holds a target (per-slot LDS bins, twice
// over with line values, so SEL_B2 stays small); pass 3 the last SEL_B3 bits
// of keys whose 20-bit prefix holds a target (global counters: few qualify).
constexpr int SEL_B1 = 12;
constexpr int SEL_B2 = 8;
constexpr int SEL_B3 = 11;
constexpr int SEL_SH1 = 31 - SEL_B1;           // 19
constexpr int SEL_SH2 = SEL_SH1 - SEL_B2;      // 11
constexpr uint32_t SEL_N1 = 1u << SEL_B1;      // 4096
constexpr uint32_t SEL_N2 = 1u << SEL_B2;      // 256
constexpr uint32_t SEL_N3 = 1u << SEL_B3;      // 2048
constexpr uint8_t NO_SLOT = 0xFF;

// Threshold-rank lookup table of the sweep: RHO_TABLE buckets of the key's
// bit pattern between the smallest and the largest threshold.
constexpr int RHO_BITS = 12;
constexpr uint32_t RHO_TABLE = 1u << RHO_BITS;
constexpr uint32_t RHO_MULTI = 0x10000u;       // entry.y >= this: >1 threshold in bucket

constexpr int LMIN_MAX = 16;

// Per-series descriptor (device copy built by the host for every call).
struct SeriesDesc {
    const float* y;        // device pointer to the series
    uint32_t n;            // samples
    uint32_t nv;           // delay vectors n - (m-1) tau
    uint32_t m, tau, norm, w, lmin;
    uint32_t K;            // targets / thresholds
    uint64_t M;            // pairs (nv-w)(nv-w+1)/2
    uint32_t B;            // bands of TILE_W diagonals: ceil((nv-w)/64)
    uint32_t T;            // segment length along a diagonal (multiple of 64)
    uint32_t q;            // T / 64
    uint32_t Smax;         // segments: ceil((nv-w)/T)
    uint32_t ntiles;       // (band, segment) tiles
    uint32_t chunk_begin;  // first global chunk index of this series
    uint32_t nchunks;      // chunks of this series
    uint32_t variant;      // kernel variant (norm/m/lmin class), host bookkeeping
    uint64_t seed;         // sketch sampling stream
    float f_logn, f_m;     // sketch features log2(n)/16 and m/4
};

// Distance sketch: SKETCH_P sampled pairs, SKETCH_BINS bins of a quarter
// binade around the sample median, plus two shape features.
constexpr int SKETCH_P = 4096;
constexpr int SKETCH_BINS = 64;
constexpr int SKETCH_FEATURES = SKETCH_BINS + 2;

// Per-series working state in device memory.
struct SeriesWork {
    // exact selection (targets in caller order)
    uint64_t k[RQA_MAX_K];        // target rank
    uint64_t below[RQA_MAX_K];    // keys below the target's current bucket
    uint32_t prefix[RQA_MAX_K];   // resolved high bits of the target's key
    uint32_t slot[RQA_MAX_K];     // slot of the target in the current pass
    uint32_t nslots2, nslots3;
    uint32_t eps_bits[RQA_MAX_K]; // selected (or given) thresholds, caller order
    uint64_t count[RQA_MAX_K];    // #{key <= eps} from selection
    // line values riding along with the keys (selection with lines): the
    // line value of a cell is the smallest threshold at which it lies on a
    // diagonal line of length >= lmin, so D(eps) = #{line value <= eps}
    uint64_t belowL[RQA_MAX_K];   // line values below the target's current bucket
    uint64_t dcount[RQA_MAX_K];   // D = #{line value <= eps}
    // sweep
    uint32_t esorted[RQA_MAX_K];  // distinct thresholds, ascending
    uint32_t dmap[RQA_MAX_K];     // caller index -> distinct index
    uint32_t Kp;                  // distinct thresholds
    uint32_t shift, emin, emax;   // rank-table geometry
    uint32_t multi;               // some bucket of the rank table holds several thresholds
    uint64_t hrho[RQA_MAX_K + 1]; // cells with rank rho (rho < Kp)
    uint64_t hlam[RQA_MAX_K + 1]; // cells with line rank lambda (lambda < Kp)
    uint32_t nonfinite;           // set when a sample is NaN or infinite
    uint32_t status;              // device-side error bits (0 = fine)
    uint32_t scale;               // sketch: bit pattern of the sample median
    // window selection (learned or sampled bracket)
    uint32_t win_lo, win_span;    // window [win_lo, win_lo + win_span] of key bit patterns
    uint32_t win_shift, win_ok;   // fine-bin width 2^win_shift; win_ok = 0: no usable window
    uint64_t win_below;           // #{key < win_lo}
    uint64_t win_belowL;          // #{line value < win_lo}
    uint32_t win_hit[RQA_MAX_K];  // target resolved inside the window
    uint32_t win_fbin[RQA_MAX_K]; // fine bin of the target's key
    uint32_t win_slot[RQA_MAX_K]; // pass-2 slot of that fine bin
    uint64_t win_base[RQA_MAX_K]; // #{key < start of the fine bin}
    uint64_t win_baseL[RQA_MAX_K];// #{line value < start of the fine bin}
    uint32_t win_nslots;
};

// Window selection: WIN_BINS fine bins over the window; the last
// win_shift <= WIN_MAX_SHIFT bits are resolved in a second pass.
constexpr int WIN_BITS = 13;
constexpr uint32_t WIN_BINS = 1u << WIN_BITS;
constexpr uint32_t WIN_MAX_SHIFT = 14;

// Device buffers of one call (host-side handle).
struct DevBufs {
    SeriesDesc* sd;     // [S]
    SeriesWork* work;   // [S]
    uint8_t* T1;        // [S][SEL_N1] pass-1 bucket -> pass-2 slot
    uint8_t* T2;        // [S][K][SEL_N2] (pass-2 slot, sub-bucket) -> pass-3 slot
    uint2* rtab;        // [S][RHO_TABLE] sweep rank table
    uint64_t* h1;       // [S][SEL_N1]
    uint64_t* h2;       // [S][K][SEL_N2]
    uint64_t* h3;       // [S][K][SEL_N3]
    uint64_t* h1L;      // line-value histograms of the same shapes (selection with lines)
    uint64_t* h2L;
    uint64_t* h3L;
    uint32_t lines;     // selection with lines: line values ride along with the keys
    uint32_t* tickets;  // work-queue counters, one per launch
    uint32_t S, K;
    uint32_t nchunks;   // over all series
    uint32_t chunk_tiles;
};

constexpr int NUM_TICKETS = 256;

// Kernel launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_zero(hipStream_t st, void* p, size_t bytes);
hipError_t launch_check_finite(hipStream_t st, const DevBufs& b, uint32_t maxn);
hipError_t launch_select_pass(hipStream_t st, const DevBufs& b, int pass, int variant,
                              uint32_t grid, uint32_t block, uint32_t groups, uint32_t group_slots,
                              uint32_t ticket_base);
hipError_t launch_select_scan(hipStream_t st, const DevBufs& b, int pass);   // honours b.lines
hipError_t launch_sweep_prep(hipStream_t st, const DevBufs& b);
hipError_t launch_sweep(hipStream_t st, const DevBufs& b, int variant, uint32_t grid,
                        uint32_t block, uint32_t ticket);
// Window selection.  Sources of the window: predicted offsets [S][20] with
// half-widths (network), or the sorted sketch sample (sample quantiles).
struct WinBufs {
    uint64_t* bins;      // [S][WIN_BINS] pass-1 counts
    uint8_t* table;      // [S][WIN_BINS] fine bin -> pass-2 slot
    uint64_t* fine;      // [S][K][1 << WIN_MAX_SHIFT] pass-2 counts
    uint64_t* binsL;     // line values, same shapes (selection with lines)
    uint64_t* fineL;
};
hipError_t launch_window_from_offsets(hipStream_t st, const DevBufs& b, const float* pred, const float* delta_dev);
hipError_t launch_window_fixed(hipStream_t st, const DevBufs& b, uint32_t lo, uint32_t hi);
hipError_t launch_window_from_sample(hipStream_t st, const DevBufs& b, const uint32_t* sample_sorted, const double* rr_dev,
                                     float z);
hipError_t launch_window_pass(hipStream_t st, const DevBufs& b, const WinBufs& w, int pass, int variant, uint32_t grid,
                              uint32_t block, uint32_t ticket);
hipError_t launch_window_scan(hipStream_t st, const DevBufs& b, const WinBufs& w, int pass);
size_t window_lds_bytes(int pass, bool lines);
int window_blocks_per_cu(int pass, int variant, uint32_t block);

// Sketch of every series: features [S][SKETCH_FEATURES], sorted sample bits
// [S][SKETCH_P] (may be NULL), scale into SeriesWork.
hipError_t launch_sketch(hipStream_t st, const DevBufs& b, float* features, uint32_t* sample_sorted);

// Kernel variants.  Embedding class: 0 any (m, tau) at run time, 1 m = 1,
// 2 m = 3 with tau = 3, 3 m = 3 with tau = 5.  Line class: 0 any lmin,
// 1 lmin = 1, 2 lmin = 2.  select variant = norm * 4 + embedding class;
// sweep variant = select variant * 3 + line class.  Selection with lines
// adds a line-value class (0 none: plain selection or lmin = 1, where every
// recurrence lies on a line; 1 lmin = 2; 2 any lmin, embedding class 0):
// selection variant = line-value class * 8 + select variant.
constexpr int NUM_MCLASS = 4;
constexpr int NUM_SELECT_VARIANTS = 2 * NUM_MCLASS;
constexpr int NUM_SWEEP_VARIANTS = NUM_SELECT_VARIANTS * 3;
int select_variant_of(uint32_t norm, uint32_t m, uint32_t tau);
int lines_variant_of(uint32_t norm, uint32_t m, uint32_t tau, uint32_t lmin);
int variant_of(uint32_t norm, uint32_t m, uint32_t tau, uint32_t lmin);

// Dynamic LDS bytes of each kernel for a K and group size.
size_t select_lds_bytes(int pass, uint32_t K, uint32_t group_slots, bool lines);
size_t sweep_lds_bytes(uint32_t K);

// Occupancy helpers (kernels.hip): max resident workgroups per CU.
int select_blocks_per_cu(int pass, int variant, uint32_t block, size_t lds);
int sweep_blocks_per_cu(int variant, uint32_t block, size_t lds);
hipError_t set_kernel_lds_limits(size_t max_dyn_lds);

}  // namespace rqa
