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
// bits of keys whose pass-1 prefix holds a target (per-slot LDS bins); the
// last SEL_B3 bits of keys whose 21-bit prefix holds a target are resolved
// either by pass 3 (selection only) or inside the line sweep (global
// counters: few keys qualify).
#ifndef RQA_SEL_B1
#define RQA_SEL_B1 12
#endif
constexpr int SEL_B1 = RQA_SEL_B1;
constexpr int SEL_B2 = 21 - SEL_B1;
constexpr int SEL_B3 = 10;
constexpr int SEL_SH1 = 31 - SEL_B1;           // 19
constexpr int SEL_SH2 = SEL_SH1 - SEL_B2;      // 10
constexpr uint32_t SEL_N1 = 1u << SEL_B1;      // 4096
constexpr uint32_t SEL_N2 = 1u << SEL_B2;      // 512
constexpr uint32_t SEL_N3 = 1u << SEL_B3;      // 1024
constexpr uint8_t NO_SLOT = 0xFF;

// Threshold-rank lookup table of the sweep: RHO_TABLE buckets of the key's
// bit pattern between the smallest and the largest threshold.
constexpr int RHO_BITS = 12;
constexpr uint32_t RHO_TABLE = 1u << RHO_BITS;
constexpr uint32_t RHO_MULTI = 0x10000u;       // entry.y >= this: >1 threshold in bucket
// Range sweep: half as many buckets, each holding up to two boundaries (a
// group's two boundaries usually share a bucket); same bytes as RHO_TABLE.
constexpr int RANGE_BITS = 11;
constexpr uint32_t RANGE_TABLE = 1u << RANGE_BITS;

constexpr int LMIN_MAX = 16;

// LDS of a CU and the unit in which gfx950 allocates it to a workgroup.  The
// unit is measured, not documented: a 53,272-byte range sweep runs three
// workgroups per CU and a 53,784-byte one two (wave-cycles per busy cycle
// drop by exactly a third), although 160 KB / 3 = 54,613 bytes would admit
// both and the runtime's occupancy query reports three for each; 1280 bytes
// (160 KB in 128 units) is the unit that separates the two.
constexpr uint32_t LDS_PER_CU = 160u * 1024u;
constexpr uint32_t LDS_UNIT = 1280u;
__host__ __device__ __forceinline__ uint32_t lds_blocks_fit(size_t bytes)
{
    const size_t units = (bytes + LDS_UNIT - 1) / LDS_UNIT;
    return units ? (uint32_t)(LDS_PER_CU / (units * LDS_UNIT)) : 1u << 16;
}

// Entries of the sweep's threshold list: K thresholds, or two boundaries per
// candidate range.
constexpr int RANK_MAX = 2 * RQA_MAX_K;

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
    uint64_t dcount[RQA_MAX_K];   // D: recurrences on lines of length >= lmin at eps
    // sweep: rank table over ascending thresholds (given thresholds) or over
    // the boundaries of the candidate ranges (range sweep)
    uint32_t esorted[RANK_MAX];   // ascending thresholds / boundaries
    uint32_t dmap[RQA_MAX_K];     // caller index -> distinct threshold index
    uint32_t Kp;                  // thresholds / boundaries in esorted
    uint32_t zbase;               // rank offset: 1 when the first range starts at key 0
    uint32_t shift, emin, emax;   // rank-table geometry
    uint32_t multi;               // some bucket of the rank table holds several thresholds
    uint64_t hrho[RANK_MAX + 2];  // cells with rank rho
    uint64_t hlam[RANK_MAX + 2];  // cells with line rank lambda
    // range sweep: after the counting passes every target's key lies in a
    // candidate range of 2^range_bits bit patterns; adjacent ranges merge into
    // groups; the sweep counts the sub-values of keys and line values that
    // fall inside a group
    uint32_t range_bits;          // log2 of the width of one range
    uint32_t nsub;                // distinct ranges (fine counters: nsub << range_bits)
    uint32_t ngroups;             // groups of adjacent ranges
    uint32_t range_ok;            // the series takes part in the range sweep
    uint32_t g_lo[RQA_MAX_K + 1]; // first bit pattern of each group
    uint32_t g_off[RQA_MAX_K + 1];// fine-counter index of each group's first value
    uint32_t t_sub[RQA_MAX_K];    // range of each target
    uint32_t t_group[RQA_MAX_K];  // group of each target
    uint32_t sub_lo[RQA_MAX_K];   // first bit pattern of each range
    uint64_t rbase[RQA_MAX_K];    // keys below the target's range (from the counting passes)
    uint32_t nonfinite;           // set when a sample is NaN or infinite
    uint32_t status;              // device-side error bits (0 = fine)
    uint32_t scale;               // sketch: bit pattern of the sample median
    // window selection (learned or sampled bracket)
    uint32_t win_lo, win_span;    // window [win_lo, win_lo + win_span] of key bit patterns
    uint32_t win_shift, win_ok;   // fine-bin width 2^win_shift; win_ok = 0: no usable window
    uint64_t win_below;           // #{key < win_lo}
    uint32_t win_hit[RQA_MAX_K];  // target resolved inside the window
    uint32_t win_fbin[RQA_MAX_K]; // fine bin of the target's key
    uint32_t win_slot[RQA_MAX_K]; // pass-2 slot of that fine bin
    uint64_t win_base[RQA_MAX_K]; // #{key < start of the fine bin}
    uint32_t win_nslots;
};

// Window selection: WIN_BINS fine bins over the window (the whole 160 KB LDS
// of a CU as 32-bit counters, one workgroup of 1024 threads per CU); the last
// win_shift <= WIN_MAX_SHIFT bits are resolved by the range sweep or a second
// window pass.
#ifndef RQA_WIN_BINS
#define RQA_WIN_BINS (39 * 1024)
#endif
constexpr uint32_t WIN_BINS = RQA_WIN_BINS;
constexpr uint32_t WIN_BLOCK = 1024;
constexpr uint32_t WIN_MAX_SHIFT = 13;

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
    uint64_t* fineK;    // range sweep: [S][fine_stride] sub-value counts of keys
    uint64_t* fineL;    //              and of line values
    uint32_t fine_stride;
    uint32_t* tickets;  // work-queue counters, one per launch
    uint32_t S, K;
    uint32_t nchunks;   // over all series
    uint32_t chunk_tiles;
};

constexpr int NUM_TICKETS = 256;

// Kernel launchers (kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_zero(hipStream_t st, void* p, size_t bytes);
// Flags non-finite samples and places the targets tgt[S][K] (ranks when
// as_rank, else threshold bit patterns) into the zeroed working state.
hipError_t launch_check_finite(hipStream_t st, const DevBufs& b, uint32_t maxn, const uint64_t* tgt, bool as_rank);
// Results the host reads, result_words(K, lines) words per series (layout at
// k_pack_results).
__host__ __device__ __forceinline__ size_t result_words(uint32_t K, bool lines) { return 3 + (size_t)(lines ? 7 : 5) * K; }
hipError_t launch_pack_results(hipStream_t st, const DevBufs& b, bool lines, uint64_t* out);
hipError_t launch_select_pass(hipStream_t st, const DevBufs& b, int pass, int variant,
                              uint32_t grid, uint32_t block, uint32_t groups, uint32_t group_slots,
                              uint32_t ticket_base);
hipError_t launch_select_scan(hipStream_t st, const DevBufs& b, int pass);
hipError_t launch_sweep_prep(hipStream_t st, const DevBufs& b);
// ranges = false: sweep at given thresholds (rank table from k_sweep_prep);
// ranges = true: range sweep (rank table from k_range_prep)
hipError_t launch_sweep(hipStream_t st, const DevBufs& b, int variant, bool ranges, uint32_t grid,
                        uint32_t block, uint32_t ticket);
// Range sweep set-up after the counting passes: from the plain selection
// state after scan 2 (window = false) or from the window state after window
// scan 1 (window = true); and the final scan giving eps, C and D.
hipError_t launch_range_prep(hipStream_t st, const DevBufs& b, bool window);
hipError_t launch_range_scan(hipStream_t st, const DevBufs& b);
// Full line-length histogram at given thresholds (after k_sweep_prep) over
// the (band, segment) tiles: difference counts dglob[S][hist_len][Kp + 1]
// (two's complement in uint64; cleared by the caller) of the lines inside a
// segment, and per tile, threshold and lane the leading and trailing run
// lengths pre / suf [tiles][Kp + 1][64] (tile index = chunk_begin *
// chunk_tiles + tile, per group); the join adds the lines across segment
// borders.  Kp <= HIST_MAX_K_HOST distinct thresholds, segments at most
// HIST_MAX_SEG_HOST long, block a multiple of 64 up to 1024.
hipError_t launch_hist(hipStream_t st, const DevBufs& b, int select_variant, uint32_t grid, uint32_t block,
                       uint64_t* dglob, uint16_t* pre, uint16_t* suf, uint32_t hist_len, uint32_t Kp, uint32_t ticket);
hipError_t launch_hist_join(hipStream_t st, const DevBufs& b, uint32_t grid, const uint16_t* pre,
                            const uint16_t* suf, uint64_t* dglob, uint32_t hist_len, uint32_t Kp);
// P_r(l) rows out[S][K][hist_len] (caller threshold order) from dglob.
hipError_t launch_hist_finish(hipStream_t st, const DevBufs& b, const uint64_t* dglob, uint64_t* out,
                              uint32_t hist_len, uint32_t Kp);
size_t hist_lds_bytes(uint32_t Kp, uint32_t block);
int hist_blocks_per_cu(int select_variant, uint32_t Kp, uint32_t block);
constexpr uint32_t HIST_MAX_K_HOST = RQA_MAX_HIST_K;
constexpr uint32_t HIST_MAX_SEG_HOST = 32768;
// Window selection.  Sources of the window: predicted offsets [S][20] with
// half-widths (network), or the sorted sketch sample (sample quantiles).
struct WinBufs {
    uint64_t* bins;      // [S][WIN_BINS] pass-1 counts
    uint8_t* table;      // [S][WIN_BINS] fine bin -> pass-2 slot
    uint64_t* fine;      // [S][K][1 << WIN_MAX_SHIFT] pass-2 counts
};
hipError_t launch_window_from_offsets(hipStream_t st, const DevBufs& b, const float* pred, const float* delta_dev);
hipError_t launch_window_fixed(hipStream_t st, const DevBufs& b, uint32_t lo, uint32_t hi);
hipError_t launch_window_from_sample(hipStream_t st, const DevBufs& b, const uint32_t* sample_sorted, const double* rr_dev,
                                     float z);
hipError_t launch_window_pass(hipStream_t st, const DevBufs& b, const WinBufs& w, int pass, int variant, uint32_t grid,
                              uint32_t block, uint32_t ticket);
hipError_t launch_window_scan(hipStream_t st, const DevBufs& b, const WinBufs& w, int pass);
size_t window_lds_bytes(int pass);
int window_blocks_per_cu(int pass, int variant, uint32_t block);

// Sketch of every series: features [S][SKETCH_FEATURES], sorted sample bits
// [S][SKETCH_P] (may be NULL), scale into SeriesWork.
hipError_t launch_sketch(hipStream_t st, const DevBufs& b, float* features, uint32_t* sample_sorted);

// Kernel variants.  Embedding class: 0 any (m, tau) at run time, 1 m = 1,
// 2 m = 3 with tau = 3, 3 m = 3 with tau = 5.  Line class: 0 any lmin,
// 1 lmin = 1, 2 lmin = 2.  select variant = norm * 4 + embedding class;
// sweep variant = select variant * 3 + line class.
constexpr int NUM_MCLASS = 4;
constexpr int NUM_SELECT_VARIANTS = 2 * NUM_MCLASS;
constexpr int NUM_SWEEP_VARIANTS = NUM_SELECT_VARIANTS * 3;
int select_variant_of(uint32_t norm, uint32_t m, uint32_t tau);
int variant_of(uint32_t norm, uint32_t m, uint32_t tau, uint32_t lmin);

// Dynamic LDS bytes of each kernel for a K and group size.  The sweep holds
// rows + 1 histogram rows per lane: rows = K for given thresholds, 2K + 1 for
// the range sweep.
size_t select_lds_bytes(int pass, uint32_t K, uint32_t group_slots);
size_t sweep_lds_bytes(uint32_t rows, bool ranges);

// Occupancy helpers (kernels.hip): max resident workgroups per CU.
int select_blocks_per_cu(int pass, int variant, uint32_t block, size_t lds);
int sweep_blocks_per_cu(int variant, bool ranges, uint32_t block, size_t lds);
hipError_t set_kernel_lds_limits(size_t max_dyn_lds);

// VALU issue-rate probe (probe.hip): kind 0 v_add_f32, 1 v_add_u32,
// 2 v_max_u32; `out` holds valu_probe_threads(blocks) words.
hipError_t launch_valu_probe(hipStream_t st, int kind, uint32_t blocks, uint32_t iters, uint32_t* out);
uint64_t valu_probe_threads(uint32_t blocks);
double valu_probe_lane_ops(uint32_t blocks, uint32_t iters);

}  // namespace rqa
