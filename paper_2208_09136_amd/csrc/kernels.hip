// kernels.hip -- gfx950 kernels of the averaged-RQA hot path.
//
// Work decomposition (every counting kernel): the pairs (i, j = i + d) of one
// series form the upper triangle of diagonals d = w .. nv-1.  A tile is one
// band of 64 consecutive diagonals times one segment of T steps along them;
// lane L of the wavefront that owns the tile walks diagonal d0 + L.  Tiles are
// enumerated segment-major (all bands of segment 0, then of segment 1, ...),
// grouped into chunks of consecutive tiles of one series, and chunks are
// handed to persistent workgroups through an atomic ticket.  The recurrence
// matrix is never stored: every key is recomputed from the series.
//
// Keys follow Eq. 1 of the paper with the maximum norm, or the squared
// Euclidean norm folded left over the embedding components; all float
// arithmetic is binary32 with round-to-nearest-even and no contraction, so the
// keys (and every count derived from them) are bit-identical to a plain CPU
// evaluation.
//
// Along a diagonal d the embedding component k of the pair (x, x + d) is the
// difference e(s) = y[s] - y[s + d] at s = x + (m-1-k) tau, so each lane keeps
// |e| or e^2 of the last (m-1) tau steps in registers and needs one new
// difference per step (the "walker").  Tiles whose every lane stays inside its
// diagonal take that path without per-lane bounds checks; border tiles and
// run-time (m, tau) take a plain per-cell path.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

#pragma clang fp contract(off)

namespace rqa {

typedef const float __attribute__((address_space(1))) gf32;  // global
typedef const float __attribute__((address_space(4))) cf32;  // constant: scalar loads for uniform indices

// A wave-uniform value held in a vector register.  gfx950 issues 32-bit add,
// sub, and, or, xor and right shifts at twice the rate of other VALU
// instructions only when no operand is a scalar register (measured: an SGPR
// source halves v_add_u32 and v_lshrrev_b32 to the rate of v_max_u32), so a
// per-series shift or offset used once per cell is copied to a VGPR once.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t s)
{
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-series scalars of the tile loops (wave-uniform).
struct SeriesScalars {
    const float* y;
    int n, nv, m, tau, w, lmin, T, q, B, Smax, ntiles;
};

__device__ __forceinline__ SeriesScalars load_scalars(const SeriesDesc& sd)
{
    SeriesScalars s;
    s.y = sd.y;
    s.n = (int)sd.n;
    s.nv = (int)sd.nv;
    s.m = (int)sd.m;
    s.tau = (int)sd.tau;
    s.w = (int)sd.w;
    s.lmin = (int)sd.lmin;
    s.T = (int)sd.T;
    s.q = (int)sd.q;
    s.B = (int)sd.B;
    s.Smax = (int)sd.Smax;
    s.ntiles = (int)sd.ntiles;
    return s;
}

__device__ __forceinline__ void tile_coords(const SeriesScalars& sd, uint32_t tile, uint32_t& band, uint32_t& seg)
{
    // Segment s holds B - s*q bands, so tiles before segment s number
    // P(s) = s*B - q*s*(s-1)/2.  Invert with the quadratic formula and fix up.
    const uint64_t B = (uint64_t)sd.B, q = (uint64_t)sd.q, Smax = (uint64_t)sd.Smax;
    auto P = [&](uint64_t s) -> uint64_t { return s * B - q * ((s * (s - 1)) / 2); };
    const double Bq = (double)B + 0.5 * (double)q;
    const double disc = Bq * Bq - 2.0 * (double)q * (double)tile;
    const double est = (Bq - sqrt(disc > 0.0 ? disc : 0.0)) / (double)q;
    uint64_t s = est > 0.0 ? (uint64_t)est : 0;
    if (s > Smax - 1) s = Smax - 1;
    while (s > 0 && P(s) > tile) --s;
    while (s + 1 < Smax && P(s + 1) <= tile) ++s;
    seg = (uint32_t)s;
    band = (uint32_t)(tile - P(s));
}

__device__ __forceinline__ uint32_t find_series(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t chunk)
{
    uint32_t lo = 0, hi = S;  // largest s with chunk_begin <= chunk
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (sds[mid].chunk_begin <= chunk) lo = mid; else hi = mid;
    }
    return lo;
}

template <int NORM>
__device__ __forceinline__ float part_of(float e)
{
    if constexpr (NORM == RQA_NORM_MAX) return fabsf(e);
    else return e * e;
}

template <int NORM>
__device__ __forceinline__ float fold(float acc, float v)
{
    if constexpr (NORM == RQA_NORM_MAX) return fmaxf(acc, v);
    else return acc + v;
}

// Distance key of vectors i and j: component k is y[i + (m-1-k) tau].
// MC > 0: m = MC and tau = TC (TC > 0) or run-time tau (TC = 0).
template <int NORM, int MC, int TC>
__device__ __forceinline__ float pair_key(const float* __restrict__ y, int i, int j, int m, int tau)
{
    const gf32* g = (const gf32*)y;
    if constexpr (MC > 0) {
        const int tt = TC > 0 ? TC : tau;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < MC; ++k) {
            const int off = (MC - 1 - k) * tt;
            const float p = part_of<NORM>(g[i + off] - g[j + off]);
            acc = (k == 0) ? p : fold<NORM>(acc, p);
        }
        return acc;
    } else {
        float acc = 0.0f;
        int off = (m - 1) * tau;
        for (int k = 0; k < m; ++k, off -= tau) {
            const float p = part_of<NORM>(g[i + off] - g[j + off]);
            acc = (k == 0) ? p : fold<NORM>(acc, p);
        }
        return acc;
    }
}

// Geometry of one tile for the calling lane.
struct TileGeo {
    int d;     // this lane's diagonal
    int d0;    // the band's first diagonal (always < nv)
    int len;   // cells on this lane's diagonal (0 past the last diagonal)
    int len0;  // cells on the band's first (longest) diagonal
    int t0;    // first step of the segment
    int t1;    // one past the last step of the segment on the band's longest diagonal
};

__device__ __forceinline__ TileGeo tile_geo(const SeriesScalars& sd, uint32_t tile, int lane)
{
    uint32_t band, seg;
    tile_coords(sd, tile, band, seg);
    TileGeo g;
    g.d0 = (int)uniform((uint32_t)sd.w + band * TILE_W);
    g.d = g.d0 + lane;
    g.len = g.d < sd.nv ? sd.nv - g.d : 0;
    g.len0 = sd.nv - g.d0;
    g.t0 = (int)uniform(seg * (uint32_t)sd.T);
    g.t1 = min(g.t0 + sd.T, g.len0);
    return g;
}

// Sequential key generator of one lane along its diagonal for compile-time
// (M, TAU).  part_of(e(s)) of W = (M-1) TAU steps ahead of the next cell is
// kept in a register ring of two halves of HU entries (HU a multiple of W, at
// least 8): each half-block writes HU new parts into one half while the last W
// parts of the other half serve as history, so the ring never moves.  Row
// samples y[s] are wave-uniform (scalar loads); column samples y[s + d] are
// one coalesced load per step at an immediate offset from the lane pointer,
// issued one half-block ahead.
template <int NORM, int M, int TAU>
struct Walker {
    static constexpr int W = (M - 1) * TAU;
    static constexpr int HU = W == 0 ? 8 : ((8 + W - 1) / W) * W;
    float ring[2 * HU];
    float cnext[HU];  // column samples of the next half-block, loaded one half ahead
    const gf32* cp;  // y + d + x (this lane's column samples)
    const cf32* rp;  // y + x (row samples, uniform)

    __device__ __forceinline__ void start(const float* y, int d, int x0)
    {
        cp = (const gf32*)y + (uint32_t)(d + x0);
        rp = (const cf32*)y + (uint32_t)x0;
#pragma unroll
        for (int i = 0; i < W; ++i) ring[2 * HU - W + i] = part_of<NORM>(rp[i] - cp[i]);
#pragma unroll
        for (int u = 0; u < HU; ++u) cnext[u] = cp[W + u];
    }
    // part at virtual position v of the half-block that writes half H: v < W is
    // history (tail of the other half), v >= W the new part of step v - W.
    template <int H>
    __device__ __forceinline__ float at(int v) const
    {
        return v >= W ? ring[H * HU + (v >= W ? v - W : 0)] : ring[(1 - H) * HU + HU - W + (v < W ? v : 0)];
    }
    // keys (binary32 bit patterns) of the next HU cells
    template <int H>
    __device__ __forceinline__ void half(uint32_t (&out)[HU])
    {
        float cv[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) cv[u] = cnext[u];
        // the next half-block's column samples, so their latency overlaps this
        // half-block's work: at most 2 HU - 1 cells past the requested range,
        // inside the walker's slack
#pragma unroll
        for (int u = 0; u < HU; ++u) cnext[u] = cp[W + HU + u];
#pragma unroll
        for (int u = 0; u < HU; ++u) ring[H * HU + u] = part_of<NORM>(rp[W + u] - cv[u]);
#pragma unroll
        for (int u = 0; u < HU; ++u) {
            float acc = at<H>(u + W);  // component 0: the newest sample
#pragma unroll
            for (int k = 1; k < M; ++k) acc = fold<NORM>(acc, at<H>(u + W - k * TAU));
            out[u] = __float_as_uint(acc);
        }
        cp += HU;
        rp += HU;
    }
};

// Margin (cells) an interior tile keeps beyond its last cell: the walker may
// compute up to HU - 1 cells past the end of the requested range.
constexpr int WALK_SLACK = 32;

// Calls fb(keys, valid) for the cells x = x0 .. x0+count-1 of the lane's
// diagonal, in order, one half-block of HU keys at a time; only the first
// `valid` keys of a call are cells of the range (valid = HU except at the
// end).  Every lane must own cells up to x0 + count - 1 + WALK_SLACK.
template <int NORM, int M, int TAU, class FB>
__device__ __forceinline__ void walk(const float* y, int d, int x0, int count, FB&& fb)
{
    using WK = Walker<NORM, M, TAU>;
    constexpr int HU = WK::HU;
    static_assert(2 * HU - 1 <= WALK_SLACK, "walker slack (the last half-block prefetches one more)");
    WK wk;
    wk.start(y, d, x0);
    int rem = count;
    while (rem >= 2 * HU) {
        uint32_t k[HU];
        wk.template half<0>(k);
        fb(k, HU);
        wk.template half<1>(k);
        fb(k, HU);
        rem -= 2 * HU;
    }
    if (rem > 0) {
        uint32_t k[HU];
        wk.template half<0>(k);
        fb(k, min(rem, HU));
        rem -= HU;
        if (rem > 0) {
            wk.template half<1>(k);
            fb(k, rem);
        }
    }
}

// Number of keys per call of a walk callback.
template <int NORM, int M, int TAU>
constexpr int walk_block() { return Walker<NORM, M, TAU>::HU; }

// End of the part of a tile the walker can take: the whole tile when every
// lane's diagonal covers [t0, t1 + WALK_SLACK] (interior tiles), else the
// longest prefix [t0, tw) whose cells and slack every lane of the band owns,
// in whole pairs of half-blocks (so that state a body carries from block to
// block is exact at tw); the cells after tw take the per-cell path.  A band
// with fewer than 64 diagonals has no walker part.
template <int HU>
__device__ __forceinline__ int walk_end(const TileGeo& g)
{
    if (g.t1 + TILE_W + WALK_SLACK <= g.len0) return g.t1;
    const int safe = g.len0 - TILE_W - WALK_SLACK;
    if (safe <= g.t0) return g.t0;
    return g.t0 + ((safe - g.t0) / (2 * HU)) * (2 * HU);
}

// ------------------------------------------------------------------ zero / checks

__global__ void k_zero(uint32_t* p, size_t words)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

hipError_t launch_zero(hipStream_t st, void* p, size_t bytes)
{
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    uint32_t grid = (uint32_t)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, st, (uint32_t*)p, words);
    return hipGetLastError();
}

// Per series: flags a NaN or infinite sample, and (block x = 0) places the
// call's targets into the zeroed working state: tgt[s * K + r] is target r's
// rank (selection) or threshold bit pattern (given thresholds).
__global__ void k_check_finite(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                               const uint64_t* __restrict__ tgt, uint32_t K, uint32_t as_rank)
{
    const SeriesDesc& sd = sds[blockIdx.y];
    SeriesWork& w = works[blockIdx.y];
    if (blockIdx.x == 0 && tgt) {
        for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) {
            const uint64_t v = tgt[(size_t)blockIdx.y * K + r];
            if (as_rank) w.k[r] = v;
            else w.eps_bits[r] = (uint32_t)v;
        }
    }
    bool bad = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sd.n; i += gridDim.x * blockDim.x) {
        const uint32_t u = __float_as_uint(sd.y[i]);
        bad |= (u & 0x7F800000u) == 0x7F800000u;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&w.nonfinite, 1u);
}

hipError_t launch_check_finite(hipStream_t st, const DevBufs& b, uint32_t maxn, const uint64_t* tgt, bool as_rank)
{
    uint32_t gx = std::min<uint32_t>((maxn + 255) / 256, 1024);
    hipLaunchKernelGGL(k_check_finite, dim3(gx, b.S), dim3(256), 0, st, b.sd, b.work, tgt, b.K, as_rank ? 1u : 0u);
    return hipGetLastError();
}

// The results the host reads, packed per series into result_words(K, lines)
// 64-bit words: [0] status | nonfinite << 32, [1] scale | range_ok << 32,
// [2] Kp, then K words each of eps_bits, k, count, dcount, win_hit | dmap
// << 32, and with lines (threshold sweep) Kp words each of hrho and hlam.
__global__ void k_pack_results(const SeriesWork* __restrict__ works, uint32_t K, uint32_t lines, uint64_t* __restrict__ out)
{
    const SeriesWork& w = works[blockIdx.x];
    uint64_t* o = out + (size_t)blockIdx.x * result_words(K, lines != 0);
    if (threadIdx.x == 0) {
        o[0] = (uint64_t)w.status | ((uint64_t)w.nonfinite << 32);
        o[1] = (uint64_t)w.scale | ((uint64_t)w.range_ok << 32);
        o[2] = w.Kp;
    }
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) {
        o[3 + r] = w.eps_bits[r];
        o[3 + K + r] = w.k[r];
        o[3 + 2 * K + r] = w.count[r];
        o[3 + 3 * K + r] = w.dcount[r];
        o[3 + 4 * K + r] = (uint64_t)w.win_hit[r] | ((uint64_t)w.dmap[r] << 32);
        if (lines) {
            o[3 + 5 * K + r] = w.hrho[r];
            o[3 + 6 * K + r] = w.hlam[r];
        }
    }
}

hipError_t launch_pack_results(hipStream_t st, const DevBufs& b, bool lines, uint64_t* out)
{
    hipLaunchKernelGGL(k_pack_results, dim3(b.S), dim3(64), 0, st, b.work, b.K, lines ? 1u : 0u, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ work loop

// Persistent work loop shared by the counting kernels (s_chunk_slot: one LDS
// word shared by the workgroup): grab chunks from the ticket, switch per-series LDS state when the series changes, process the
// chunk's tiles one per wavefront, flush accumulated counts when the series
// changes, when 32-bit LDS counters could overflow, and at the end.
template <class Body>
__device__ __forceinline__ void chunk_loop(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t nchunks,
                                           uint32_t chunk_tiles, uint32_t* __restrict__ ticket, Body& body,
                                           uint32_t* s_chunk_slot)
{
    uint32_t& s_chunk = *s_chunk_slot;
    uint32_t cur = 0xFFFFFFFFu;
    uint64_t acc = 0;
    const int wave = threadIdx.x / TILE_W;
    const int nwaves = blockDim.x / TILE_W;
    const int lane = threadIdx.x % TILE_W;
    SeriesScalars ss{};
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_chunk = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t c = uniform(s_chunk);
        if (c >= nchunks) {
            // queue drained (possibly before this workgroup drew its first chunk)
            if (cur != 0xFFFFFFFFu) body.flush(cur);
            break;
        }
        const uint32_t s = uniform(find_series(sds, S, c));
        const SeriesDesc& sd = sds[s];
        const uint64_t chunk_cells = (uint64_t)chunk_tiles * TILE_W * sd.T;
        if (s != cur || acc + chunk_cells > 0xFFFFFFFFull) {
            if (cur != 0xFFFFFFFFu) body.flush(cur);
            __syncthreads();
            body.begin(s);
            __syncthreads();
            cur = s;
            acc = 0;
            ss = load_scalars(sd);
        }
        if (body.active) {
            const uint32_t lc = c - sd.chunk_begin;
            const uint32_t tb = lc * chunk_tiles;
            const uint32_t te = min(tb + chunk_tiles, (uint32_t)ss.ntiles);
            for (uint32_t tile = tb + wave; tile < te; tile += nwaves) body.tile(ss, uniform(tile), lane);
        }
        acc += chunk_cells;
    }
}

// Adds 1 to slot base[idx] for every active lane, one atomic per distinct idx
// among the active lanes.
__device__ __forceinline__ void wave_add(unsigned long long* base, uint32_t idx, bool active)
{
    uint64_t mask = __ballot(active);
    while (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        const uint32_t li = __builtin_amdgcn_readlane(idx, leader);
        const uint64_t same = __ballot(active && idx == li);
        if ((int)__lane_id() == leader) atomicAdd(base + li, (unsigned long long)__popcll(same));
        active = active && idx != li;
        mask &= ~same;
    }
}

// wave_add kept out of line: the range sweep calls it rarely from deeply
// unrolled loops, whose registers would otherwise spill
__device__ __attribute__((noinline)) void fine_add(unsigned long long* base, uint32_t idx, bool active)
{
    wave_add(base, idx, active);
}

// ------------------------------------------------------------------ selection

// Shared tile driver of the counting passes.  For every cell of the lane's
// diagonal in the tile: look = body.look(key) (LDS table reads, issued for a
// whole block of keys first), then body.count(key, look).
template <int NORM, int MC, int TC, class Body>
__device__ __forceinline__ void select_tile(const SeriesScalars& sd, uint32_t tile_id, int lane, Body& body)
{
    const TileGeo g = tile_geo(sd, tile_id, lane);
    constexpr bool kFast = MC > 0 && (MC == 1 || TC > 0);
    int tx = g.t0;  // cells before tx are counted by the walker
    if constexpr (kFast) {
        constexpr int TW = MC == 1 ? 1 : TC;
        constexpr int HU = walk_block<NORM, MC, TW>();
        const int tw = walk_end<HU>(g);
        if (tw > g.t0) {
            // every lane's diagonal covers [t0, tw + WALK_SLACK]
            walk<NORM, MC, TW>(sd.y, g.d, g.t0, tw - g.t0, [&](const uint32_t(&k)[HU], int valid) {
                uint32_t lk[HU];
#pragma unroll
                for (int u = 0; u < HU; ++u) lk[u] = body.look(k[u]);
#pragma unroll
                for (int u = 0; u < HU; ++u)
                    if (u < valid) body.count(k[u], lk[u]);
            });
            tx = tw;
        }
    }
    for (int x = tx; x < g.t1; ++x) {
        if (x < g.len) {
            const uint32_t u = __float_as_uint(pair_key<NORM, MC, TC>(sd.y, x, x + g.d, sd.m, sd.tau));
            body.count(u, body.look(u));
        }
    }
}

#ifndef RQA_P1_COPIES
#define RQA_P1_COPIES 4
#endif
// Interleaved copies of the pass-1 histogram: lane L counts into copy L mod
// P1_COPIES, so lanes of one wave that hit the same bucket hit different words.
constexpr uint32_t P1_COPIES = RQA_P1_COPIES;

// Sets of the pass-3 prefix table (two entries each).
constexpr uint32_t P3_SETS = 4096;

// Bytes of a selection pass's LDS tables and bins; the work-queue word follows.
__host__ __device__ __forceinline__ size_t select_lds_bytes_dev(int pass, uint32_t K, uint32_t G)
{
    if (pass == 1) return SEL_N1 * 4 * P1_COPIES;
    if (pass == 2) return SEL_N1 * 2 + (size_t)G * SEL_N2 * 4 + TILE_W * 4;
    return P3_SETS * 8 + RQA_MAX_K * 2 + 16;
}

// Pass 1: histogram of the top SEL_B1 bits of every key.
template <int NORM, int MC, int TC>
struct SelPass1 {
    uint32_t* bins;   // LDS [SEL_N1][P1_COPIES]
    uint64_t* h1;     // global [S][SEL_N1]
    bool active = true;
    uint32_t copy = 0;
    __device__ void begin(uint32_t)
    {
        for (uint32_t i = threadIdx.x; i < SEL_N1 * P1_COPIES; i += blockDim.x) bins[i] = 0u;
    }
    __device__ void flush(uint32_t s)
    {
        for (uint32_t i = threadIdx.x; i < SEL_N1; i += blockDim.x) {
            uint32_t v = 0;
            for (uint32_t c = 0; c < P1_COPIES; ++c) v += bins[i * P1_COPIES + c];
            if (v) atomicAdd((unsigned long long*)&h1[(size_t)s * SEL_N1 + i], (unsigned long long)v);
        }
    }
    __device__ __forceinline__ uint32_t look(uint32_t) const { return 0u; }
    __device__ __forceinline__ void count(uint32_t u, uint32_t) const
    {
        if constexpr (P1_COPIES == 1) atomicAdd(&bins[__builtin_amdgcn_ubfe(u, SEL_SH1, SEL_B1)], 1u);
        else atomicAdd(&bins[__builtin_amdgcn_ubfe(u, SEL_SH1, SEL_B1) * P1_COPIES + copy], 1u);
    }
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        copy = (uint32_t)lane & (P1_COPIES - 1);
        select_tile<NORM, MC, TC>(sd, tile_id, lane, *this);
    }
};

// Pass 2: for keys whose pass-1 bucket holds a target (slot in [lo, hi)),
// histogram the next SEL_B2 bits per slot.
constexpr uint16_t NO_BIN = 0xFFFF;
template <int NORM, int MC, int TC>
struct SelPass2 {
    uint16_t* sOff;   // LDS [SEL_N1]: first bin of the bucket's slot in this group, or NO_BIN
    uint32_t* bins;   // LDS [G][SEL_N2] + one spare word per lane
    const uint8_t* T1;
    const SeriesWork* works;
    uint64_t* h2;     // global [S][K][SEL_N2]
    uint32_t K, G, lo, hi;
    bool active = true;
    __device__ void begin(uint32_t s)
    {
        const uint32_t ns = works[s].nslots2;
        hi = min(lo + G, ns);
        active = lo < ns;
        for (uint32_t i = threadIdx.x; i < SEL_N1; i += blockDim.x) {
            const uint32_t t = T1[(size_t)s * SEL_N1 + i];
            sOff[i] = (t >= lo && t < hi) ? (uint16_t)((t - lo) * SEL_N2) : NO_BIN;
        }
        for (uint32_t i = threadIdx.x; i < G * SEL_N2; i += blockDim.x) bins[i] = 0u;
    }
    __device__ void flush(uint32_t s)
    {
        if (!active) return;
        const uint32_t n = (hi - lo) * SEL_N2;
        uint64_t* dst = h2 + ((size_t)s * K + lo) * SEL_N2;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t v = bins[i];
            if (v) atomicAdd((unsigned long long*)&dst[i], (unsigned long long)v);
        }
    }
    // first bin of the key's pass-1 bucket's slot (NO_BIN: not a target bucket of this group)
    __device__ __forceinline__ uint32_t look(uint32_t u) const
    {
        return sOff[__builtin_amdgcn_ubfe(u, SEL_SH1, SEL_B1)];
    }
    // keys outside this group's target buckets count into a spare word per
    // lane, so the count needs no branch (and no divergence)
    uint32_t dummy = 0;
    __device__ __forceinline__ void count(uint32_t u, uint32_t off) const
    {
        atomicAdd(&bins[off != NO_BIN ? off + __builtin_amdgcn_ubfe(u, SEL_SH2, SEL_B2) : dummy], 1u);
    }
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        dummy = G * SEL_N2 + (uint32_t)lane;
        select_tile<NORM, MC, TC>(sd, tile_id, lane, *this);
    }
};

// Pass 3 (selection only): for keys whose 21-bit prefix holds a target,
// count the last SEL_B3 bits per pass-3 slot directly in global memory (few
// keys qualify).  The target prefixes sit in an LDS table of P3_SETS sets of
// two entries (prefix << 7 | pass-3 slot), indexed by the prefix's low bits,
// so a key takes one 8-byte table read.  A series with three target prefixes
// in one set (rare) looks its keys up in the pass-1 and pass-2 slot tables in
// global memory instead, two dependent reads.
constexpr uint32_t P3_EMPTY = 0xFFFFFFFFu;  // prefix field above every 21-bit prefix
constexpr uint32_t P3_NONE = 0xFFFFFFFFu;   // key outside every target prefix
static_assert(RQA_MAX_K <= 128, "pass-3 slots take 7 bits of a prefix-table entry");

template <int NORM, int MC, int TC>
struct SelPass3 {
    uint2* sH;        // LDS [P3_SETS]: two entries prefix << 7 | pass-3 slot
    uint16_t* sB;     // LDS [RQA_MAX_K]: pass-1 bucket of each pass-2 slot
    uint32_t* sOver;  // LDS word: some set overflowed
    const uint8_t* T1;
    const uint8_t* T2;
    const SeriesWork* works;
    uint64_t* h3;     // global [S][K][SEL_N3]
    uint32_t K;
    unsigned long long* dst;
    const uint8_t* gT1;  // this series' slot tables (overflow lookups)
    const uint8_t* gT2;
    bool over = false;
    bool active = true;
    __device__ void begin(uint32_t s)
    {
        const uint32_t n2 = works[s].nslots2;
        gT1 = T1 + (size_t)s * SEL_N1;
        gT2 = T2 + (size_t)s * K * SEL_N2;
        for (uint32_t i = threadIdx.x; i < P3_SETS; i += blockDim.x) sH[i] = make_uint2(P3_EMPTY, P3_EMPTY);
        for (uint32_t i = threadIdx.x; i < SEL_N1; i += blockDim.x) {
            const uint32_t t = gT1[i];
            if (t != NO_SLOT) sB[t] = (uint16_t)i;
        }
        if (threadIdx.x == 0) *sOver = 0u;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n2 * SEL_N2; i += blockDim.x) {
            const uint32_t s3 = gT2[i];
            if (s3 == NO_SLOT) continue;
            const uint32_t pfx = ((uint32_t)sB[i / SEL_N2] << SEL_B2) | (i % SEL_N2);
            const uint32_t ent = (pfx << 7) | s3;
            uint2& e = sH[pfx & (P3_SETS - 1)];
            if (atomicCAS(&e.x, P3_EMPTY, ent) != P3_EMPTY && atomicCAS(&e.y, P3_EMPTY, ent) != P3_EMPTY)
                *sOver = 1u;
        }
        __syncthreads();
        over = uniform(*sOver) != 0u;
        dst = (unsigned long long*)(h3 + (size_t)s * K * SEL_N3);
    }
    __device__ void flush(uint32_t) {}
    // counter index of the key (P3_NONE: outside every target prefix): one
    // table read at a byte offset made by a right shift and a mask
    struct Table {
        const SelPass3& b;
        __device__ __forceinline__ uint32_t look(uint32_t u) const
        {
            const uint32_t off = (u >> (SEL_SH2 - 3)) & ((P3_SETS - 1u) << 3);
            const uint2 e = *(const uint2*)((const unsigned char*)b.sH + off);
            const uint32_t pfx = u >> SEL_SH2, lo = u & (SEL_N3 - 1);
            const bool hx = (e.x >> 7) == pfx, hy = (e.y >> 7) == pfx;
            const uint32_t ent = hx ? e.x : e.y;
            return (hx || hy) ? ((ent & 127u) << SEL_B3) | lo : P3_NONE;
        }
        __device__ __forceinline__ void count(uint32_t, uint32_t idx) const { wave_add(b.dst, idx, idx != P3_NONE); }
    };
    struct Slots {
        const SelPass3& b;
        __device__ __forceinline__ uint32_t look(uint32_t u) const
        {
            const uint32_t s2 = b.gT1[__builtin_amdgcn_ubfe(u, SEL_SH1, SEL_B1)];
            if (s2 == NO_SLOT) return P3_NONE;
            const uint32_t s3 = b.gT2[s2 * SEL_N2 + __builtin_amdgcn_ubfe(u, SEL_SH2, SEL_B2)];
            return s3 != NO_SLOT ? s3 * SEL_N3 + (u & (SEL_N3 - 1)) : P3_NONE;
        }
        __device__ __forceinline__ void count(uint32_t, uint32_t idx) const { wave_add(b.dst, idx, idx != P3_NONE); }
    };
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        if (over) {
            Slots v{*this};
            select_tile<NORM, MC, TC>(sd, tile_id, lane, v);
        } else {
            Table v{*this};
            select_tile<NORM, MC, TC>(sd, tile_id, lane, v);
        }
    }
};

template <int PASS, int NORM, int MC, int TC>
__global__ void __launch_bounds__(1024)
k_select(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t nchunks, uint32_t chunk_tiles,
         uint32_t* __restrict__ tickets, SeriesWork* __restrict__ works, const uint8_t* __restrict__ T1,
         const uint8_t* __restrict__ T2, uint64_t* __restrict__ hist, uint32_t K, uint32_t G)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* ticket = tickets + blockIdx.y;
    uint32_t* slot = (uint32_t*)(smem + select_lds_bytes_dev(PASS, K, G));
    if constexpr (PASS == 1) {
        SelPass1<NORM, MC, TC> body{(uint32_t*)smem, hist};
        chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, slot);
    } else if constexpr (PASS == 2) {
        SelPass2<NORM, MC, TC> body;
        body.sOff = (uint16_t*)smem;
        body.bins = (uint32_t*)(smem + SEL_N1 * 2);
        body.T1 = T1;
        body.works = works;
        body.h2 = hist;
        body.K = K;
        body.G = G;
        body.lo = blockIdx.y * G;
        body.hi = body.lo;
        chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, slot);
    } else {
        SelPass3<NORM, MC, TC> body;
        body.sH = (uint2*)smem;
        body.sB = (uint16_t*)(smem + P3_SETS * 8);
        body.sOver = (uint32_t*)(smem + P3_SETS * 8 + RQA_MAX_K * 2);
        body.T1 = T1;
        body.T2 = T2;
        body.works = works;
        body.h3 = hist;
        body.K = K;
        body.dst = nullptr;
        chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, slot);
    }
}

size_t select_lds_bytes(int pass, uint32_t K, uint32_t G) { return select_lds_bytes_dev(pass, K, G) + 16; }

static int mclass_of(uint32_t m, uint32_t tau)
{
    if (m == 1) return 1;
    if (m == 3 && tau == 3) return 2;
    if (m == 3 && tau == 5) return 3;
    return 0;
}

int select_variant_of(uint32_t norm, uint32_t m, uint32_t tau) { return (int)norm * NUM_MCLASS + mclass_of(m, tau); }

int variant_of(uint32_t norm, uint32_t m, uint32_t tau, uint32_t lmin)
{
    const int lc = (lmin == 1) ? 1 : (lmin == 2) ? 2 : 0;
    return select_variant_of(norm, m, tau) * 3 + lc;
}

using SelFn = void (*)(const SeriesDesc*, uint32_t, uint32_t, uint32_t, uint32_t*, SeriesWork*, const uint8_t*,
                       const uint8_t*, uint64_t*, uint32_t, uint32_t);

template <int PASS, int NORM>
static SelFn select_fn_n(int mclass)
{
    switch (mclass) {
    case 1: return k_select<PASS, NORM, 1, 0>;
    case 2: return k_select<PASS, NORM, 3, 3>;
    case 3: return k_select<PASS, NORM, 3, 5>;
    default: return k_select<PASS, NORM, 0, 0>;
    }
}

template <int PASS>
static SelFn select_fn(int variant)
{
    const int norm = variant / NUM_MCLASS, mc = variant % NUM_MCLASS;
    return norm == RQA_NORM_MAX ? select_fn_n<PASS, RQA_NORM_MAX>(mc) : select_fn_n<PASS, RQA_NORM_EUCLIDEAN>(mc);
}

static SelFn select_fn_pass(int pass, int variant)
{
    if (pass == 1) return select_fn<1>(variant);
    if (pass == 2) return select_fn<2>(variant);
    return select_fn<3>(variant);
}

hipError_t launch_select_pass(hipStream_t st, const DevBufs& b, int pass, int variant, uint32_t grid,
                              uint32_t block, uint32_t groups, uint32_t G, uint32_t ticket_base)
{
    const size_t lds = select_lds_bytes(pass, b.K, G);
    uint64_t* hist = pass == 1 ? b.h1 : pass == 2 ? b.h2 : b.h3;
    hipLaunchKernelGGL(select_fn_pass(pass, variant), dim3(grid, groups), dim3(block), lds, st, b.sd, b.S,
                       b.nchunks, b.chunk_tiles, b.tickets + ticket_base, b.work, b.T1, b.T2, hist, b.K, G);
    return hipGetLastError();
}

// Workgroups of `block` threads with `lds` bytes of dynamic LDS that one CU
// runs at once: the runtime's occupancy query, capped by the LDS allocation
// unit it does not apply.
int blocks_per_cu(const void* f, uint32_t block, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, (int)block, lds) != hipSuccess || n < 1) return 1;
    const int fit = (int)lds_blocks_fit(lds);
    return n < fit ? n : (fit > 0 ? fit : 1);
}

int select_blocks_per_cu(int pass, int variant, uint32_t block, size_t lds)
{
    return blocks_per_cu((const void*)select_fn_pass(pass, variant), block, lds);
}

// ------------------------------------------------------------------ scans

// Exclusive prefix over the workgroup of one u64 per thread (blockDim.x a
// multiple of 64, at most 1024): shuffles inside each wave, then the wave
// totals.  *total receives the sum over the workgroup.  Called by every
// thread.
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* total)
{
    __shared__ uint64_t wsum[16];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (lane >= (uint32_t)off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
    for (uint32_t i = 0; i < nw; ++i) {
        const uint64_t t = wsum[i];
        base += i < wid ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// Sum over the workgroup of one u64 per thread (every thread gets it).
__device__ __forceinline__ uint64_t block_sum(uint64_t v)
{
    uint64_t tot;
    (void)block_excl_scan(v, &tot);
    return tot;
}

// Inclusive prefix sums of n (multiple of blockDim.x) u64 values into LDS.
__device__ void block_cumsum(const uint64_t* __restrict__ src, uint64_t* cum, uint32_t n)
{
    const uint32_t per = n / blockDim.x;
    const uint32_t base = threadIdx.x * per;
    uint64_t s = 0;
    for (uint32_t i = 0; i < per; ++i) {
        s += src[base + i];
        cum[base + i] = s;
    }
    uint64_t tot;
    const uint64_t off = block_excl_scan(s, &tot);
    for (uint32_t i = 0; i < per; ++i) cum[base + i] += off;
    __syncthreads();
}

// A u64 moved between lanes by a DPP control (row_mask and bank_mask all
// rows and banks).
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Sum of a u64 over each aligned group of eight lanes, every lane of the
// group getting it: lane ^ 1 and lane ^ 2 (quad permutations), then the
// other half of the eight (row half mirror: lane i takes lane 7 - i).  DPP
// moves read the neighbouring lanes' registers directly, with no LDS round
// trip.  Called with the whole wave active.
__device__ __forceinline__ uint64_t sum8_lanes(uint64_t x)
{
    x += dpp_u64<0xB1>(x);
    x += dpp_u64<0x4E>(x);
    x += dpp_u64<0x141>(x);
    return x;
}

// Prefix sums of n u64 counts in blockDim.x contiguous chunks of
// ceil(n / blockDim.x): pre[t] = sum of the chunks before chunk t,
// pre[blockDim.x] = the total.  Short chunks are summed by their thread
// (its up to 16 loads issued before any is summed);
// long ones (more than 16 counts) by eight lanes of the thread's wave, wave
// w taking chunks 64 w .. 64 w + 63 eight at a time (each load then reads
// eight runs of eight consecutive counts), so that no lane walks a long
// chunk alone and the eight partial sums meet through DPP moves.  Then
// first_in_chunks finds, for one count kk <= total, the first index whose
// inclusive prefix reaches kk.
__device__ void chunk_prefix(const uint64_t* __restrict__ c, uint32_t n, uint64_t* pre /* LDS [blockDim.x + 1] */)
{
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t lane = threadIdx.x & 63, wbase = threadIdx.x & ~63u;
    uint64_t mine = 0;
    if (per <= 16) {
        const uint32_t b0 = min(threadIdx.x * per, n), b1 = min(b0 + per, n);
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) mine += b0 + k < b1 ? c[b0 + k] : 0ull;
    } else {
        // lanes 8 g .. 8 g + 7 sum chunk wbase + 8 i + g in part[i]
        const uint32_t g = lane >> 3, j = lane & 7;
        const uint32_t nk = (per + 7) / 8;
        uint64_t part[8];
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) part[i] = 0;
        for (uint32_t k = 0; k < nk; ++k) {
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) {
                const uint32_t b0 = min((wbase + 8 * i + g) * per, n), b1 = min(b0 + per, n);
                const uint32_t e = b0 + 8 * k + j;
                part[i] += e < b1 ? c[e] : 0ull;
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
            const uint64_t v = sum8_lanes(part[i]);
            if (j == 0) pre[wbase + 8 * i + g] = v;
        }
        // per is the same on every thread, so is this branch
        __syncthreads();
        mine = pre[threadIdx.x];
    }
    uint64_t tot;
    pre[threadIdx.x] = block_excl_scan(mine, &tot);
    if (threadIdx.x == 0) pre[blockDim.x] = tot;
    __syncthreads();
}

// Called by all 64 lanes of one wave with the same arguments (every lane
// gets the result): the first index i with pre-sum + c[..i] >= kk, found by
// a binary search over the chunk prefixes and a wave scan of 64 counts at a
// time through the chunk; the chunk's last index if none reaches kk.
// *before = the sum of the counts below the index.
__device__ uint32_t first_in_chunks(const uint64_t* __restrict__ c, uint32_t n, const uint64_t* pre, uint64_t kk,
                                    uint64_t* before)
{
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    uint32_t lo = 0, hi = blockDim.x;  // pre[lo] < kk <= pre[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] < kk) lo = mid; else hi = mid;
    }
    uint64_t run = pre[lo];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t b0 = lo * per, b1 = min(b0 + per, n);
    for (uint32_t base = b0; base < b1; base += 64) {
        const uint32_t i = base + lane;
        const uint64_t v = i < b1 ? c[i] : 0;
        uint64_t x = v;  // inclusive prefix over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t y = __shfl_up(x, off);
            if (lane >= (uint32_t)off) x += y;
        }
        const unsigned long long hit = __ballot(i < b1 && (run + x >= kk || i + 1 == b1));
        if (hit) {
            const int l = __ffsll(hit) - 1;
            *before = run + __shfl(x, l) - __shfl(v, l);
            return base + (uint32_t)l;
        }
        run += __shfl(x, 63);
    }
    *before = run;
    return b0;
}

// First index i in [0, n) with cum[i] >= k (cum inclusive, nondecreasing);
// n-1 if none.
__device__ __forceinline__ uint32_t first_reaching(const uint64_t* cum, uint32_t n, uint64_t k)
{
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cum[mid] >= k) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// The distinct values of v[0..n) in ascending order, written to out[] (which
// must not overlap v), over the entries with keep[i] != 0 (all entries when
// keep is null); pos[i] = the position of v[i] among them, for kept entries.
// flag is LDS scratch of n words.  One entry per thread, in parallel (a
// serial sort on one thread waits on an LDS round trip per step), so n is at
// most RQA_MAX_K and every caller runs at least that many threads.  Called by
// the whole block; synchronises it.  Returns the number of distinct values.
static_assert(RQA_MAX_K <= 256, "the set-up kernels give every target a thread of 256");
__device__ uint32_t block_sort_unique(const uint32_t* v, const uint32_t* keep, uint32_t n, uint32_t* out,
                                      uint32_t* pos, uint32_t* flag)
{
    const uint32_t i = threadIdx.x;
    const bool mine = i < n && (keep == nullptr || keep[i] != 0u);
    const uint32_t x = mine ? v[i] : 0u;
    // the first kept entry of each value stands for it
    bool first = mine;
    if (mine)
        for (uint32_t j = 0; j < i; ++j)
            if ((keep == nullptr || keep[j] != 0u) && v[j] == x) first = false;
    if (i < n) flag[i] = first ? 1u : 0u;
    const uint32_t nu = (uint32_t)__syncthreads_count(first);
    if (mine) {
        uint32_t p = 0;
        for (uint32_t j = 0; j < n; ++j) p += (flag[j] != 0u && v[j] < x) ? 1u : 0u;
        pos[i] = p;
        if (first) out[p] = x;
    }
    __syncthreads();
    return nu;
}

// After pass 1: locate each target's bucket, assign pass-2 slots, fill T1.
__global__ void __launch_bounds__(256) k_scan1(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                                               uint8_t* __restrict__ T1, const uint64_t* __restrict__ h1)
{
    __shared__ uint64_t cum[SEL_N1];
    __shared__ uint32_t s_pre[RQA_MAX_K], uniq[RQA_MAX_K], s_pos[RQA_MAX_K], s_flag[RQA_MAX_K];
    const uint32_t s = blockIdx.x;
    const uint32_t K = sds[s].K;
    SeriesWork& w = works[s];
    block_cumsum(h1 + (size_t)s * SEL_N1, cum, SEL_N1);
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) {
        const uint64_t k = w.k[r];
        const uint32_t b = first_reaching(cum, SEL_N1, k);
        if (cum[b] < k) atomicOr(&w.status, 1u);
        w.prefix[r] = b;
        w.below[r] = b ? cum[b - 1] : 0;
        s_pre[r] = b;
    }
    uint8_t* t1 = T1 + (size_t)s * SEL_N1;
    for (uint32_t i = threadIdx.x; i < SEL_N1; i += blockDim.x) t1[i] = NO_SLOT;
    __syncthreads();
    const uint32_t nu = block_sort_unique(s_pre, nullptr, K, uniq, s_pos, s_flag);
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) w.slot[r] = s_pos[r];
    for (uint32_t u = threadIdx.x; u < nu; u += blockDim.x) t1[uniq[u]] = (uint8_t)u;
    if (threadIdx.x == 0) w.nslots2 = nu;
}

// After pass 2: resolve SEL_B2 more bits per target, assign pass-3 slots,
// fill T2 (per pass-2 slot and sub-bucket).
__global__ void __launch_bounds__(256) k_scan2(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                                               uint8_t* __restrict__ T2, const uint64_t* __restrict__ h2all)
{
    __shared__ uint32_t s_pre[RQA_MAX_K], uniq[RQA_MAX_K], s_pos[RQA_MAX_K], s_flag[RQA_MAX_K];
    const uint32_t s = blockIdx.x;
    const uint32_t K = sds[s].K;
    SeriesWork& w = works[s];
    uint8_t* t2 = T2 + (size_t)s * K * SEL_N2;
    const uint32_t n2 = w.nslots2;
    const uint64_t* h2 = h2all + (size_t)s * K * SEL_N2;
    (void)h2;
    for (uint32_t i = threadIdx.x; i < n2 * SEL_N2; i += blockDim.x) t2[i] = NO_SLOT;
    // below / prefix of every target come from k_scan2_find
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) s_pre[r] = w.prefix[r];
    __syncthreads();
    const uint32_t nu = block_sort_unique(s_pre, nullptr, K, uniq, s_pos, s_flag);
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x)
        t2[w.slot[r] * SEL_N2 + (s_pre[r] & (SEL_N2 - 1))] = (uint8_t)s_pos[r];
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) w.slot[r] = s_pos[r];
    if (threadIdx.x == 0) w.nslots3 = nu;
}

// First bin of a target's histogram row whose prefix reaches want: one
// workgroup (series, target); *c and *run (the sum below the bin) land in
// LDS for thread 0.  A row that does not reach want (inconsistent counts)
// gives its last bin, the row's total and status |= flag.
__device__ void target_bin(const uint64_t* __restrict__ h, uint32_t n, uint64_t want, SeriesWork& w, uint32_t flag,
                           uint64_t* pre, uint32_t* c, uint64_t* run)
{
    chunk_prefix(h, n, pre);
    if (threadIdx.x < 64) {  // wave 0
        if (pre[blockDim.x] >= want) {
            uint64_t r;
            const uint32_t i = first_in_chunks(h, n, pre, want, &r);
            if (threadIdx.x == 0) {
                *c = i;
                *run = r;
            }
        } else if (threadIdx.x == 0) {
            *c = n - 1;
            *run = pre[blockDim.x];
            atomicOr(&w.status, flag);
        }
    }
}

// Pass-2 bins of every target (workgroup per series and target), before k_scan2.
__global__ void __launch_bounds__(256) k_scan2_find(const SeriesDesc* __restrict__ sds,
                                                    SeriesWork* __restrict__ works, const uint64_t* __restrict__ h2all)
{
    __shared__ uint64_t pre[257];
    __shared__ uint32_t s_c;
    __shared__ uint64_t s_run;
    const uint32_t s = blockIdx.x, r = blockIdx.y;
    const uint32_t K = sds[s].K;
    if (r >= K) return;
    SeriesWork& w = works[s];
    const uint64_t* h = h2all + (size_t)s * K * SEL_N2 + (size_t)w.slot[r] * SEL_N2;
    target_bin(h, SEL_N2, w.k[r] - w.below[r], w, 2u, pre, &s_c, &s_run);
    if (threadIdx.x == 0) {
        w.below[r] += s_run;
        w.prefix[r] = (w.prefix[r] << SEL_B2) | s_c;
    }
}

// After pass 3: the last SEL_B3 bits give the threshold; count = #{key <= eps}.
// Workgroup per series and target.
__global__ void __launch_bounds__(256) k_scan3(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                                               const uint64_t* __restrict__ h3)
{
    __shared__ uint64_t pre[257];
    __shared__ uint32_t s_c;
    __shared__ uint64_t s_run;
    const uint32_t s = blockIdx.x, r = blockIdx.y;
    const uint32_t K = sds[s].K;
    if (r >= K) return;
    SeriesWork& w = works[s];
    const uint64_t* h = h3 + ((size_t)s * K + w.slot[r]) * SEL_N3;
    target_bin(h, SEL_N3, w.k[r] - w.below[r], w, 4u, pre, &s_c, &s_run);
    if (threadIdx.x == 0) {
        w.eps_bits[r] = (w.prefix[r] << SEL_B3) | s_c;
        w.count[r] = w.below[r] + s_run + h[s_c];
    }
}

hipError_t launch_select_scan(hipStream_t st, const DevBufs& b, int pass)
{
    if (pass == 1) hipLaunchKernelGGL(k_scan1, dim3(b.S), dim3(256), 0, st, b.sd, b.work, b.T1, b.h1);
    else if (pass == 2) {
        hipLaunchKernelGGL(k_scan2_find, dim3(b.S, b.K), dim3(256), 0, st, b.sd, b.work, b.h2);
        hipLaunchKernelGGL(k_scan2, dim3(b.S), dim3(256), 0, st, b.sd, b.work, b.T2, b.h2);
    } else hipLaunchKernelGGL(k_scan3, dim3(b.S, b.K), dim3(256), 0, st, b.sd, b.work, b.h3);
    return hipGetLastError();
}

// ------------------------------------------------------------------ sweep

// Rank of a key among the sorted thresholds e_0 < ... < e_{Kp-1}, plus a
// per-series base z: rho = z + #{e < key}.  Given thresholds: z = 0 and the
// pair recurs at threshold j iff rho <= j.  Range sweep: the thresholds are
// the group boundaries (first value - 1, last value) and z = 1 when the first
// group starts at key 0, so rho is odd exactly for keys inside a group,
// group (rho - 1) / 2.  The bucket of the key (clamped to [e_0, e_{Kp-1}])
// gives the rank below the bucket and the bucket's first threshold; buckets
// holding several thresholds compare each of them.
struct RhoCtx {
    const uint2* table;     // LDS [RHO_TABLE]: x = first threshold in bucket (or ~0), y = rank base
    const uint32_t* es;     // LDS [Kp] thresholds
    float emin, emax;       // smallest and largest threshold
    uint32_t shift, Kp, z;
};

// MULTI: some bucket holds more than one threshold (rare; flagged per series).
template <bool MULTI>
__device__ __forceinline__ uint32_t rho_of(uint32_t u, const RhoCtx& c)
{
    // keys and thresholds are non-negative floats: they order like their bits
    const uint32_t cl = __float_as_uint(__builtin_amdgcn_fmed3f(__uint_as_float(u), c.emin, c.emax));
    const uint2 e = c.table[__builtin_amdgcn_ubfe(cl, c.shift, RHO_BITS)];
    uint32_t r = e.y + (u > e.x ? 1u : 0u);
    if constexpr (MULTI) {
        if (e.y >= RHO_MULTI) {
            const uint32_t base = e.y & 0xFFFFu, cnt = e.y >> 16;
            r = base;
            for (uint32_t i = 0; i < cnt; ++i) r += (u > c.es[base - c.z + i]) ? 1u : 0u;
        }
    }
    return r;
}

// rho_of for a table without multi-threshold buckets and a bucket shift of
// at least 3, written with double-rate instructions: the bucket's byte offset
// as a right shift by sh3 = shift - 3 (held in a VGPR) and a mask (the table
// sits at LDS byte 0; the kernels check it), and the compare as the sign bit
// of b - u (keys are at most 0x7F800000, an empty bucket's b is 0x7FFFFFFF:
// the table is loaded with rho_table_entry).
__device__ __forceinline__ uint32_t rho_fast(uint32_t u, const RhoCtx& c, uint32_t sh3)
{
    const uint32_t cl = __float_as_uint(__builtin_amdgcn_fmed3f(__uint_as_float(u), c.emin, c.emax));
    const uint32_t off = (cl >> sh3) & ((RHO_TABLE - 1u) << 3);
    const __attribute__((address_space(3))) uint32_t* e = (const __attribute__((address_space(3))) uint32_t*)(size_t)off;
    return e[1] + ((e[0] - u) >> 31);
}

// A rank-table entry as the sweeps keep it in LDS: an empty bucket's first
// threshold 0xFFFFFFFF becomes 0x7FFFFFFF, above every key either way.
__device__ __forceinline__ uint2 rho_table_entry(uint2 e)
{
    e.x = min(e.x, 0x7FFFFFFFu);
    return e;
}

// Range sweep: buckets of 2^shift bit patterns hold up to two boundaries
// (x, y) and the rank base z (z + boundaries below the bucket); w > 0 marks a
// bucket with w > 2 boundaries, compared one by one (rare).
struct RangeCtx {
    const uint4* table;     // LDS [RANGE_TABLE], at LDS byte 0
    const uint32_t* es;     // LDS [Kp] boundaries
    float emin, emax;
    uint32_t sh4, Kp, z;    // sh4 = bucket shift - 4 (the shift is at least 4)
};

// Written with the operations gfx950 issues at the double rate (32-bit add,
// sub, and, or, right shifts): the bucket's byte offset is a right shift and
// a mask instead of a bit-field extract and a scaled add, and the two
// compares are sign bits of differences instead of compare-and-select pairs.
// Keys are at most +inf (0x7F800000) and boundaries at most 0x7FFFFFFF (the
// absent-boundary value), so b - u cannot wrap and its sign bit is u > b.
template <bool MULTI>
__device__ __forceinline__ uint32_t rank_of(uint32_t u, const RangeCtx& c)
{
    const uint32_t cl = __float_as_uint(__builtin_amdgcn_fmed3f(__uint_as_float(u), c.emin, c.emax));
    const uint32_t off = (cl >> c.sh4) & ((RANGE_TABLE - 1u) << 4);
    // the table sits at LDS byte 0 (k_range_sweep checks it), so its byte
    // offset is the LDS address: no base to add per key
    const __attribute__((address_space(3))) uint32_t* e = (const __attribute__((address_space(3))) uint32_t*)(size_t)off;
    const uint32_t ex = e[0], ey = e[1], ez = e[2];
    uint32_t r = ez + ((ex - u) >> 31) + ((ey - u) >> 31);
    if constexpr (MULTI) {
        const uint32_t ew = e[3];
        if (ew) {
            r = ez;
            for (uint32_t i = 0; i < ew; ++i) r += (u > c.es[ez - c.z + i]) ? 1u : 0u;
        }
    }
    return r;
}

// Line rank lambda_t: the smallest threshold index at which cell t lies on a
// diagonal line of length >= lmin, i.e. the minimum over windows of lmin
// consecutive cells containing t of the window's largest rho (cells outside
// the diagonal have rho = Kp).  lmin = 2: max(rho_t, min(rho_{t-1},
// rho_{t+1})).  Because rho is monotone in the key, lambda is also the rank
// of the cell's line value: the same expression over keys, i.e. the smallest
// threshold at which the cell lies on such a line (Eq. 4 and the line
// definition after it).
template <int NORM, int MC, int TC, int LMC>
struct SweepBody {
    uint2* stab;          // LDS [RHO_TABLE]
    uint32_t* ses;        // LDS [RANK_MAX]
    uint32_t* brho;       // LDS [Kcap+1][64]: row Kp collects cells that recur at no threshold
    uint32_t* blam;       // LDS [Kcap+1][64]
    const uint2* rtab;    // global [S][RHO_TABLE]
    SeriesWork* works;
    uint32_t Kcap;
    RhoCtx rc;
    uint32_t lmin;
    bool multi;
    bool active = true;

    __device__ void begin(uint32_t s)
    {
        const SeriesWork& w = works[s];
        for (uint32_t i = threadIdx.x; i < RHO_TABLE; i += blockDim.x) stab[i] = rtab[(size_t)s * RHO_TABLE + i];
        for (uint32_t i = threadIdx.x; i < RANK_MAX; i += blockDim.x) ses[i] = w.esorted[i];
        for (uint32_t i = threadIdx.x; i < (Kcap + 1) * TILE_W; i += blockDim.x) { brho[i] = 0u; blam[i] = 0u; }
        rc.table = stab;
        rc.es = ses;
        rc.emin = __uint_as_float(uniform(w.emin));
        rc.emax = __uint_as_float(uniform(w.emax));
        rc.shift = uniform(w.shift);
        rc.Kp = uniform(w.Kp);
        rc.z = 0;
        multi = uniform(w.multi) != 0;
    }
    __device__ void flush(uint32_t s)
    {
        SeriesWork& w = works[s];
        const uint32_t Kp = rc.Kp;
        for (uint32_t j = threadIdx.x; j < 2 * Kp; j += blockDim.x) {
            const uint32_t* row = (j < Kp) ? brho + j * TILE_W : blam + (j - Kp) * TILE_W;
            uint64_t sum = 0;
            for (int l = 0; l < TILE_W; ++l) sum += row[l];
            if (sum) atomicAdd((unsigned long long*)((j < Kp) ? &w.hrho[j] : &w.hlam[j - Kp]),
                               (unsigned long long)sum);
        }
    }
    // rho, lam <= Kp: the row Kp absorbs cells that recur at no threshold, so
    // the counting is branch-free and every lane hits its own bank.
    __device__ __forceinline__ void emit(uint32_t rho, uint32_t lam, int lane) const
    {
        atomicAdd(&brho[rho * TILE_W + lane], 1u);
        atomicAdd(&blam[lam * TILE_W + lane], 1u);
    }
    template <bool MULTI>
    __device__ __forceinline__ uint32_t rho_at(const SeriesScalars& sd, const TileGeo& g, int x) const
    {
        const bool ok = (x >= 0) && (x < g.len);
        const int i = ok ? x : 0;
        const int j = ok ? x + g.d : g.d0;
        const uint32_t r = rho_of<MULTI>(__float_as_uint(pair_key<NORM, MC, TC>(sd.y, i, j, sd.m, sd.tau)), rc);
        return ok ? r : rc.Kp;
    }
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        if (multi) tile_impl<true>(sd, tile_id, lane);
        else tile_impl<false>(sd, tile_id, lane);
    }
    template <bool MULTI>
    __device__ __forceinline__ void tile_impl(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        const TileGeo g = tile_geo(sd, tile_id, lane);
        constexpr bool kFast = (LMC == 1 || LMC == 2) && MC > 0 && (MC == 1 || TC > 0);
        constexpr int TW = MC == 1 ? 1 : TC;
        int tx = g.t0;  // cells before tx are counted by the walker
        // lmin = 2: ranks of the cells before and at the next one counted
        uint32_t rm1 = 0, r0 = 0;
        if constexpr (LMC == 2) {
            rm1 = rho_at<MULTI>(sd, g, g.t0 - 1);
            r0 = rho_at<MULTI>(sd, g, g.t0);
        }
        if constexpr (kFast) {
            constexpr int HU = walk_block<NORM, MC, TW>();
            const int tw = walk_end<HU>(g);
            if (tw > g.t0) {
                // every lane's diagonal covers [t0 - 1, tw + WALK_SLACK]
                const RhoCtx c = rc;
                if constexpr (LMC == 1) {
                    walk<NORM, MC, TW>(sd.y, g.d, g.t0, tw - g.t0, [&](const uint32_t(&k)[HU], int valid) {
                        uint32_t r[HU];
#pragma unroll
                        for (int u = 0; u < HU; ++u) r[u] = rho_of<MULTI>(k[u], c);
#pragma unroll
                        for (int u = 0; u < HU; ++u)
                            if (u < valid) emit(r[u], r[u], lane);
                    });
                } else {
                    walk<NORM, MC, TW>(sd.y, g.d, g.t0 + 1, tw - g.t0, [&](const uint32_t(&k)[HU], int valid) {
                        uint32_t r[HU];
#pragma unroll
                        for (int u = 0; u < HU; ++u) r[u] = rho_of<MULTI>(k[u], c);
#pragma unroll
                        for (int u = 0; u < HU; ++u) {
                            if (u < valid) {
                                emit(r0, max(r0, min(rm1, r[u])), lane);
                                rm1 = r0;
                                r0 = r[u];
                            }
                        }
                    });
                }
                tx = tw;
            }
        }
        if constexpr (LMC == 1) {
            for (int x = tx; x < g.t1; ++x) {
                const uint32_t r = rho_at<MULTI>(sd, g, x);
                emit(r, r, lane);
            }
        } else if constexpr (LMC == 2) {
            for (int x = tx; x < g.t1; ++x) {
                const uint32_t rp1 = rho_at<MULTI>(sd, g, x + 1);
                emit(r0, max(r0, min(rm1, rp1)), lane);
                rm1 = r0;
                r0 = rp1;
            }
        } else {
            // general lmin <= LMIN_MAX: rings of the last lmin ranks and of the
            // last lmin window maxima; output lags the newest rank by h = lmin-1.
            const int h = (int)lmin - 1;
            uint32_t rr[LMIN_MAX], ww[LMIN_MAX];
#pragma unroll
            for (int i = 0; i < LMIN_MAX; ++i) { rr[i] = rc.Kp; ww[i] = rc.Kp; }
            for (int x = g.t0 - h; x < g.t1 + h; ++x) {
                const uint32_t r = rho_at<MULTI>(sd, g, x);
#pragma unroll
                for (int i = 0; i < LMIN_MAX - 1; ++i) rr[i] = rr[i + 1];
                rr[LMIN_MAX - 1] = r;
                uint32_t wmax = 0, rold = rc.Kp;
#pragma unroll
                for (int i = 0; i < LMIN_MAX; ++i) {
                    if (i >= LMIN_MAX - 1 - h) wmax = max(wmax, rr[i]);
                    if (i == LMIN_MAX - 1 - h) rold = rr[i];
                }
#pragma unroll
                for (int i = 0; i < LMIN_MAX - 1; ++i) ww[i] = ww[i + 1];
                ww[LMIN_MAX - 1] = wmax;
                if (x >= g.t0 + h) {
                    uint32_t lam = rc.Kp;
#pragma unroll
                    for (int i = 0; i < LMIN_MAX; ++i)
                        if (i >= LMIN_MAX - 1 - h) lam = min(lam, ww[i]);
                    emit(rold, lam, lane);
                }
            }
        }
    }
};

// Range sweep.  The ranks are taken against the group boundaries (odd rank:
// inside group rank/2, see RangeCtx), and only the line ranks are
// histogrammed: C comes from the counting passes plus the fine counters, D
// from the line ranks below the target's group plus the fine counters of
// line values inside it.  A key or line value inside a group adds one to
// the group's fine counter at its offset from the group start (global
// memory, rare).  lmin = 1 needs no line values (D = C).
// Range-sweep LDS: rank table (at byte 0), per-column line-rank histograms
// of rows + 1 rows, the boundaries, then the group starts and fine offsets.
// A histogram row has 64 columns (one per lane) or, where 64 would cost a
// CU its third workgroup, 32 (lanes L and L + 32 share a column): the third
// workgroup is worth more than the shared columns cost (K = 48: sweep 7.36
// -> 6.07 ms; K = 20, where both layouts fit three: 64 columns 0.3% faster).
__host__ __device__ __forceinline__ size_t range_lds_layout(uint32_t rows, uint32_t cols)
{
    return RANGE_TABLE * sizeof(uint4) + (size_t)(rows + 1) * cols * 4 + (size_t)(rows - 1) * 4 +
           2 * (size_t)((rows + 1) / 2 + 1) * 4;
}
__host__ __device__ __forceinline__ uint32_t range_cols(uint32_t rows)
{
    return lds_blocks_fit(range_lds_layout(rows, 64) + 16) >= 3 ? 64u : 32u;
}

template <int NORM, int MC, int TC, int LMC>
struct RangeBody {
    uint4* stab;          // LDS [RANGE_TABLE], at byte 0
    uint32_t* blam;       // LDS [rows+1][cols]: the last row collects cells outside the diagonal
    uint32_t* ses;        // LDS [rows - 1] boundaries (rows - 1 = 2K >= Kp)
    uint32_t* sglo;       // LDS [gcap] group starts (gcap = K + 2 > ngroups)
    uint32_t* sgoff;      // LDS [gcap] group fine offsets
    uint32_t cols, csh, gcap;  // histogram columns, log2 of a row's bytes
    uint32_t lcol;        // this lane's column byte offset
    const uint4* rtab;    // global [S][RANGE_TABLE]
    SeriesWork* works;
    uint64_t* fineK;      // global [S][fine_stride]
    uint64_t* fineL;
    uint32_t fine_stride;
    unsigned long long* dk;
    unsigned long long* dl;
    uint32_t rows;
    RangeCtx rc;
    uint32_t lmin;
    uint32_t spare;       // rank above every boundary (and of cells outside the diagonal)
    uint32_t ngroups, nfine;
    bool multi;
    bool active = true;

    __device__ void begin(uint32_t s)
    {
        const SeriesWork& w = works[s];
        active = uniform(w.range_ok) != 0;
        for (uint32_t i = threadIdx.x; i < RANGE_TABLE; i += blockDim.x) stab[i] = rtab[(size_t)s * RANGE_TABLE + i];
        for (uint32_t i = threadIdx.x; i < rows - 1; i += blockDim.x) ses[i] = w.esorted[i];
        for (uint32_t i = threadIdx.x; i < (rows + 1) * cols; i += blockDim.x) blam[i] = 0u;
        for (uint32_t i = threadIdx.x; i < gcap; i += blockDim.x) {
            sglo[i] = w.g_lo[i];
            sgoff[i] = w.g_off[i];
        }
        rc.table = stab;
        rc.es = ses;
        rc.emin = __uint_as_float(uniform(w.emin));
        rc.emax = __uint_as_float(uniform(w.emax));
        rc.sh4 = uniform(w.shift) - 4u;
        rc.Kp = uniform(w.Kp);
        rc.z = uniform(w.zbase);
        spare = rc.Kp + rc.z;
        ngroups = uniform(w.ngroups);
        nfine = active ? uniform(w.nsub) << uniform(w.range_bits) : 0u;
        multi = uniform(w.multi) != 0;
        dk = (unsigned long long*)(fineK + (size_t)s * fine_stride);
        dl = (unsigned long long*)(fineL + (size_t)s * fine_stride);
    }
    __device__ void flush(uint32_t s)
    {
        if (!active || LMC == 1) return;
        SeriesWork& w = works[s];
        for (uint32_t j = threadIdx.x; j < spare; j += blockDim.x) {
            const uint32_t* row = blam + j * cols;
            uint64_t sum = 0;
            for (uint32_t l = 0; l < cols; ++l) sum += row[l];
            if (sum) atomicAdd((unsigned long long*)&w.hlam[j], (unsigned long long)sum);
        }
    }
    // row lam, this lane's column: one shift-and-add for the byte offset
    __device__ __forceinline__ void emit(uint32_t lam, int) const
    {
        atomicAdd((uint32_t*)((unsigned char*)blam + ((lam << csh) + lcol)), 1u);
    }
    // count value x of rank r if r is odd (inside group r/2); group and
    // counter index are checked, so no rank can address outside the counters
    __device__ __forceinline__ void fine(unsigned long long* dst, uint32_t r, uint32_t x) const
    {
        const uint32_t g = min(r >> 1, ngroups);
        const uint32_t idx = sgoff[g] + (x - sglo[g]);
        fine_add(dst, idx, (r & 1u) != 0 && g < ngroups && idx < nfine);
    }
    __device__ __forceinline__ uint32_t key_at(const SeriesScalars& sd, const TileGeo& g, int x) const
    {
        const bool ok = (x >= 0) && (x < g.len);
        const int i = ok ? x : 0;
        const int j = ok ? x + g.d : g.d0;
        const uint32_t k = __float_as_uint(pair_key<NORM, MC, TC>(sd.y, i, j, sd.m, sd.tau));
        return ok ? k : 0xFFFFFFFFu;  // outside the diagonal: above every boundary
    }
    template <bool MULTI>
    __device__ __forceinline__ uint32_t rank_at(uint32_t key) const
    {
        return key == 0xFFFFFFFFu ? spare : rank_of<MULTI>(key, rc);
    }
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        if (multi) tile_impl<true>(sd, tile_id, lane);
        else tile_impl<false>(sd, tile_id, lane);
    }
    template <bool MULTI>
    __device__ __forceinline__ void tile_impl(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        const TileGeo g = tile_geo(sd, tile_id, lane);
        constexpr bool kFast = (LMC == 1 || LMC == 2) && MC > 0 && (MC == 1 || TC > 0);
        constexpr int TW = MC == 1 ? 1 : TC;
        int tx = g.t0;  // cells before tx are counted by the walker
        // lmin = 2: keys and ranks of the cells before and at the next one counted
        uint32_t km1 = 0, k0 = 0, rm1 = 0, r0 = 0;
        if constexpr (LMC == 2) {
            km1 = key_at(sd, g, g.t0 - 1);
            k0 = key_at(sd, g, g.t0);
            rm1 = rank_at<MULTI>(km1);
            r0 = rank_at<MULTI>(k0);
        }
        if constexpr (kFast) {
            constexpr int HU = walk_block<NORM, MC, TW>();
            const int tw = walk_end<HU>(g);
            if (tw > g.t0) {
                // every lane's diagonal covers [t0 - 1, tw + WALK_SLACK]
                RangeCtx c = rc;
                c.sh4 = in_vgpr(rc.sh4);
                if constexpr (LMC == 1) {
                    walk<NORM, MC, TW>(sd.y, g.d, g.t0, tw - g.t0, [&](const uint32_t(&k)[HU], int valid) {
                        uint32_t r[HU];
                        uint32_t acc = 0;
#pragma unroll
                        for (int u = 0; u < HU; ++u) {
                            r[u] = rank_of<MULTI>(k[u], c);
                            if (u < valid) acc |= r[u];
                        }
                        if (__ballot(acc & 1u)) {   // rare: a key of the block lies inside a group
#pragma unroll
                            for (int u = 0; u < HU; ++u)
                                if (u < valid && __ballot(r[u] & 1u)) fine(dk, r[u], k[u]);
                        }
                    });
                } else {
                    // the walk runs one cell ahead: block keys are the right
                    // neighbours of the cells counted in the block
                    walk<NORM, MC, TW>(sd.y, g.d, g.t0 + 1, tw - g.t0, [&](const uint32_t(&k)[HU], int valid) {
                        uint32_t r[HU];
                        // a line value is one of the ranks of its cell and the two
                        // neighbours, so an odd rank among those of the block and the
                        // two before it covers every odd key rank and line rank
                        uint32_t acc = rm1 | r0;
#pragma unroll
                        for (int u = 0; u < HU; ++u) {
                            r[u] = rank_of<MULTI>(k[u], c);
                            acc |= r[u];
                        }
#pragma unroll
                        for (int u = 0; u < HU; ++u) {
                            if (u < valid) {
                                const uint32_t cr = u == 0 ? r0 : r[u - 1];
                                const uint32_t left = u == 0 ? rm1 : (u == 1 ? r0 : r[u - 2]);
                                emit(max(cr, min(left, r[u])), lane);
                            }
                        }
                        if (__ballot(acc & 1u)) {
                            // rare: some key or line value of the block lies inside a
                            // group; walk the block again for the fine counters
#pragma unroll
                            for (int u = 0; u < HU; ++u) {
                                if (u < valid) {
                                    const uint32_t cr = u == 0 ? r0 : r[u - 1];
                                    const uint32_t left = u == 0 ? rm1 : (u == 1 ? r0 : r[u - 2]);
                                    const uint32_t lam = max(cr, min(left, r[u]));
                                    if (__ballot((cr | lam) & 1u)) {
                                        const uint32_t ck = u == 0 ? k0 : k[u - 1];
                                        const uint32_t lk = u == 0 ? km1 : (u == 1 ? k0 : k[u - 2]);
                                        fine(dk, cr, ck);
                                        fine(dl, lam, max(ck, min(lk, k[u])));
                                    }
                                }
                            }
                        }
                        // state for the next block (the walk covers whole blocks
                        // only, so after it: the keys and ranks at tw - 1 and tw)
                        km1 = k[HU - 2];
                        k0 = k[HU - 1];
                        rm1 = r[HU - 2];
                        r0 = r[HU - 1];
                    });
                }
                tx = tw;
            }
        }
        if constexpr (LMC == 1) {
            for (int x = tx; x < g.t1; ++x) {
                const uint32_t k = key_at(sd, g, x);
                const uint32_t r = rank_at<MULTI>(k);
                if (__ballot(r & 1u)) fine(dk, r, k);
            }
        } else if constexpr (LMC == 2) {
            for (int x = tx; x < g.t1; ++x) {
                const uint32_t kp1 = key_at(sd, g, x + 1);
                const uint32_t rp1 = rank_at<MULTI>(kp1);
                const uint32_t lam = max(r0, min(rm1, rp1));
                emit(lam, lane);
                if (__ballot((r0 | lam) & 1u)) {
                    fine(dk, r0, k0);
                    fine(dl, lam, max(k0, min(km1, kp1)));
                }
                km1 = k0;
                k0 = kp1;
                rm1 = r0;
                r0 = rp1;
            }
        } else {
            // general lmin <= LMIN_MAX: rings of the last lmin keys and of the
            // last lmin window maxima (keys; ranks follow); the counted cell lags
            // the newest key by h = lmin-1
            const int h = (int)lmin - 1;
            uint32_t kk[LMIN_MAX], wk[LMIN_MAX];
#pragma unroll
            for (int i = 0; i < LMIN_MAX; ++i) { kk[i] = 0xFFFFFFFFu; wk[i] = 0xFFFFFFFFu; }
            for (int x = g.t0 - h; x < g.t1 + h; ++x) {
                const uint32_t key = key_at(sd, g, x);
#pragma unroll
                for (int i = 0; i < LMIN_MAX - 1; ++i) kk[i] = kk[i + 1];
                kk[LMIN_MAX - 1] = key;
                uint32_t wmax = 0, kold = 0xFFFFFFFFu;
#pragma unroll
                for (int i = 0; i < LMIN_MAX; ++i) {
                    if (i >= LMIN_MAX - 1 - h) wmax = max(wmax, kk[i]);
                    if (i == LMIN_MAX - 1 - h) kold = kk[i];
                }
#pragma unroll
                for (int i = 0; i < LMIN_MAX - 1; ++i) wk[i] = wk[i + 1];
                wk[LMIN_MAX - 1] = wmax;
                if (x >= g.t0 + h) {
                    uint32_t lkey = 0xFFFFFFFFu;
#pragma unroll
                    for (int i = 0; i < LMIN_MAX; ++i)
                        if (i >= LMIN_MAX - 1 - h) lkey = min(lkey, wk[i]);
                    const uint32_t rk = rank_at<MULTI>(kold), lam = rank_at<MULTI>(lkey);
                    emit(lam, lane);
                    if (__ballot((rk | lam) & 1u)) {
                        fine(dk, rk, kold);
                        fine(dl, lam, lkey);
                    }
                }
            }
        }
    }
};

// LDS of the sweeps: rank table, thresholds, per-lane histograms with a spare
// row (two for given thresholds, one for the range sweep, which also holds
// the group arrays), then the work-queue word.
__host__ __device__ __forceinline__ size_t sweep_lds_bytes_dev(uint32_t rows, bool ranges)
{
    if (ranges)
        return range_lds_layout(rows, range_cols(rows));
    return RHO_TABLE * sizeof(uint2) + RANK_MAX * 4 + 2 * (size_t)(rows + 1) * TILE_W * 4;
}

// Launched with 512 threads, or 1024 where its LDS admits one workgroup per
// CU (large K), so that more waves share the one copy of the tables.
template <int NORM, int MC, int TC, int LMC>
__global__ void __launch_bounds__(1024)
k_sweep(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t nchunks, uint32_t chunk_tiles,
        uint32_t* __restrict__ ticket, SeriesWork* __restrict__ works, const uint2* __restrict__ rtab, uint32_t Kcap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    SweepBody<NORM, MC, TC, LMC> body;
    body.stab = (uint2*)smem;
    body.ses = (uint32_t*)(smem + RHO_TABLE * sizeof(uint2));
    body.brho = body.ses + RANK_MAX;
    body.blam = body.brho + (size_t)(Kcap + 1) * TILE_W;
    body.rtab = rtab;
    body.works = works;
    body.Kcap = Kcap;
    body.multi = false;
    // the generic line class reads lmin from the descriptors: launches group
    // series of one lmin
    body.lmin = LMC == 0 ? sds[0].lmin : (uint32_t)LMC;
    chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, (uint32_t*)(smem + sweep_lds_bytes_dev(Kcap, false)));
}

// Six waves per SIMD (three workgroups of 512 per CU, which the LDS allows up
// to K = 38 with 64 histogram columns and up to K = 76 with 32, in 1280-byte
// units): the register budget drops to 80 and a few spill, but the
// extra waves hide the rank-table and series loads better (about 10% faster
// at K = 20 than the four waves 105 registers allow).
template <int NORM, int MC, int TC, int LMC>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
k_range_sweep(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t nchunks, uint32_t chunk_tiles,
              uint32_t* __restrict__ ticket, SeriesWork* __restrict__ works, const uint2* __restrict__ rtab,
              uint32_t rows, uint64_t* __restrict__ fineK, uint64_t* __restrict__ fineL, uint32_t fine_stride)
{
    extern __shared__ __align__(16) unsigned char smem[];
    RangeBody<NORM, MC, TC, LMC> body;
    body.cols = range_cols(rows);
    body.csh = body.cols == 64 ? 8u : 7u;
    body.gcap = (rows + 1) / 2 + 1;
    body.lcol = ((uint32_t)threadIdx.x & (body.cols - 1)) * 4u;
    body.stab = (uint4*)smem;
    body.blam = (uint32_t*)(smem + RANGE_TABLE * sizeof(uint4));
    body.ses = body.blam + (size_t)(rows + 1) * body.cols;
    body.sglo = body.ses + (rows - 1);
    body.sgoff = body.sglo + body.gcap;
    body.rtab = (const uint4*)rtab;
    body.works = works;
    body.fineK = fineK;
    body.fineL = fineL;
    body.fine_stride = fine_stride;
    body.dk = nullptr;
    body.dl = nullptr;
    body.rows = rows;
    body.ngroups = 0;
    body.nfine = 0;
    body.multi = false;
    body.lmin = LMC == 0 ? sds[0].lmin : (uint32_t)LMC;
    // rank_of addresses the rank table by its offset from LDS byte 0: the
    // kernel's dynamic LDS must start there (it has no static LDS); a launch
    // where it does not marks every series (the host reports a device error)
    if ((uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char*)smem != 0u) {
        if (threadIdx.x == 0)
            for (uint32_t s = 0; s < S; ++s) atomicOr(&works[s].status, 64u);
        return;
    }
    chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, (uint32_t*)(smem + sweep_lds_bytes_dev(rows, true)));
}

size_t sweep_lds_bytes(uint32_t rows, bool ranges) { return sweep_lds_bytes_dev(rows, ranges) + 16; }

using SweepFn = void (*)(const SeriesDesc*, uint32_t, uint32_t, uint32_t, uint32_t*, SeriesWork*, const uint2*,
                         uint32_t);
using RangeFn = void (*)(const SeriesDesc*, uint32_t, uint32_t, uint32_t, uint32_t*, SeriesWork*, const uint2*,
                         uint32_t, uint64_t*, uint64_t*, uint32_t);

template <int NORM, int MC, int TC>
static SweepFn sweep_fn_l(int lc)
{
    if (lc == 1) return k_sweep<NORM, MC, TC, 1>;
    if (lc == 2) return k_sweep<NORM, MC, TC, 2>;
    return k_sweep<NORM, MC, TC, 0>;
}

template <int NORM, int MC, int TC>
static RangeFn range_fn_l(int lc)
{
    if (lc == 1) return k_range_sweep<NORM, MC, TC, 1>;
    if (lc == 2) return k_range_sweep<NORM, MC, TC, 2>;
    return k_range_sweep<NORM, MC, TC, 0>;
}

template <int NORM>
static SweepFn sweep_fn_n(int mclass, int lc)
{
    switch (mclass) {
    case 1: return sweep_fn_l<NORM, 1, 0>(lc);
    case 2: return sweep_fn_l<NORM, 3, 3>(lc);
    case 3: return sweep_fn_l<NORM, 3, 5>(lc);
    default: return sweep_fn_l<NORM, 0, 0>(lc);
    }
}

template <int NORM>
static RangeFn range_fn_n(int mclass, int lc)
{
    switch (mclass) {
    case 1: return range_fn_l<NORM, 1, 0>(lc);
    case 2: return range_fn_l<NORM, 3, 3>(lc);
    case 3: return range_fn_l<NORM, 3, 5>(lc);
    default: return range_fn_l<NORM, 0, 0>(lc);
    }
}

static SweepFn sweep_fn(int variant)
{
    const int lc = variant % 3, sv = variant / 3;
    const int norm = sv / NUM_MCLASS, mc = sv % NUM_MCLASS;
    return norm == RQA_NORM_MAX ? sweep_fn_n<RQA_NORM_MAX>(mc, lc) : sweep_fn_n<RQA_NORM_EUCLIDEAN>(mc, lc);
}

static RangeFn range_fn(int variant)
{
    const int lc = variant % 3, sv = variant / 3;
    const int norm = sv / NUM_MCLASS, mc = sv % NUM_MCLASS;
    return norm == RQA_NORM_MAX ? range_fn_n<RQA_NORM_MAX>(mc, lc) : range_fn_n<RQA_NORM_EUCLIDEAN>(mc, lc);
}

static uint32_t sweep_rows(uint32_t K, bool ranges) { return ranges ? 2 * K + 1 : K; }

hipError_t launch_sweep(hipStream_t st, const DevBufs& b, int variant, bool ranges, uint32_t grid, uint32_t block,
                        uint32_t ticket)
{
    const uint32_t rows = sweep_rows(b.K, ranges);
    if (ranges)
        hipLaunchKernelGGL(range_fn(variant), dim3(grid), dim3(block), sweep_lds_bytes(rows, true), st, b.sd, b.S,
                           b.nchunks, b.chunk_tiles, b.tickets + ticket, b.work, b.rtab, rows, b.fineK, b.fineL,
                           b.fine_stride);
    else
        hipLaunchKernelGGL(sweep_fn(variant), dim3(grid), dim3(block), sweep_lds_bytes(rows, false), st, b.sd, b.S,
                           b.nchunks, b.chunk_tiles, b.tickets + ticket, b.work, b.rtab, rows);
    return hipGetLastError();
}

int sweep_blocks_per_cu(int variant, bool ranges, uint32_t block, size_t lds)
{
    return blocks_per_cu(ranges ? (const void*)range_fn(variant) : (const void*)sweep_fn(variant), block, lds);
}

// Threads of the sweeps' set-up kernels: each looks up a few table buckets
// (binary searches whose steps wait on LDS), so more threads finish sooner.
constexpr uint32_t PREP_THREADS = 1024;

// Number of entries of the ascending array es[0..n) below x (a binary
// search: the table builders below look up both edges of every bucket).
__device__ __forceinline__ uint32_t count_below(const uint32_t* es, uint32_t n, uint64_t x)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)es[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Rank table of one series over the ascending thresholds es[0..kp) with rank
// base z: spans the buckets (key >> shift) from es[0] to es[kp-1] with the
// smallest shift that fits RHO_TABLE buckets; bucket a (mod RHO_TABLE) stores
// z + the number of thresholds below a << shift, and the first threshold
// inside the bucket (several inside: flagged, the count in the high half).
// Called by a whole block after es is complete in LDS.
__device__ void build_rank_table(SeriesWork& w, const uint32_t* es, uint32_t kp, uint32_t z, uint2* tab,
                                 uint32_t* s_shift)
{
    if (threadIdx.x == 0) {
        uint32_t sh = 0;
        while (sh < 31 && (es[kp - 1] >> sh) - (es[0] >> sh) >= RHO_TABLE) ++sh;
        *s_shift = sh;
        w.multi = 0u;  // set before the barrier; table entries below may raise it
    }
    __syncthreads();
    const uint32_t sh = *s_shift;
    const uint32_t emin = es[0], emax = es[kp - 1];
    for (uint32_t i = threadIdx.x; i < RANK_MAX; i += blockDim.x) w.esorted[i] = (i < kp) ? es[i] : 0xFFFFFFFFu;
    for (uint32_t i = threadIdx.x; i < RANK_MAX + 2; i += blockDim.x) { w.hrho[i] = 0; w.hlam[i] = 0; }
    if (threadIdx.x == 0) {
        w.Kp = kp;
        w.zbase = z;
        w.shift = sh;
        w.emin = emin;
        w.emax = emax;
    }
    const uint32_t a0 = emin >> sh, a1 = emax >> sh;
    for (uint32_t idx = threadIdx.x; idx < RHO_TABLE; idx += blockDim.x) {
        const uint32_t a = a0 + ((idx - a0) & (RHO_TABLE - 1));
        uint2 e = make_uint2(0xFFFFFFFFu, z);
        if (a <= a1) {
            const uint64_t lo = (uint64_t)a << sh, hi = (uint64_t)(a + 1) << sh;
            const uint32_t below = count_below(es, kp, lo), inside = count_below(es, kp, hi) - below;
            e.x = inside ? es[below] : 0xFFFFFFFFu;
            e.y = (inside >= 2) ? ((z + below) | (inside << 16)) : z + below;
            if (inside >= 2) w.multi = 1u;
        }
        tab[idx] = e;
    }
}

// Sweep at given thresholds: per series the distinct sorted thresholds, the
// caller->distinct map and the rank table.
__global__ void __launch_bounds__(PREP_THREADS) k_sweep_prep(const SeriesDesc* __restrict__ sds,
                                                    SeriesWork* __restrict__ works, uint2* __restrict__ rtab)
{
    __shared__ uint32_t s_eps[RQA_MAX_K], es[RQA_MAX_K], s_pos[RQA_MAX_K], s_flag[RQA_MAX_K];
    __shared__ uint32_t s_shift;
    const uint32_t s = blockIdx.x;
    const uint32_t K = sds[s].K;
    SeriesWork& w = works[s];
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) s_eps[r] = w.eps_bits[r];
    __syncthreads();
    const uint32_t kp = block_sort_unique(s_eps, nullptr, K, es, s_pos, s_flag);
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) w.dmap[r] = s_pos[r];
    build_rank_table(w, es, kp, 0u, rtab + (size_t)s * RHO_TABLE, &s_shift);
}

hipError_t launch_sweep_prep(hipStream_t st, const DevBufs& b)
{
    hipLaunchKernelGGL(k_sweep_prep, dim3(b.S), dim3(PREP_THREADS), 0, st, b.sd, b.work, b.rtab);
    return hipGetLastError();
}

// ------------------------------------------------------------------ full line-length histogram

// Full line-length histogram P_j(l) at given thresholds (the histogram behind
// Eq. 4).  Tiles are the (band, segment) tiles of the sweep.  Each lane keeps
// a stack of the cells of its segment that were larger in rank than every
// later cell so far ("previous greater" chain): ranks strictly decrease from
// the bottom (a sentinel at position t0 - 1, above every rank) to the top.
// A new cell of rank r at position t pops every entry of rank <= r; popping
// entry (r_i, p_i) with (r_n, p_n) below it ends, for every threshold j in
// [r_i, min(r_n, r)), the run of cells p_n + 1 .. t - 1 (at threshold j the
// last cell before t that is not recurrent is p_n).  A run inside the
// segment is a line: one +1 / -1 pair in a difference histogram over j for
// its length, so the work per cell is amortised O(1) whatever the number of
// thresholds, and P_j(l) is the prefix sum over j.  A run that starts at the
// segment's first cell (p_n is the sentinel) or ends at its last may continue
// in the neighbouring segment: per lane and threshold the segment records
// the length of its leading run (pre_j) and trailing run (suf_j), and a join
// pass walks each diagonal's segments in order and counts the lines that
// cross segment borders.  Cells past the end of a diagonal have rank Kp
// (recurrent at no threshold).  The top two stack entries live in registers;
// entries pack (rank << 24) | (position + 1).
constexpr uint32_t HIST_SHORT = 64;     // lengths below this count in LDS
constexpr uint32_t HIST_MAX_K = RQA_MAX_HIST_K;  // distinct thresholds
static_assert(HIST_MAX_K == HIST_MAX_K_HOST, "histogram limits");
static_assert(HIST_MAX_K + 1 < 256, "ranks are packed into 8 bits");
static_assert(HIST_MAX_SEG_HOST < 65536, "run lengths are stored in 16 bits");

__host__ __device__ __forceinline__ size_t hist_lds_bytes_dev(uint32_t Kp, uint32_t block)
{
    return RHO_TABLE * sizeof(uint2) + RANK_MAX * 4 + (size_t)(Kp + 1) * block * 4 +
           (size_t)HIST_SHORT * (Kp + 1) * 4;
}

template <int NORM, int MC, int TC>
struct HistBody {
    uint2* stab;          // LDS [RHO_TABLE]
    uint32_t* ses;        // LDS [RANK_MAX]
    uint32_t* stk;        // LDS [Kp + 1][blockDim] stack entries below the top two (column = thread)
    uint32_t* dsh;        // LDS [Kp + 1][HIST_SHORT] difference counts of short lines
    const SeriesDesc* sds;
    const uint2* rtab;
    SeriesWork* works;
    uint64_t* dglob;      // global [S][hist_len][kcap] difference counts (signed, two's complement)
    uint16_t* pre;        // global [tiles][kcap][64] leading run per threshold
    uint16_t* suf;        // global [tiles][kcap][64] trailing run per threshold
    uint32_t hist_len;
    uint32_t kcap;        // Kp + 1 of the launch (row stride)
    uint32_t chunk_tiles;
    RhoCtx rc;
    uint64_t* dser;       // this series' rows
    uint32_t tbase;       // this series' first tile in pre / suf
    bool multi;
    bool active = true;
    // lane state: the top and next entries of the stack (packed); LDS rows
    // [0, sp) hold the bottom sentinel and then the entries below next (sp >= 1),
    // addressed by byte offsets: so = row sp of this lane, so0 / so1 = rows 0 / 1;
    // pm is the largest rank so far in the segment.  A cell of rank Kp ends every
    // run: it replaces the whole stack as a new bottom sentinel (rank Kp + 1 at
    // its position), so runs of such cells cost no pops.  Only the segment's own
    // sentinel has position t0.
    uint32_t top, nx, so, so0, so1, bd4, pm, t0;
    uint32_t sh3;         // bucket shift - 3
    uint16_t* lpre;       // this lane's pre / suf column in the current tile
    uint16_t* lsuf;

    __device__ __forceinline__ void begin(uint32_t s)
    {
        const SeriesWork& w = works[s];
        for (uint32_t i = threadIdx.x; i < RHO_TABLE; i += blockDim.x)
            stab[i] = rho_table_entry(rtab[(size_t)s * RHO_TABLE + i]);
        for (uint32_t i = threadIdx.x; i < RANK_MAX; i += blockDim.x) ses[i] = w.esorted[i];
        for (uint32_t i = threadIdx.x; i < HIST_SHORT * kcap; i += blockDim.x) dsh[i] = 0u;
        rc.table = stab;
        rc.es = ses;
        rc.emin = __uint_as_float(uniform(w.emin));
        rc.emax = __uint_as_float(uniform(w.emax));
        rc.shift = uniform(w.shift);
        rc.Kp = uniform(w.Kp);
        rc.z = 0;
        // rho_fast needs a bucket shift of at least 3; narrower tables take
        // the general lookup
        multi = uniform(w.multi) != 0 || rc.shift < 3u;
        sh3 = rc.shift - 3u;
        sh3 = in_vgpr(sh3);
        active = uniform(w.nonfinite) == 0u;  // no ranks for a series with NaN or infinite samples
        dser = dglob + (size_t)s * hist_len * kcap;
        tbase = uniform(sds[s].chunk_begin) * chunk_tiles;
    }
    __device__ __forceinline__ void flush(uint32_t)
    {
        for (uint32_t i = threadIdx.x; i < HIST_SHORT * kcap; i += blockDim.x) {
            const uint32_t j = i / HIST_SHORT, l = i % HIST_SHORT;
            const int32_t v = (int32_t)dsh[i];
            if (v && l < hist_len)
                atomicAdd((unsigned long long*)&dser[(size_t)l * kcap + j], (unsigned long long)(int64_t)v);
        }
    }
    // one line of length l at thresholds [a, b)
    __device__ __forceinline__ void line(uint32_t l, uint32_t a, uint32_t b)
    {
        const uint32_t lb = min(l, hist_len - 1);
        if (lb < HIST_SHORT) {
            atomicAdd(&dsh[a * HIST_SHORT + lb], 1u);
            atomicAdd(&dsh[b * HIST_SHORT + lb], 0xFFFFFFFFu);
        } else {
            atomicAdd((unsigned long long*)&dser[(size_t)lb * kcap + a], 1ull);
            atomicAdd((unsigned long long*)&dser[(size_t)lb * kcap + b], ~0ull);
        }
    }
    __device__ __forceinline__ uint32_t& at(uint32_t off) { return *(uint32_t*)((unsigned char*)stk + off); }
    static constexpr uint32_t POS = 0xFFFFFFu;
    __device__ __forceinline__ void pop()
    {
        top = nx;
        // row 0 is the bottom sentinel: below it is the sentinel again
        nx = at(so - bd4);
        so = max(so - bd4, so1);
    }
    // rank of a key (at most Kp)
    template <bool MULTI>
    __device__ __forceinline__ uint32_t rank(uint32_t u, const RhoCtx& c) const
    {
        if constexpr (MULTI) return rho_of<true>(u, c);
        else return rho_fast(u, c, sh3);
    }
    // cell of rank r <= Kp at position t
    __device__ __forceinline__ void cell(uint32_t r, uint32_t t)
    {
        if (r > pm) {
            // first cell above thresholds [pm, r): the leading runs there end before t
#pragma unroll 1
            for (uint32_t j = pm; j < r; ++j) lpre[(size_t)j * TILE_W] = (uint16_t)(t - t0);
            pm = r;
        }
        // pop while the top's rank is <= r (ranks sit in the high byte)
        const uint32_t rhi = (r << 24) | POS;
        while (top <= rhi) {
            const uint32_t tr = top >> 24, np1 = nx & POS;
            // next is the segment's sentinel: a leading run, recorded above
            const uint32_t b = np1 == t0 ? tr : min(nx >> 24, r);
            if (tr < b) line(t - np1, tr, b);
            pop();
        }
        const bool reset = r == rc.Kp;
        const uint32_t snt = ((rc.Kp + 1) << 24) | (t + 1);
        // push: a cell below the top sends next to LDS (a sentinel next is row 0 already)
        at(reset ? so0 : so) = reset ? snt : nx;
        so = reset ? so1 : so + (nx < ((rc.Kp + 1) << 24) ? bd4 : 0u);
        nx = reset ? snt : top;
        top = reset ? snt : (r << 24) | (t + 1);
    }
    __device__ __forceinline__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        if (multi) tile_impl<true>(sd, tile_id, lane);
        else tile_impl<false>(sd, tile_id, lane);
    }
    template <bool MULTI>
    __device__ __forceinline__ void tile_impl(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        const TileGeo g = tile_geo(sd, tile_id, lane);
        const uint32_t Kp = rc.Kp;
        const size_t col = ((size_t)(tbase + tile_id) * kcap) * TILE_W + lane;
        lpre = pre + col;
        lsuf = suf + col;
        t0 = (uint32_t)g.t0;
        // sentinel (rank Kp + 1 at position t0 - 1) as top, next and LDS row 0
        bd4 = blockDim.x * 4u;
        so0 = threadIdx.x * 4u;
        so1 = so0 + bd4;
        so = so1;
        top = nx = ((Kp + 1) << 24) | t0;
        at(so0) = top;
        pm = 0;
        constexpr bool kFast = MC > 0 && (MC == 1 || TC > 0);
        int tx = g.t0;  // cells before tx are taken by the walker
        if constexpr (kFast) {
            constexpr int TW = MC == 1 ? 1 : TC;
            constexpr int HU = walk_block<NORM, MC, TW>();
            const int tw = walk_end<HU>(g);
            if (tw > g.t0) {
                // every lane's diagonal covers [t0, tw + WALK_SLACK]
                const RhoCtx c = rc;
                uint32_t t = t0;
                walk<NORM, MC, TW>(sd.y, g.d, g.t0, tw - g.t0, [&](const uint32_t(&k)[HU], int valid) {
                    uint32_t rk[HU];
#pragma unroll
                    for (int u = 0; u < HU; ++u) rk[u] = rank<MULTI>(k[u], c);
#pragma unroll
                    for (int u = 0; u < HU; ++u)
                        if (u < valid) cell(rk[u], t + (uint32_t)u);
                    t += HU;
                });
                tx = tw;
            }
        }
        {
            for (int x = tx; x < g.t1; ++x) {
                uint32_t r = Kp;
                if (x < g.len)
                    r = min(rho_of<MULTI>(__float_as_uint(pair_key<NORM, MC, TC>(sd.y, x, x + g.d, sd.m, sd.tau)), rc),
                            Kp);
                cell(r, (uint32_t)x);
            }
        }
        // trailing runs: below the last cell's rank empty, then one per stack entry
        const uint32_t e = (uint32_t)g.t1;
        #pragma unroll 1
        for (uint32_t j = 0; j < min(top >> 24, Kp); ++j) lsuf[(size_t)j * TILE_W] = 0;
        while ((top >> 24) <= Kp) {
            const uint32_t tr = top >> 24, hi = min(nx >> 24, Kp), np1 = nx & POS;
            if (np1 == t0) {
                // every cell of the segment recurrent at [tr, Kp)
                #pragma unroll 1
                for (uint32_t j = tr; j < hi; ++j) {
                    lpre[(size_t)j * TILE_W] = (uint16_t)(e - t0);
                    lsuf[(size_t)j * TILE_W] = (uint16_t)(e - t0);
                }
            } else {
                #pragma unroll 1
                for (uint32_t j = tr; j < hi; ++j) lsuf[(size_t)j * TILE_W] = (uint16_t)(e - np1);
            }
            pop();
        }
    }
};

template <int NORM, int MC, int TC>
__global__ void __launch_bounds__(1024)
k_hist(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t nchunks, uint32_t chunk_tiles,
       uint32_t* __restrict__ ticket, SeriesWork* __restrict__ works, const uint2* __restrict__ rtab,
       uint64_t* __restrict__ dglob, uint16_t* __restrict__ pre, uint16_t* __restrict__ suf, uint32_t hist_len,
       uint32_t Kp)
{
    extern __shared__ __align__(16) unsigned char smem[];
    HistBody<NORM, MC, TC> body;
    body.stab = (uint2*)smem;
    body.ses = (uint32_t*)(smem + RHO_TABLE * sizeof(uint2));
    body.stk = body.ses + RANK_MAX;
    body.dsh = body.stk + (size_t)(Kp + 1) * blockDim.x;
    body.sds = sds;
    body.rtab = rtab;
    body.works = works;
    body.dglob = dglob;
    body.pre = pre;
    body.suf = suf;
    body.hist_len = hist_len;
    body.kcap = Kp + 1;
    body.chunk_tiles = chunk_tiles;
    body.multi = false;
    // rank() addresses the rank table by its offset from LDS byte 0
    if ((uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char*)smem != 0u) {
        if (threadIdx.x == 0)
            for (uint32_t s = 0; s < S; ++s) atomicOr(&works[s].status, 64u);
        return;
    }
    chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, (uint32_t*)(smem + hist_lds_bytes_dev(Kp, blockDim.x)));
}

// Lines across segment borders: thread (diagonal, threshold) walks the
// diagonal's segments in order, carrying the run that reaches the segment's
// end into the next segment's leading run (or through a segment recurrent
// everywhere at that threshold).  A leading run of the first segment and a
// trailing run of the last are lines too.  A workgroup (64 diagonals x 4
// thresholds per step) strides over (band, threshold group) items and counts
// short lines in LDS; one flush per workgroup.
constexpr uint32_t HIST_JOIN_BLOCK = 256;

__global__ void __launch_bounds__(HIST_JOIN_BLOCK)
k_hist_join(const SeriesDesc* __restrict__ sds, const SeriesWork* __restrict__ works, uint32_t chunk_tiles,
            const uint16_t* __restrict__ pre, const uint16_t* __restrict__ suf, uint64_t* __restrict__ dglob,
            uint32_t hist_len, uint32_t kcap)
{
    __shared__ uint32_t cnt[HIST_SHORT * (HIST_MAX_K + 1)];
    const uint32_t s = blockIdx.y;
    const SeriesDesc& sd = sds[s];
    const uint32_t Kp = works[s].Kp;
    if (works[s].nonfinite) return;  // uniform over the workgroup
    for (uint32_t i = threadIdx.x; i < HIST_SHORT * kcap; i += blockDim.x) cnt[i] = 0u;
    __syncthreads();
    uint64_t* dser = dglob + (size_t)s * hist_len * kcap;
    const uint32_t jb = (Kp + 3) / 4;
    const uint32_t lane = threadIdx.x % TILE_W;
    const uint64_t B = sd.B, q = sd.q;
    const uint32_t T = sd.T;
    auto emit = [&](uint32_t l, uint32_t j) {
        const uint32_t lb = min(l, hist_len - 1);
        if (lb < HIST_SHORT) {
            atomicAdd(&cnt[lb * kcap + j], 1u);
        } else {
            atomicAdd((unsigned long long*)&dser[(size_t)lb * kcap + j], 1ull);
            atomicAdd((unsigned long long*)&dser[(size_t)lb * kcap + j + 1], ~0ull);
        }
    };
    for (uint32_t item = blockIdx.x; item < sd.B * jb; item += gridDim.x) {
        const uint32_t band = item / jb;
        const uint32_t j = (item % jb) * 4 + threadIdx.x / TILE_W;
        const uint32_t d = sd.w + band * TILE_W + lane;
        if (j >= Kp || d >= sd.nv) continue;
        const uint32_t len = sd.nv - d;
        const uint32_t nseg = (len + T - 1) / T;
        uint32_t carry = 0;
        for (uint32_t g = 0; g < nseg; ++g) {
            const uint64_t tile = (uint64_t)g * B - q * ((uint64_t)g * (g - 1) / 2) + band;
            const size_t at = (((size_t)sd.chunk_begin * chunk_tiles + tile) * kcap + j) * TILE_W + lane;
            const uint32_t seglen = min(T, len - g * T);
            const uint32_t a = pre[at];
            if (a == seglen) {
                carry += seglen;
            } else {
                if (carry + a) emit(carry + a, j);
                carry = suf[at];
            }
        }
        if (carry) emit(carry, j);
    }
    __syncthreads();
    // counts of one threshold: +c at j and -c at j + 1 of the difference rows
    for (uint32_t i = threadIdx.x; i < HIST_SHORT * kcap; i += blockDim.x) {
        const uint32_t c = cnt[i];
        const uint32_t l = i / kcap, j = i % kcap;
        if (c && l < hist_len) {
            atomicAdd((unsigned long long*)&dser[(size_t)l * kcap + j], (unsigned long long)c);
            atomicAdd((unsigned long long*)&dser[(size_t)l * kcap + j + 1], (unsigned long long)(-(int64_t)c));
        }
    }
}

// P_r(l) from the difference counts: the prefix over thresholds up to the
// caller's threshold r (dmap), written as rows out[s][r][l] (thread per l).
__global__ void __launch_bounds__(256)
k_hist_finish(const SeriesDesc* __restrict__ sds, const SeriesWork* __restrict__ works,
              const uint64_t* __restrict__ dglob, uint64_t* __restrict__ out, uint32_t hist_len, uint32_t kcap)
{
    const uint32_t s = blockIdx.y;
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= hist_len) return;
    const uint32_t K = sds[s].K;
    const SeriesWork& w = works[s];
    const uint64_t* d = dglob + ((size_t)s * hist_len + l) * kcap;
    uint64_t* o = out + (size_t)s * K * hist_len + l;
    for (uint32_t r = 0; r < K; ++r) {
        const uint32_t top = min(w.dmap[r], kcap - 1);
        uint64_t acc = 0;  // two's complement: the sum of the signed differences
        for (uint32_t j = 0; j <= top; ++j) acc += d[j];
        o[(size_t)r * hist_len] = acc;
    }
}

hipError_t launch_hist_finish(hipStream_t st, const DevBufs& b, const uint64_t* dglob, uint64_t* out,
                              uint32_t hist_len, uint32_t Kp)
{
    hipLaunchKernelGGL(k_hist_finish, dim3((hist_len + 255) / 256, b.S), dim3(256), 0, st, b.sd, b.work, dglob, out,
                       hist_len, Kp + 1);
    return hipGetLastError();
}

size_t hist_lds_bytes(uint32_t Kp, uint32_t block) { return hist_lds_bytes_dev(Kp, block) + 16; }

using HistFn = void (*)(const SeriesDesc*, uint32_t, uint32_t, uint32_t, uint32_t*, SeriesWork*, const uint2*,
                        uint64_t*, uint16_t*, uint16_t*, uint32_t, uint32_t);

template <int NORM>
static HistFn hist_fn_n(int mclass)
{
    switch (mclass) {
    case 1: return k_hist<NORM, 1, 0>;
    case 2: return k_hist<NORM, 3, 3>;
    case 3: return k_hist<NORM, 3, 5>;
    default: return k_hist<NORM, 0, 0>;
    }
}

static HistFn hist_fn(int select_variant)
{
    const int norm = select_variant / NUM_MCLASS, mc = select_variant % NUM_MCLASS;
    return norm == RQA_NORM_MAX ? hist_fn_n<RQA_NORM_MAX>(mc) : hist_fn_n<RQA_NORM_EUCLIDEAN>(mc);
}

hipError_t launch_hist(hipStream_t st, const DevBufs& b, int select_variant, uint32_t grid, uint32_t block,
                       uint64_t* dglob, uint16_t* pre, uint16_t* suf, uint32_t hist_len, uint32_t Kp, uint32_t ticket)
{
    hipLaunchKernelGGL(hist_fn(select_variant), dim3(grid), dim3(block), hist_lds_bytes(Kp, block), st, b.sd, b.S,
                       b.nchunks, b.chunk_tiles, b.tickets + ticket, b.work, b.rtab, dglob, pre, suf, hist_len, Kp);
    return hipGetLastError();
}

hipError_t launch_hist_join(hipStream_t st, const DevBufs& b, uint32_t grid, const uint16_t* pre,
                            const uint16_t* suf, uint64_t* dglob, uint32_t hist_len, uint32_t Kp)
{
    hipLaunchKernelGGL(k_hist_join, dim3(grid, b.S), dim3(HIST_JOIN_BLOCK), 0, st, b.sd, b.work, b.chunk_tiles, pre,
                       suf, dglob, hist_len, Kp + 1);
    return hipGetLastError();
}

int hist_blocks_per_cu(int select_variant, uint32_t Kp, uint32_t block)
{
    return blocks_per_cu((const void*)hist_fn(select_variant), block, hist_lds_bytes(Kp, block));
}


// Range table of one series over the ascending boundaries es[0..kp) with rank
// base z: RANGE_TABLE buckets of 2^shift bit patterns (shift >= 4) from es[0]
// to es[kp-1]; each holds the first two boundaries inside it (x, y;
// 0x7FFFFFFF, above every key, when absent), z + the boundaries below it, and
// w = the count when more than two lie inside (compared one by one).  Called
// by a whole block.
__device__ void build_range_table(SeriesWork& w, const uint32_t* es, uint32_t kp, uint32_t z, uint4* tab,
                                  uint32_t* s_shift)
{
    if (threadIdx.x == 0) {
        uint32_t sh = 4;
        while (sh < 31 && (es[kp - 1] >> sh) - (es[0] >> sh) >= RANGE_TABLE) ++sh;
        *s_shift = sh;
        w.multi = 0u;  // set before the barrier; table entries below may raise it
    }
    __syncthreads();
    const uint32_t sh = *s_shift;
    const uint32_t emin = es[0], emax = es[kp - 1];
    for (uint32_t i = threadIdx.x; i < RANK_MAX; i += blockDim.x) w.esorted[i] = (i < kp) ? es[i] : 0xFFFFFFFFu;
    for (uint32_t i = threadIdx.x; i < RANK_MAX + 2; i += blockDim.x) { w.hrho[i] = 0; w.hlam[i] = 0; }
    if (threadIdx.x == 0) {
        w.Kp = kp;
        w.zbase = z;
        w.shift = sh;
        w.emin = emin;
        w.emax = emax;
    }
    const uint32_t a0 = emin >> sh, a1 = emax >> sh;
    for (uint32_t idx = threadIdx.x; idx < RANGE_TABLE; idx += blockDim.x) {
        const uint32_t a = a0 + ((idx - a0) & (RANGE_TABLE - 1));
        uint4 e = make_uint4(0x7FFFFFFFu, 0x7FFFFFFFu, z, 0u);
        if (a <= a1) {
            const uint64_t lo = (uint64_t)a << sh, hi = (uint64_t)(a + 1) << sh;
            const uint32_t below = count_below(es, kp, lo), inside = count_below(es, kp, hi) - below;
            e.x = inside >= 1 ? es[below] : 0x7FFFFFFFu;
            e.y = inside >= 2 ? es[below + 1] : 0x7FFFFFFFu;
            e.z = z + below;
            e.w = inside >= 3 ? inside : 0u;
            if (inside >= 3) w.multi = 1u;
        }
        tab[idx] = e;
    }
}

// Range sweep set-up.  Every target's key lies in a candidate range of
// 2^bits bit patterns starting at a_r, with rbase_r keys below it: after
// plain scan 2 (a_r = 21-bit prefix << SEL_B3, rbase = keys below the
// prefix) or after window scan 1 (a_r = fine-bin start, rbase = keys below
// the fine bin; a series with a target outside its window is left out).
// Distinct ranges are sorted, adjacent ones merge into groups, and the
// group boundaries (first value - 1, last value) form the rank table; the
// fine counters of the ranges are cleared.
__global__ void __launch_bounds__(PREP_THREADS) k_range_prep(const SeriesDesc* __restrict__ sds,
                                                    SeriesWork* __restrict__ works, uint2* __restrict__ rtab,
                                                    uint64_t* __restrict__ fineK, uint64_t* __restrict__ fineL,
                                                    uint32_t fine_stride, uint32_t window)
{
    __shared__ uint32_t es[RANK_MAX];
    __shared__ uint32_t sub[RQA_MAX_K];
    // the per-target inputs and the group arrays in LDS, worked on by one
    // thread per target or range (serially, each step would wait on a round
    // trip to memory or LDS)
    __shared__ uint32_t s_addr[RQA_MAX_K], s_tsub[RQA_MAX_K], s_tgroup[RQA_MAX_K];
    __shared__ uint32_t s_flag[RQA_MAX_K], s_gid[RQA_MAX_K];
    __shared__ uint32_t s_glo[RQA_MAX_K + 1], s_goff[RQA_MAX_K + 1];
    __shared__ uint32_t s_kp, s_z, s_shift, s_miss;
    const uint32_t s = blockIdx.x;
    const uint32_t K = sds[s].K;
    SeriesWork& w = works[s];
    const uint32_t bits = window ? w.win_shift : (uint32_t)SEL_B3;
    if (threadIdx.x == 0) s_miss = 0u;
    __syncthreads();
    // each target's range start and base count, loaded in parallel
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) {
        if (window) {
            if (!w.win_hit[r]) atomicOr(&s_miss, 1u);
            s_addr[r] = w.win_lo + (w.win_fbin[r] << bits);
            w.rbase[r] = w.win_base[r];
        } else {
            s_addr[r] = w.prefix[r] << SEL_B3;
            w.rbase[r] = w.below[r];
        }
    }
    __syncthreads();
    // series with a NaN or infinite sample end in an error; keep them out
    // (the same value on every thread)
    const bool ok = w.nonfinite == 0u && (!window || (w.win_ok != 0u && s_miss == 0u));
    uint32_t ns = 0, ng = 0;
    if (ok) {
        ns = block_sort_unique(s_addr, nullptr, K, sub, s_tsub, s_flag);
        // groups of adjacent ranges: a range starts a group unless it follows
        // the one before it directly
        const uint64_t width = 1ull << bits;
        const uint32_t j = threadIdx.x;
        const bool start = j < ns && (j == 0 || (uint64_t)sub[j] != (uint64_t)sub[j - 1] + width);
        if (j < ns) s_flag[j] = start ? 1u : 0u;
        ng = (uint32_t)__syncthreads_count(start);
        if (j < ns) {
            uint32_t gi = 0;  // starts after the first one, up to j
            for (uint32_t i = 1; i <= j; ++i) gi += s_flag[i];
            s_gid[j] = gi;
            if (start) {
                s_glo[gi] = sub[j];
                s_goff[gi] = j << bits;
            }
        }
        __syncthreads();
        if (j < K) s_tgroup[j] = s_gid[s_tsub[j]];
        // the rank table's boundaries, per group: its first value - 1 (unless
        // that value is 0, which only the first group can start at) and its
        // last value, in group order
        const uint32_t z = s_glo[0] == 0u ? 1u : 0u;
        if (j < ng) {
            const uint32_t glo = s_glo[j];
            const uint32_t nj = (j + 1 < ng ? (s_goff[j + 1] >> bits) : ns) - (s_goff[j] >> bits);
            // keys never exceed +inf
            const uint64_t last = (uint64_t)glo + ((uint64_t)nj << bits) - 1;
            const uint32_t at = j == 0 ? 0u : 2u * j - z;
            if (glo > 0u) es[at] = glo - 1u;
            es[at + (glo > 0u ? 1u : 0u)] = (uint32_t)(last < 0x7F800000ull ? last : 0x7F800000ull);
        }
        if (j == 0) {
            s_glo[ng] = 0;
            s_goff[ng] = 0;
            s_kp = 2u * ng - z;
            s_z = z;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        w.range_ok = ok ? 1u : 0u;
        w.range_bits = bits;
        if (ok) {
            w.nsub = ns;
            w.ngroups = ng;
        }
    }
    if (!ok) return;
    // the group and target arrays back to the series' working state
    for (uint32_t j = threadIdx.x; j < ns; j += blockDim.x) w.sub_lo[j] = sub[j];
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) {
        w.t_sub[r] = s_tsub[r];
        w.t_group[r] = s_tgroup[r];
    }
    for (uint32_t g = threadIdx.x; g <= ng; g += blockDim.x) {
        w.g_lo[g] = s_glo[g];
        w.g_off[g] = s_goff[g];
    }
    // clear the fine counters of the ranges
    const uint32_t nfine = ns << bits;
    uint64_t* fk = fineK + (size_t)s * fine_stride;
    uint64_t* fl = fineL + (size_t)s * fine_stride;
    for (uint32_t i = threadIdx.x; i < nfine; i += blockDim.x) {
        fk[i] = 0;
        fl[i] = 0;
    }
    build_range_table(w, es, s_kp, s_z, (uint4*)(rtab + (size_t)s * RHO_TABLE), &s_shift);
}

hipError_t launch_range_prep(hipStream_t st, const DevBufs& b, bool window)
{
    hipLaunchKernelGGL(k_range_prep, dim3(b.S), dim3(PREP_THREADS), 0, st, b.sd, b.work, b.rtab, b.fineK, b.fineL,
                       b.fine_stride, window ? 1u : 0u);
    return hipGetLastError();
}

// This thread's share of c[b, e) (indices b + threadIdx.x + m blockDim.x),
// eight loads issued before any is summed.
__device__ __forceinline__ uint64_t strided_sum(const uint64_t* __restrict__ c, uint32_t b, uint32_t e)
{
    uint64_t sum = 0;
    for (uint32_t i0 = b + threadIdx.x; i0 < e; i0 += 8 * blockDim.x) {
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            sum += i < e ? c[i] : 0ull;
        }
    }
    return sum;
}

// Threads of a range-scan workgroup (one per series and target).  A batch
// of many short series launches thousands of these small, latency-bound
// workgroups: 128 threads fit twice as many per CU as 256 (the 600-series
// ensemble's scan 285 -> 140 us) and cost a few series nothing (6.2 against
// 7.0 us for the two N = 1e5 series; 64 threads: 136 and 7.8 us).
constexpr uint32_t RANGE_SCAN_THREADS = 128;

// After the range sweep: per target, the fine counters of its range resolve
// the last bits of eps (rank k - rbase inside the range); C = rbase + the
// keys of the range up to eps; D = line values of rank below the target's
// group (line ranks 0 .. 2 g) + those from the group start up to eps.
__global__ void __launch_bounds__(RANGE_SCAN_THREADS) k_range_scan(const SeriesDesc* __restrict__ sds,
                                                    SeriesWork* __restrict__ works,
                                                    const uint64_t* __restrict__ fineK,
                                                    const uint64_t* __restrict__ fineL, uint32_t fine_stride)
{
    // workgroup (series, target)
    __shared__ uint64_t pre[RANGE_SCAN_THREADS + 1];
    __shared__ uint32_t s_c;
    __shared__ uint64_t s_run;
    const uint32_t s = blockIdx.x, r = blockIdx.y;
    SeriesWork& w = works[s];
    if (r >= sds[s].K || !w.range_ok) return;  // uniform over the workgroup
    const uint32_t bits = w.range_bits, width = 1u << bits;
    const uint64_t* fk = fineK + (size_t)s * fine_stride;
    const uint64_t* fl = fineL + (size_t)s * fine_stride;
    const uint32_t j = w.t_sub[r], gi = w.t_group[r];
    const uint32_t f0 = w.g_off[gi], fj = j << bits;
    // line values below the target's fine range: line-rank rows and fine bins
    uint64_t part = 0;
    for (uint32_t row = threadIdx.x; row < 2 * gi + 1; row += blockDim.x) part += w.hlam[row];
    part += strided_sum(fl, f0, fj);
    // the target's fine bin: first c with rbase + keys up to bin c >= k
    const uint64_t want = w.k[r] - w.rbase[r];
    chunk_prefix(fk + fj, width, pre);
    if (threadIdx.x < 64) {  // wave 0
        if (pre[blockDim.x] >= want) {
            uint64_t before;
            const uint32_t i = first_in_chunks(fk + fj, width, pre, want, &before);
            if (threadIdx.x == 0) {
                s_c = i;
                s_run = before;
            }
        } else if (threadIdx.x == 0) {
            s_c = width - 1;
            s_run = pre[blockDim.x];
            atomicOr(&w.status, 32u);
        }
    }
    __syncthreads();
    const uint32_t c = s_c;
    part += strided_sum(fl, fj, fj + c + 1);
    const uint64_t cl = block_sum(part);
    if (threadIdx.x == 0) {
        w.eps_bits[r] = w.sub_lo[j] + c;
        w.count[r] = w.rbase[r] + s_run + fk[fj + c];
        w.dcount[r] = cl;
    }
}

hipError_t launch_range_scan(hipStream_t st, const DevBufs& b)
{
    hipLaunchKernelGGL(k_range_scan, dim3(b.S, b.K), dim3(RANGE_SCAN_THREADS), 0, st, b.sd, b.work, b.fineK, b.fineL, b.fine_stride);
    return hipGetLastError();
}


// ------------------------------------------------------------------ window selection

// Window of key bit patterns [lo, hi] (clamped to [0, +inf]) -> the smallest
// fine-bin shift that covers it with WIN_BINS bins; unusable if the shift
// exceeds WIN_MAX_SHIFT.
__device__ void set_window(SeriesWork& w, int64_t lo, int64_t hi, bool valid)
{
    lo = lo < 0 ? 0 : lo;
    hi = hi > 0x7F800000ll ? 0x7F800000ll : hi;
    w.win_below = 0;
    w.win_nslots = 0;
    if (!valid || hi < lo) {
        w.win_ok = 0u;
        w.win_lo = 0u;
        w.win_span = 0u;
        w.win_shift = 0u;
        return;
    }
    const uint32_t span = (uint32_t)(hi - lo);
    // at least 2: window pass 1 forms a bin's byte offset as a right shift
    // by win_shift - 2 and a mask
    uint32_t sh = 2;
    while (sh < 31 && (span >> sh) >= WIN_BINS) ++sh;
    w.win_lo = (uint32_t)lo;
    w.win_span = span;
    w.win_shift = sh;
    // window pass 1 counts keys below the window in the fine bin below its
    // start, so the start must be at least one fine bin above key 0 (keys
    // that small are denormals or zeros; such series take the plain passes)
    w.win_ok = (sh <= WIN_MAX_SHIFT && (uint64_t)lo >= (1ull << sh)) ? 1u : 0u;
}

// Window from predicted offsets t_r (network output) and half-widths d_r:
// [scale + (t_r - d_r) 2^23, scale + (t_r + d_r) 2^23] over all outputs.
__global__ void k_window_from_offsets(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works, uint32_t S,
                                      const float* __restrict__ pred, const float* __restrict__ delta, int nout)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    SeriesWork& w = works[s];
    const double sc = (double)w.scale;
    double lo = 1e300, hi = -1e300;
    bool valid = true;
    for (int r = 0; r < nout; ++r) {
        const double t = pred[(size_t)s * nout + r], d = delta[r];
        valid &= isfinite(t);
        lo = fmin(lo, sc + floor((t - d) * 8388608.0));
        hi = fmax(hi, sc + ceil((t + d) * 8388608.0));
    }
    valid &= lo > -4.0e9 && hi < 4.0e9;
    set_window(w, valid ? (int64_t)lo : 0, valid ? (int64_t)hi : -1, valid);
}

// Window from the sorted sketch sample: for each target rate q = k/M, the
// sample keys at ranks q P -/+ z sqrt(P q (1 - q)) (one more below), over
// all targets.  One wave per series, a lane per target (each lane's loads
// depend on its target's count, so one thread walking the targets would wait
// on two memory round trips per target); the bounds meet in a wave min / max.
__global__ void __launch_bounds__(64) k_window_from_sample(const SeriesDesc* __restrict__ sds,
                                                           SeriesWork* __restrict__ works, uint32_t S,
                                                           const uint32_t* __restrict__ sample, float z)
{
    const uint32_t s = blockIdx.x;
    if (s >= S) return;  // uniform over the wave
    SeriesWork& w = works[s];
    const uint32_t* smp = sample + (size_t)s * SKETCH_P;
    const uint32_t K = sds[s].K;
    const double M = (double)sds[s].M;
    long long lo = 0x7F800000ll, hi = 0;
    for (uint32_t r = threadIdx.x; r < K; r += 64) {
        const double q = (double)w.k[r] / M;
        const double c = q * SKETCH_P, sd = sqrt(SKETCH_P * q * (1.0 - q)) * z;
        const int ilo = (int)floor(c - sd) - 1, ihi = (int)ceil(c + sd);
        lo = min(lo, ilo < 0 ? 0ll : (long long)smp[ilo]);
        hi = max(hi, ihi >= (int)SKETCH_P ? 0x7F800000ll : (long long)smp[ihi]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
    }
    if (threadIdx.x == 0) set_window(w, lo, hi, true);
}

// A window given by the caller, the same for every series.
__global__ void k_window_fixed(SeriesWork* __restrict__ works, uint32_t S, uint32_t lo, uint32_t hi)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) set_window(works[s], (int64_t)lo, (int64_t)hi, true);
}

hipError_t launch_window_fixed(hipStream_t st, const DevBufs& b, uint32_t lo, uint32_t hi)
{
    hipLaunchKernelGGL(k_window_fixed, dim3((b.S + 63) / 64), dim3(64), 0, st, b.work, b.S, lo, hi);
    return hipGetLastError();
}

hipError_t launch_window_from_offsets(hipStream_t st, const DevBufs& b, const float* pred, const float* delta_dev)
{
    hipLaunchKernelGGL(k_window_from_offsets, dim3((b.S + 63) / 64), dim3(64), 0, st, b.sd, b.work, b.S, pred, delta_dev,
                       20);
    return hipGetLastError();
}

hipError_t launch_window_from_sample(hipStream_t st, const DevBufs& b, const uint32_t* sample_sorted, const double*,
                                     float z)
{
    hipLaunchKernelGGL(k_window_from_sample, dim3(b.S), dim3(64), 0, st, b.sd, b.work, b.S, sample_sorted, z);
    return hipGetLastError();
}

// Window pass 1: count keys below the window and histogram the window in
// WIN_BINS fine bins.
template <int NORM, int MC, int TC>
struct WinPass1 {
    uint32_t* bins;       // LDS [1 + WIN_BINS]: [0] keys below the window, [1 + f] fine bin f
    uint64_t* gbins;      // global [S][WIN_BINS]
    SeriesWork* works;
    uint32_t base;        // win_lo - 2^shift: the key one fine bin below the window start
    uint32_t hi, shift, sh2;
    bool active = true;
    __device__ void begin(uint32_t s)
    {
        const SeriesWork& w = works[s];
        const uint32_t lo = uniform(w.win_lo);
        shift = uniform(w.win_shift);
        sh2 = shift - 2u;
        hi = lo + uniform(w.win_span);
        base = lo - (1u << shift);  // the window set-up keeps win_lo >= 2^shift
        sh2 = in_vgpr(sh2);
        base = in_vgpr(base);
        active = uniform(w.win_ok) != 0;
        for (uint32_t i = threadIdx.x; i <= WIN_BINS; i += blockDim.x) bins[i] = 0u;
    }
    __device__ void flush(uint32_t s)
    {
        if (!active) return;
        for (uint32_t i = threadIdx.x; i < WIN_BINS; i += blockDim.x) {
            const uint32_t v = bins[1 + i];
            if (v) atomicAdd((unsigned long long*)&gbins[(size_t)s * WIN_BINS + i], (unsigned long long)v);
        }
        if (threadIdx.x == 0 && bins[0]) atomicAdd((unsigned long long*)&works[s].win_below, (unsigned long long)bins[0]);
    }
    __device__ __forceinline__ uint32_t look(uint32_t) const { return 0u; }
    // Keys at most the window end count in LDS bin (key - base) >> shift,
    // saturated at 0: every key below the window start lands in bin 0 and a
    // window key v in bin ((v - win_lo) >> shift) + 1.  A branch: most keys
    // lie above the window, and an atomic per key would cost more than the
    // divergence.
    __device__ __forceinline__ void count(uint32_t u, uint32_t)
    {
        // the bins sit at LDS byte 0 (k_window checks it): the bin's byte
        // offset is its LDS address
        if (u <= hi) {
            const uint32_t a = (__builtin_elementwise_sub_sat(u, base) >> sh2) & ~3u;
            __hip_atomic_fetch_add((__attribute__((address_space(3))) uint32_t*)(size_t)a, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        select_tile<NORM, MC, TC>(sd, tile_id, lane, *this);
    }
};

// Window pass 2: keys in a target's fine bin add to that bin's 2^shift
// sub-bins in global memory (few keys qualify).
template <int NORM, int MC, int TC>
struct WinPass2 {
    uint8_t* table;       // LDS [WIN_BINS] fine bin -> slot
    const uint8_t* gtable;
    uint64_t* fine;       // global [S][K][1 << WIN_MAX_SHIFT]
    SeriesWork* works;
    uint32_t K;
    uint32_t lo, span, shift;
    unsigned long long* dst;
    bool active = true;
    __device__ void begin(uint32_t s)
    {
        const SeriesWork& w = works[s];
        lo = uniform(w.win_lo);
        span = uniform(w.win_span);
        shift = uniform(w.win_shift);
        active = uniform(w.win_ok) != 0 && uniform(w.win_nslots) != 0;
        for (uint32_t i = threadIdx.x; i < WIN_BINS; i += blockDim.x) table[i] = gtable[(size_t)s * WIN_BINS + i];
        dst = (unsigned long long*)(fine + (size_t)s * K * (1u << WIN_MAX_SHIFT));
    }
    __device__ void flush(uint32_t) {}
    __device__ __forceinline__ uint32_t look(uint32_t u) const
    {
        const uint32_t rel = u - lo;
        const uint32_t fb = min(rel >> shift, WIN_BINS - 1);
        const uint32_t sl = table[fb];
        return rel <= span ? sl : (uint32_t)NO_SLOT;
    }
    __device__ __forceinline__ void count(uint32_t u, uint32_t sl) const
    {
        const uint32_t sub = (u - lo) & ((1u << shift) - 1u);
        wave_add(dst, sl * (1u << WIN_MAX_SHIFT) + sub, sl != NO_SLOT);
    }
    __device__ void tile(const SeriesScalars& sd, uint32_t tile_id, int lane)
    {
        select_tile<NORM, MC, TC>(sd, tile_id, lane, *this);
    }
};

__host__ __device__ __forceinline__ size_t window_lds_bytes_dev(int pass) { return (pass == 1 ? (WIN_BINS + 1) * 4 : WIN_BINS) + 16; }

size_t window_lds_bytes(int pass) { return window_lds_bytes_dev(pass); }

template <int PASS, int NORM, int MC, int TC>
__global__ void __launch_bounds__(1024)
k_window(const SeriesDesc* __restrict__ sds, uint32_t S, uint32_t nchunks, uint32_t chunk_tiles,
         uint32_t* __restrict__ ticket, SeriesWork* __restrict__ works, uint64_t* __restrict__ bins,
         const uint8_t* __restrict__ table, uint64_t* __restrict__ fine, uint32_t K)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* slot = (uint32_t*)(smem + window_lds_bytes_dev(PASS) - 16);
    if constexpr (PASS == 1) {
        // WinPass1 addresses its bins by their offset from LDS byte 0: the
        // kernel's dynamic LDS must start there (it has no static LDS); a
        // launch where it does not marks every series (a device error)
        if ((uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char*)smem != 0u) {
            if (threadIdx.x == 0)
                for (uint32_t s = 0; s < S; ++s) atomicOr(&works[s].status, 64u);
            return;
        }
        WinPass1<NORM, MC, TC> body;
        body.bins = (uint32_t*)smem;
        body.gbins = bins;
        body.works = works;
        chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, slot);
    } else {
        WinPass2<NORM, MC, TC> body;
        body.table = (uint8_t*)smem;
        body.gtable = table;
        body.fine = fine;
        body.works = works;
        body.K = K;
        body.dst = nullptr;
        chunk_loop(sds, S, nchunks, chunk_tiles, ticket, body, slot);
    }
}

using WinFn = void (*)(const SeriesDesc*, uint32_t, uint32_t, uint32_t, uint32_t*, SeriesWork*, uint64_t*,
                       const uint8_t*, uint64_t*, uint32_t);

template <int PASS, int NORM>
static WinFn window_fn_n(int mclass)
{
    switch (mclass) {
    case 1: return k_window<PASS, NORM, 1, 0>;
    case 2: return k_window<PASS, NORM, 3, 3>;
    case 3: return k_window<PASS, NORM, 3, 5>;
    default: return k_window<PASS, NORM, 0, 0>;
    }
}

static WinFn window_fn(int pass, int variant)
{
    const int norm = variant / NUM_MCLASS, mc = variant % NUM_MCLASS;
    if (pass == 1)
        return norm == RQA_NORM_MAX ? window_fn_n<1, RQA_NORM_MAX>(mc) : window_fn_n<1, RQA_NORM_EUCLIDEAN>(mc);
    return norm == RQA_NORM_MAX ? window_fn_n<2, RQA_NORM_MAX>(mc) : window_fn_n<2, RQA_NORM_EUCLIDEAN>(mc);
}

hipError_t launch_window_pass(hipStream_t st, const DevBufs& b, const WinBufs& w, int pass, int variant, uint32_t grid,
                              uint32_t block, uint32_t ticket)
{
    hipLaunchKernelGGL(window_fn(pass, variant), dim3(grid), dim3(block), window_lds_bytes(pass), st, b.sd, b.S,
                       b.nchunks, b.chunk_tiles, b.tickets + ticket, b.work, w.bins, w.table, w.fine, b.K);
    return hipGetLastError();
}

int window_blocks_per_cu(int pass, int variant, uint32_t block)
{
    return blocks_per_cu((const void*)window_fn(pass, variant), block, window_lds_bytes(pass));
}

// After window pass 1: per target, hit if its rank falls inside the window;
// its fine bin and the count below that bin; pass-2 slots and table.
__global__ void __launch_bounds__(1024) k_window_scan1(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                                                       uint64_t* __restrict__ bins, uint8_t* __restrict__ table,
                                                       uint64_t* __restrict__ fine, uint32_t clear_fine)
{
    // up to 1024 threads (each then sums 39 of the 39,936 fine bins)
    __shared__ uint64_t pre[1025];
    __shared__ uint32_t uniq[RQA_MAX_K], s_pos[RQA_MAX_K], s_flag[RQA_MAX_K];
    __shared__ uint32_t s_hit[RQA_MAX_K], s_fbin[RQA_MAX_K];
    const uint32_t s = blockIdx.x;
    const uint32_t K = sds[s].K;
    SeriesWork& w = works[s];
    uint8_t* tb = table + (size_t)s * WIN_BINS;
    for (uint32_t i = threadIdx.x; i < WIN_BINS; i += blockDim.x) tb[i] = NO_SLOT;
    const bool ok = w.win_ok != 0;
    const uint64_t below = w.win_below;
    const uint64_t* cb = bins + (size_t)s * WIN_BINS;
    chunk_prefix(cb, WIN_BINS, pre);
    const uint64_t total = pre[blockDim.x];
    // one wave per target
    for (uint32_t r = threadIdx.x >> 6; r < K; r += blockDim.x >> 6) {
        const uint64_t k = w.k[r];
        const bool hit = ok && k > below && k - below <= total;
        uint32_t fb = 0;
        uint64_t before = 0;
        if (hit) fb = first_in_chunks(cb, WIN_BINS, pre, k - below, &before);
        if ((threadIdx.x & 63) == 0) {
            w.win_hit[r] = hit ? 1u : 0u;
            s_hit[r] = hit ? 1u : 0u;
            s_fbin[r] = fb;
            if (hit) {
                w.win_fbin[r] = fb;
                w.win_base[r] = below + before;
            }
        }
    }
    __syncthreads();
    const uint32_t nu = block_sort_unique(s_fbin, s_hit, K, uniq, s_pos, s_flag);
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x)
        w.win_slot[r] = s_hit[r] ? s_pos[r] : (uint32_t)NO_SLOT;
    __syncthreads();
    for (uint32_t u = threadIdx.x; u < nu; u += blockDim.x) tb[uniq[u]] = (uint8_t)u;
    if (threadIdx.x == 0) w.win_nslots = nu;
    // clear the sub-bins window pass 2 will count into
    if (clear_fine) {
        const uint32_t nsub = 1u << w.win_shift;
        uint64_t* f = fine + (size_t)s * K * (1u << WIN_MAX_SHIFT);
        for (uint32_t u = 0; u < nu; ++u)
            for (uint32_t i = threadIdx.x; i < nsub; i += blockDim.x) f[(size_t)u * (1u << WIN_MAX_SHIFT) + i] = 0;
    }
}

// After window pass 2: the sub-bin of each hit target gives its threshold;
// count = #{key <= eps}.
__global__ void __launch_bounds__(256) k_window_scan2(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                                                      const uint64_t* __restrict__ fine)
{
    // workgroup (series, target)
    __shared__ uint64_t pre[257];
    const uint32_t s = blockIdx.x, r = blockIdx.y;
    const uint32_t K = sds[s].K;
    SeriesWork& w = works[s];
    if (r >= K || !w.win_hit[r]) return;  // uniform over the workgroup
    const uint32_t nsub = 1u << w.win_shift;
    const uint64_t* c = fine + ((size_t)s * K + w.win_slot[r]) * (1u << WIN_MAX_SHIFT);
    const uint64_t want = w.k[r] - w.win_base[r];
    chunk_prefix(c, nsub, pre);
    if (threadIdx.x < 64) {  // wave 0
        if (pre[blockDim.x] >= want) {
            uint64_t before;
            const uint32_t idx = first_in_chunks(c, nsub, pre, want, &before);
            if (threadIdx.x == 0) {
                w.eps_bits[r] = w.win_lo + (w.win_fbin[r] << w.win_shift) + idx;
                w.count[r] = w.win_base[r] + before + c[idx];
            }
        } else if (threadIdx.x == 0) {
            w.win_hit[r] = 0u;
            atomicOr(&w.status, 8u);
        }
    }
}

hipError_t launch_window_scan(hipStream_t st, const DevBufs& b, const WinBufs& w, int pass)
{
    // scan 1 clears the fine counters of window pass 2 unless the range sweep
    // (which clears its own) follows
    if (pass == 1)
        // few series: 1024 threads share each series' bins; many: 256, so
        // that several series' workgroups share a CU
        hipLaunchKernelGGL(k_window_scan1, dim3(b.S), dim3(b.S <= 128 ? 1024 : 256), 0, st, b.sd, b.work, w.bins, w.table, w.fine,
                           w.fine ? 1u : 0u);
    else hipLaunchKernelGGL(k_window_scan2, dim3(b.S, b.K), dim3(256), 0, st, b.sd, b.work, w.fine);
    return hipGetLastError();
}

// ------------------------------------------------------------------ sketch

// SplitMix64 output for counter s of stream `seed` (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t s)
{
    uint64_t z = seed + (s + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One workgroup per series: SKETCH_P pairs drawn uniformly (counter-based
// SplitMix64, pair index v mod M in diagonal-major order), their keys sorted
// in LDS, the median as scale, and the histogram of (bits - scale) >> 21
// clamped to SKETCH_BINS quarter-binade bins.
constexpr uint32_t SKETCH_THREADS = 1024;
__global__ void __launch_bounds__(SKETCH_THREADS) k_sketch(const SeriesDesc* __restrict__ sds, SeriesWork* __restrict__ works,
                                                float* __restrict__ features, uint32_t* __restrict__ sample_sorted)
{
    __shared__ uint32_t keys[SKETCH_P];
    __shared__ uint32_t keys2[SKETCH_P];
    __shared__ uint32_t hist[SKETCH_BINS];
    const uint32_t s = blockIdx.x;
    const SeriesDesc& sd = sds[s];
    const uint64_t M = sd.M;
    const uint64_t L0 = (uint64_t)sd.nv - sd.w;
    for (uint32_t i = threadIdx.x; i < SKETCH_BINS; i += blockDim.x) hist[i] = 0u;
    for (uint32_t q = threadIdx.x; q < (uint32_t)SKETCH_P; q += blockDim.x) {
        const uint64_t p = splitmix64(sd.seed, q) % M;
        // diagonal offset dl: the largest with C(dl) = dl*L0 - dl(dl-1)/2 <= p
        auto C = [&](uint64_t dl) { return dl * L0 - (dl * (dl - 1)) / 2; };
        const double b = 2.0 * (double)L0 + 1.0;
        const double disc = b * b - 8.0 * (double)p;
        double est = 0.5 * (b - sqrt(disc > 0.0 ? disc : 0.0));
        uint64_t dl = est > 0.0 ? (uint64_t)est : 0;
        if (dl > L0 - 1) dl = L0 - 1;
        while (dl > 0 && C(dl) > p) --dl;
        while (dl + 1 < L0 && C(dl + 1) <= p) ++dl;
        const int t = (int)(p - C(dl));
        const int j = t + (int)sd.w + (int)dl;
        const float key = sd.norm == RQA_NORM_MAX ? pair_key<RQA_NORM_MAX, 0, 0>(sd.y, t, j, sd.m, sd.tau)
                                                  : pair_key<RQA_NORM_EUCLIDEAN, 0, 0>(sd.y, t, j, sd.m, sd.tau);
        keys[q] = __float_as_uint(key);
    }
    __syncthreads();
    // bitonic sort of the sampled key bits, ascending.  Thread t holds
    // elements 4t .. 4t+3 in registers: partners at distance 1 and 2 are in
    // the same thread, at 4 .. 128 in another lane of the same wave
    // (shuffles), and only the ten stages at 256 .. 2048 go through LDS (two
    // buffers, one barrier each).
    static_assert(SKETCH_P == 4 * SKETCH_THREADS, "four sample keys per thread");
    const uint32_t t = threadIdx.x;
    uint32_t x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = keys[4 * t + c];
    int cur = 0;
    __syncthreads();
    for (uint32_t k = 2; k <= (uint32_t)SKETCH_P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (j >= 4 * 64) {
                uint32_t* buf = cur ? keys2 : keys;
#pragma unroll
                for (int c = 0; c < 4; ++c) buf[4 * t + c] = x[c];
                __syncthreads();
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint32_t i = 4 * t + c, b = buf[i ^ j];
                    const bool keep_min = ((i & k) == 0) == ((i & j) == 0);
                    x[c] = keep_min ? min(x[c], b) : max(x[c], b);
                }
                cur ^= 1;
            } else if (j >= 4) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint32_t i = 4 * t + c, b = (uint32_t)__shfl_xor((int)x[c], (int)(j >> 2));
                    const bool keep_min = ((i & k) == 0) == ((i & j) == 0);
                    x[c] = keep_min ? min(x[c], b) : max(x[c], b);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if ((c & (int)j) == 0) {
                        const uint32_t i = 4 * t + c;
                        const uint32_t a = x[c], b = x[c | (int)j];
                        const bool up = (i & k) == 0;
                        x[c] = up ? min(a, b) : max(a, b);
                        x[c | (int)j] = up ? max(a, b) : min(a, b);
                    }
                }
            }
        }
    }
    // the sorted keys back to LDS, once every thread has read its last
    // partner there
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) keys[4 * t + c] = x[c];
    __syncthreads();
    const uint32_t scale = keys[SKETCH_P / 2 - 1];
    for (uint32_t q = threadIdx.x; q < (uint32_t)SKETCH_P; q += blockDim.x) {
        int idx = (int)(((int64_t)keys[q] - (int64_t)scale) >> 21) + SKETCH_BINS / 2;
        idx = min(max(idx, 0), SKETCH_BINS - 1);
        atomicAdd(&hist[idx], 1u);
        if (sample_sorted) sample_sorted[(size_t)s * SKETCH_P + q] = keys[q];
    }
    __syncthreads();
    float* f = features + (size_t)s * SKETCH_FEATURES;
    for (uint32_t i = threadIdx.x; i < SKETCH_BINS; i += blockDim.x) f[i] = (float)hist[i] * (1.0f / SKETCH_P);
    if (threadIdx.x == 0) {
        f[SKETCH_BINS] = sd.f_logn;
        f[SKETCH_BINS + 1] = sd.f_m;
        works[s].scale = scale;
    }
}

hipError_t launch_sketch(hipStream_t st, const DevBufs& b, float* features, uint32_t* sample_sorted)
{
    // 1024 threads: four sample keys per thread through the 78 bitonic stages
    hipLaunchKernelGGL(k_sketch, dim3(b.S), dim3(SKETCH_THREADS), 0, st, b.sd, b.work, features, sample_sorted);
    return hipGetLastError();
}

hipError_t set_kernel_lds_limits(size_t max_dyn_lds)
{
    hipError_t err = hipSuccess;
    auto set = [&](const void* f) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn_lds);
        if (e != hipSuccess) err = e;
    };
    for (int v = 0; v < NUM_SELECT_VARIANTS; ++v) {
        for (int p = 1; p <= 3; ++p) set((const void*)select_fn_pass(p, v));
        for (int p = 1; p <= 2; ++p) set((const void*)window_fn(p, v));
        for (int l = 0; l < 3; ++l) {
            set((const void*)sweep_fn(v * 3 + l));
            set((const void*)range_fn(v * 3 + l));
        }
        set((const void*)hist_fn(v));
    }
    return err;
}

}  // namespace rqa
