// capi.hip -- host runtime and C ABI of the averaged-RQA library (include/rqa.h).
//
// A call builds one descriptor per series, uploads it with the targets, and
// runs the phases on the context stream without a host round trip:
//   finite check -> [selection: pass 1, scan 1, pass 2, scan 2, pass 3, scan 3]
//   -> [sweep: rank tables, line sweep] -> one copy of the results to the host.
// The host then turns the integer counts into RR, DET and the averaged DET in
// double precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp.h"

using namespace rqa;

namespace {

thread_local char g_err[512] = "";

rqa_status fail(rqa_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(RQA_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

// Device scratch of rqa_batch_static, for callers that cannot allocate
// device memory.  Each GPU holds its own copy of this array from the first
// use of the library on it until the process ends.  Host code never passes
// the array's name to a kernel or a copy: it holds a host-side stand-in, not
// a device address.  The device address of each GPU's copy is resolved once
// per device with hipGetSymbolAddress (resolve_static_scratch, called by
// rqa_create) and only that address is used.
constexpr size_t STATIC_SCRATCH_BYTES = RQA_STATIC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// Device address of `device`'s copy of the static scratch; the device must
// be current.
rqa_status resolve_static_scratch(int device, void** out)
{
    if (device < 0 || device >= MAX_DEVICES)
        return fail(RQA_ERR_UNSUPPORTED, "device %d: the static scratch serves devices 0..%d", device, MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(RQA_ERR_DEVICE, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
        }
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return RQA_OK;
}

enum Phase { PH_P1 = 0, PH_P2 = 1, PH_P3 = 2, PH_SWEEP = 3, PH_OTHER = 4, PH_HIST = 5, PH_N = 6 };

// Size bucket of the autotuner: log2 of the number of vectors, the kernel
// variant (norm, embedding class, line class) and K up to 32 or beyond.  The
// bucket with nvlog2 = -1 holds the chunk size of multi-series calls.
struct TuneKey {
    int nvlog2, variant, kcls;
    bool operator<(const TuneKey& o) const
    {
        if (nvlog2 != o.nvlog2) return nvlog2 < o.nvlog2;
        if (variant != o.variant) return variant < o.variant;
        return kcls < o.kcls;
    }
};
struct Shape {
    uint32_t seg, chunk;
};

}  // namespace

struct rqa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cu = 256;
    size_t max_lds = 65536;
    uint32_t seg = 0;          // segment length override (0: tuned table or heuristic)
    uint32_t chunk_tiles = 0;  // chunk size override (0: tuned table or heuristic)
    uint32_t grid = 0;         // workgroups per launch override (0: automatic)
    std::map<TuneKey, Shape> tune;  // autotuned shapes per size bucket
    // threshold-bracket network: device params | grad | Adam m | Adam v
    float* mlp = nullptr;
    float* mlp_acts = nullptr;   // activations for up to mlp_cap rows
    uint32_t mlp_cap = 0;
    float* mlp_partial = nullptr;
    uint64_t adam_t = 0;
    bool has_model = false;
    float sample_z = 5.0f;       // width of the sample-quantile window in standard deviations
    uint32_t win_lo = 0, win_hi = 0x7F800000u;  // caller-given window (RQA_SEL_WINDOW)
    // statistics of the last selection: full counting passes over all pairs,
    // series that fell back to the plain path, targets outside their window
    uint32_t stat_passes = 0, stat_fallback = 0, stat_missed = 0;
    float bracket_delta[MLP_OUT] = {};  // calibrated half-widths of the bracket (offset units)
    // device pool
    void* pool = nullptr;
    size_t pool_bytes = 0;
    // host staging (pinned)
    void* host = nullptr;
    size_t host_bytes = 0;
    // rqa_batch_static: this device's copy of the static scratch area (its
    // device address, resolved once per device), and, while such a call
    // runs, use_static = true: the call's device scratch comes from that
    // area and its host staging from static_host (ordinary host memory)
    void* static_dev = nullptr;
    bool use_static = false;
    std::vector<unsigned char> static_host;
    // second stream (default priority) and fork/join events: the variant
    // groups of one phase run concurrently, the first on the context stream
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // timing
    bool timing = false;
    hipEvent_t ev[2 * PH_N * 8] = {};
    bool ev_ready = false;
    double phase_ms[PH_N] = {};
};

namespace {

struct Series {
    uint64_t offset;  // element offset into the device buffer
    uint64_t n;
    rqa_params p;
};

rqa_status check_params(const rqa_params* p, uint64_t n, uint64_t* nv_out, uint64_t* M_out)
{
    if (!p) return fail(RQA_ERR_INVALID_ARG, "params is NULL");
    if (p->m == 0 || p->tau == 0) return fail(RQA_ERR_INVALID_ARG, "m and tau must be >= 1");
    if (p->theiler == 0) return fail(RQA_ERR_INVALID_ARG, "theiler window must be >= 1");
    if (p->lmin == 0 || p->lmin > (uint32_t)LMIN_MAX)
        return fail(p->lmin == 0 ? RQA_ERR_INVALID_ARG : RQA_ERR_UNSUPPORTED, "lmin must be in 1..%d", LMIN_MAX);
    if (p->norm != RQA_NORM_MAX && p->norm != RQA_NORM_EUCLIDEAN)
        return fail(RQA_ERR_INVALID_ARG, "unknown norm %u", p->norm);
    if (n >= (1ull << 31)) return fail(RQA_ERR_UNSUPPORTED, "series length must be < 2^31");
    const uint64_t span = (uint64_t)(p->m - 1) * p->tau;
    const uint64_t nv = span < n ? n - span : 0;
    if (nv <= p->theiler) return fail(RQA_ERR_TOO_SHORT, "%llu vectors leave no pair beyond the Theiler window",
                                      (unsigned long long)nv);
    const uint64_t a = nv - p->theiler;
    *nv_out = nv;
    *M_out = a * (a + 1) / 2;
    return RQA_OK;
}

// k = ceil(q * M / 1e9) with q = round(rr * 1e9), clamped to [1, M].
rqa_status target_rank(double rr, uint64_t M, uint64_t* k)
{
    if (!(rr > 0.0) || !(rr <= 1.0)) return fail(RQA_ERR_INVALID_ARG, "RR target %g outside (0, 1]", rr);
    long long q = llround(rr * 1e9);
    q = std::min(std::max(q, 1LL), 1000000000LL);
    const unsigned __int128 prod = (unsigned __int128)(uint64_t)q * M;
    uint64_t kk = (uint64_t)((prod + 999999999u) / 1000000000u);
    *k = std::min(std::max<uint64_t>(kk, 1), M);
    return RQA_OK;
}

rqa_status check_eps(float e, uint32_t* bits)
{
    if (std::isnan(e)) return fail(RQA_ERR_INVALID_ARG, "threshold is NaN");
    if (e < 0.0f) return fail(RQA_ERR_INVALID_ARG, "threshold %g is negative", (double)e);
    if (e == 0.0f) e = 0.0f;  // -0 -> +0
    std::memcpy(bits, &e, 4);
    return RQA_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int log2_floor(uint64_t v)
{
    int l = 0;
    while (v >>= 1) ++l;
    return l;
}

TuneKey tune_key(uint64_t nv, const rqa_params& p, uint32_t K)
{
    return {log2_floor(nv), variant_of(p.norm, p.m, p.tau, p.lmin), K <= 32 ? 0 : 1};
}

// Default segment length when nothing is tuned: about 16 segments per series,
// a power of two between 64 and 1024.
uint32_t default_segment(uint64_t L0)
{
    uint64_t t = 64;
    while (t * 2 <= L0 / 16 && t < 1024) t *= 2;
    return (uint32_t)t;
}

constexpr uint32_t DEFAULT_CHUNK = 8;

uint32_t segment_for(const rqa_ctx* c, uint64_t nv, const rqa_params& p, uint32_t K)
{
    if (c->seg) return c->seg;
    auto it = c->tune.find(tune_key(nv, p, K));
    if (it != c->tune.end()) return it->second.seg;
    return default_segment(nv - p.theiler);
}

// The threshold sweep runs 1024-thread workgroups when its LDS (rank table,
// per-lane histograms of K + 1 rows) admits only one workgroup per CU: at
// K = 99 on two N = 1e5 series 6.1 -> 4.5 ms.
bool wide_sweep(const rqa_ctx* c, uint32_t K) { return sweep_lds_bytes(K, false) * 2 > c->max_lds; }

// Segment of the histogram pass: the caller's override (at most
// HIST_MAX_SEG_HOST), else about 96 segments on the longest diagonal
// (256 .. 4096).
uint32_t hist_segment_for(const rqa_ctx* c, uint64_t L0)
{
    if (c->seg) return std::min<uint32_t>(c->seg, HIST_MAX_SEG_HOST);
    const uint64_t t = (L0 + 95) / 96;
    return (uint32_t)std::min<uint64_t>(std::max<uint64_t>((t + TILE_W - 1) / TILE_W * TILE_W, 256), 4096);
}

uint32_t chunk_for(const rqa_ctx* c, uint32_t S, uint64_t nv0, const rqa_params& p0, uint32_t K)
{
    if (c->chunk_tiles) return c->chunk_tiles;
    const TuneKey key = S == 1 ? tune_key(nv0, p0, K) : TuneKey{-1, 0, K <= 32 ? 0 : 1};
    auto it = c->tune.find(key);
    if (it != c->tune.end()) return it->second.chunk;
    return DEFAULT_CHUNK;
}

rqa_status ensure_pool(rqa_ctx* c, size_t bytes)
{
    if (c->pool_bytes >= bytes) return RQA_OK;
    const size_t want = std::max(bytes, c->pool_bytes * 3 / 2);
    if (c->pool) (void)hipFree(c->pool);
    c->pool = nullptr;
    c->pool_bytes = 0;
    if (hipMalloc(&c->pool, want) != hipSuccess) {
        c->pool = nullptr;
        (void)hipGetLastError();
        return fail(RQA_ERR_NOMEM, "hipMalloc of %zu bytes of scratch failed", want);
    }
    c->pool_bytes = want;
    return RQA_OK;
}

rqa_status ensure_host(rqa_ctx* c, size_t bytes)
{
    if (c->host_bytes >= bytes) return RQA_OK;
    if (c->host) (void)hipHostFree(c->host);
    c->host = nullptr;
    c->host_bytes = 0;
    if (hipHostMalloc(&c->host, bytes, hipHostMallocDefault) != hipSuccess) {
        c->host = nullptr;
        (void)hipGetLastError();
        return fail(RQA_ERR_NOMEM, "hipHostMalloc of %zu bytes failed", bytes);
    }
    c->host_bytes = bytes;
    return RQA_OK;
}

void reset_phases(rqa_ctx* c)
{
    for (int i = 0; i < PH_N; ++i) c->phase_ms[i] = 0.0;
}

struct Timer {
    rqa_ctx* c;
    int used = 0;
    int phase[PH_N * 8];
    Timer(rqa_ctx* ctx) : c(ctx) {}
    hipError_t begin(int ph)
    {
        if (!c->timing || used >= PH_N * 8) return hipSuccess;
        phase[used] = ph;
        return hipEventRecord(c->ev[2 * used], c->stream);
    }
    hipError_t end()
    {
        if (!c->timing || used >= PH_N * 8) return hipSuccess;
        hipError_t e = hipEventRecord(c->ev[2 * used + 1], c->stream);
        ++used;
        return e;
    }
    // adds this job's phase times to the call's totals (reset at the start
    // of every computing entry point)
    void collect()
    {
        if (!c->timing) return;
        for (int i = 0; i < used; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) c->phase_ms[phase[i]] += ms;
        }
    }
};

// MODE_FUSED: counting passes, then the range sweep, which resolves the
// last bits of every threshold and counts C and D at it in one pass.
// MODE_BOTH: three counting passes, then the sweep at the thresholds found.
// MODE_HIST: full line-length histogram at given thresholds (whole-diagonal
// tiles, after the rank tables of the sweep).
enum Mode { MODE_SELECT = 1, MODE_SWEEP = 2, MODE_BOTH = 3, MODE_SKETCH = 4, MODE_LINES = 8, MODE_FUSED = 9,
            MODE_HIST = 16 };

struct Job {
    std::vector<Series> series;
    const float* base = nullptr;     // device
    uint32_t K = 0;
    int mode = MODE_BOTH;
    uint64_t seed = 0;               // sketch stream of series 0 (series s uses seed + s)
    int sel = 0;                     // selection: 0 plain radix, 1 network window, 2 sample window, 3 given window
    std::vector<uint64_t> k;         // S*K, selection targets
    std::vector<uint32_t> eps_bits;  // S*K, sweep-only thresholds
    // results
    std::vector<float> eps;
    std::vector<uint64_t> kout, count_sel, count;
    std::vector<uint64_t> dcount;    // S*K, D (fused mode)
    std::vector<double> rr, det, det_mean;
    std::vector<uint64_t> M;
    std::vector<float> features;     // S*SKETCH_FEATURES (sketch mode)
    std::vector<uint32_t> scale;     // S (sketch mode)
    bool want_sample = false;        // sketch mode: also the sorted sample keys
    std::vector<uint32_t> sample;    // S*SKETCH_P (want_sample)
    std::vector<uint8_t> hit;        // S*K, window selection: target resolved in the window
    uint32_t hist_len = 0;           // histogram mode: entries per row (length 0 .. hist_len-1)
    uint32_t hist_kp = 0;            // histogram mode: largest number of distinct thresholds
    uint64_t* hist_dst = nullptr;    // histogram mode: host rows P_r(l), caller order: series s's K rows
                                     // of hist_len entries start at hist_dst + s * hist_series_stride
    size_t hist_series_stride = 0;   // 0: K * hist_len (rows of consecutive series back to back)
};

rqa_status ensure_acts(rqa_ctx* c, uint32_t B, MlpActs& a);

// Pass-2 slots (targets counted per launch) that fit the LDS next to the
// bucket table; false if not even one does.
bool pass2_slots(const rqa_ctx* c, uint32_t K, uint32_t* G)
{
    const size_t fixed = select_lds_bytes(2, K, 0);
    const size_t room = c->max_lds > fixed ? c->max_lds - fixed : 0;
    *G = (uint32_t)std::min<size_t>(K, room / (SEL_N2 * 4));
    return *G != 0;
}

// Runs selection and/or sweep for every series of the job.
rqa_status run_job(rqa_ctx* c, Job& job)
{
    const uint32_t S = (uint32_t)job.series.size();
    const uint32_t K = job.K;
    const bool hist = (job.mode & MODE_HIST) != 0;
    // histogram pass: the largest workgroup whose stacks fit in LDS, one tile per wave and chunk
    uint32_t hist_block = 0;
    if (hist) {
        for (uint32_t b : {1024u, 512u, 256u, 128u, 64u})
            if (hist_lds_bytes(job.hist_kp, b) <= c->max_lds) {
                hist_block = b;
                break;
            }
        if (!hist_block) return fail(RQA_ERR_UNSUPPORTED, "the histogram pass does not fit in LDS");
    }
    uint32_t CT;
    {
        const Series& z0 = job.series[0];
        CT = hist ? hist_block / TILE_W : chunk_for(c, S, z0.n - (uint64_t)(z0.p.m - 1) * z0.p.tau, z0.p, K);
        // the wide threshold sweep needs a tile per wave of its 1024-thread workgroups
        if ((job.mode & MODE_SWEEP) && !((job.mode & MODE_SELECT) && (job.mode & MODE_LINES)) && wide_sweep(c, K))
            CT = std::max<uint32_t>(CT, 1024 / TILE_W);
    }

    // descriptors, ordered by kernel variant so each launch sees a contiguous range
    std::vector<uint32_t> order(S);
    std::vector<SeriesDesc> sd(S);
    std::vector<int> sel_var(S), swp_var(S);
    job.M.assign(S, 0);
    for (uint32_t s = 0; s < S; ++s) {
        const Series& z = job.series[s];
        uint64_t nv, M;
        rqa_status st = check_params(&z.p, z.n, &nv, &M);
        if (st) return st;
        job.M[s] = M;
        sel_var[s] = select_variant_of(z.p.norm, z.p.m, z.p.tau);
        swp_var[s] = variant_of(z.p.norm, z.p.m, z.p.tau, z.p.lmin);
        order[s] = s;
    }
    // largest series first inside a variant: their chunks leave the queue first
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (swp_var[a] != swp_var[b]) return swp_var[a] < swp_var[b];
        if (job.series[a].p.lmin != job.series[b].p.lmin) return job.series[a].p.lmin < job.series[b].p.lmin;
        return job.M[a] > job.M[b];
    });
    // groups: consecutive device series sharing the sweep variant (and lmin for the generic one)
    struct Group { uint32_t begin, end; int sel, swp; uint32_t nchunks; };
    const bool fused = (job.mode & MODE_SELECT) && (job.mode & MODE_LINES);
    std::vector<Group> groups;
    uint32_t maxn = 0;
    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t s = order[i];
        const Series& z = job.series[s];
        const bool same = !groups.empty() && groups.back().swp == swp_var[s] &&
                          (swp_var[s] % 3 != 0 || job.series[order[groups.back().begin]].p.lmin == z.p.lmin);
        if (!same) groups.push_back({i, i, sel_var[s], swp_var[s], 0});
        Group& g = groups.back();
        g.end = i + 1;
        const uint64_t nv = z.n - (uint64_t)(z.p.m - 1) * z.p.tau;
        const uint64_t L0 = nv - z.p.theiler;
        SeriesDesc& d = sd[i];
        const uint32_t T = hist ? hist_segment_for(c, L0) : segment_for(c, nv, z.p, K);
        d.y = job.base + z.offset;
        d.n = (uint32_t)z.n;
        d.nv = (uint32_t)nv;
        d.m = z.p.m;
        d.tau = z.p.tau;
        d.norm = z.p.norm;
        d.w = z.p.theiler;
        d.lmin = z.p.lmin;
        d.K = K;
        d.M = job.M[s];
        d.T = T;
        d.q = T / TILE_W;
        d.B = (uint32_t)((L0 + TILE_W - 1) / TILE_W);
        d.Smax = (uint32_t)((L0 + T - 1) / T);
        const uint64_t ntiles = (uint64_t)d.Smax * d.B - (uint64_t)d.q * ((uint64_t)d.Smax * (d.Smax - 1) / 2);
        if (ntiles >= (1ull << 31)) return fail(RQA_ERR_UNSUPPORTED, "too many tiles; raise the segment length");
        d.ntiles = (uint32_t)ntiles;
        d.variant = (uint32_t)swp_var[s];
        d.seed = job.seed + s;
        d.f_logn = (float)(std::log2((double)z.n) / 16.0);
        d.f_m = (float)((double)z.p.m / 4.0);
        maxn = std::max<uint32_t>(maxn, (uint32_t)z.n);
    }
    // pass 2 of plain selection takes 1024-thread workgroups where its bins
    // admit one workgroup per CU (large K); a chunk then needs a tile for each
    // of their 16 waves
    if ((job.mode & MODE_SELECT) && job.sel == 0) {
        uint32_t G = 0;
        const bool fits = pass2_slots(c, K, &G);
        for (const Group& g : groups)
            if (fits && select_blocks_per_cu(2, g.sel, 512, select_lds_bytes(2, K, G)) == 1)
                CT = std::max<uint32_t>(CT, 1024 / TILE_W);
    }
    // The window pass flushes WIN_BINS fine bins (nearly all non-zero) each
    // time a workgroup moves to another series: give windowed jobs chunks
    // large enough that a workgroup sees about eight of them in all.
    if ((job.mode & MODE_SELECT) && job.sel != 0) {
        uint64_t tiles = 0;
        for (uint32_t i = 0; i < S; ++i) tiles += sd[i].ntiles;
        const uint64_t wgs = (uint64_t)c->num_cu * 2;
        const uint64_t want = tiles / (wgs * 8);
        CT = (uint32_t)std::max<uint64_t>(CT, std::min<uint64_t>(want, 1024));
    }
    for (Group& g : groups) {
        for (uint32_t i = g.begin; i < g.end; ++i) {
            SeriesDesc& d = sd[i];
            d.nchunks = (d.ntiles + CT - 1) / CT;
            d.chunk_begin = g.nchunks;  // chunk numbering restarts in every group
            g.nchunks += d.nchunks;
        }
    }

    // device layout
    size_t off = 0;
    auto carve = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_sd = carve(sizeof(SeriesDesc) * S);
    const size_t o_tgt = carve(sizeof(uint64_t) * S * K);
    const bool lines_out = (job.mode & MODE_SWEEP) != 0;
    const size_t res_words = result_words(K, lines_out);
    const size_t o_res = carve(sizeof(uint64_t) * S * res_words);
    const size_t o_tick = carve(sizeof(uint32_t) * NUM_TICKETS);
    // the working state is cleared with the tickets and histograms; the
    // targets are placed into it on the device
    const size_t o_work = carve(sizeof(SeriesWork) * S);
    const size_t o_h1 = carve(sizeof(uint64_t) * S * SEL_N1);
    const size_t o_h2 = carve(sizeof(uint64_t) * S * K * SEL_N2);
    const size_t o_h3 = carve(sizeof(uint64_t) * S * K * SEL_N3);
    const bool window = (job.mode & MODE_SELECT) && job.sel != 0;
    const size_t o_wbins = window ? carve(sizeof(uint64_t) * S * WIN_BINS) : 0;
    const size_t hist_words = hist ? (size_t)S * job.hist_len * (job.hist_kp + 1) : 0;
    const size_t o_dh = hist ? carve(sizeof(uint64_t) * hist_words) : 0;
    // histogram: leading / trailing runs per tile, threshold and lane (written before read)
    std::vector<size_t> g_tile(groups.size(), 0);
    size_t hist_tiles = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        g_tile[gi] = hist_tiles;
        hist_tiles += (size_t)groups[gi].nchunks * CT;
    }
    const size_t run_words = hist ? hist_tiles * (job.hist_kp + 1) * TILE_W : 0;
    const size_t o_pre = hist ? carve(sizeof(uint16_t) * run_words) : 0;
    const size_t o_suf = hist ? carve(sizeof(uint16_t) * run_words) : 0;
    const size_t zero_end = off;  // tickets and histograms are cleared every call
    // histogram rows: every entry written by the finishing kernel
    const size_t o_hout = hist ? carve(sizeof(uint64_t) * (size_t)S * K * job.hist_len) : 0;
    const size_t o_T1 = carve((size_t)S * SEL_N1);
    const size_t o_T2 = carve((size_t)S * K * SEL_N2);
    const size_t o_rt = carve(sizeof(uint2) * S * RHO_TABLE);
    const bool sketch = (job.mode & MODE_SKETCH) || window;
    const size_t o_feat = sketch ? carve(sizeof(float) * S * SKETCH_FEATURES) : 0;
    const bool keep_sample = window || ((job.mode & MODE_SKETCH) && job.want_sample);
    const size_t o_smp = keep_sample ? carve(sizeof(uint32_t) * S * SKETCH_P) : 0;
    const size_t o_wtab = window ? carve((size_t)S * WIN_BINS) : 0;
    const size_t o_wfine = window && !fused ? carve(sizeof(uint64_t) * S * K * (1u << WIN_MAX_SHIFT)) : 0;
    // range sweep: fine counters of keys and line values, cleared by the set-up kernel
    const uint32_t fine_stride = fused ? K << (window ? WIN_MAX_SHIFT : (uint32_t)SEL_B3) : 0;
    const size_t o_fineK = fused ? carve(sizeof(uint64_t) * S * fine_stride) : 0;
    const size_t o_fineL = fused ? carve(sizeof(uint64_t) * S * fine_stride) : 0;
    const size_t o_pred = window ? carve(sizeof(float) * S * MLP_OUT) : 0;
    const size_t o_delta = window ? carve(sizeof(float) * MLP_OUT) : 0;
    if (window && window_lds_bytes(1) > c->max_lds)
        return fail(RQA_ERR_UNSUPPORTED, "the window pass needs %zu bytes of LDS per workgroup", window_lds_bytes(1));
    rqa_status st = RQA_OK;
    char* pool = nullptr;
    if (c->use_static) {
        // rqa_batch_static: the fixed device area; nothing is allocated
        if (off > STATIC_SCRATCH_BYTES)
            return fail(RQA_ERR_NOMEM, "this call needs %zu bytes of device scratch; the static area holds %zu "
                        "(fewer series or targets per call, or rqa_batch)", off, STATIC_SCRATCH_BYTES);
        pool = (char*)c->static_dev;
    } else {
        if ((st = ensure_pool(c, off))) return st;
        pool = (char*)c->pool;
    }
    DevBufs all;
    all.sd = (SeriesDesc*)(pool + o_sd);
    all.work = (SeriesWork*)(pool + o_work);
    all.tickets = (uint32_t*)(pool + o_tick);
    all.h1 = (uint64_t*)(pool + o_h1);
    all.h2 = (uint64_t*)(pool + o_h2);
    all.h3 = (uint64_t*)(pool + o_h3);
    all.fineK = fused ? (uint64_t*)(pool + o_fineK) : nullptr;
    all.fineL = fused ? (uint64_t*)(pool + o_fineL) : nullptr;
    all.fine_stride = fine_stride;
    all.T1 = (uint8_t*)(pool + o_T1);
    all.T2 = (uint8_t*)(pool + o_T2);
    all.rtab = (uint2*)(pool + o_rt);
    all.S = S;
    all.K = K;
    all.chunk_tiles = CT;
    all.nchunks = 0;

    // host staging: descriptors and targets (in), packed results and sketch
    // features (out)
    const size_t hs_sd = sizeof(SeriesDesc) * S, hs_tgt = sizeof(uint64_t) * S * K;
    const size_t hs_res = sizeof(uint64_t) * S * res_words;
    const size_t hs_feat = (job.mode & MODE_SKETCH) ? sizeof(float) * S * SKETCH_FEATURES : 0;
    const size_t hs_smp = ((job.mode & MODE_SKETCH) && job.want_sample) ? sizeof(uint32_t) * S * SKETCH_P : 0;
    const size_t hs_all = hs_sd + hs_tgt + hs_res + hs_feat + sizeof(float) * MLP_OUT + hs_smp;
    char* hbase = nullptr;
    if (c->use_static) {
        // ordinary host memory (no pinned allocation); the copies below then
        // stage through the runtime, and the call synchronises before return
        if (c->static_host.size() < hs_all) c->static_host.resize(hs_all);
        hbase = (char*)c->static_host.data();
    } else {
        if ((st = ensure_host(c, hs_all))) return st;
        hbase = (char*)c->host;
    }
    SeriesDesc* h_sd = (SeriesDesc*)hbase;
    uint64_t* h_tgt = (uint64_t*)(hbase + hs_sd);
    uint64_t* h_res = (uint64_t*)(hbase + hs_sd + hs_tgt);
    float* h_feat = (float*)(hbase + hs_sd + hs_tgt + hs_res);
    float* h_delta = (float*)(hbase + hs_sd + hs_tgt + hs_res + hs_feat);
    uint32_t* h_smp = (uint32_t*)(hbase + hs_sd + hs_tgt + hs_res + hs_feat + sizeof(float) * MLP_OUT);
    std::memcpy(h_delta, c->bracket_delta, sizeof(float) * MLP_OUT);
    if (window && job.sel == 1 && !c->has_model)
        return fail(RQA_ERR_INVALID_ARG, "RQA_SEL_LEARNED needs a network (rqa_mlp_init / rqa_mlp_set_params)");
    std::memcpy(h_sd, sd.data(), hs_sd);
    const bool as_rank = (job.mode & MODE_SELECT) != 0;
    const bool has_tgt = as_rank || (job.mode & (MODE_SWEEP | MODE_HIST));
    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t s = order[i];
        for (uint32_t r = 0; r < K; ++r)
            h_tgt[(size_t)i * K + r] = !has_tgt ? 0 : as_rank ? job.k[(size_t)s * K + r] : job.eps_bits[(size_t)s * K + r];
    }

    Timer tm(c);
    hipStream_t sm = c->stream;
    HIP_TRY(tm.begin(PH_OTHER));
    HIP_TRY(hipMemcpyAsync(all.sd, h_sd, hs_sd, hipMemcpyHostToDevice, sm));
    HIP_TRY(hipMemcpyAsync(pool + o_tgt, h_tgt, hs_tgt, hipMemcpyHostToDevice, sm));
    HIP_TRY(launch_zero(sm, pool + o_tick, zero_end - o_tick));
    HIP_TRY(launch_check_finite(sm, all, maxn, (const uint64_t*)(pool + o_tgt), as_rank));
    if (sketch)
        HIP_TRY(launch_sketch(sm, all, (float*)(pool + o_feat), keep_sample ? (uint32_t*)(pool + o_smp) : nullptr));
    if (window) {
        HIP_TRY(hipMemcpyAsync(pool + o_delta, h_delta, sizeof(float) * MLP_OUT, hipMemcpyHostToDevice, sm));
        if (job.sel == 3) {
            HIP_TRY(launch_window_fixed(sm, all, c->win_lo, c->win_hi));
        } else if (job.sel == 1) {
            MlpActs acts;
            if ((st = ensure_acts(c, S, acts))) return st;
            HIP_TRY(mlp_forward(sm, c->mlp, (const float*)(pool + o_feat), (int)S, acts, (float*)(pool + o_pred)));
            HIP_TRY(launch_window_from_offsets(sm, all, (const float*)(pool + o_pred), (const float*)(pool + o_delta)));
        } else {
            HIP_TRY(launch_window_from_sample(sm, all, (const uint32_t*)(pool + o_smp), nullptr, c->sample_z));
        }
    }
    HIP_TRY(tm.end());

    auto view = [&](const Group& g) {
        DevBufs v = all;
        v.sd = all.sd + g.begin;
        v.work = all.work + g.begin;
        v.h1 = all.h1 + (size_t)g.begin * SEL_N1;
        v.h2 = all.h2 + (size_t)g.begin * K * SEL_N2;
        v.h3 = all.h3 + (size_t)g.begin * K * SEL_N3;
        if (fused) {
            v.fineK = all.fineK + (size_t)g.begin * fine_stride;
            v.fineL = all.fineL + (size_t)g.begin * fine_stride;
        }
        v.T1 = all.T1 + (size_t)g.begin * SEL_N1;
        v.T2 = all.T2 + (size_t)g.begin * K * SEL_N2;
        v.rtab = all.rtab + (size_t)g.begin * RHO_TABLE;
        v.S = g.end - g.begin;
        v.nchunks = g.nchunks;
        return v;
    };

    uint32_t ticket = 0;
    auto take = [&](uint32_t n) -> int {
        if (ticket + n > (uint32_t)NUM_TICKETS) return -1;
        int t = (int)ticket;
        ticket += n;
        return t;
    };
    // The variant groups of one phase (each its own persistent launch) run
    // concurrently: the first on the context stream, the others on the
    // second stream, forked from and joined back into the context stream by
    // events, so the workgroups of one group take the CUs as those of the
    // other drain instead of each launch ending in its own tail.
    const bool multi = groups.size() > 1 && c->aux;
    auto gstream = [&](size_t gi) { return (multi && gi > 0) ? c->aux : sm; };
    auto fork = [&]() -> hipError_t {
        if (!multi) return hipSuccess;
        hipError_t e = hipEventRecord(c->ev_fork, sm);
        return e != hipSuccess ? e : hipStreamWaitEvent(c->aux, c->ev_fork, 0);
    };
    auto join = [&]() -> hipError_t {
        if (!multi) return hipSuccess;
        hipError_t e = hipEventRecord(c->ev_join, c->aux);
        return e != hipSuccess ? e : hipStreamWaitEvent(sm, c->ev_join, 0);
    };

    if (window) {
        WinBufs wb;
        wb.bins = (uint64_t*)(pool + o_wbins);
        wb.table = (uint8_t*)(pool + o_wtab);
        wb.fine = fused ? nullptr : (uint64_t*)(pool + o_wfine);
        // fused: window pass 1 only; the range sweep resolves the fine bins
        for (int pass = 1; pass <= (fused ? 1 : 2); ++pass) {
            HIP_TRY(tm.begin(pass - 1));
            HIP_TRY(fork());
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                const Group& g = groups[gi];
                DevBufs v = view(g);
                WinBufs wv = wb;
                wv.bins = wb.bins + (size_t)g.begin * WIN_BINS;
                wv.table = wb.table + (size_t)g.begin * WIN_BINS;
                wv.fine = fused ? nullptr : wb.fine + (size_t)g.begin * K * (1u << WIN_MAX_SHIFT);
                const int var = g.sel;
                const uint32_t block = pass == 1 ? WIN_BLOCK : 512;
                const int per_cu = window_blocks_per_cu(pass, var, block);
                const uint32_t grid = c->grid ? c->grid
                                              : std::max<uint32_t>(1, std::min<uint32_t>(g.nchunks, (uint32_t)(c->num_cu * per_cu)));
                const int t = take(1);
                if (t < 0) return fail(RQA_ERR_UNSUPPORTED, "too many kernel launches in one call");
                HIP_TRY(launch_window_pass(gstream(gi), v, wv, pass, var, grid, block, (uint32_t)t));
            }
            HIP_TRY(join());
            HIP_TRY(tm.end());
            HIP_TRY(tm.begin(PH_OTHER));
            HIP_TRY(launch_window_scan(sm, all, wb, pass));
            HIP_TRY(tm.end());
        }
    } else if (job.mode & MODE_SELECT) {
        // fused: passes 1 and 2; the range sweep takes the place of pass 3
        for (int pass = 1; pass <= (fused ? 2 : 3); ++pass) {
            HIP_TRY(tm.begin(pass - 1));
            HIP_TRY(fork());
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                const Group& g = groups[gi];
                DevBufs v = view(g);
                const int var = g.sel;
                uint32_t block = 512;
                uint32_t G = 1, ngroups = 1;
                if (pass == 2) {
                    if (!pass2_slots(c, K, &G)) return fail(RQA_ERR_UNSUPPORTED, "pass 2 does not fit the LDS");
                    ngroups = (K + G - 1) / G;
                } else if (pass == 3 && select_lds_bytes(3, K, 0) > c->max_lds) {
                    return fail(RQA_ERR_UNSUPPORTED, "K=%u does not fit the LDS of pass 3", K);
                }
                const size_t lds = select_lds_bytes(pass, K, G);
                int per_cu = select_blocks_per_cu(pass, var, block, lds);
                // pass 2 at large K: when the bins admit one workgroup per CU,
                // a 1024-thread one puts twice the waves on the same bins
                if (pass == 2 && per_cu == 1) block = 1024;
                const uint32_t grid = c->grid ? c->grid
                                              : std::max<uint32_t>(1, std::min<uint32_t>(g.nchunks, (uint32_t)(c->num_cu * per_cu)));
                const int t = take(ngroups);
                if (t < 0) return fail(RQA_ERR_UNSUPPORTED, "too many kernel launches in one call");
                HIP_TRY(launch_select_pass(gstream(gi), v, pass, var, grid, block, ngroups, G, (uint32_t)t));
            }
            HIP_TRY(join());
            HIP_TRY(tm.end());
            HIP_TRY(tm.begin(PH_OTHER));
            HIP_TRY(launch_select_scan(sm, all, pass));
            HIP_TRY(tm.end());
        }
    }
    if (hist) {
        HIP_TRY(tm.begin(PH_OTHER));
        HIP_TRY(launch_sweep_prep(sm, all));
        HIP_TRY(tm.end());
        HIP_TRY(tm.begin(PH_HIST));
        const uint32_t kc = job.hist_kp + 1;
        HIP_TRY(fork());
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group& g = groups[gi];
            DevBufs v = view(g);
            const int per_cu = hist_blocks_per_cu(g.sel, job.hist_kp, hist_block);
            const uint32_t grid = c->grid ? c->grid
                                          : std::max<uint32_t>(1, std::min<uint32_t>(g.nchunks, (uint32_t)(c->num_cu * per_cu)));
            const int t = take(1);
            if (t < 0) return fail(RQA_ERR_UNSUPPORTED, "too many kernel launches in one call");
            uint64_t* dg = (uint64_t*)(pool + o_dh) + (size_t)g.begin * job.hist_len * kc;
            uint16_t* pre = (uint16_t*)(pool + o_pre) + g_tile[gi] * kc * TILE_W;
            uint16_t* suf = (uint16_t*)(pool + o_suf) + g_tile[gi] * kc * TILE_W;
            HIP_TRY(launch_hist(gstream(gi), v, g.sel, grid, hist_block, dg, pre, suf, job.hist_len, job.hist_kp,
                                (uint32_t)t));
            uint32_t items = 1;
            for (uint32_t i = g.begin; i < g.end; ++i) items = std::max(items, sd[i].B * ((job.hist_kp + 3) / 4));
            const uint32_t jgrid = std::min<uint32_t>(items, (uint32_t)c->num_cu * 4);
            HIP_TRY(launch_hist_join(gstream(gi), v, jgrid, pre, suf, dg, job.hist_len, job.hist_kp));
        }
        HIP_TRY(join());
        HIP_TRY(launch_hist_finish(sm, all, (const uint64_t*)(pool + o_dh), (uint64_t*)(pool + o_hout), job.hist_len,
                                   job.hist_kp));
        HIP_TRY(tm.end());
    }
    if ((job.mode & MODE_SWEEP) || fused) {
        HIP_TRY(tm.begin(PH_OTHER));
        if (fused) HIP_TRY(launch_range_prep(sm, all, window));
        else HIP_TRY(launch_sweep_prep(sm, all));
        HIP_TRY(tm.end());
        HIP_TRY(tm.begin(PH_SWEEP));
        HIP_TRY(fork());
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Group& g = groups[gi];
            DevBufs v = view(g);
            const uint32_t block = (!fused && wide_sweep(c, K)) ? 1024 : 512;
            const size_t lds = sweep_lds_bytes(fused ? 2 * K + 1 : K, fused);
            const int per_cu = sweep_blocks_per_cu(g.swp, fused, block, lds);
            const uint32_t grid = c->grid ? c->grid
                                          : std::max<uint32_t>(1, std::min<uint32_t>(g.nchunks, (uint32_t)(c->num_cu * per_cu)));
            const int t = take(1);
            if (t < 0) return fail(RQA_ERR_UNSUPPORTED, "too many kernel launches in one call");
            HIP_TRY(launch_sweep(gstream(gi), v, g.swp, fused, grid, block, (uint32_t)t));
        }
        HIP_TRY(join());
        HIP_TRY(tm.end());
        if (fused) {
            HIP_TRY(tm.begin(PH_OTHER));
            HIP_TRY(launch_range_scan(sm, all));
            HIP_TRY(tm.end());
        }
    }
    HIP_TRY(launch_pack_results(sm, all, lines_out, (uint64_t*)(pool + o_res)));
    HIP_TRY(hipMemcpyAsync(h_res, pool + o_res, hs_res, hipMemcpyDeviceToHost, sm));
    if (hs_feat) HIP_TRY(hipMemcpyAsync(h_feat, pool + o_feat, hs_feat, hipMemcpyDeviceToHost, sm));
    if (hs_smp) HIP_TRY(hipMemcpyAsync(h_smp, pool + o_smp, hs_smp, hipMemcpyDeviceToHost, sm));
    if (hist) {
        // rows straight into the caller's buffer, series back in caller order
        if (!job.hist_dst) return fail(RQA_ERR_INVALID_ARG, "histogram destination is NULL");
        const size_t rows = (size_t)K * job.hist_len;
        const size_t stride = job.hist_series_stride ? job.hist_series_stride : rows;
        for (uint32_t i = 0; i < S; ++i)
            HIP_TRY(hipMemcpyAsync(job.hist_dst + (size_t)order[i] * stride, (uint64_t*)(pool + o_hout) + (size_t)i * rows,
                                   sizeof(uint64_t) * rows, hipMemcpyDeviceToHost, sm));
    }
    HIP_TRY(hipStreamSynchronize(sm));
    tm.collect();

    // results, back in caller order
    job.eps.assign((size_t)S * K, 0.f);
    job.kout.assign((size_t)S * K, 0);
    job.count_sel.assign((size_t)S * K, 0);
    if (fused) job.dcount.assign((size_t)S * K, 0);
    job.count.assign((size_t)S * K, 0);
    job.rr.assign((size_t)S * K, 0.0);
    job.det.assign((size_t)S * K, 0.0);
    job.det_mean.assign(S, 0.0);
    if (job.mode & MODE_SKETCH) {
        job.features.assign((size_t)S * SKETCH_FEATURES, 0.f);
        job.scale.assign(S, 0);
        if (hs_smp) job.sample.assign((size_t)S * SKETCH_P, 0u);
    }
    if (window) job.hit.assign((size_t)S * K, 0);
    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t s = order[i];
        // packed results of device series i (layout at k_pack_results)
        const uint64_t* w = h_res + (size_t)i * res_words;
        const uint32_t status = (uint32_t)w[0], nonfinite = (uint32_t)(w[0] >> 32);
        const uint32_t scale = (uint32_t)w[1], range_ok = (uint32_t)(w[1] >> 32);
        const uint64_t* w_eps = w + 3;
        const uint64_t* w_k = w_eps + K;
        const uint64_t* w_count = w_k + K;
        const uint64_t* w_dcount = w_count + K;
        const uint64_t* w_hitmap = w_dcount + K;
        if (nonfinite) return fail(RQA_ERR_NONFINITE, "series %u holds a NaN or infinite sample", s);
        if (status & ~8u) return fail(RQA_ERR_DEVICE, "selection of series %u is inconsistent (code %u)", s, status);
        if (job.mode & MODE_SKETCH) {
            std::memcpy(&job.features[(size_t)s * SKETCH_FEATURES], h_feat + (size_t)i * SKETCH_FEATURES,
                        sizeof(float) * SKETCH_FEATURES);
            if (hs_smp)
                std::memcpy(&job.sample[(size_t)s * SKETCH_P], h_smp + (size_t)i * SKETCH_P,
                            sizeof(uint32_t) * SKETCH_P);
            job.scale[s] = scale;
        }
        for (uint32_t r = 0; r < K; ++r) {
            float e;
            const uint32_t bits = (uint32_t)w_eps[r];
            std::memcpy(&e, &bits, 4);
            job.eps[(size_t)s * K + r] = e;
            job.kout[(size_t)s * K + r] = w_k[r];
            job.count_sel[(size_t)s * K + r] = w_count[r];
            if (fused) job.dcount[(size_t)s * K + r] = job.series[s].p.lmin <= 1 ? w_count[r] : w_dcount[r];
            // fused window mode resolves a series only when every target hit
            if (window) job.hit[(size_t)s * K + r] = ((uint32_t)w_hitmap[r] && (!fused || range_ok)) ? 1 : 0;
        }
        if (job.mode & MODE_SWEEP) {
            const uint32_t Kp = (uint32_t)w[2];
            const uint64_t* w_hrho = w_hitmap + K;
            const uint64_t* w_hlam = w_hrho + K;
            std::vector<uint64_t> C(Kp), D(Kp);
            uint64_t cr = 0, cl = 0;
            for (uint32_t j = 0; j < Kp; ++j) {
                cr += w_hrho[j];
                cl += w_hlam[j];
                C[j] = cr;
                D[j] = cl;
            }
            double sum = 0.0;
            for (uint32_t r = 0; r < K; ++r) {
                const uint32_t j = (uint32_t)(w_hitmap[r] >> 32);
                const uint64_t cnt = C[j];
                const double det = cnt ? (double)D[j] / (double)cnt : NAN;
                job.count[(size_t)s * K + r] = cnt;
                job.rr[(size_t)s * K + r] = (double)cnt / (double)job.M[s];
                job.det[(size_t)s * K + r] = det;
                sum += det;
            }
            job.det_mean[s] = sum / (double)K;
        }
    }
    return RQA_OK;
}

rqa_status check_ctx(rqa_ctx* c)
{
    if (!c) return fail(RQA_ERR_INVALID_ARG, "context is NULL");
    HIP_TRY(hipSetDevice(c->device));
    return RQA_OK;
}

rqa_status check_k(uint32_t K)
{
    if (K == 0 || K > RQA_MAX_K) return fail(RQA_ERR_INVALID_ARG, "K=%u outside 1..%d", K, RQA_MAX_K);
    return RQA_OK;
}

// Selection method of the flags: 0 plain radix passes, 1 network window,
// 2 sample window, 3 caller window, -1 automatic (resolve_method).
rqa_status check_flags_select(uint32_t flags, int* sel)
{
    const uint32_t known = RQA_SEL_LEARNED | RQA_FULL_HIST | RQA_SEL_SAMPLE | RQA_SEL_WINDOW | RQA_SEL_PLAIN;
    if (flags & ~known) return fail(RQA_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (flags & RQA_FULL_HIST)
        return fail(RQA_ERR_UNSUPPORTED, "RQA_FULL_HIST is a flag of rqa_det_curve (rqa_batch_hist gives the "
                                         "histogram with the whole path)");
    const uint32_t m = flags & (RQA_SEL_LEARNED | RQA_SEL_SAMPLE | RQA_SEL_WINDOW | RQA_SEL_PLAIN);
    if (m & (m - 1)) return fail(RQA_ERR_INVALID_ARG, "choose one selection method");
    *sel = (m == RQA_SEL_LEARNED) ? 1 : (m == RQA_SEL_SAMPLE) ? 2 : (m == RQA_SEL_WINDOW) ? 3
         : (m == RQA_SEL_PLAIN) ? 0 : -1;
    return RQA_OK;
}

// RQA_SEL_AUTO: the sample window (two passes over the pairs, exact, plain
// fallback) for calls of at least AUTO_WINDOW_PAIRS pairs in all, else the
// plain radix passes.  Measured on MI355X at K = 20 (ms per call, plain /
// sample window): two N = 1e5 series 9.2 / 7.3, the 600-series ensemble
// 12.4 / 11.3, 15 series of N = 1e4 in one call 1.54 / 1.49, ten of N = 1e3
// 0.33 / 0.44, one N = 1e4 series 0.43 / 0.49 (the sketch and window set-up
// cost about 0.1 ms per call).
constexpr uint64_t AUTO_WINDOW_PAIRS = 1ull << 29;

int resolve_method(const Job& job, int sel)
{
    if (sel >= 0) return sel;
    uint64_t pairs = 0;
    for (const Series& z : job.series) {
        const uint64_t a = z.n - (uint64_t)(z.p.m - 1) * z.p.tau - z.p.theiler;
        pairs += a * (a + 1) / 2;
    }
    return pairs >= AUTO_WINDOW_PAIRS ? 2 : 0;
}

rqa_status single_job_setup(rqa_ctx* c, Job& job, const float* series, uint64_t n, const rqa_params* p,
                            const double* rr, uint32_t K)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (!series) return fail(RQA_ERR_INVALID_ARG, "series pointer is NULL");
    if ((st = check_k(K))) return st;
    uint64_t nv, M;
    if ((st = check_params(p, n, &nv, &M))) return st;
    if (!rr) return fail(RQA_ERR_INVALID_ARG, "rr is NULL");
    job.series.push_back({0, n, *p});
    job.base = series;
    job.K = K;
    job.mode = MODE_FUSED;
    job.k.resize(K);
    for (uint32_t r = 0; r < K; ++r)
        if ((st = target_rank(rr[r], M, &job.k[r]))) return st;
    return RQA_OK;
}

rqa_status single_job(rqa_ctx* c, Job& job, const float* series, uint64_t n, const rqa_params* p,
                      const double* rr, const float* eps, uint32_t K, int mode)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (!series) return fail(RQA_ERR_INVALID_ARG, "series pointer is NULL");
    if ((st = check_k(K))) return st;
    uint64_t nv, M;
    if ((st = check_params(p, n, &nv, &M))) return st;
    job.series.push_back({0, n, *p});
    job.base = series;
    job.K = K;
    job.mode = mode;
    if (mode & MODE_SELECT) {
        if (!rr) return fail(RQA_ERR_INVALID_ARG, "rr is NULL");
        job.k.resize(K);
        for (uint32_t r = 0; r < K; ++r)
            if ((st = target_rank(rr[r], M, &job.k[r]))) return st;
    } else {
        if (!eps) return fail(RQA_ERR_INVALID_ARG, "eps is NULL");
        job.eps_bits.resize(K);
        for (uint32_t r = 0; r < K; ++r)
            if ((st = check_eps(eps[r], &job.eps_bits[r]))) return st;
    }
    return run_job(c, job);
}

// Exact thresholds by the window method; every series with a target outside
// its window (or without a usable window) is selected again by the plain
// radix passes.  Leaves job.eps / kout / count_sel complete.
rqa_status select_windowed(rqa_ctx* c, Job& job)
{
    const uint32_t S = (uint32_t)job.series.size(), K = job.K;
    job.mode = MODE_SELECT | (job.mode & MODE_LINES);
    rqa_status st = run_job(c, job);
    if (st) return st;
    std::vector<uint32_t> redo;
    uint32_t missed = 0;
    for (uint32_t s = 0; s < S; ++s) {
        uint32_t m = 0;
        for (uint32_t r = 0; r < K; ++r) m += job.hit[(size_t)s * K + r] ? 0 : 1;
        missed += m;
        if (m) redo.push_back(s);
    }
    c->stat_passes = 2;
    c->stat_fallback = (uint32_t)redo.size();
    c->stat_missed = missed;
    if (redo.empty()) return RQA_OK;
    Job plain;
    plain.base = job.base;
    plain.K = K;
    plain.mode = job.mode;
    for (uint32_t s : redo) {
        plain.series.push_back(job.series[s]);
        plain.k.insert(plain.k.end(), job.k.begin() + (size_t)s * K, job.k.begin() + (size_t)(s + 1) * K);
    }
    if ((st = run_job(c, plain))) return st;
    for (size_t i = 0; i < redo.size(); ++i)
        for (uint32_t r = 0; r < K; ++r) {
            const size_t a = (size_t)redo[i] * K + r, b = i * K + r;
            job.eps[a] = plain.eps[b];
            job.kout[a] = plain.kout[b];
            job.count_sel[a] = plain.count_sel[b];
            if (job.mode & MODE_LINES) job.dcount[a] = plain.dcount[b];
        }
    c->stat_passes += 3;
    return RQA_OK;
}

// RR, DET and the averaged DET from C = #{key <= eps} and D = #{line value
// <= eps} (Eq. 3, Eq. 4 and the averaged-determinism equation), in double.
void finish_lines(Job& job)
{
    const uint32_t S = (uint32_t)job.series.size(), K = job.K;
    job.count.assign((size_t)S * K, 0);
    job.rr.assign((size_t)S * K, 0.0);
    job.det.assign((size_t)S * K, 0.0);
    job.det_mean.assign(S, 0.0);
    for (uint32_t s = 0; s < S; ++s) {
        double sum = 0.0;
        for (uint32_t r = 0; r < K; ++r) {
            const size_t i = (size_t)s * K + r;
            const uint64_t C = job.count_sel[i], D = job.dcount[i];
            const double det = C ? (double)D / (double)C : NAN;
            job.count[i] = C;
            job.rr[i] = (double)C / (double)job.M[s];
            job.det[i] = det;
            sum += det;
        }
        job.det_mean[s] = sum / (double)K;
    }
}

// Exact thresholds (plain or windowed counting passes) and RR, DET at them.
// Normally the last pass is the range sweep, which finishes the thresholds and
// counts C and D in the same pass.  With many targets its histograms do not
// fit the LDS: then the thresholds are selected completely first and a sweep
// at them follows.  stat_passes counts every full pass over the pairs.
// The range sweep (counting passes, then ranks against the candidate ranges
// left by them) while it is the faster path, else complete selection and the
// threshold sweep.  The range sweep's cost grows with K (line-rank histograms
// of 2K + 1 rows in LDS, which keep three workgroups per CU up to K = 76, and
// more keys inside candidate ranges take its fine-counter path), the
// threshold sweep's hardly does.  Measured on MI355X (two N = 1e5 series,
// targets 1..K %, range sweep / complete selection, ms per step): plain
// selection 12.7 / 13.6 at K = 56, 13.4 / 13.8 at 64, 14.1 / 14.1 at 72,
// 17.5 / 14.5 at 80; with the sample window, whose candidate ranges are
// wider, 8.9 / 9.5 at K = 36, 9.4 / 9.6 at 40, 10.5 / 9.8 at 48.
#ifndef RQA_FUSED_MAX_K_PLAIN
#define RQA_FUSED_MAX_K_PLAIN 64
#endif
#ifndef RQA_FUSED_MAX_K_WINDOW
#define RQA_FUSED_MAX_K_WINDOW 40
#endif
constexpr uint32_t FUSED_MAX_K_PLAIN = RQA_FUSED_MAX_K_PLAIN;
constexpr uint32_t FUSED_MAX_K_WINDOW = RQA_FUSED_MAX_K_WINDOW;

bool use_fused(const rqa_ctx* c, uint32_t K, int sel)
{
    return K <= (sel == 0 ? FUSED_MAX_K_PLAIN : FUSED_MAX_K_WINDOW) && sweep_lds_bytes(2 * K + 1, true) <= c->max_lds;
}

rqa_status select_and_sweep(rqa_ctx* c, Job& job)
{
    rqa_status st;
    if (use_fused(c, job.K, job.sel)) {
        job.mode = MODE_FUSED;
        if (job.sel == 0) {
            c->stat_passes = 3;
            c->stat_fallback = 0;
            c->stat_missed = 0;
            st = run_job(c, job);
        } else {
            st = select_windowed(c, job);
        }
        if (st) return st;
        finish_lines(job);
        return RQA_OK;
    }
    if (job.sel == 0) {
        job.mode = MODE_BOTH;
        c->stat_passes = 4;
        c->stat_fallback = 0;
        c->stat_missed = 0;
        return run_job(c, job);
    }
    job.mode = MODE_SELECT;
    if ((st = select_windowed(c, job))) return st;
    Job sw;
    sw.base = job.base;
    sw.K = job.K;
    sw.mode = MODE_SWEEP;
    sw.series = job.series;
    sw.eps_bits.resize(job.eps.size());
    std::memcpy(sw.eps_bits.data(), job.eps.data(), sizeof(uint32_t) * job.eps.size());
    if ((st = run_job(c, sw))) return st;
    c->stat_passes += 1;
    job.count = sw.count;
    job.rr = sw.rr;
    job.det = sw.det;
    job.det_mean = sw.det_mean;
    job.M = sw.M;
    return RQA_OK;
}

rqa_status build_batch_job(Job& job, uint32_t S, const float* concat, const uint64_t* offsets, const rqa_params* p,
                           const double* rr, uint32_t K)
{
    rqa_status st;
    if ((st = check_k(K))) return st;
    if (S == 0 || !concat || !offsets || !p || !rr) return fail(RQA_ERR_INVALID_ARG, "S is 0 or a required pointer is NULL");
    job.base = concat;
    job.K = K;
    job.mode = MODE_FUSED;
    job.k.resize((size_t)S * K);
    for (uint32_t s = 0; s < S; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(RQA_ERR_INVALID_ARG, "offsets decrease at series %u", s);
        const uint64_t n = offsets[s + 1] - offsets[s];
        uint64_t nv, M;
        if ((st = check_params(&p[s], n, &nv, &M))) {
            char msg[512];
            std::snprintf(msg, sizeof msg, "series %u: %s", s, g_err);
            return fail(st, "%s", msg);
        }
        job.series.push_back({offsets[s], n, p[s]});
        for (uint32_t r = 0; r < K; ++r)
            if ((st = target_rank(rr[(size_t)s * K + r], M, &job.k[(size_t)s * K + r]))) return st;
    }
    return RQA_OK;
}

// Best host wall time (ms) of `reps` calls of the job; each call synchronises.
// Device time of the job's phases (HIP events on the context stream), the
// fastest of `reps` runs: the host's share of a call does not depend on the
// launch shape and would only add noise to the comparison.
rqa_status time_job(rqa_ctx* c, Job& job, int reps, double* best)
{
    *best = 1e300;
    if (!c->ev_ready) {
        for (auto& e : c->ev) HIP_TRY(hipEventCreate(&e));
        c->ev_ready = true;
    }
    const bool save_timing = c->timing;
    c->timing = true;
    rqa_status st = RQA_OK;
    for (int i = 0; i < reps && !st; ++i) {
        Job j = job;
        reset_phases(c);
        st = run_job(c, j);
        if (!st) {
            double ms = 0.0;
            for (int p = 0; p < PH_N; ++p) ms += c->phase_ms[p];
            *best = std::min(*best, ms);
        }
    }
    c->timing = save_timing;
    reset_phases(c);
    return st;
}

// Candidate segment lengths: powers of two from 64 up to the longest diagonal
// (at most 4096).
std::vector<uint32_t> segment_candidates(uint64_t L0)
{
    std::vector<uint32_t> v;
    for (uint32_t t = 64; t <= 4096; t *= 2) {
        v.push_back(t);
        if (t >= L0) break;
    }
    return v;
}

const uint32_t CHUNK_CANDIDATES[] = {2, 8, 32, 128, 512};

// Tunes the segment length of each size bucket present in the job (on up to
// 64 of its series, chunk size at the default) and then the chunk size of the
// whole job, with the job's selection method; records everything in the
// context's table.
rqa_status tune_job(rqa_ctx* c, Job& job, uint32_t* seg_out, uint32_t* chunk_out)
{
    const uint32_t save_seg = c->seg, save_chunk = c->chunk_tiles;
    const uint32_t K = job.K;
    std::map<TuneKey, std::vector<uint32_t>> buckets;
    uint64_t maxL0 = 0;
    for (uint32_t s = 0; s < (uint32_t)job.series.size(); ++s) {
        const Series& z = job.series[s];
        const uint64_t nv = z.n - (uint64_t)(z.p.m - 1) * z.p.tau;
        buckets[tune_key(nv, z.p, K)].push_back(s);
        maxL0 = std::max<uint64_t>(maxL0, nv - z.p.theiler);
    }
    rqa_status st = RQA_OK;
    uint32_t last_seg = 0;
    // tune the path the calls take (see select_and_sweep)
    const int mode = (job.mode == MODE_FUSED && !use_fused(c, K, job.sel)) ? MODE_BOTH : job.mode;
    for (auto& kv : buckets) {
        Job sub;
        sub.base = job.base;
        sub.K = K;
        sub.mode = mode;
        // a size bucket that is the whole call is tuned with the call's
        // selection method; buckets of a larger batch with plain selection
        // (measured on the 600-series ensemble: segments tuned per bucket on
        // the sample window's path made the whole call 10.3 ms instead of 8.4)
        sub.sel = buckets.size() == 1 ? job.sel : 0;
        uint64_t L0 = 0;
        for (size_t i = 0; i < kv.second.size() && i < 64; ++i) {
            const uint32_t s = kv.second[i];
            sub.series.push_back(job.series[s]);
            sub.k.insert(sub.k.end(), job.k.begin() + (size_t)s * K, job.k.begin() + (size_t)(s + 1) * K);
            const Series& z = job.series[s];
            L0 = std::max<uint64_t>(L0, z.n - (uint64_t)(z.p.m - 1) * z.p.tau - z.p.theiler);
        }
        double best = 1e300;
        uint32_t best_seg = 64;
        c->chunk_tiles = DEFAULT_CHUNK;
        // one untimed run first: a GPU that has been idle raises its clocks
        // during the first candidates, which would favour the later ones
        c->seg = default_segment(L0);
        {
            double warm;
            if ((st = time_job(c, sub, 1, &warm))) break;
        }
        for (uint32_t T : segment_candidates(L0)) {
            c->seg = T;
            double ms;
            if ((st = time_job(c, sub, 3, &ms))) break;
            if (ms < best) { best = ms; best_seg = T; }
        }
        if (st) break;
        c->tune[kv.first] = {best_seg, DEFAULT_CHUNK};
        last_seg = best_seg;
    }
    uint32_t best_chunk = DEFAULT_CHUNK;
    if (!st) {
        c->seg = 0;  // the table just filled
        double best = 1e300;
        Job whole = job;
        whole.mode = mode;
        // the largest chunk within 3% of the fastest: shorter chunks cost
        // per-chunk set-up that some paths feel much more than the one tuned
        // (plain selection's pass 2 at 2 tiles per chunk: twice the time)
        double ms_of[sizeof(CHUNK_CANDIDATES) / sizeof(CHUNK_CANDIDATES[0])];
        int n = 0;
        for (uint32_t CT : CHUNK_CANDIDATES) {
            c->chunk_tiles = CT;
            double ms;
            if ((st = time_job(c, whole, 3, &ms))) break;
            ms_of[n++] = ms;
            best = std::min(best, ms);
        }
        if (!st)
            for (int i = 0; i < n; ++i)
                if (ms_of[i] <= best * 1.03) best_chunk = CHUNK_CANDIDATES[i];
    }
    c->seg = save_seg;
    c->chunk_tiles = save_chunk;
    if (st) return st;
    if (job.series.size() == 1) {
        auto& e = c->tune[buckets.begin()->first];
        e.chunk = best_chunk;
    } else {
        c->tune[TuneKey{-1, 0, K <= 32 ? 0 : 1}] = {0, best_chunk};
    }
    if (seg_out) *seg_out = job.series.size() == 1 ? last_seg : 0;
    if (chunk_out) *chunk_out = best_chunk;
    (void)maxL0;
    return RQA_OK;
}

// Full line-length histogram P_r(l) (lengths 0 .. hist_len-1) of every
// series of `src` at the thresholds eps_bits[S*K] (caller order), written to
// hist_out[S][K][hist_len].  One histogram pass takes at most
// HIST_MAX_K_HOST thresholds (its ranks and per-lane stacks are sized for
// them), so larger K runs in ceil(K / HIST_MAX_K_HOST) passes of balanced
// slices of the targets, inside this one call.
rqa_status hist_in_passes(rqa_ctx* c, const Job& src, const std::vector<uint32_t>& eps_bits, uint32_t hist_len,
                          uint64_t* hist_out)
{
    const uint32_t S = (uint32_t)src.series.size(), K = src.K;
    for (uint32_t s = 0; s < S; ++s) {
        const Series& z = src.series[s];
        const uint64_t nv = z.n - (uint64_t)(z.p.m - 1) * z.p.tau;
        if (nv >= (1ull << 24) - 1)
            return fail(RQA_ERR_UNSUPPORTED, "series %u has %llu embedded vectors; the full histogram takes fewer than "
                        "2^24 - 1", s, (unsigned long long)nv);
    }
    const uint32_t passes = (K + HIST_MAX_K_HOST - 1) / HIST_MAX_K_HOST;
    const uint32_t per = (K + passes - 1) / passes;
    for (uint32_t r0 = 0; r0 < K; r0 += per) {
        const uint32_t kc = std::min(per, K - r0);
        Job hj;
        hj.series = src.series;
        hj.base = src.base;
        hj.K = kc;
        hj.mode = MODE_HIST;
        hj.hist_len = hist_len;
        hj.eps_bits.resize((size_t)S * kc);
        uint32_t kp = 1;
        for (uint32_t s = 0; s < S; ++s) {
            std::vector<uint32_t> d(eps_bits.begin() + (size_t)s * K + r0, eps_bits.begin() + (size_t)s * K + r0 + kc);
            std::copy(d.begin(), d.end(), hj.eps_bits.begin() + (size_t)s * kc);
            std::sort(d.begin(), d.end());
            kp = std::max(kp, (uint32_t)(std::unique(d.begin(), d.end()) - d.begin()));
        }
        hj.hist_kp = kp;
        // this slice's rows go straight to their place in the caller's rows
        hj.hist_dst = hist_out + (size_t)r0 * hist_len;
        hj.hist_series_stride = (size_t)K * hist_len;
        rqa_status st = run_job(c, hj);
        if (st) return st;
    }
    return RQA_OK;
}

}  // namespace

extern "C" {

rqa_status rqa_create(rqa_ctx** out, int device, void* hip_stream)
{
    if (!out) return fail(RQA_ERR_INVALID_ARG, "out is NULL");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(RQA_ERR_INVALID_ARG, "device %d of %d", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(RQA_ERR_UNSUPPORTED, "built for gfx950, device is %s", prop.gcnArchName);
    void* static_dev = nullptr;
    rqa_status sst = resolve_static_scratch(device, &static_dev);
    if (sst) return sst;
    rqa_ctx* c = new rqa_ctx();
    c->device = device;
    c->static_dev = static_dev;
    c->num_cu = prop.multiProcessorCount;
    c->max_lds = std::max<size_t>(prop.sharedMemPerBlock, 65536);
    if (prop.maxSharedMemoryPerMultiProcessor > 0)
        c->max_lds = std::min<size_t>(std::max<size_t>(c->max_lds, prop.sharedMemPerBlockOptin),
                                      prop.maxSharedMemoryPerMultiProcessor);
    if (c->max_lds > 65536 && set_kernel_lds_limits(c->max_lds) != hipSuccess) {
        (void)hipGetLastError();
        c->max_lds = 65536;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(RQA_ERR_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        rqa_destroy(c);
        return fail(RQA_ERR_DEVICE, "creating the context's second stream or its events failed");
    }
    *out = c;
    return RQA_OK;
}

void rqa_destroy(rqa_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->pool) (void)hipFree(c->pool);
    if (c->host) (void)hipHostFree(c->host);
    if (c->mlp) (void)hipFree(c->mlp);
    if (c->mlp_acts) (void)hipFree(c->mlp_acts);
    if (c->mlp_partial) (void)hipFree(c->mlp_partial);
    if (c->ev_ready)
        for (auto& e : c->ev) (void)hipEventDestroy(e);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

rqa_status rqa_set_timing(rqa_ctx* c, int enable)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (enable && !c->ev_ready) {
        for (auto& e : c->ev) HIP_TRY(hipEventCreate(&e));
        c->ev_ready = true;
    }
    c->timing = enable != 0;
    return RQA_OK;
}

int rqa_phase_times(rqa_ctx* c, double* out, int n)
{
    if (!c || !out) return 0;
    int k = std::min(n, (int)PH_N);
    for (int i = 0; i < k; ++i) out[i] = c->phase_ms[i];
    return k;
}

rqa_status rqa_valu_rate(rqa_ctx* c, uint32_t kind, double* lane_ops_per_s, double* ms_out)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (kind > 3) return fail(RQA_ERR_INVALID_ARG, "probe kind %u outside 0..3", kind);
    if (!lane_ops_per_s) return fail(RQA_ERR_INVALID_ARG, "lane_ops_per_s is NULL");
    // 32 waves per CU (8 per SIMD) with 16 independent chains each keep every
    // SIMD's issue port busy; 8 launches of a few milliseconds, the fastest counts
    const uint32_t blocks = (uint32_t)c->num_cu * 8;
    const uint32_t iters = 2048;
    if ((st = ensure_pool(c, sizeof(uint32_t) * valu_probe_threads(blocks)))) return st;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RQA_ERR_DEVICE, "hipEventCreate failed");
    }
    double best = 1e300;
    hipError_t e = launch_valu_probe(c->stream, (int)kind, blocks, iters, (uint32_t*)c->pool);  // warm-up
    for (int rep = 0; rep < 8 && e == hipSuccess; ++rep) {
        float ms = 0.f;
        e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess) e = launch_valu_probe(c->stream, (int)kind, blocks, iters, (uint32_t*)c->pool);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms > 0.f) best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(RQA_ERR_DEVICE, "VALU probe failed: %s", hipGetErrorString(e));
    *lane_ops_per_s = valu_probe_lane_ops(blocks, iters) / (best * 1e-3);
    if (ms_out) *ms_out = best;
    return RQA_OK;
}

rqa_status rqa_set_shape(rqa_ctx* c, uint32_t segment, uint32_t chunk_tiles)
{
    if (!c) return fail(RQA_ERR_INVALID_ARG, "context is NULL");
    if (segment && (segment % TILE_W || segment > 65536))
        return fail(RQA_ERR_INVALID_ARG, "segment %u must be a multiple of 64 in 64..65536", segment);
    if (chunk_tiles > 4096) return fail(RQA_ERR_INVALID_ARG, "chunk_tiles %u > 4096", chunk_tiles);
    c->seg = segment;
    c->chunk_tiles = chunk_tiles;
    return RQA_OK;
}

rqa_status rqa_set_grid(rqa_ctx* c, uint32_t workgroups)
{
    if (!c) return fail(RQA_ERR_INVALID_ARG, "context is NULL");
    if (workgroups > 65536) return fail(RQA_ERR_INVALID_ARG, "workgroups %u > 65536", workgroups);
    c->grid = workgroups;
    return RQA_OK;
}

rqa_status rqa_select_thresholds(rqa_ctx* c, const float* series, uint64_t n, const rqa_params* p,
                                 const double* rr, uint32_t K, uint32_t flags, float* eps_out,
                                 uint64_t* k_out, uint64_t* count_out)
{
    if (c) reset_phases(c);
    int sel = 0;
    rqa_status st = check_flags_select(flags, &sel);
    if (st) return st;
    if (!eps_out) return fail(RQA_ERR_INVALID_ARG, "eps_out is NULL");
    Job job;
    if ((st = single_job_setup(c, job, series, n, p, rr, K))) return st;
    job.sel = resolve_method(job, sel);
    job.mode = MODE_SELECT;
    if (job.sel) {
        if ((st = select_windowed(c, job))) return st;
    } else {
        c->stat_passes = 3;
        c->stat_fallback = 0;
        c->stat_missed = 0;
        if ((st = run_job(c, job))) return st;
    }
    for (uint32_t r = 0; r < K; ++r) {
        eps_out[r] = job.eps[r];
        if (k_out) k_out[r] = job.kout[r];
        if (count_out) count_out[r] = job.count_sel[r];
    }
    return RQA_OK;
}

rqa_status rqa_det_curve(rqa_ctx* c, const float* series, uint64_t n, const rqa_params* p, const float* eps,
                         uint32_t K, uint32_t flags, uint64_t* count_out, double* rr_out, double* det_out,
                         double* det_mean_out, uint64_t* hist_out, uint64_t hist_len)
{
    if (c) reset_phases(c);
    if (flags & ~(uint32_t)RQA_FULL_HIST) return fail(RQA_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const bool full = (flags & RQA_FULL_HIST) != 0;
    if (!full && (hist_out || hist_len)) return fail(RQA_ERR_INVALID_ARG, "hist_out/hist_len need RQA_FULL_HIST");
    if (full && !hist_out) return fail(RQA_ERR_INVALID_ARG, "RQA_FULL_HIST with hist_out NULL");
    if (full && (hist_len < 1 || hist_len > RQA_MAX_HIST_LEN))
        return fail(RQA_ERR_INVALID_ARG, "hist_len=%llu outside 1..%u", (unsigned long long)hist_len,
                    (unsigned)RQA_MAX_HIST_LEN);
    if (!count_out || !rr_out || !det_out || !det_mean_out) return fail(RQA_ERR_INVALID_ARG, "an output is NULL");
    Job job;
    rqa_status st = single_job(c, job, series, n, p, nullptr, eps, K, MODE_SWEEP);
    if (st) return st;
    if (full && (st = hist_in_passes(c, job, job.eps_bits, (uint32_t)hist_len, hist_out))) return st;
    for (uint32_t r = 0; r < K; ++r) {
        count_out[r] = job.count[r];
        rr_out[r] = job.rr[r];
        det_out[r] = job.det[r];
    }
    *det_mean_out = job.det_mean[0];
    return RQA_OK;
}

rqa_status rqa_run(rqa_ctx* c, const float* series, uint64_t n, const rqa_params* p, const double* rr, uint32_t K,
                   uint32_t flags, float* eps_out, uint64_t* k_out, uint64_t* count_out, double* rr_out,
                   double* det_out, double* det_mean_out)
{
    if (c) reset_phases(c);
    int sel = 0;
    rqa_status st = check_flags_select(flags, &sel);
    if (st) return st;
    if (!det_mean_out) return fail(RQA_ERR_INVALID_ARG, "det_mean_out is NULL");
    Job job;
    if ((st = single_job_setup(c, job, series, n, p, rr, K))) return st;
    job.sel = resolve_method(job, sel);
    if ((st = select_and_sweep(c, job))) return st;
    for (uint32_t r = 0; r < K; ++r) {
        if (eps_out) eps_out[r] = job.eps[r];
        if (k_out) k_out[r] = job.kout[r];
        if (count_out) count_out[r] = job.count[r];
        if (rr_out) rr_out[r] = job.rr[r];
        if (det_out) det_out[r] = job.det[r];
    }
    *det_mean_out = job.det_mean[0];
    return RQA_OK;
}

rqa_status rqa_batch(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets, const rqa_params* p,
                     const double* rr, uint32_t K, uint32_t flags, float* eps_out, double* rr_out, double* det_out,
                     double* det_mean_out, uint64_t* count_out)
{
    if (c) reset_phases(c);
    rqa_status st = check_ctx(c);
    if (st) return st;
    int sel = 0;
    if ((st = check_flags_select(flags, &sel))) return st;
    if (!eps_out || !rr_out || !det_out || !det_mean_out) return fail(RQA_ERR_INVALID_ARG, "an output is NULL");
    Job job;
    if ((st = build_batch_job(job, S, concat, offsets, p, rr, K))) return st;
    job.sel = resolve_method(job, sel);
    if ((st = select_and_sweep(c, job))) return st;
    for (size_t i = 0; i < (size_t)S * K; ++i) {
        eps_out[i] = job.eps[i];
        rr_out[i] = job.rr[i];
        det_out[i] = job.det[i];
        if (count_out) count_out[i] = job.count[i];
    }
    for (uint32_t s = 0; s < S; ++s) det_mean_out[s] = job.det_mean[s];
    return RQA_OK;
}

rqa_status rqa_batch_static(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets,
                            const rqa_params* p, const double* rr, uint32_t K, uint32_t flags, float* eps_out,
                            double* rr_out, double* det_out, double* det_mean_out, uint64_t* count_out)
{
    if (c) reset_phases(c);
    rqa_status st = check_ctx(c);
    if (st) return st;
    int sel = 0;
    if ((st = check_flags_select(flags, &sel))) return st;
    // the network's activations live in allocated memory
    if (sel == 1)
        return fail(RQA_ERR_UNSUPPORTED, "rqa_batch_static takes RQA_SEL_AUTO, RQA_SEL_PLAIN, RQA_SEL_SAMPLE or "
                                         "RQA_SEL_WINDOW");
    if (!c->static_dev) return fail(RQA_ERR_DEVICE, "the static scratch of device %d is not resolved", c->device);
    c->use_static = true;
    st = rqa_batch(c, S, concat, offsets, p, rr, K, flags, eps_out, rr_out, det_out, det_mean_out, count_out);
    c->use_static = false;
    return st;
}

rqa_status rqa_batch_hist(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets, const rqa_params* p,
                          const double* rr, uint32_t K, uint32_t flags, float* eps_out, double* rr_out,
                          double* det_out, double* det_mean_out, uint64_t* count_out, uint64_t* hist_out,
                          uint64_t hist_len)
{
    if (c) reset_phases(c);
    rqa_status st = check_ctx(c);
    if (st) return st;
    int sel = 0;
    if ((st = check_flags_select(flags, &sel))) return st;
    if (!eps_out || !rr_out || !det_out || !det_mean_out || !hist_out)
        return fail(RQA_ERR_INVALID_ARG, "an output is NULL");
    if (hist_len < 1 || hist_len > RQA_MAX_HIST_LEN)
        return fail(RQA_ERR_INVALID_ARG, "hist_len=%llu outside 1..%u", (unsigned long long)hist_len,
                    (unsigned)RQA_MAX_HIST_LEN);
    Job job;
    if ((st = build_batch_job(job, S, concat, offsets, p, rr, K))) return st;
    job.sel = resolve_method(job, sel);
    if ((st = select_and_sweep(c, job))) return st;
    std::vector<uint32_t> bits((size_t)S * K);
    std::memcpy(bits.data(), job.eps.data(), sizeof(uint32_t) * bits.size());
    if ((st = hist_in_passes(c, job, bits, (uint32_t)hist_len, hist_out))) return st;
    for (size_t i = 0; i < (size_t)S * K; ++i) {
        eps_out[i] = job.eps[i];
        rr_out[i] = job.rr[i];
        det_out[i] = job.det[i];
        if (count_out) count_out[i] = job.count[i];
    }
    for (uint32_t s = 0; s < S; ++s) det_mean_out[s] = job.det_mean[s];
    return RQA_OK;
}

rqa_status rqa_autotune(rqa_ctx* c, const float* series, uint64_t n, const rqa_params* p, const double* rr, uint32_t K,
                        uint32_t* segment_out, uint32_t* chunk_tiles_out)
{
    Job job;
    rqa_status st = single_job_setup(c, job, series, n, p, rr, K);
    if (st) return st;
    job.sel = resolve_method(job, -1);  // the method a call with default flags takes
    return tune_job(c, job, segment_out, chunk_tiles_out);
}

rqa_status rqa_autotune_batch(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets,
                              const rqa_params* p, const double* rr, uint32_t K, uint32_t* chunk_tiles_out)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    Job job;
    if ((st = build_batch_job(job, S, concat, offsets, p, rr, K))) return st;
    job.sel = resolve_method(job, -1);  // the method a call with default flags takes
    return tune_job(c, job, nullptr, chunk_tiles_out);
}

static rqa_status sketch_job(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets,
                             const rqa_params* p, uint64_t seed, bool want_sample, Job& job)
{
    rqa_status st;
    job.base = concat;
    job.K = 1;
    job.mode = MODE_SKETCH;
    job.seed = seed;
    job.want_sample = want_sample;
    for (uint32_t s = 0; s < S; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(RQA_ERR_INVALID_ARG, "offsets decrease at series %u", s);
        uint64_t nv, M;
        if ((st = check_params(&p[s], offsets[s + 1] - offsets[s], &nv, &M))) return st;
        job.series.push_back({offsets[s], offsets[s + 1] - offsets[s], p[s]});
    }
    return run_job(c, job);
}

rqa_status rqa_sketch_sample(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets,
                             const rqa_params* p, uint64_t seed, uint32_t* sample_out)
{
    if (c) reset_phases(c);
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (S == 0 || !concat || !offsets || !p || !sample_out) return fail(RQA_ERR_INVALID_ARG, "a required pointer is NULL");
    Job job;
    if ((st = sketch_job(c, S, concat, offsets, p, seed, true, job))) return st;
    std::memcpy(sample_out, job.sample.data(), sizeof(uint32_t) * job.sample.size());
    return RQA_OK;
}

rqa_status rqa_sketch_batch(rqa_ctx* c, uint32_t S, const float* concat, const uint64_t* offsets,
                            const rqa_params* p, uint64_t seed, float* features_out, uint32_t* scale_out)
{
    if (c) reset_phases(c);
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (S == 0 || !concat || !offsets || !p || !features_out) return fail(RQA_ERR_INVALID_ARG, "a required pointer is NULL");
    Job job;
    job.base = concat;
    job.K = 1;
    job.mode = MODE_SKETCH;
    job.seed = seed;
    for (uint32_t s = 0; s < S; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(RQA_ERR_INVALID_ARG, "offsets decrease at series %u", s);
        uint64_t nv, M;
        if ((st = check_params(&p[s], offsets[s + 1] - offsets[s], &nv, &M))) return st;
        job.series.push_back({offsets[s], offsets[s + 1] - offsets[s], p[s]});
    }
    if ((st = run_job(c, job))) return st;
    std::memcpy(features_out, job.features.data(), sizeof(float) * job.features.size());
    if (scale_out) std::memcpy(scale_out, job.scale.data(), sizeof(uint32_t) * S);
    return RQA_OK;
}

rqa_status rqa_set_window(rqa_ctx* c, float lo, float hi)
{
    if (!c) return fail(RQA_ERR_INVALID_ARG, "context is NULL");
    uint32_t a, b;
    rqa_status st;
    if ((st = check_eps(lo, &a)) || (st = check_eps(hi, &b))) return st;
    if (b < a) return fail(RQA_ERR_INVALID_ARG, "window upper end below lower end");
    c->win_lo = a;
    c->win_hi = b;
    return RQA_OK;
}

rqa_status rqa_set_sample_width(rqa_ctx* c, float z)
{
    if (!c) return fail(RQA_ERR_INVALID_ARG, "context is NULL");
    if (!(z > 0.f) || !std::isfinite(z)) return fail(RQA_ERR_INVALID_ARG, "width must be positive");
    c->sample_z = z;
    return RQA_OK;
}

rqa_status rqa_selection_stats(rqa_ctx* c, uint32_t* full_passes, uint32_t* series_fallback, uint32_t* targets_missed)
{
    if (!c) return fail(RQA_ERR_INVALID_ARG, "context is NULL");
    if (full_passes) *full_passes = c->stat_passes;
    if (series_fallback) *series_fallback = c->stat_fallback;
    if (targets_missed) *targets_missed = c->stat_missed;
    return RQA_OK;
}

rqa_status rqa_tune_save(rqa_ctx* c, const char* path)
{
    if (!c || !path) return fail(RQA_ERR_INVALID_ARG, "context or path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(RQA_ERR_INVALID_ARG, "cannot write %s", path);
    std::fprintf(f, "{\"rqa_tune\": 1, \"entries\": [");
    bool first = true;
    for (const auto& kv : c->tune) {
        std::fprintf(f, "%s\n  {\"nvlog2\": %d, \"variant\": %d, \"kcls\": %d, \"segment\": %u, \"chunk_tiles\": %u}",
                     first ? "" : ",", kv.first.nvlog2, kv.first.variant, kv.first.kcls, kv.second.seg, kv.second.chunk);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    std::fclose(f);
    return RQA_OK;
}

rqa_status rqa_tune_load(rqa_ctx* c, const char* path)
{
    if (!c || !path) return fail(RQA_ERR_INVALID_ARG, "context or path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(RQA_ERR_INVALID_ARG, "cannot read %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    if (text.find("\"rqa_tune\": 1") == std::string::npos) return fail(RQA_ERR_INVALID_ARG, "%s is not a tuning table", path);
    std::map<TuneKey, Shape> table;
    size_t pos = 0;
    while ((pos = text.find("{\"nvlog2\":", pos)) != std::string::npos) {
        int nvlog2, variant, kcls;
        unsigned seg, chunk;
        if (std::sscanf(text.c_str() + pos,
                        "{\"nvlog2\": %d, \"variant\": %d, \"kcls\": %d, \"segment\": %u, \"chunk_tiles\": %u}",
                        &nvlog2, &variant, &kcls, &seg, &chunk) != 5)
            return fail(RQA_ERR_INVALID_ARG, "malformed entry in %s", path);
        if ((seg && (seg % TILE_W || seg > 65536)) || chunk == 0 || chunk > 4096)
            return fail(RQA_ERR_INVALID_ARG, "out-of-range shape in %s", path);
        table[TuneKey{nvlog2, variant, kcls}] = {seg, chunk};
        ++pos;
    }
    c->tune = table;
    return RQA_OK;
}

rqa_status rqa_averaged_det(const double* det, uint32_t K, double* curve_out)
{
    if (!det || !curve_out || K == 0) return fail(RQA_ERR_INVALID_ARG, "det or curve_out is NULL, or K is 0");
    double sum = 0.0;
    for (uint32_t r = 0; r < K; ++r) {
        sum += det[r];
        curve_out[r] = sum / (double)(r + 1);
    }
    return RQA_OK;
}

rqa_status rqa_line_measures(const uint64_t* hist, uint32_t K, uint64_t hist_len, uint32_t lmin, double* L_out,
                             uint64_t* lmax_out)
{
    if (!hist || K == 0 || hist_len == 0 || lmin == 0)
        return fail(RQA_ERR_INVALID_ARG, "hist is NULL, or K, hist_len or lmin is 0");
    for (uint32_t r = 0; r < K; ++r) {
        const uint64_t* row = hist + (size_t)r * hist_len;
        double num = 0.0, den = 0.0;
        uint64_t lmax = 0;
        for (uint64_t l = 0; l < hist_len; ++l) {
            if (!row[l]) continue;
            lmax = l;
            if (l >= lmin) {
                num += (double)l * (double)row[l];
                den += (double)row[l];
            }
        }
        if (L_out) L_out[r] = den > 0.0 ? num / den : NAN;
        if (lmax_out) lmax_out[r] = lmax;
    }
    return RQA_OK;
}

const char* rqa_status_string(rqa_status s)
{
    switch (s) {
    case RQA_OK: return "ok";
    case RQA_ERR_INVALID_ARG: return "invalid argument";
    case RQA_ERR_TOO_SHORT: return "series too short";
    case RQA_ERR_NONFINITE: return "non-finite sample";
    case RQA_ERR_DEVICE: return "device error";
    case RQA_ERR_NOMEM: return "out of device memory";
    case RQA_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* rqa_last_error(void) { return g_err; }

}  // extern "C"

// ------------------------------------------------------------------ network

namespace {

rqa_status ensure_mlp(rqa_ctx* c)
{
    if (c->mlp) return RQA_OK;
    if (hipMalloc(&c->mlp, sizeof(float) * 4 * MLP_PARAMS) != hipSuccess) {
        c->mlp = nullptr;
        (void)hipGetLastError();
        return fail(RQA_ERR_NOMEM, "hipMalloc of the network failed");
    }
    if (hipMalloc(&c->mlp_partial, sizeof(float) * 4096) != hipSuccess) {
        c->mlp_partial = nullptr;
        (void)hipGetLastError();
        return fail(RQA_ERR_NOMEM, "hipMalloc of the loss buffer failed");
    }
    HIP_TRY(launch_zero(c->stream, c->mlp, sizeof(float) * 4 * MLP_PARAMS));
    return RQA_OK;
}

rqa_status ensure_acts(rqa_ctx* c, uint32_t B, MlpActs& a)
{
    if (B > c->mlp_cap) {
        if (c->mlp_acts) (void)hipFree(c->mlp_acts);
        c->mlp_acts = nullptr;
        c->mlp_cap = 0;
        const size_t per = 5 * MLP_H + 2 * MLP_OUT + MLP_H;  // Z1 A1 Z2 A2 dZ2 dZ1 + Y dY
        if (hipMalloc(&c->mlp_acts, sizeof(float) * per * B) != hipSuccess) {
            c->mlp_acts = nullptr;
            (void)hipGetLastError();
            return fail(RQA_ERR_NOMEM, "hipMalloc of network activations failed");
        }
        c->mlp_cap = B;
    }
    float* p = c->mlp_acts;
    const size_t cap = c->mlp_cap;
    a.Z1 = p; p += cap * MLP_H;
    a.A1 = p; p += cap * MLP_H;
    a.Z2 = p; p += cap * MLP_H;
    a.A2 = p; p += cap * MLP_H;
    a.dZ2 = p; p += cap * MLP_H;
    a.dZ1 = p; p += cap * MLP_H;
    a.Y = p; p += cap * MLP_OUT;
    a.dY = p;
    return RQA_OK;
}

rqa_status check_model(rqa_ctx* c, uint32_t B)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (!c->has_model) return fail(RQA_ERR_INVALID_ARG, "no network: call rqa_mlp_init or rqa_mlp_set_params");
    if (B == 0 || B > 65536) return fail(RQA_ERR_INVALID_ARG, "batch %u outside 1..65536", B);
    return RQA_OK;
}

// forward + backward into the gradient buffer; loss summed on the host
rqa_status mlp_grad(rqa_ctx* c, const float* x, const float* t, uint32_t B, double* loss)
{
    MlpActs a;
    rqa_status st = ensure_acts(c, B, a);
    if (st) return st;
    float* params = c->mlp;
    float* grad = c->mlp + MLP_PARAMS;
    HIP_TRY(mlp_forward(c->stream, params, x, (int)B, a, a.Y));
    int np = 0;
    HIP_TRY(mlp_backward(c->stream, params, x, t, (int)B, a, grad, c->mlp_partial, &np));
    if (np > 4096) return fail(RQA_ERR_INVALID_ARG, "batch too large for the loss buffer");
    float part[4096];
    HIP_TRY(hipMemcpyAsync(part, c->mlp_partial, sizeof(float) * np, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (int i = 0; i < np; ++i) sum += part[i];
    if (loss) *loss = sum;
    return RQA_OK;
}

}  // namespace

extern "C" {

rqa_status rqa_mlp_init(rqa_ctx* c, uint64_t seed)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if ((st = ensure_mlp(c))) return st;
    // He-uniform weights from the SplitMix64 stream `seed`, zero biases
    std::vector<float> h(MLP_PARAMS, 0.f);
    const MlpOffsets o;
    uint64_t ctr = 0;
    auto uni = [&]() {
        uint64_t z = seed + (++ctr) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int fan_in, int count) {
        const double lim = std::sqrt(6.0 / fan_in);
        for (int i = 0; i < count; ++i) h[off + i] = (float)((2.0 * uni() - 1.0) * lim);
    };
    fill(o.W1, MLP_IN, MLP_IN * MLP_H);
    fill(o.W2, MLP_H, MLP_H * MLP_H);
    fill(o.W3, MLP_H, MLP_H * MLP_OUT);
    HIP_TRY(hipMemcpyAsync(c->mlp, h.data(), sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_zero(c->stream, c->mlp + MLP_PARAMS, sizeof(float) * 3 * MLP_PARAMS));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    c->has_model = true;
    return RQA_OK;
}

rqa_status rqa_mlp_set_params(rqa_ctx* c, const float* params, uint64_t count)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (!params || count != (uint64_t)MLP_PARAMS) return fail(RQA_ERR_INVALID_ARG, "need %d parameters", MLP_PARAMS);
    for (uint64_t i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return fail(RQA_ERR_NONFINITE, "parameter %llu is not finite", (unsigned long long)i);
    if ((st = ensure_mlp(c))) return st;
    HIP_TRY(hipMemcpyAsync(c->mlp, params, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_zero(c->stream, c->mlp + MLP_PARAMS, sizeof(float) * 3 * MLP_PARAMS));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    c->has_model = true;
    return RQA_OK;
}

rqa_status rqa_mlp_get_params(rqa_ctx* c, float* params, uint64_t count)
{
    rqa_status st = check_model(c, 1);
    if (st) return st;
    if (!params || count != (uint64_t)MLP_PARAMS) return fail(RQA_ERR_INVALID_ARG, "need %d parameters", MLP_PARAMS);
    HIP_TRY(hipMemcpyAsync(params, c->mlp, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return RQA_OK;
}

rqa_status rqa_mlp_forward(rqa_ctx* c, const float* x_dev, uint32_t B, float* y_dev)
{
    rqa_status st = check_model(c, B);
    if (st) return st;
    if (!x_dev || !y_dev) return fail(RQA_ERR_INVALID_ARG, "a device pointer is NULL");
    MlpActs a;
    if ((st = ensure_acts(c, B, a))) return st;
    HIP_TRY(mlp_forward(c->stream, c->mlp, x_dev, (int)B, a, y_dev));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return RQA_OK;
}

rqa_status rqa_mlp_gradients(rqa_ctx* c, const float* x_dev, const float* t_dev, uint32_t B, float* grad_out,
                             double* loss_out)
{
    rqa_status st = check_model(c, B);
    if (st) return st;
    if (!x_dev || !t_dev || !grad_out) return fail(RQA_ERR_INVALID_ARG, "a pointer is NULL");
    if ((st = mlp_grad(c, x_dev, t_dev, B, loss_out))) return st;
    HIP_TRY(hipMemcpyAsync(grad_out, c->mlp + MLP_PARAMS, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return RQA_OK;
}

rqa_status rqa_mlp_train_step(rqa_ctx* c, const float* x_dev, const float* t_dev, uint32_t B, float lr,
                              double* loss_out)
{
    rqa_status st = check_model(c, B);
    if (st) return st;
    if (!x_dev || !t_dev) return fail(RQA_ERR_INVALID_ARG, "a device pointer is NULL");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(RQA_ERR_INVALID_ARG, "learning rate must be positive");
    if ((st = mlp_grad(c, x_dev, t_dev, B, loss_out))) return st;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    c->adam_t += 1;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)c->adam_t));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)c->adam_t));
    HIP_TRY(mlp_adam(c->stream, c->mlp, c->mlp + MLP_PARAMS, c->mlp + 2 * MLP_PARAMS, c->mlp + 3 * MLP_PARAMS, lr, b1,
                     b2, eps, c1, c2));
    return RQA_OK;
}

rqa_status rqa_mlp_set_bracket(rqa_ctx* c, const float* delta, uint32_t n)
{
    rqa_status st = check_ctx(c);
    if (st) return st;
    if (!delta || n != (uint32_t)MLP_OUT) return fail(RQA_ERR_INVALID_ARG, "need %d half-widths", MLP_OUT);
    for (uint32_t i = 0; i < n; ++i)
        if (!(delta[i] >= 0.f) || !std::isfinite(delta[i])) return fail(RQA_ERR_INVALID_ARG, "half-width %u invalid", i);
    std::memcpy(c->bracket_delta, delta, sizeof(float) * MLP_OUT);
    return RQA_OK;
}

}  // extern "C"
