/*
 * rqa_oracle.c -- plain CPU oracle for averaged recurrence quantification
 * analysis (Panis, Adamek & Marwan, "Averaged Recurrence Quantification
 * Analysis", arXiv 2208.09136).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no FMA contraction, IEEE binary32 with round-to-nearest-even, denormals
 * kept; x86-64 evaluates float in SSE registers, so there is no excess
 * precision).
 *
 * What is computed, step by step (the numbers refer to the paper):
 *   - delay vectors x(t) = [y(t), y(t-tau), ..., y(t-(m-1)tau)]
 *     (Methodology, Lorenz-system subsection).  With 0-based vector index
 *     i = t-(m-1)tau, component k of vector i is y[i + (m-1-k)tau].
 *   - a distance key per pair of vectors: the maximum norm of the paper
 *     (Recurrence quantification analysis section, after Eq. 1), or the
 *     squared Euclidean norm summed left to right over k = 0..m-1.
 *   - the recurrence matrix R_ij of Eq. 1 over the upper triangle j > i
 *     (Technical implementation on a GPU), with a Theiler window w >= 1 that
 *     removes pairs with j - i < w.  The threshold test is key <= eps (the
 *     paper's strict Heaviside with eps' = the next float above eps gives
 *     the same matrix).
 *   - eps for a preselected recurrence rate (Averaged RQA section): the
 *     k-th smallest key, k = ceil(RR * M) on the RR quantised to 1e-9.
 *   - RR (Eq. 3) as C / M over the same pair set, the diagonal-line length
 *     histogram P(l) (Eq. 4), DET = sum_{l >= lmin} l P(l) / sum R, and the
 *     averaged DET (the averaged-determinism equation of the Averaged RQA
 *     section) as the plain mean over the given RR targets.
 *
 * Parity status of each function is stated at the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_TOO_SHORT (-2)
#define ORC_ERR_NONFINITE (-3)
#define ORC_ERR_NOMEM (-5)

#define ORC_NORM_MAX 0
#define ORC_NORM_EUCLID 1

/* Number of delay vectors: N - (m-1) tau, or 0 if the series is too short. */
uint64_t orc_num_vectors(uint64_t n, uint32_t m, uint32_t tau)
{
    uint64_t span = (uint64_t)(m - 1) * (uint64_t)tau;
    if (m == 0 || span >= n) return 0;
    return n - span;
}

/* Number of pairs (i, j) with 0 <= i < j < nv and j - i >= w. */
uint64_t orc_num_pairs(uint64_t nv, uint32_t w)
{
    if (w == 0 || nv <= (uint64_t)w) return 0;
    uint64_t a = nv - w;
    return a * (a + 1) / 2;
}

/* Rank of the threshold for a target recurrence rate rr in (0, 1]:
 * q = round(rr * 1e9), k = ceil(q * M / 1e9), clamped to [1, M].
 * Exact 128-bit integer arithmetic.  Returns 0 for an invalid rr or M = 0. */
uint64_t orc_rank(double rr, uint64_t M)
{
    if (!(rr > 0.0) || !(rr <= 1.0) || M == 0) return 0;
    long long q = llround(rr * 1e9);
    if (q < 1) q = 1;
    if (q > 1000000000LL) q = 1000000000LL;
    unsigned __int128 prod = (unsigned __int128)(uint64_t)q * (unsigned __int128)M;
    unsigned __int128 k = (prod + 999999999u) / 1000000000u;
    if (k < 1) k = 1;
    if (k > M) k = M;
    return (uint64_t)k;
}

/* Distance key of delay vectors i and j (0-based).  Max norm: max_k |d_k|.
 * Euclidean: the squared norm d_0^2 + d_1^2 + ... folded left in k, with
 * every product and sum rounded to binary32.  d_k = y[i+(m-1-k)tau] -
 * y[j+(m-1-k)tau]. */
float orc_key(const float *y, uint32_t m, uint32_t tau, uint32_t norm,
              uint64_t i, uint64_t j)
{
    float acc = 0.0f;
    for (uint32_t k = 0; k < m; ++k) {
        uint64_t off = (uint64_t)(m - 1 - k) * tau;
        float d = y[i + off] - y[j + off];
        if (norm == ORC_NORM_MAX) {
            float a = fabsf(d);
            if (a > acc) acc = a;
        } else {
            float sq = d * d;
            acc = (k == 0) ? sq : acc + sq;
        }
    }
    return acc;
}

static int check_common(const float *y, uint64_t n, uint32_t m, uint32_t tau,
                        uint32_t norm, uint32_t w, uint64_t *nv, uint64_t *M)
{
    if (!y || m == 0 || tau == 0 || w == 0) return ORC_ERR_INVALID;
    if (norm != ORC_NORM_MAX && norm != ORC_NORM_EUCLID) return ORC_ERR_INVALID;
    for (uint64_t i = 0; i < n; ++i)
        if (!isfinite(y[i])) return ORC_ERR_NONFINITE;
    *nv = orc_num_vectors(n, m, tau);
    *M = orc_num_pairs(*nv, w);
    if (*M == 0) return ORC_ERR_TOO_SHORT;
    return ORC_OK;
}

/* All keys in diagonal-major order: d = w .. nv-1, then t = 0 .. nv-1-d,
 * pair (t, t+d).  out must hold M floats.  Used by the tests to compare with
 * an independent brute force. */
int orc_keys(const float *y, uint64_t n, uint32_t m, uint32_t tau,
             uint32_t norm, uint32_t w, float *out)
{
    uint64_t nv, M;
    int st = check_common(y, n, m, tau, norm, w, &nv, &M);
    if (st) return st;
    uint64_t pos = 0;
    for (uint64_t d = w; d < nv; ++d)
        for (uint64_t t = 0; t + d < nv; ++t)
            out[pos++] = orc_key(y, m, tau, norm, t, t + d);
    return ORC_OK;
}

/* For each value v[r] (r < K), count keys with key < v[r] (lt) and
 * key <= v[r] (le).  One brute-force pass over all pairs.  lt may be NULL. */
int orc_count(const float *y, uint64_t n, uint32_t m, uint32_t tau,
              uint32_t norm, uint32_t w, const float *v, uint32_t K,
              uint64_t *lt, uint64_t *le)
{
    uint64_t nv, M;
    int st = check_common(y, n, m, tau, norm, w, &nv, &M);
    if (st) return st;
    if (!v || !le || K == 0) return ORC_ERR_INVALID;
    for (uint32_t r = 0; r < K; ++r) { le[r] = 0; if (lt) lt[r] = 0; }
#pragma omp parallel
    {
        uint64_t *my_le = calloc(K, sizeof(uint64_t));
        uint64_t *my_lt = calloc(K, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
        for (int64_t d = (int64_t)w; d < (int64_t)nv; ++d) {
            for (uint64_t t = 0; t + (uint64_t)d < nv; ++t) {
                float key = orc_key(y, m, tau, norm, t, t + (uint64_t)d);
                for (uint32_t r = 0; r < K; ++r) {
                    if (key <= v[r]) my_le[r]++;
                    if (key < v[r]) my_lt[r]++;
                }
            }
        }
#pragma omp critical
        for (uint32_t r = 0; r < K; ++r) {
            le[r] += my_le[r];
            if (lt) lt[r] += my_lt[r];
        }
        free(my_le);
        free(my_lt);
    }
    return ORC_OK;
}

static int cmp_float(const void *a, const void *b)
{
    float x = *(const float *)a, y = *(const float *)b;
    return (x > y) - (x < y);
}

static float bits_to_float(uint32_t u)
{
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

/* Exact threshold selection: eps[r] = the k_r-th smallest key (1-based) over
 * all M pairs, k_r = orc_rank(rr[r], M).  count[r] = #{key <= eps[r]}.
 *
 * method 1: materialise every key and sort (the definition written out).
 * method 2: bisection on the binary32 pattern: eps[r] is the smallest float
 *           v with #{key <= v} >= k_r; all targets share each counting pass.
 * method 0: 1 when M <= 2e8, else 2.
 * Keys are >= +0 and at most +inf, so the search interval is [0, +inf]. */
int orc_select(const float *y, uint64_t n, uint32_t m, uint32_t tau,
               uint32_t norm, uint32_t w, const double *rr, uint32_t K,
               int method, float *eps, uint64_t *kout, uint64_t *count)
{
    uint64_t nv, M;
    int st = check_common(y, n, m, tau, norm, w, &nv, &M);
    if (st) return st;
    if (!rr || !eps || K == 0) return ORC_ERR_INVALID;
    uint64_t *k = malloc(K * sizeof(uint64_t));
    if (!k) return ORC_ERR_NOMEM;
    for (uint32_t r = 0; r < K; ++r) {
        k[r] = orc_rank(rr[r], M);
        if (k[r] == 0) { free(k); return ORC_ERR_INVALID; }
    }
    if (method == 0) method = (M <= 200000000ull) ? 1 : 2;

    if (method == 1) {
        float *all = malloc(M * sizeof(float));
        if (!all) { free(k); return ORC_ERR_NOMEM; }
        orc_keys(y, n, m, tau, norm, w, all);
        qsort(all, M, sizeof(float), cmp_float);
        for (uint32_t r = 0; r < K; ++r) {
            eps[r] = all[k[r] - 1];
            /* count of keys <= eps: first index past the run of equal keys */
            uint64_t c = k[r];
            while (c < M && all[c] <= eps[r]) ++c;
            if (count) count[r] = c;
        }
        free(all);
    } else if (method == 2) {
        uint32_t *lo = malloc(K * sizeof(uint32_t));
        uint32_t *hi = malloc(K * sizeof(uint32_t));
        float *mid = malloc(K * sizeof(float));
        uint64_t *le = malloc(K * sizeof(uint64_t));
        for (uint32_t r = 0; r < K; ++r) { lo[r] = 0u; hi[r] = 0x7F800000u; }
        for (;;) {
            int open = 0;
            for (uint32_t r = 0; r < K; ++r) {
                uint32_t md = (lo[r] < hi[r]) ? lo[r] + (hi[r] - lo[r]) / 2 : lo[r];
                mid[r] = bits_to_float(md);
                open |= lo[r] < hi[r];
            }
            if (!open) break;
            orc_count(y, n, m, tau, norm, w, mid, K, NULL, le);
            for (uint32_t r = 0; r < K; ++r) {
                if (lo[r] >= hi[r]) continue;
                uint32_t md = lo[r] + (hi[r] - lo[r]) / 2;
                if (le[r] >= k[r]) hi[r] = md; else lo[r] = md + 1;
            }
        }
        for (uint32_t r = 0; r < K; ++r) eps[r] = bits_to_float(lo[r]);
        if (count) orc_count(y, n, m, tau, norm, w, eps, K, NULL, count);
        free(lo); free(hi); free(mid); free(le);
    } else {
        free(k);
        return ORC_ERR_INVALID;
    }
    if (kout) memcpy(kout, k, K * sizeof(uint64_t));
    free(k);
    return ORC_OK;
}

/* Diagonal-line statistics for each threshold separately.
 *
 * For threshold r, R(i, j) = [key(i, j) <= eps[r]].  Every diagonal
 * d = w .. nv-1 is walked over t = 0 .. nv-1-d (cells (t, t+d)); each maximal
 * run of recurrences of length l adds one to P_r(l).  Runs that touch the
 * border of the plot are counted with the length they have inside it.
 *
 *   count[r] = sum_l l P_r(l)                     (= sum of R over the pairs)
 *   rr[r]    = count[r] / M                        (Eq. 3 as a fraction)
 *   det[r]   = sum_{l >= lmin} l P_r(l) / count[r] (Eq. 4; NaN when count = 0)
 *   det_mean = (det[0] + ... + det[K-1]) / K, summed left to right.
 *
 * hist (optional, K rows of hist_len entries) receives P_r(l) for
 * l = 0 .. hist_len-1; lines longer than hist_len-1 are added to the last
 * entry.  Row r starts at hist + r * hist_len.  P_r(0) is always 0. */
int orc_lines(const float *y, uint64_t n, uint32_t m, uint32_t tau,
              uint32_t norm, uint32_t w, uint32_t lmin, const float *eps,
              uint32_t K, uint64_t *hist, uint64_t hist_len, uint64_t *count,
              double *rr, double *det, double *det_mean)
{
    uint64_t nv, M;
    int st = check_common(y, n, m, tau, norm, w, &nv, &M);
    if (st) return st;
    if (!eps || K == 0 || lmin == 0) return ORC_ERR_INVALID;
    if (hist && hist_len == 0) return ORC_ERR_INVALID;
    uint64_t maxlen = nv - w; /* the longest diagonal has nv - w cells */
    double sum_det = 0.0;
    for (uint32_t r = 0; r < K; ++r) {
        if (isnan(eps[r])) return ORC_ERR_INVALID;
        uint64_t *P = calloc(maxlen + 1, sizeof(uint64_t));
        if (!P) return ORC_ERR_NOMEM;
        const float e = eps[r];
#pragma omp parallel
        {
            uint64_t *myP = calloc(maxlen + 1, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
            for (int64_t d = (int64_t)w; d < (int64_t)nv; ++d) {
                uint64_t run = 0;
                for (uint64_t t = 0; t + (uint64_t)d < nv; ++t) {
                    float key = orc_key(y, m, tau, norm, t, t + (uint64_t)d);
                    if (key <= e) {
                        run++;
                    } else {
                        if (run) myP[run]++;
                        run = 0;
                    }
                }
                if (run) myP[run]++;
            }
#pragma omp critical
            for (uint64_t l = 0; l <= maxlen; ++l) P[l] += myP[l];
            free(myP);
        }
        uint64_t c = 0, c_long = 0;
        for (uint64_t l = 1; l <= maxlen; ++l) {
            c += l * P[l];
            if (l >= lmin) c_long += l * P[l];
        }
        if (count) count[r] = c;
        if (rr) rr[r] = (double)c / (double)M;
        double dr = (c == 0) ? NAN : (double)c_long / (double)c;
        if (det) det[r] = dr;
        sum_det += dr;
        if (hist) {
            uint64_t *row = hist + (uint64_t)r * hist_len;
            for (uint64_t l = 0; l < hist_len; ++l) row[l] = 0;
            for (uint64_t l = 1; l <= maxlen; ++l) {
                uint64_t slot = (l < hist_len) ? l : hist_len - 1;
                row[slot] += P[l];
            }
        }
        free(P);
    }
    if (det_mean) *det_mean = sum_det / (double)K;
    return ORC_OK;
}

/* Number of OpenMP threads the oracle runs with (for the benchmark report). */
int orc_num_threads(void)
{
    return omp_get_max_threads();
}
