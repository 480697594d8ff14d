"""Distance sketch of a series: the input of the threshold-bracket network.

TEST INFRASTRUCTURE ONLY (part of the oracle; the GPU library computes the
same sketch in its own kernel and shares no code with this file).

Definition (the learned-bracket extension of the method; the paper itself
has no such step):
  * P = 4096 pairs are drawn from the M pairs of the recurrence plot (upper
    triangle, Theiler window w) with a counter-based generator: the SplitMix64
    output function (Steele, Lea and Flood, OOPSLA 2014) applied to
    seed + (s + 1) * 0x9E3779B97F4A7C15 gives v_s, and pair index p_s =
    v_s mod M.  Pairs are numbered diagonal by diagonal: diagonal d = w + delta
    holds L0 - delta pairs (L0 = nv - w), so p -> (delta, t) with
    C(delta) <= p < C(delta + 1), C(delta) = delta L0 - delta (delta - 1) / 2,
    and the pair is (t, t + w + delta).
  * scale = the 2048-th smallest sampled key (binary32 bit pattern).
  * bin of a sampled key = clamp(((bits - scale) >> 21) + 32, 0, 63): 64
    bins of a quarter binade each around the median (the float bit pattern
    is a piecewise-linear log2 of the value).
  * features[0:64] = bin counts / 4096; features[64] = log2(N) / 16;
    features[65] = m / 4.
The exact per-target output the network learns is
  t_r = (bits(eps_r) - scale) / 2^23
(a log2-like offset of the exact threshold from the sample median).
"""
import math

import numpy as np

from . import key as orc_key, num_pairs, num_vectors

P = 4096
GOLDEN = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def splitmix64(seed, s):
    """SplitMix64 output for counter s of stream `seed` (both 64-bit)."""
    z = (seed + (s + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def pair_of(p, L0, w):
    """Pair (i, j) of diagonal-major index p: the largest delta with
    C(delta) <= p, then t = p - C(delta)."""
    def C(dl):
        return dl * L0 - dl * (dl - 1) // 2
    lo, hi = 0, L0 - 1          # C is increasing on [0, L0]
    while lo < hi:               # plain bisection on the definition
        mid = (lo + hi + 1) // 2
        if C(mid) <= p:
            lo = mid
        else:
            hi = mid - 1
    t = p - C(lo)
    return t, t + w + lo


def sample_keys(y, m, tau, norm, w, seed):
    nv = num_vectors(len(y), m, tau)
    M = num_pairs(nv, w)
    L0 = nv - w
    out = np.empty(P, dtype=np.float32)
    for s in range(P):
        p = splitmix64(seed, s) % M
        i, j = pair_of(p, L0, w)
        out[s] = orc_key(y, m, tau, norm, i, j)
    return out


def bin_of(bits, scale):
    """Sketch bin of a key bit pattern: clamp(floor((bits - scale) / 2^21)
    + 32, 0, 63), i.e. quarter binades counted from the median's, bin 32
    starting at the median itself (Python's >> on a negative int floors)."""
    idx = ((int(bits) - int(scale)) >> 21) + 32
    return min(max(idx, 0), 63)


def features_from_keys(keys, n, m):
    """(features float32[66], scale_bits) from the P sampled keys of a
    series of n samples with embedding dimension m."""
    keys = np.asarray(keys, dtype=np.float32)
    if keys.size != P:
        raise ValueError(f"need {P} sampled keys")
    bits = np.sort(keys.view(np.uint32).astype(np.int64))
    scale = int(bits[P // 2 - 1])
    counts = np.zeros(64, dtype=np.int64)
    for b in bits:
        counts[bin_of(b, scale)] += 1
    f = np.zeros(66, dtype=np.float32)
    f[:64] = (counts / P).astype(np.float32)
    f[64] = np.float32(math.log2(n) / 16.0)
    f[65] = np.float32(m / 4.0)
    return f, scale


def sketch(y, m, tau, norm, w, seed):
    """(features float32[66], scale_bits) of the series."""
    keys = sample_keys(y, m, tau, norm, w, seed)
    return features_from_keys(keys, len(y), m)


def target_offsets(eps, scale):
    """t_r = (bits(eps_r) - scale) / 2^23 as float32."""
    b = np.asarray(eps, dtype=np.float32).view(np.uint32).astype(np.int64)
    return ((b - scale) / float(1 << 23)).astype(np.float32)
