"""Seeded synthetic inputs for averaged RQA (arXiv 2208.09136).

This module only produces input series; it contains none of the method's
arithmetic and serves both the GPU path and the CPU oracle.

Systems follow the Methodology section of the paper: a periodic signal, the
logistic map x_{n+1} = r x_n (1 - x_n) and the x-component of the Lorenz
system (sigma = 10, rho = 28, beta = 8/3, Runge-Kutta, step 0.01), each
corrupted by additive Gaussian white noise at a signal-to-noise ratio
SNR = var(signal) / var(noise).  The workload configurations give SNR in dB,
the logistic parameter r = 4, a plain sine of period 37.3 samples instead of
the paper's light-curve generator, and 5000 discarded Lorenz transient steps.

Everything is generated in float64 and cast to float32 once at the end.
"""
import math

import numpy as np

SYSTEMS = ("sine", "logistic", "lorenz")
RR_20 = tuple(k / 100.0 for k in range(1, 21))   # 0.01, 0.02, ..., 0.20
NORM_MAX = 0
NORM_EUCLID = 1


def rng_for(*key):
    """PCG64 stream for an integer key tuple (config, system, snr, realisation)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def logistic(n, rng, r=4.0, transient=1000):
    """Logistic map in float64 from x0 ~ U(0.1, 0.9), transient discarded."""
    x = rng.uniform(0.1, 0.9)
    for _ in range(transient):
        x = r * x * (1.0 - x)
    out = np.empty(n, dtype=np.float64)
    for i in range(n):
        out[i] = x
        x = r * x * (1.0 - x)
    return out


def sine(n, rng, period=37.3):
    """sin(2 pi t / period + phi) with phi ~ U(0, 2 pi)."""
    phi = rng.uniform(0.0, 2.0 * math.pi)
    t = np.arange(n, dtype=np.float64)
    return np.sin(2.0 * math.pi * t / period + phi)


def _lorenz_rhs(x, y, z, sigma, rho, beta):
    return sigma * (y - x), x * (rho - z) - y, x * y - beta * z


def lorenz_x(n, rng, dt=0.01, transient=5000, sigma=10.0, rho=28.0, beta=8.0 / 3.0,
             znorm=True):
    """x-component of the Lorenz system by classical RK4, started at
    (1, 1, 1) + N(0, 0.01^2), transient discarded, z-normalised."""
    s = np.array([1.0, 1.0, 1.0]) + rng.normal(0.0, 0.01, size=3)
    x, y, z = float(s[0]), float(s[1]), float(s[2])
    out = np.empty(n, dtype=np.float64)
    h = dt
    for i in range(transient + n):
        if i >= transient:
            out[i - transient] = x
        k1 = _lorenz_rhs(x, y, z, sigma, rho, beta)
        k2 = _lorenz_rhs(x + 0.5 * h * k1[0], y + 0.5 * h * k1[1], z + 0.5 * h * k1[2],
                         sigma, rho, beta)
        k3 = _lorenz_rhs(x + 0.5 * h * k2[0], y + 0.5 * h * k2[1], z + 0.5 * h * k2[2],
                         sigma, rho, beta)
        k4 = _lorenz_rhs(x + h * k3[0], y + h * k3[1], z + h * k3[2], sigma, rho, beta)
        x += h / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
        y += h / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
        z += h / 6.0 * (k1[2] + 2.0 * k2[2] + 2.0 * k3[2] + k4[2])
    if znorm:
        out = (out - out.mean()) / out.std()
    return out


def add_noise(signal, snr_db, rng):
    """Add N(0, s^2) noise with s^2 = var(signal) / 10^(snr_db / 10)
    (population variance)."""
    var = float(np.var(signal))
    sigma = math.sqrt(var / (10.0 ** (snr_db / 10.0)))
    return signal + rng.standard_normal(len(signal)) * sigma


def clean(system, n, rng):
    if system == "sine":
        return sine(n, rng)
    if system == "logistic":
        return logistic(n, rng)
    if system == "lorenz":
        return lorenz_x(n, rng)
    raise ValueError(system)


def series(system, n, snr_db, key):
    """float32 series of a system plus noise at snr_db, seeded by key.
    snr_db=None gives the noise-free signal."""
    rng = rng_for(*key)
    s = clean(system, n, rng)
    if snr_db is not None:
        s = add_noise(s, snr_db, rng)
    y = s.astype(np.float32)
    if not np.all(np.isfinite(y)) or float(np.std(y)) <= 0.0:
        raise RuntimeError(f"degenerate synthetic series {system} {key}")
    return y


def embedding_for(system):
    """(m, tau) per system in the workload configurations."""
    return (3, 5) if system == "lorenz" else (1, 1)


def _case(name, y, m, tau, norm, w=1, lmin=2, rr=RR_20):
    return {"name": name, "y": y, "m": m, "tau": tau, "norm": norm, "theiler": w,
            "lmin": lmin, "rr": np.array(rr, dtype=np.float64)}


def config_small(seed=0):
    """Logistic r = 4 with 10 dB noise, N = 1000, m = 1, max norm, w = 1,
    l_min = 2, K = 20 targets 0.01..0.20."""
    y = series("logistic", 1000, 10.0, (0, 1, 0, seed))
    return _case(f"logistic_n1000_snr10_seed{seed}", y, 1, 1, NORM_MAX)


SNRS_MEDIUM = (20.0, 10.0, 0.0, -10.0, -20.0)


def config_medium(n=10_000):
    """Sine (period 37.3), logistic r = 4 and Lorenz-x at 20, 10, 0, -10 and
    -20 dB, N = 10^4, Euclidean norm, m = 3 / tau = 5 for Lorenz and m = 1
    otherwise: 15 series."""
    out = []
    for si, system in enumerate(SYSTEMS):
        for qi, snr in enumerate(SNRS_MEDIUM):
            m, tau = embedding_for(system)
            y = series(system, n, snr, (1, si, qi, 0))
            out.append(_case(f"{system}_n{n}_snr{int(snr)}", y, m, tau, NORM_EUCLID))
    return out


def config_large(n=100_000, which=None):
    """Lorenz-x at 0 dB and logistic at -10 dB, N = 10^5, m = 3, tau = 5,
    Euclidean norm, w = 1, l_min = 2, K = 20."""
    cases = [("lorenz", 0.0, 2), ("logistic", -10.0, 1)]
    out = []
    for system, snr, si in cases:
        if which is not None and system != which:
            continue
        y = series(system, n, snr, (2, si, 0, 0))
        out.append(_case(f"{system}_n{n}_snr{int(snr)}", y, 3, 5, NORM_EUCLID))
    return out


SNRS_BATCH = tuple(float(20 - 5 * i) for i in range(10))   # 20 .. -25 dB


def batch_lengths(count=600, lo=100, hi=20_000, seed=3):
    """Series lengths floor(10^U(log10 lo, log10 hi)) from a fixed seed."""
    rng = rng_for(3, 99, 0, seed)
    u = rng.uniform(math.log10(lo), math.log10(hi), size=count)
    return np.floor(10.0 ** u).astype(np.int64)


def config_batch(realisations=20, lo=100, hi=20_000):
    """3 systems x 10 SNRs (20 .. -25 dB) x realisations series with lengths
    log-uniform in [lo, hi]; m = 1 for sine and logistic, m = 3 / tau = 5 for
    Lorenz; Euclidean norm, w = 1, l_min = 2, K = 20 each."""
    total = len(SYSTEMS) * len(SNRS_BATCH) * realisations
    lengths = batch_lengths(total, lo, hi)
    out = []
    idx = 0
    for si, system in enumerate(SYSTEMS):
        m, tau = embedding_for(system)
        for qi, snr in enumerate(SNRS_BATCH):
            for r in range(realisations):
                n = int(lengths[idx])
                idx += 1
                y = series(system, n, snr, (3, si, qi, r))
                out.append(_case(f"{system}_n{n}_snr{int(snr)}_r{r}", y, m, tau,
                                 NORM_EUCLID))
    return out


def periodic_integer(n, period, seed=0):
    """y_t = c_{t mod period} with distinct integer levels c: recurrences at
    threshold 0 are exactly the diagonals that are multiples of the period."""
    rng = rng_for(100, period, n, seed)
    levels = rng.permutation(period).astype(np.float64) * 3.0 + 1.0
    return levels[np.arange(n) % period].astype(np.float32)


# ---------------------------------------------------------------------------
# Many series at once (training and evaluation sets of the threshold-bracket
# network).  Same systems and noise model as above, iterated in float64 with
# the state of all series of one system held in one array, so that tens of
# thousands of series take seconds instead of hours.  Series are stored
# back to back (concatenated) with offsets.


def _iterate_many(lengths, transient, init, step, observe):
    """Run `step` on the states of all series (sorted by length, longest
    first; `step(state, a)` advances the first `a` in place) and record
    `observe(state)` for t < length of each series."""
    order = np.argsort(-lengths, kind="stable")
    lens = lengths[order]
    offs = np.concatenate([[0], np.cumsum(lens)])
    out = np.empty(int(offs[-1]), dtype=np.float64)
    state = np.ascontiguousarray(init(len(lens))[..., order])   # drawn in input order
    for _ in range(transient):
        step(state, len(lens))
    active = len(lens)
    for t in range(int(lens[0]) if len(lens) else 0):
        while active and lens[active - 1] <= t:
            active -= 1
        out[offs[:active] + t] = observe(state)[:active]
        step(state, active)
    res = [None] * len(lens)
    for pos, idx in enumerate(order):
        res[idx] = out[offs[pos]:offs[pos + 1]]
    return res


def _logistic_many(lengths, rng, r=4.0, transient=1000):
    def step(x, a):
        v = x[:a]
        v *= r * (1.0 - v)
    return _iterate_many(lengths, transient, lambda k: rng.uniform(0.1, 0.9, size=k), step, lambda x: x)


def _lorenz_many(lengths, rng, dt=0.01, transient=5000, sigma=10.0, rho=28.0, beta=8.0 / 3.0):
    h = dt

    def f(x, y, z):
        return sigma * (y - x), x * (rho - z) - y, x * y - beta * z

    def step(s, a):
        x, y, z = s[0, :a], s[1, :a], s[2, :a]
        k1 = f(x, y, z)
        k2 = f(x + 0.5 * h * k1[0], y + 0.5 * h * k1[1], z + 0.5 * h * k1[2])
        k3 = f(x + 0.5 * h * k2[0], y + 0.5 * h * k2[1], z + 0.5 * h * k2[2])
        k4 = f(x + h * k3[0], y + h * k3[1], z + h * k3[2])
        x += h / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
        y += h / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
        z += h / 6.0 * (k1[2] + 2.0 * k2[2] + 2.0 * k3[2] + k4[2])

    def init(k):
        return np.array([1.0, 1.0, 1.0])[:, None] + rng.normal(0.0, 0.01, size=(3, k)).reshape(k, 3).T.copy()

    res = _iterate_many(lengths, transient, init, step, lambda s: s[0])
    return [(v - v.mean()) / v.std() for v in res]


GROUP = 512   # series per independently seeded group of one system


def _group(args):
    system, si, seed, g, lengths, snrs = args
    rng = rng_for(5, seed, si, g)
    if system == "sine":
        clean_ = [sine(int(n), rng) for n in lengths]
    elif system == "logistic":
        clean_ = _logistic_many(lengths, rng)
    else:
        clean_ = _lorenz_many(lengths, rng)
    out = []
    for c, snr in zip(clean_, snrs):
        y = add_noise(c, snr, rng).astype(np.float32)
        if not np.all(np.isfinite(y)) or float(np.std(y)) <= 0.0:
            raise RuntimeError(f"degenerate synthetic series {system} group {g}")
        out.append(y)
    return out


def many_series(systems, lengths, snrs, seed, workers=None):
    """float32 series (list) for parallel lists of system names, lengths and
    SNRs in dB.  The series of each system are cut, in input order, into
    groups of GROUP, each generated from its own seed (seed, system, group),
    so the result does not depend on the number of worker processes."""
    import concurrent.futures
    import os
    systems = list(systems)
    lengths = np.asarray(lengths, dtype=np.int64)
    snrs = np.asarray(snrs, dtype=np.float64)
    jobs, where = [], []
    for si, system in enumerate(SYSTEMS):
        idx = [i for i, s in enumerate(systems) if s == system]
        for g in range(0, len(idx), GROUP):
            part = idx[g:g + GROUP]
            jobs.append((system, si, seed, g // GROUP, lengths[part], snrs[part]))
            where.append(part)
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    out = [None] * len(systems)
    if workers <= 1 or len(jobs) <= 1:
        results = map(_group, jobs)
    else:
        ex = concurrent.futures.ProcessPoolExecutor(max_workers=min(workers, len(jobs)))
        results = ex.map(_group, jobs)
    for part, ys in zip(where, results):
        for i, y in zip(part, ys):
            out[i] = y
    if workers > 1 and len(jobs) > 1:
        ex.shutdown()
    return out


def bracket_set(count, seed, lo=1000, hi=100_000, snr_lo=-25.0, snr_hi=20.0, m=None):
    """Series for training or evaluating the threshold-bracket network:
    system uniform over the three, SNR ~ U[snr_lo, snr_hi] dB, length
    log-uniform in [lo, hi] (lo == hi gives a fixed length), Euclidean norm,
    w = 1, l_min = 2, K = 20 targets 0.01..0.20.  Embedding m = 3, tau = 5
    when m == 3; m = 1 when m == 1; m=None draws 3 (tau = 5) with
    probability 2/3 and 1 otherwise.  Returns (concat float32, offsets
    uint64[count + 1], params list, systems, snrs)."""
    rng = rng_for(6, seed)
    systems = [SYSTEMS[i] for i in rng.integers(0, len(SYSTEMS), size=count)]
    snrs = rng.uniform(snr_lo, snr_hi, size=count)
    if lo == hi:
        lengths = np.full(count, lo, dtype=np.int64)
    else:
        lengths = np.floor(10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=count)).astype(np.int64)
    if m is None:
        ms = np.where(rng.uniform(size=count) < 2.0 / 3.0, 3, 1)
    else:
        ms = np.full(count, int(m))
    ys = many_series(systems, lengths, snrs, seed)
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint64)
    params = [(int(mm), 5 if mm == 3 else 1, NORM_EUCLID, 1, 2) for mm in ms]
    return np.concatenate(ys), offs, params, systems, snrs


# ---------------------------------------------------------------------------
# The sorting-rate ensemble of the Methodology section: for each system, SNR
# level and length, 10 equidistant SNRs (a linear variance ratio) x R noise
# realisations.  The periodic signal is a sine of 25 cycles over the series
# (the paper's light-curve generator set to equidistant sine sampling with 25
# observed cycles), the logistic map uses r = 3.679 (band merging), the
# Lorenz x-component the same integration as above.

SNR_LEVELS = {
    "0.1": tuple(k / 100.0 for k in range(1, 11)),   # 0.01, 0.02, ..., 0.1
    "1": tuple(k / 10.0 for k in range(1, 11)),      # 0.1, 0.2, ..., 1
    "10": tuple(float(k) for k in range(1, 11)),     # 1, 2, ..., 10
}
PAPER_LOGISTIC_R = 3.679
PAPER_SINE_CYCLES = 25


def paper_embedding(system):
    """(m, tau) of the sorting-rate experiments: m = 3, tau = 3 for Lorenz
    (the values the paper gives); m = 1 otherwise."""
    return (3, 3) if system == "lorenz" else (1, 1)


def paper_ensemble(system, n, level, realisations=10, seed=0):
    """Series of one (system, length, SNR level) cell of the sorting-rate
    ensemble: a list over realisations of lists over the 10 SNRs (ascending)
    of float32 series of length n.  Each realisation draws its own clean
    signal (initial condition or phase) and noise, from the key (seed,
    system, level, n)."""
    snrs = SNR_LEVELS[level]
    si = SYSTEMS.index(system)
    li = list(SNR_LEVELS).index(level)
    rng = rng_for(7, seed, si, li, int(n))
    count = realisations * len(snrs)
    lengths = np.full(count, int(n), dtype=np.int64)
    if system == "sine":
        clean_ = [sine(int(n), rng, period=n / PAPER_SINE_CYCLES) for _ in range(count)]
    elif system == "logistic":
        clean_ = _logistic_many(lengths, rng, r=PAPER_LOGISTIC_R)
    else:
        clean_ = _lorenz_many(lengths, rng)
    out = []
    for r in range(realisations):
        row = []
        for q, snr in enumerate(snrs):
            c = clean_[r * len(snrs) + q]
            y = add_noise(c, 10.0 * math.log10(snr), rng).astype(np.float32)
            if not np.all(np.isfinite(y)) or float(np.std(y)) <= 0.0:
                raise RuntimeError(f"degenerate synthetic series {system} {n} {level}")
            row.append(y)
        out.append(row)
    return out
