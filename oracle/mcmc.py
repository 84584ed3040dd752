"""Reference DE-MCz sampler with snooker updates and delayed acceptance (oracle; test
infrastructure only).

Sec. 3, Sec. 4 item 10, Sec. 5: BART's MC3 samples with differential-evolution MCMC;
its DEMCzs (ter Braak & Vrugt 2008) proposes from an archive of past states and mixes
parallel-direction moves with snooker moves. The step definitions follow ter Braak &
Vrugt (2008) and, for the two-stage acceptance, Christen & Fox (2005); the random numbers
are SplitMix64 outputs (Steele, Lea & Flood 2014) addressed by (generation, chain, slot)
counters, written here from that definition in plain Python integers.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
SLOTS = 64
SLOT_R1, SLOT_R2, SLOT_U, SLOT_U1, SLOT_NORMAL = 0, 1, 2, 3, 8
SLOT_MOVE, SLOT_Z, SLOT_GAMMA_S = 4, 5, 6   # snooker: move choice, archive row z, gamma_s
INIT_XOR = 0xA5A5A5A5A5A5A5A5


def splitmix64(seed: int, k: int) -> int:
    """Output k (0-based) of the SplitMix64 stream with the given seed."""
    z = (seed + (k + 1) * GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def u01(seed: int, k: int) -> float:
    """Uniform in [0, 1) from the top 53 bits."""
    return (splitmix64(seed, k) >> 11) * 2.0 ** -53


def counter(g: int, c: int, n_chains: int, slot: int) -> int:
    return ((g * n_chains + c) * SLOTS + slot)


def normal(seed: int, g: int, c: int, n_chains: int, j: int) -> float:
    """Box-Muller on the uniform pair (2j, 2j+1) of the normal slots."""
    u1 = u01(seed, counter(g, c, n_chains, SLOT_NORMAL + 2 * j))
    u2 = u01(seed, counter(g, c, n_chains, SLOT_NORMAL + 2 * j + 1))
    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)


def init_state(seed: int, n_chains: int, z_init: int, lo, hi):
    """Archive of z_init uniform prior draws, then C chain starts, from the init stream."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = lo.size
    draws = np.empty((z_init + n_chains, d))
    for i in range(z_init + n_chains):
        for p in range(d):
            draws[i, p] = lo[p] + (hi[p] - lo[p]) * u01(seed ^ INIT_XOR, i * SLOTS + p)
    return draws[z_init:].copy(), draws[:z_init].copy()


def free_count(lo, hi) -> int:
    """Number of free parameters (Sec. 5 sizes the chain count by them): those whose prior
    box has non-zero width. A parameter with lo = hi is held fixed: every archive row and
    state holds its value, so its DE difference and its jitter are zero and no move changes
    it, and the chains move in the space of the others. All fixed reads as d."""
    k = int(np.sum(np.asarray(hi, np.float64) > np.asarray(lo, np.float64)))
    return k if k > 0 else len(lo)


def propose(x, z, m: int, g: int, seed: int, lo, hi, eps_scale: float, gamma_scale: float = 1.0):
    """DE-MCz proposals of generation g: y = x + gamma (z_r1 - z_r2) + e, r1 != r2 uniform
    over the m archive rows, gamma = gamma_scale 2.38/sqrt(2k) over the k free parameters
    (1 every 10th generation; ter Braak's value for Gaussian targets at gamma_scale = 1),
    e ~ N(0, (eps_scale * width)^2). Returns (y, r1, r2)."""
    n_chains, d = x.shape
    y = np.empty_like(x)
    r1s, r2s = np.empty(n_chains, int), np.empty(n_chains, int)
    k = free_count(lo, hi)
    gamma = 1.0 if g % 10 == 9 else gamma_scale * (2.38 / math.sqrt(2.0 * k))
    for c in range(n_chains):
        r1 = min(int(u01(seed, counter(g, c, n_chains, SLOT_R1)) * m), m - 1)
        r2 = min(int(u01(seed, counter(g, c, n_chains, SLOT_R2)) * (m - 1)), m - 2)
        if r2 >= r1:
            r2 += 1
        r1s[c], r2s[c] = r1, r2
        for p in range(d):
            width = hi[p] - lo[p]
            e = (eps_scale * width) * normal(seed, g, c, n_chains, p)
            y[c, p] = (x[c, p] + gamma * (z[r1, p] - z[r2, p])) + e
    return y, r1s, r2s


def snooker(x, zz, z1, z2, gamma_s: float, k: int | None = None):
    """ter Braak & Vrugt (2008) snooker move of one chain: z_R1 and z_R2 are projected
    orthogonally onto the line through the state x and the archive member zz, and x moves
    along that line by gamma_s times the difference of the projections,
        y = x + gamma_s ((z_R1 - z_R2) . u) u,   u = (x - zz) / |x - zz|.
    The move is accepted with the extra factor (|y - zz| / |x - zz|)^(k - 1), k the
    dimension of the space the chains move in (the free parameters; all d by default);
    returns y and the log of that factor (-inf when x = zz, where the line is undefined and
    y = x). Sums run over the parameters in order; every operation is written out."""
    d = len(x)
    k = d if k is None else k
    nn, dot = 0.0, 0.0
    for p in range(d):
        e = x[p] - zz[p]
        nn = nn + e * e
        dot = dot + (z1[p] - z2[p]) * e
    y = np.array(x, dtype=np.float64)
    if not nn > 0.0:
        return y, -math.inf
    coef = gamma_s * (dot / nn)
    n2 = 0.0
    for p in range(d):
        y[p] = x[p] + coef * (x[p] - zz[p])
        f = y[p] - zz[p]
        n2 = n2 + f * f
    if not n2 > 0.0:
        return y, -math.inf
    return y, (0.5 * (k - 1)) * (math.log(n2) - math.log(nn))


def third_row(u: float, m: int, r1: int, r2: int) -> int:
    """An archive row uniform over the m - 2 rows other than r1 and r2."""
    rz = min(int(u * (m - 2)), m - 3)
    a, b = min(r1, r2), max(r1, r2)
    if rz >= a:
        rz += 1
    if rz >= b:
        rz += 1
    return rz


def propose_zs(x, z, m: int, g: int, seed: int, lo, hi, eps_scale: float, p_snooker: float,
               gamma_scale: float = 1.0):
    """DEMCzs proposals of generation g: chain c takes a snooker move when its move-choice
    uniform is below p_snooker (and the archive has at least 3 rows), otherwise the
    parallel-direction move of propose(). Returns (y, log_q) with log_q the log proposal
    factor of each chain (0 for parallel-direction moves)."""
    y, r1s, r2s = propose(x, z, m, g, seed, lo, hi, eps_scale, gamma_scale)
    n_chains, d = x.shape
    log_q = np.zeros(n_chains)
    if p_snooker <= 0.0 or m < 3:
        return y, log_q
    k = free_count(lo, hi)
    for c in range(n_chains):
        if not u01(seed, counter(g, c, n_chains, SLOT_MOVE)) < p_snooker:
            continue
        rz = third_row(u01(seed, counter(g, c, n_chains, SLOT_Z)), m, r1s[c], r2s[c])
        gamma_s = 1.2 + u01(seed, counter(g, c, n_chains, SLOT_GAMMA_S))
        y[c], log_q[c] = snooker(x[c], z[rz], z[r1s[c]], z[r2s[c]], gamma_s, k)
    return y, log_q


def log_post(y, chi2: float, flags: int, lo, hi) -> float:
    """-chi^2/2 inside the uniform prior box; -inf outside or for a flagged model."""
    if not (np.all(y >= lo) and np.all(y <= hi)) or flags != 0 or not np.isfinite(chi2):
        return -math.inf
    return -0.5 * chi2


def accept(x, lp, y, chi2, flags, g: int, seed: int, lo, hi, log_q=None):
    """Metropolis-Hastings: accept y_c with probability min(1, exp(lp(y_c) - lp(x_c) +
    log_q_c)), log_q the log proposal factor (0 for symmetric moves)."""
    x, lp = x.copy(), lp.copy()
    taken = np.zeros(len(x), bool)
    for c in range(len(x)):
        lpy = log_post(y[c], chi2[c], 0 if flags is None else int(flags[c]), lo, hi)
        u = u01(seed, counter(g, c, len(x), SLOT_U))
        lq = 0.0 if log_q is None else log_q[c]
        if math.isfinite(lpy) and math.log(u) < (lpy - lp[c]) + lq:
            x[c], lp[c], taken[c] = y[c], lpy, True
    return x, lp, taken


def da_screen(y, chi2_surr, lp_surr, g: int, seed: int, lo, hi, log_q=None):
    """Delayed acceptance stage 1: pass with probability min(1, exp(ls(y) - ls(x) +
    log_q)). Stage 2 needs no proposal factor: it cancels against stage 1's."""
    act = np.zeros(len(y), np.int32)
    for c in range(len(y)):
        if np.all(y[c] >= lo) and np.all(y[c] <= hi) and np.isfinite(chi2_surr[c]):
            u = u01(seed, counter(g, c, len(y), SLOT_U1))
            lq = 0.0 if log_q is None else log_q[c]
            act[c] = math.log(u) < (-0.5 * chi2_surr[c] - lp_surr[c]) + lq
    return act


def da_accept(x, lp, lp_surr, y, chi2, flags, chi2_surr, active, g: int, seed: int, lo, hi):
    """Stage 2: among stage-1 survivors accept with
    min(1, exp((lp(y) - lp(x)) - (ls(y) - ls(x))))."""
    x, lp, lp_surr = x.copy(), lp.copy(), lp_surr.copy()
    for c in range(len(x)):
        if not active[c]:
            continue
        lpy = log_post(y[c], chi2[c], 0 if flags is None else int(flags[c]), lo, hi)
        lsy = -0.5 * chi2_surr[c]
        u = u01(seed, counter(g, c, len(x), SLOT_U))
        if math.isfinite(lpy) and math.log(u) < (lpy - lp[c]) - (lsy - lp_surr[c]):
            x[c], lp[c], lp_surr[c] = y[c], lpy, lsy
    return x, lp, lp_surr


def run(loglike_chi2, n_chains: int, n_gen: int, lo, hi, seed: int, thin: int = 10,
        eps_scale: float = 1e-6, z_init: int | None = None, surrogate_chi2=None,
        p_snooker: float = 0.0):
    """Full reference sampler; loglike_chi2(y[C][d]) -> chi^2[C]. With surrogate_chi2,
    delayed acceptance; with p_snooker > 0, DEMCzs (snooker moves at that rate).
    Returns the chain history [n_gen][C][d] and acceptance counts."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = lo.size
    z_init = z_init if z_init is not None else 10 * d
    x, z = init_state(seed, n_chains, z_init, lo, hi)
    chi2 = loglike_chi2(x)
    lp = np.array([log_post(x[c], chi2[c], 0, lo, hi) for c in range(n_chains)])
    lp_surr = -0.5 * surrogate_chi2(x) if surrogate_chi2 is not None else None
    hist = np.empty((n_gen, n_chains, d))
    n_acc = np.zeros(n_chains, int)
    for g in range(n_gen):
        y, log_q = propose_zs(x, z, len(z), g, seed, lo, hi, eps_scale, p_snooker)
        if surrogate_chi2 is None:
            x, lp, taken = accept(x, lp, y, loglike_chi2(y), None, g, seed, lo, hi, log_q)
            n_acc += taken
        else:
            cs = surrogate_chi2(y)
            act = da_screen(y, cs, lp_surr, g, seed, lo, hi, log_q)
            x_new, lp, lp_surr = da_accept(x, lp, lp_surr, y, loglike_chi2(y), None, cs, act, g,
                                           seed, lo, hi)
            n_acc += np.any(x_new != x, axis=1)
            x = x_new
        hist[g] = x
        if (g + 1) % thin == 0:
            z = np.vstack([z, x])
    return hist, n_acc
