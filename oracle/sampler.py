"""CPU oracle of the GPU-resident parallel-tempered Metropolis sampler.

TEST INFRASTRUCTURE.  Only the test-suite may use this module; it shares no
code with the HIP implementation.

The paper names a fully GPU-resident parallel-tempered MCMC as the inference
layer its likelihood is built for (Sect. 6).  The sampler here is standard
parallel tempering with random-walk Metropolis moves:

* state: C chains at each of T inverse temperatures beta_0 = 1 > beta_1 > ...;
  chain (t, c) holds a parameter record and its log-likelihood L;
* move at step n: theta' = theta + s_j / sqrt(beta_t) * z_j on the free
  parameter slots j (z standard normal), accepted when
  log u < beta_t (L' - L) and theta' lies inside the uniform prior box
  (the target of temperature t is prior x likelihood^beta_t);
* swap after every swap_every-th step: for each chain c the pairs (t, t + 1)
  of one parity (even pairs on even swap rounds, odd on odd) exchange their
  states when log u < (beta_t - beta_{t+1}) (L_{t+1} - L_t).

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC11), a counter-based
generator: counter (n mod 2^32, n div 2^32, t C + c, purpose << 16 | k), key
(seed mod 2^32, seed div 2^32); purpose 0 = proposal (k = pair of free
slots), 1 = acceptance, 2 = swap.  A 53-bit uniform is taken from two output
words (high word first); Box-Muller turns two uniforms into two normals.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)
PURPOSE_PROPOSE, PURPOSE_ACCEPT, PURPOSE_SWAP = 0, 1, 2


def philox4x32_10(ctr, key):
    """Philox4x32 with ten rounds.  ctr: uint32-valued array [..., 4], key:
    two uint32 values.  Each round multiplies words 0 and 2 by the two
    multipliers, and the new words are (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
    hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by the two Weyl
    constants between rounds."""
    c = np.asarray(ctr, dtype=np.uint64) & MASK32
    k0 = np.uint64(key[0]) & MASK32
    k1 = np.uint64(key[1]) & MASK32
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c[..., 0]
        p1 = PHILOX_M1 * c[..., 2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = np.stack([hi1 ^ c[..., 1] ^ k0, lo1, hi0 ^ c[..., 3] ^ k1, lo0], axis=-1)
    return c


def uniform53(w_hi, w_lo):
    """Uniform on [0, 1) from the top 53 bits of the 64-bit word hi:lo."""
    w = (np.asarray(w_hi, dtype=np.uint64) << np.uint64(21)) | (np.asarray(w_lo, dtype=np.uint64) >> np.uint64(11))
    return w.astype(np.float64) * 2.0 ** -53


def counters(step, slot, purpose, k):
    step = int(step)
    slot = np.asarray(slot, dtype=np.uint64)
    shape = np.broadcast(slot, np.asarray(k)).shape
    ctr = np.zeros(shape + (4,), dtype=np.uint64)
    ctr[..., 0] = step & 0xFFFFFFFF
    ctr[..., 1] = step >> 32
    ctr[..., 2] = slot
    ctr[..., 3] = (np.uint64(purpose) << np.uint64(16)) | np.asarray(k, dtype=np.uint64)
    return ctr


def seed_key(seed):
    return (int(seed) & 0xFFFFFFFF, int(seed) >> 32)


def normals(step, slot, n_pairs, seed):
    """Standard normals z[slot, 2 n_pairs] of a proposal (purpose 0)."""
    slot = np.atleast_1d(np.asarray(slot))
    k = np.arange(n_pairs)
    w = philox4x32_10(counters(step, slot[:, None], PURPOSE_PROPOSE, k[None, :]), seed_key(seed))
    ua = uniform53(w[..., 0], w[..., 1])
    ub = uniform53(w[..., 2], w[..., 3])
    r = np.sqrt(-2.0 * np.log(1.0 - ua))
    z = np.empty((slot.size, 2 * n_pairs))
    z[:, 0::2] = r * np.cos(2.0 * np.pi * ub)
    z[:, 1::2] = r * np.sin(2.0 * np.pi * ub)
    return z


def uniforms(step, slot, purpose, seed):
    w = philox4x32_10(counters(step, np.atleast_1d(slot), purpose, 0), seed_key(seed))
    return uniform53(w[..., 0], w[..., 1])


class PTConfig:
    def __init__(self, n_chains, betas, free_slots, lo, hi, step_scale, seed, swap_every=1):
        self.C = int(n_chains)
        self.beta = np.asarray(betas, dtype=np.float64)
        self.T = self.beta.size
        self.free = np.asarray(free_slots, dtype=np.int64)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.step = np.asarray(step_scale, dtype=np.float64)
        self.seed = int(seed)
        self.swap_every = int(swap_every)


def propose(cfg: PTConfig, params, step):
    """params [T, C, 16] -> proposals [T, C, 16] of step `step`."""
    T, C = cfg.T, cfg.C
    nf = cfg.free.size
    slots = np.arange(T * C)
    z = normals(step, slots, (nf + 1) // 2, cfg.seed)[:, :nf].reshape(T, C, nf)
    out = np.array(params, dtype=np.float64, copy=True)
    scale = cfg.step[None, None, :] / np.sqrt(cfg.beta)[:, None, None]
    out[:, :, cfg.free] = out[:, :, cfg.free] + scale * z
    return out


def accept_and_swap(cfg: PTConfig, params, logl, prop, prop_logl, step):
    """Metropolis decisions of step `step`, then the swap round when due.
    Returns (params, logl, accepted [T, C] bool, swapped [T - 1, C] bool)."""
    T, C = cfg.T, cfg.C
    params = np.array(params, dtype=np.float64, copy=True)
    logl = np.array(logl, dtype=np.float64, copy=True)
    prop_logl = np.asarray(prop_logl, dtype=np.float64)
    fp = prop[:, :, cfg.free]
    in_box = np.all((fp >= cfg.lo) & (fp <= cfg.hi), axis=-1)
    u = uniforms(step, np.arange(T * C), PURPOSE_ACCEPT, cfg.seed).reshape(T, C)
    with np.errstate(invalid="ignore"):
        log_alpha = cfg.beta[:, None] * (prop_logl - logl)
        acc = in_box & np.isfinite(prop_logl) & (np.log(u) < log_alpha)
    params[acc] = prop[acc]
    logl[acc] = prop_logl[acc]
    swapped = np.zeros((max(T - 1, 0), C), dtype=bool)
    if cfg.swap_every > 0 and T > 1 and (step + 1) % cfg.swap_every == 0:
        parity = (step // cfg.swap_every) % 2
        for t in range(parity, T - 1, 2):
            us = uniforms(step, t * C + np.arange(C), PURPOSE_SWAP, cfg.seed)
            with np.errstate(invalid="ignore"):
                log_r = (cfg.beta[t] - cfg.beta[t + 1]) * (logl[t + 1] - logl[t])
                sw = np.log(us) < log_r
            a, b = params[t, sw].copy(), params[t + 1, sw].copy()
            params[t, sw], params[t + 1, sw] = b, a
            la, lb = logl[t, sw].copy(), logl[t + 1, sw].copy()
            logl[t, sw], logl[t + 1, sw] = lb, la
            swapped[t] = sw
    return params, logl, acc, swapped


def run(cfg: PTConfig, params0, loglike_fn, n_steps):
    """Runs n_steps of the sampler with a CPU likelihood loglike_fn(params
    [N, 16]) -> [N]; returns the cold chain [n_steps, C, 16], its logL and
    the acceptance / swap counts."""
    params = np.array(params0, dtype=np.float64, copy=True)
    logl = loglike_fn(params.reshape(-1, params.shape[-1])).reshape(cfg.T, cfg.C)
    chain = np.zeros((n_steps, cfg.C, params.shape[-1]))
    chain_l = np.zeros((n_steps, cfg.C))
    n_acc = np.zeros((cfg.T, cfg.C), dtype=np.int64)
    n_sw = np.zeros((max(cfg.T - 1, 0), cfg.C), dtype=np.int64)
    for n in range(n_steps):
        prop = propose(cfg, params, n)
        pl = loglike_fn(prop.reshape(-1, prop.shape[-1])).reshape(cfg.T, cfg.C)
        params, logl, acc, sw = accept_and_swap(cfg, params, logl, prop, pl, n)
        n_acc += acc
        n_sw += sw
        chain[n] = params[0]
        chain_l[n] = logl[0]
    return chain, chain_l, n_acc, n_sw, params, logl
