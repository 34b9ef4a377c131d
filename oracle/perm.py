"""Keyed surrogate permutations.  TEST INFRASTRUCTURE ONLY.

The paper builds surrogates by shuffling the embedded source samples within a
trial when replications are too few (Maximum statistic test section), and by
shuffling the selected sources' realisations jointly for the omnibus test
(Omnibus test section).  It does not say which random generator draws the
shuffle, so this project fixes one counter-based definition that both the
library and this oracle implement independently, each from the published
constructions it combines:

  mix64(z)      SplitMix64 output function (Steele, Lea and Flood 2014):
                z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
                z *= 0x94D049BB133111EB; z ^= z>>31                 (mod 2^64)
  key           h = mix64(mix64(seed + G) ^ (c<<32 | s)), G = 0x9E3779B97F4A7C15,
                for surrogate s of candidate test c
  rounds        R(N) = max(24, 6*ceil(log2 N))
  round keys    rk_r = mix64(h + (r+1)*G), K_r = ((rk_r >> 32) * N) >> 32, r < R
  pi(i)         swap-or-not shuffle (Hoang, Morris and Rogaway 2012): x = i; for
                each round r: x' = (K_r - x) mod N; if the top bit of
                mix64(max(x, x') ^ rk_r) is 1 then x = x'.  Each round pairs x
                with K_r - x and swaps both or neither, so pi is a bijection of
                {0..N-1} for every N >= 1.

Surrogate row i takes the source value of row pi(i).
"""

from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB


def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * C1) & M64
    z = ((z ^ (z >> 27)) * C2) & M64
    return z ^ (z >> 31)


def splitmix64(seed: int, count: int):
    """The first `count` outputs of the SplitMix64 generator started at seed."""
    state, out = seed & M64, []
    for _ in range(count):
        state = (state + GOLDEN) & M64
        out.append(mix64(state))
    return out


def surrogate_key(seed: int, cand: int, s: int) -> int:
    return mix64(mix64((seed + GOLDEN) & M64) ^ (((cand & 0xFFFFFFFF) << 32) | (s & 0xFFFFFFFF)))


def n_rounds(n: int) -> int:
    return max(24, 6 * (n - 1).bit_length())


def round_keys_from_hash(h: int, n: int):
    """[(rk_r, K_r)] for r < R(n), from the key hash h."""
    out = []
    for r in range(n_rounds(n)):
        rk = mix64((h + (r + 1) * GOLDEN) & M64)
        out.append((rk, ((rk >> 32) * n) >> 32))
    return out


def round_keys(seed: int, cand: int, s: int, n: int):
    """[(rk_r, K_r)] for r < R(n)."""
    return round_keys_from_hash(surrogate_key(seed, cand, s), n)


def permutation_scalar(seed: int, cand: int, s: int, n: int):
    """pi_{seed,cand,s} as a Python list, element by element (slow)."""
    keys = round_keys(seed, cand, s, n)
    out = []
    for i in range(n):
        x = i
        for rk, k in keys:
            xp = k - x if x <= k else k - x + n
            if mix64(max(x, xp) ^ rk) >> 63:
                x = xp
        out.append(x)
    return out


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(C1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(C2)
    return z ^ (z >> np.uint64(31))


def permutation_from_hash(h: int, n: int) -> np.ndarray:
    """The swap-or-not permutation keyed by hash h over {0..n-1} (uint32)."""
    x = np.arange(n, dtype=np.int64)
    with np.errstate(over="ignore"):
        for rk, k in round_keys_from_hash(h, n):
            xp = np.where(x <= k, k - x, k - x + n)
            hi = np.maximum(x, xp).astype(np.uint64)
            bit = (_mix64_np(hi ^ np.uint64(rk)) >> np.uint64(63)).astype(bool)
            x = np.where(bit, xp, x)
    return x.astype(np.uint32)


def permutation(seed: int, cand: int, s: int, n: int) -> np.ndarray:
    """pi_{seed,cand,s} over {0..n-1} as a uint32 numpy array (the same
    definition as permutation_scalar, evaluated for all indices at once)."""
    return permutation_from_hash(surrogate_key(seed, cand, s), n)


# ---------------------------------------------------------------- replications
# With R replications (trials) the rows of an estimate are the embedded rows
# of every replication, replication after replication: row i = r * n_r + t,
# N = R * n_r.  The Maximum statistic test section prefers surrogates that
# shuffle the order of the replications of the candidate, keeping the other
# variables in place, and falls back to shuffling the embedded samples within
# each trial when the replications allow too few permutations.  Readings:
#   * "enough" replications: R! >= S (at least S distinct orderings);
#   * replication shuffle: sigma = pi_{seed,cand,s} over {0..R-1}; row (r, t)
#     takes the candidate's row (sigma(r), t);
#   * within-trial shuffle: row (r, t) takes (r, pi_r(t)), pi_r the swap-or-not
#     permutation over {0..n_r-1} keyed by h_r = mix64(h XOR ((r+1) G mod 2^64))
#     for R > 1, h = surrogate_key(seed, cand, s); for R = 1 it is keyed by h
#     itself, i.e. it is pi_{seed,cand,s} over all N rows.

REPLICATIONS, WITHIN = "replications", "within"


def shuffle_mode(reps: int, n_surr: int) -> str:
    f = 1
    for r in range(2, reps + 1):
        f *= r
        if f >= n_surr:
            break
    return REPLICATIONS if reps > 1 and f >= n_surr else WITHIN


def replication_source_rows(seed: int, cand: int, s: int, n_rows: int, reps: int, mode: str) -> np.ndarray:
    """Source row of every row of surrogate s (uint32 [n_rows])."""
    if reps < 1 or n_rows % reps:
        raise ValueError("n_rows must be a multiple of reps")
    n_r = n_rows // reps
    h = surrogate_key(seed, cand, s)
    t = np.arange(n_r, dtype=np.int64)
    out = np.empty(n_rows, dtype=np.int64)
    if mode == REPLICATIONS:
        sigma = permutation_from_hash(h, reps)
        for r in range(reps):
            out[r * n_r:(r + 1) * n_r] = int(sigma[r]) * n_r + t
    elif mode == WITHIN:
        if reps == 1:
            return permutation_from_hash(h, n_rows)
        for r in range(reps):
            h_r = mix64(h ^ (((r + 1) * GOLDEN) & M64))
            out[r * n_r:(r + 1) * n_r] = r * n_r + permutation_from_hash(h_r, n_r).astype(np.int64)
    else:
        raise ValueError(f"unknown mode {mode!r}")
    return out.astype(np.uint32)
