"""Seeded generators for the synthetic workloads.

Every generator takes an explicit integer seed and returns float32 arrays, which
is the precision the estimator consumes. Simulations run in float64 and are cast
once at the end.

Workloads (paper, Validation tasks section, and the configurations measured here):

* ``c1_gaussian``: jointly Gaussian X, Y, Z with partial correlation rho given Z.
* ``var_network``: linear VAR on a directed Erdos-Renyi graph with link
  probability 3/P (expected in-degree 3), self-term 0.4, random lags 1..5 and
  couplings U(0.1, 0.5) scaled by one common factor so that the spectral radius
  of the VAR companion matrix is 0.9; unit Gaussian noise.
* ``paper_var_network``: the paper's own VAR variant (self-coupling 0.5, couplings
  normalised to sum 0.4 per target, noise s.d. 0.1).
* ``empty_network``: independent AR(1) processes (no links).
* ``clm_network``: coupled logistic maps, coupling applied after the map.
* ``paper_clm_network``: the paper's CLM variant (the map applied to the weighted
  input: self-coupling 0.5, couplings normalised to sum 0.4, noise s.d. 0.1).
* ``random_points``: sample matrices with ties and duplicate rows for parity tests.
"""

from __future__ import annotations

import numpy as np

MAX_LAG = 5
BURN_IN = 1000


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


# --------------------------------------------------------------------------- C1
def c1_gaussian(n: int, seed: int, rho: float = 0.6, r: float = 0.3):
    """Jointly Gaussian (X, Y, Z), each 1-D, with corr(X,Z)=corr(Y,Z)=r and
    partial correlation rho between X and Y given Z.

    Construction: Z ~ N(0,1), (U,V) ~ N(0, [[1,rho],[rho,1]]),
    X = r Z + sqrt(1-r^2) U, Y = r Z + sqrt(1-r^2) V.  The true conditional
    mutual information is -0.5*log(1-rho^2) nats.

    Returns (X, Y, Z, true_cmi) with X, Y, Z of shape [1][n] float32.
    """
    g = _rng(seed)
    z = g.standard_normal(n)
    u = g.standard_normal(n)
    w = g.standard_normal(n)
    v = rho * u + np.sqrt(1.0 - rho * rho) * w
    s = np.sqrt(1.0 - r * r)
    x = r * z + s * u
    y = r * z + s * v
    f = lambda a: np.ascontiguousarray(a.astype(np.float32)[None, :])
    return f(x), f(y), f(z), float(-0.5 * np.log(1.0 - rho * rho))


# ---------------------------------------------------------------- graphs
def er_digraph(p_nodes: int, seed: int, in_degree: float = 3.0):
    """Directed Erdos-Renyi graph without self-loops, link probability
    in_degree/P.  Returns parents[i] = sorted list of source nodes of i."""
    g = _rng(seed)
    prob = in_degree / p_nodes
    mask = g.random((p_nodes, p_nodes)) < prob
    np.fill_diagonal(mask, False)
    return [sorted(np.nonzero(mask[i])[0].tolist()) for i in range(p_nodes)]


def _companion_radius(self_coef: float, coup, p_nodes: int) -> float:
    """Spectral radius of the VAR(MAX_LAG) companion matrix."""
    a = np.zeros((MAX_LAG, p_nodes, p_nodes))
    a[0][np.arange(p_nodes), np.arange(p_nodes)] = self_coef
    for (i, j, lag, c) in coup:
        a[lag - 1][i, j] += c
    m = p_nodes * MAX_LAG
    comp = np.zeros((m, m))
    comp[:p_nodes, :] = np.concatenate(list(a), axis=1)
    comp[p_nodes:, :-p_nodes] = np.eye(m - p_nodes)
    return float(np.max(np.abs(np.linalg.eigvals(comp))))


def var_network(p_nodes: int, n_rows: int, seed: int, radius: float = 0.9,
                self_coef: float = 0.4, noise_sd: float = 1.0):
    """Linear VAR x_i(t) = self_coef*x_i(t-1) + sum_j c*a_ij*x_j(t-l_ij) + noise.

    a_ij ~ U(0.1, 0.5), l_ij ~ U{1..5}; c is found by bisection so that the
    companion spectral radius equals ``radius`` (the radius is monotone in c
    because every coefficient is non-negative).  A graph without cycles keeps
    the radius at self_coef, so it is redrawn with seed+1.

    Returns (series [P][n_rows+MAX_LAG] float32, links) where links is a list of
    (target, source, lag, coefficient).
    """
    graph_seed = seed
    while True:
        parents = er_digraph(p_nodes, graph_seed)
        g = _rng(graph_seed * 7919 + 1)
        base = []
        for i in range(p_nodes):
            for j in parents[i]:
                lag = int(g.integers(1, MAX_LAG + 1))
                base.append((i, j, lag, float(g.uniform(0.1, 0.5))))
        if base and _companion_radius(self_coef, [(i, j, l, 1e3 * c) for (i, j, l, c) in base],
                                      p_nodes) > radius:
            break
        graph_seed += 1
    lo, hi = 0.0, 1.0
    while _companion_radius(self_coef, [(i, j, l, hi * c) for (i, j, l, c) in base], p_nodes) < radius:
        hi *= 2.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        rad = _companion_radius(self_coef, [(i, j, l, mid * c) for (i, j, l, c) in base], p_nodes)
        if rad < radius:
            lo = mid
        else:
            hi = mid
    scale = 0.5 * (lo + hi)
    links = [(i, j, l, scale * c) for (i, j, l, c) in base]
    return _simulate_linear(p_nodes, n_rows, seed, self_coef, links, noise_sd), links


def paper_var_network(p_nodes: int, n_rows: int, seed: int):
    """The paper's VAR variant: self-coupling 0.5, cross-couplings uniform and
    normalised to sum 0.4 per target, noise s.d. 0.1 (VAR section)."""
    parents = er_digraph(p_nodes, seed)
    g = _rng(seed * 7919 + 1)
    links = []
    for i in range(p_nodes):
        if parents[i]:
            c = 0.4 / len(parents[i])
            for j in parents[i]:
                links.append((i, j, int(g.integers(1, MAX_LAG + 1)), c))
    return _simulate_linear(p_nodes, n_rows, seed, 0.5, links, 0.1), links


def _simulate_linear(p_nodes, n_rows, seed, self_coef, links, noise_sd):
    g = _rng(seed * 104729 + 3)
    total = BURN_IN + n_rows + MAX_LAG
    a = np.zeros((MAX_LAG, p_nodes, p_nodes))
    a[0][np.arange(p_nodes), np.arange(p_nodes)] = self_coef
    for (i, j, lag, c) in links:
        a[lag - 1][i, j] += c
    x = np.zeros((total, p_nodes))
    noise = g.standard_normal((total, p_nodes)) * noise_sd
    for t in range(total):
        acc = noise[t].copy()
        for lag in range(1, MAX_LAG + 1):
            if t - lag >= 0:
                acc += a[lag - 1] @ x[t - lag]
        x[t] = acc
    return np.ascontiguousarray(x[BURN_IN:].T.astype(np.float32))


def var_network_trials(p_nodes: int, n_rows: int, reps: int, seed: int, radius: float = 0.9,
                       self_coef: float = 0.4, noise_sd: float = 1.0):
    """R replications (trials) of the same VAR network: the coefficients of
    var_network(p_nodes, n_rows, seed), each trial simulated from its own
    burn-in with its own noise (seeds seed*1000 + r).  Returns
    (series [R][P][n_rows+MAX_LAG] float32, links)."""
    _, links = var_network(p_nodes, 8, seed, radius, self_coef, noise_sd)
    trials = [_simulate_linear(p_nodes, n_rows, seed * 1000 + r, self_coef, links, noise_sd) for r in range(reps)]
    return np.ascontiguousarray(np.stack(trials)), links


def empty_network(p_nodes: int, n_rows: int, seed: int, self_coef: float = 0.4, noise_sd: float = 1.0):
    """P independent AR(1) processes x_i(t) = self_coef * x_i(t-1) + noise: a
    network without links, where every inferred link is a false positive
    (Validation of false positive rate).  Returns series [P][n_rows+MAX_LAG]."""
    return _simulate_linear(p_nodes, n_rows, seed, self_coef, [], noise_sd)


# ---------------------------------------------------------------- CLM
def clm_network(p_nodes: int, n_rows: int, seed: int, coupling: float = 0.5,
                noise_sd: float = 0.1):
    """Coupled logistic maps with the coupling applied after the map:
    x_i(t) = [(1-c) f(x_i(t-1)) + c * mean_j f(x_j(t-l_ij)) + eta] mod 1,
    f(x) = 4x(1-x).  A node without sources evolves as [f(x_i(t-1)) + eta] mod 1.

    Returns (series [P][n_rows+MAX_LAG] float32, links (target, source, lag, c)).
    """
    parents = er_digraph(p_nodes, seed)
    g = _rng(seed * 7919 + 1)
    links = []
    for i in range(p_nodes):
        for j in parents[i]:
            links.append((i, j, int(g.integers(1, MAX_LAG + 1)), coupling / len(parents[i])))
    h = _rng(seed * 104729 + 3)
    total = BURN_IN + n_rows + MAX_LAG
    x = np.zeros((total, p_nodes))
    x[:MAX_LAG] = h.random((MAX_LAG, p_nodes))
    noise = h.standard_normal((total, p_nodes)) * noise_sd
    f = lambda v: 4.0 * v * (1.0 - v)
    # coupling matrices per lag: w[lag-1][i, j] = 1/|parents(i)| (mean over sources)
    w = np.zeros((MAX_LAG, p_nodes, p_nodes))
    self_w = np.ones(p_nodes)
    for (i, j, lag, _) in links:
        w[lag - 1][i, j] += 1.0 / len(parents[i])
        self_w[i] = 1.0 - coupling
    fx = np.zeros((total, p_nodes))
    fx[:MAX_LAG] = f(x[:MAX_LAG])
    for t in range(MAX_LAG, total):
        acc = self_w * fx[t - 1]
        for lag in range(1, MAX_LAG + 1):
            acc = acc + coupling * (w[lag - 1] @ fx[t - lag])
        v = np.mod(acc + noise[t], 1.0)
        v[v >= 1.0] = 0.0
        x[t] = v
        fx[t] = f(v)
    return np.ascontiguousarray(x[BURN_IN:].T.astype(np.float32)), links


def paper_clm_network(p_nodes: int, n_rows: int, seed: int):
    """The paper's coupled-logistic-map variant (CLM section): the map acts on
    the weighted input, a_i(t) = 0.5 x_i(t-1) + sum_j alpha x_j(t-l_ij) with the
    couplings uniform and normalised to sum 0.4 per target (the VAR section's
    conditions), then x_i(t) = [f(a_i(t)) + eta] mod 1, f(a) = 4a(1-a),
    eta ~ N(0, 0.1^2).  A node without sources keeps the self term alone.

    Returns (series [P][n_rows+MAX_LAG] float32, links (target, source, lag, alpha)).
    """
    parents = er_digraph(p_nodes, seed)
    g = _rng(seed * 7919 + 1)
    links = []
    for i in range(p_nodes):
        if parents[i]:
            c = 0.4 / len(parents[i])
            for j in parents[i]:
                links.append((i, j, int(g.integers(1, MAX_LAG + 1)), c))
    h = _rng(seed * 104729 + 3)
    total = BURN_IN + n_rows + MAX_LAG
    w = np.zeros((MAX_LAG, p_nodes, p_nodes))
    w[0][np.arange(p_nodes), np.arange(p_nodes)] = 0.5
    for (i, j, lag, c) in links:
        w[lag - 1][i, j] += c
    x = np.zeros((total, p_nodes))
    x[:MAX_LAG] = h.random((MAX_LAG, p_nodes))
    noise = h.standard_normal((total, p_nodes)) * 0.1
    for t in range(MAX_LAG, total):
        a = np.zeros(p_nodes)
        for lag in range(1, MAX_LAG + 1):
            a = a + w[lag - 1] @ x[t - lag]
        v = np.mod(4.0 * a * (1.0 - a) + noise[t], 1.0)
        v[v >= 1.0] = 0.0
        x[t] = v
    return np.ascontiguousarray(x[BURN_IN:].T.astype(np.float32)), links


def truth_adjacency(p_nodes: int, links):
    """A[s][t] = 1 for every (target t, source s, lag, c) link of a generator."""
    adj = np.zeros((p_nodes, p_nodes), dtype=np.uint8)
    for (t, s, _lag, _c) in links:
        adj[s, t] = 1
    return adj


# ---------------------------------------------------------------- slicing
def window(series: np.ndarray, node: int, lag: int, n_rows: int, t0: int = MAX_LAG):
    """Rows t0..t0+n_rows-1 of one node's series delayed by ``lag`` samples
    (a plain slice, returned as a [1][n_rows] float32 array)."""
    s = series[node, t0 - lag: t0 - lag + n_rows]
    assert s.shape[0] == n_rows
    return np.ascontiguousarray(s[None, :].astype(np.float32))


def c2_te_inputs(n_rows: int = 10000, seed: int = 2, p_nodes: int = 10):
    """One transfer-entropy estimate on the 10-node VAR: X = the first parent of
    the lowest-index node that has one, at its true lag; Y = that node's present;
    Z = its own past at lags 1..5.  Returns (X [1][N], Y [1][N], Z [5][N], meta)."""
    series, links = var_network(p_nodes, n_rows, seed)
    tgt = min(i for (i, _, _, _) in links)
    src, lag = sorted((j, l) for (i, j, l, _) in links if i == tgt)[0]
    x = window(series, src, lag, n_rows)
    y = window(series, tgt, 0, n_rows)
    z = np.concatenate([window(series, tgt, l, n_rows) for l in range(1, MAX_LAG + 1)], axis=0)
    return x, y, np.ascontiguousarray(z), {"target": tgt, "source": src, "lag": lag,
                                          "series": series, "links": links}


# ---------------------------------------------------------------- parity inputs
def random_points(n: int, dims, seed: int, kind: str = "normal"):
    """Random sample matrices for parity tests, one float32 array [d][n] per
    entry of ``dims`` (a d of 0 gives None).

    kind: "normal" (continuous), "grid" (values on a coarse dyadic grid, so many
    exact distance ties), "dup" (normal values with a quarter of the rows
    duplicated), "tiny" (denormal-range magnitudes), "wide" (mixed magnitudes),
    "cells" (every value s * 3e38 + u with a random sign s per value and
    u ~ U(-0.25e38, 0.25e38): two values of one sign differ by at most 0.5e38,
    two of opposite signs by more than the largest float, so in any subspace a
    row is at a finite distance only from the rows whose signs all agree with
    its own, and at +inf from the rest), "split" (the same values with one sign
    per row, shared by all its coordinates: two clusters of exactly n // 2 and
    n - n // 2 rows, finite within a cluster and +inf across).
    """
    g = _rng(seed)
    if kind == "split":
        sign = np.where(g.permutation(n) < n // 2, -1.0, 1.0)
    out = []
    for d in dims:
        if d == 0:
            out.append(None)
            continue
        if kind == "normal":
            a = g.standard_normal((d, n))
        elif kind == "grid":
            a = g.integers(-8, 9, size=(d, n)) * 0.25
        elif kind == "dup":
            a = g.standard_normal((d, n))
        elif kind == "tiny":
            a = g.standard_normal((d, n)) * 1e-39
        elif kind == "wide":
            a = g.standard_normal((d, n)) * np.exp2(g.integers(-20, 21, size=(d, n)))
        elif kind in ("cells", "split"):
            s = np.where(g.random((d, n)) < 0.5, -1.0, 1.0) if kind == "cells" else np.tile(sign, (d, 1))
            a = s * 3e38 + g.uniform(-0.25e38, 0.25e38, size=(d, n))
        else:
            raise ValueError(kind)
        out.append(a.astype(np.float32))
    if kind == "dup" and n >= 4:
        src = g.integers(0, n, size=n // 4)
        dst = g.choice(n, size=n // 4, replace=False)
        for a in out:
            if a is not None:
                a[:, dst] = a[:, src]
    return [None if a is None else np.ascontiguousarray(a) for a in out]
