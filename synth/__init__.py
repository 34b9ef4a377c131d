"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package only draws random numbers and simulates the synthetic processes the
paper validates on (Erdos-Renyi networks driving a linear VAR or coupled logistic
maps, Validation tasks section). It holds none of the estimator's arithmetic: no
distances, neighbour searches, counts, digamma sums, permutations or tests.
"""

from .gen import (  # noqa: F401
    c1_gaussian,
    c2_te_inputs,
    clm_network,
    empty_network,
    er_digraph,
    paper_clm_network,
    paper_var_network,
    random_points,
    truth_adjacency,
    var_network,
    var_network_trials,
    window,
)
