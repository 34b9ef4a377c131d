"""Plain CPU oracle for the KSG conditional-mutual-information hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything from this package; only the tests, the smoke check and the benchmark's
CPU baseline do.  It shares no code with the HIP library: it re-derives every
step from the paper and from the estimator definition the paper cites.

Modules
  ksg     brute-force KSG CMI estimator (numpy, float32 subtraction, float64 sums),
          with an optional Theiler window
  perm    keyed surrogate permutation (swap-or-not shuffle keyed by SplitMix64)
  stats   maximum-statistic, minimum-statistic and omnibus tests
  act     autocorrelation decay time (the Theiler window heuristic)
  gauss   Gaussian (linear) CMI estimator and its analytic chi^2 null
  greedy  the four-step greedy multivariate TE inference for one target (surrogate
          tests with KSG, or analytic tests with the Gaussian estimator)
  network every target, Benjamini-Hochberg over omnibus p-values, adjacency,
          precision / recall / specificity / false positive rate
  cksg    ctypes loader for ksg_oracle.c, the same brute force in plain C (timed)

Parity status: ksg, perm, stats, act and gauss are pinned by tests/test_oracle_*.py against
closed forms, hand-counted cases, invariances and published generator outputs.
greedy's and network's selections on real data are pinned only statistically (recovery of
known parents, no selection on independent data): beyond that, parity
unpinned, since the paper prints no CMI or TE values.
"""
