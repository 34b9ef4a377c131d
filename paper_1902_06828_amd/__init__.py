"""MI355X (gfx950) library for the hot path of greedy multivariate
transfer-entropy network inference (arXiv:1902.06828): the KSG
conditional-mutual-information estimator with permutation surrogates, the
maximum/minimum-statistic and omnibus tests, the four-step greedy source
selection and a continuous-batching request loop; the Gaussian estimator with
its analytic null as the alternative estimator of the greedy search.

All work runs in libmte.so (HIP kernels and C++ runtime); this package only
marshals arguments.  The C ABI is declared in include/mte.h.
"""

from ._lib import (  # noqa: F401
    ESTIMATORS,
    MteError,
    cmi_gauss,
    cmi_ksg,
    cmi_ksg_dev,
    cmi_ksg_diag,
    cmi_ksg_surrogates,
    cmi_ksg_surrogates_rep,
    cmi_ksg_surrogates_dev,
    cmi_ksg_surrogates_dev_noalloc,
    lib,
    mte_autocorr_decay_time,
    mte_chi2_sf,
    mte_fdr_bh,
    mte_gauss_cmi_sets,
    mte_gauss_covariance_dev,
    mte_infer_network,
    mte_init,
    mte_link_metrics,
    mte_kernel_timing,
    mte_kernel_timing_read,
    mte_kernel_timing_stage,
    mte_list_stats,
    mte_list_stats_enable,
    mte_max_statistic,
    mte_min_statistic,
    mte_omnibus,
    mte_permutation,
    mte_permutation_rep,
    mte_select_sources,
    mte_select_sources_sid,
    mte_serve_cancel,
    mte_serve_get_stats,
    mte_series_register,
    mte_series_release,
    mte_shuffle_mode,
    mte_standardise,
    mte_shutdown,
    mte_submit,
    mte_tile_configs,
    mte_tune_report,
    mte_wait,
)
