"""MI355X-native all-pairs Pearson/Spearman correlation with pairwise deletion
of missing values (the method of NApy, arXiv 2505.00448), as hand-written HIP
kernels for gfx950 behind a C ABI (include/napy.h).

Importing the package does not load the library; the functions load
``libnapy.so`` on first use and raise if it is not built.
"""

__version__ = "0.1.0"

from .api import (  # noqa: F401,E402
    pearson,
    spearman,
    pearson_corr,
    PearsonCorr,
    pearson_subset,
    SpearmanBase,
    spearman_pair_ranks,
    pvalue_device,
    adjust_pvalues,
    ttest,
    anova,
    chi2,
    mannwhitney,
    kruskal,
)
