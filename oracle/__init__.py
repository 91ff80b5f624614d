"""FP64 CPU oracle for pairwise-deletion Pearson/Spearman (test infrastructure
only: imported by tests, the smoke check and the benchmark's CPU baseline)."""
