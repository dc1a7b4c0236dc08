"""Seeded synthetic workloads (tree ensembles and explained samples)."""
from .ensembles import (CONFIGS, Ensemble, Workload, make_workload, stump, from_nested,
                        random_small_ensemble, build_grow, SEED_BASE)

__all__ = ["CONFIGS", "Ensemble", "Workload", "make_workload", "stump", "from_nested",
           "random_small_ensemble", "build_grow", "SEED_BASE"]
