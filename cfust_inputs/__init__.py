"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the EM method itself.  It draws
  * data sets from the generative hierarchy of the CFUST mixture (Sec. 3, eq. 6),
  * parameter sets Psi of the shapes used by the workloads,
  * the quasi-Monte Carlo design (a rank-1 lattice generating vector and the
    random shifts) that both the oracle and the HIP path take as *inputs*,
  * starting partitions for the restarts of the initialisation (also inputs).
"""
from .synth import (Params, Dataset, draw_params, sample_hierarchy, workload,
                    WORKLOADS, random_spd, draw_mvt_problems)
from .qmc_design import QmcDesign, korobov_vector, make_design
from .partitions import random_partitions, kmeans_partitions

__all__ = ["Params", "Dataset", "draw_params", "sample_hierarchy", "workload",
           "WORKLOADS", "random_spd", "draw_mvt_problems",
           "QmcDesign", "korobov_vector", "make_design", "random_partitions", "kmeans_partitions"]
