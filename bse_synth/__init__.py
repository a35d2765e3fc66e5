"""Seeded synthetic inputs shaped like the paper's BSE workloads (shared by the
oracle tests, the GPU tests and the benchmark; holds none of the method)."""
from . import lattice, workloads
from .generate import make_batch_inputs, make_inputs, make_screening_inputs, screened_interaction
from .workloads import BATCHES, WORKLOADS, BatchWorkload, Workload, get

__all__ = ["lattice", "workloads", "make_inputs", "make_batch_inputs", "make_screening_inputs",
           "screened_interaction",
           "WORKLOADS", "BATCHES", "Workload", "BatchWorkload", "get"]
