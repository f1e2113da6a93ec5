"""Seeded synthetic inputs shared by the GPU path and the oracle.

This package holds only random-number draws and workload parameter tables.
It contains none of the method's arithmetic (no field solve, no correction
stencil, no shape factor, no push, no deposit), so both sides may import it.
"""
from .beam import load_beam, beam_weight
from .workloads import workload, WORKLOADS, batched_candidates, growth_cases, VARIANTS

__all__ = ["load_beam", "beam_weight", "workload", "WORKLOADS", "batched_candidates", "growth_cases", "VARIANTS"]
