"""Seeded synthetic traffic-tensor inputs shared by the oracle tests, the GPU tests and the bench.

This package only draws input data (observed tensor, sampling mask, initial factors).
It holds none of the completion method's arithmetic; see ``synth.traffic``.
"""
from .traffic import LAYOUTS, WORKLOADS, Workload, batch_specs, make_inputs, make_workload, relayout

__all__ = ["LAYOUTS", "WORKLOADS", "Workload", "batch_specs", "make_inputs", "make_workload", "relayout"]
