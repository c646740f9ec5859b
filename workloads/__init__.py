"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package draws random arrays (coupling matrix, input weights, initial
magnetisations, input series and the readout target) and names the
workload sizes.  It holds none of the simulation's arithmetic: no field
evaluation, no integrator, no readout solve, and no physical constants.
Both the CPU oracle and the HIP library receive these arrays as plain
inputs.
"""

from .inputs import (  # noqa: F401
    STREAMS,
    SWEEPS,
    Sweep,
    Workload,
    WORKLOADS,
    draw_coupling,
    draw_initial,
    draw_input_weights,
    draw_inputs,
    draw_target,
    make_paper_arrays,
    make_stream_arrays,
    make_sweep_arrays,
    make_workload_arrays,
    seed_streams,
)
