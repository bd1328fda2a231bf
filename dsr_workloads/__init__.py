"""Seeded synthetic inputs for the data-sharing runtime's workloads.

This package is shared by the CPU oracle (``oracle/``) and by the GPU path's
tests and benchmark.  It draws random numbers and lays out input structures
(scalars, arrays, loop lengths, frame compositions); it computes none of the
method's results: no loop body, no reduction and no stack logic lives here.
"""
from .gen import (GAMMA, mix64, stream_base, draws, uniform_int, uniform_f32,
                  uniform_f64, log_uniform_int, splitmix64_sequence,
                  uniform_f32_draws)
from .configs import (Cfg1, Cfg2, Cfg3, Cfg4Instance, cfg1_inputs, cfg2_inputs,
                      cfg3_arrays, cfg4_descriptors, cfg4_instance, instance_x,
                      poisson_schedule, frame_composition, CFG2_KS, CFG3_AS,
                      CFG3_LENS)

__all__ = [n for n in dir() if not n.startswith("_")]
