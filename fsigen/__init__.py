"""Seeded synthetic inputs for the Newton-step linear solves.

This package is the input fixture shared by the GPU library's tests/benchmark
and by the CPU oracle.  It builds meshes, states, assembled matrices and
right-hand sides; it contains none of the solver's arithmetic (no smoother,
transfer, Krylov or coarse-solve code).
"""
from .problem import (BSR, Level, Problem, PARAMS_DEFAULT, build_native, graded_axis,
                      make_problem, make_level, config_problem, batch_instance, serve_instance,
                      serve_request, Channel, make_channel, inflow_profile, inflow_ramp,
                      graded_breaks, CHANNEL_PARAMS)

__all__ = ["BSR", "Level", "Problem", "PARAMS_DEFAULT", "build_native", "graded_axis",
           "make_problem", "make_level", "config_problem", "batch_instance", "serve_instance",
           "serve_request", "Channel", "make_channel", "inflow_profile", "inflow_ramp",
           "graded_breaks", "CHANNEL_PARAMS"]
