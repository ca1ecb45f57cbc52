"""Seeded synthetic inputs for time-domain backprojection (TDBP).

This package is the only code shared by the FP64 oracle (``oracle/``) and the
HIP path (``paper_2101_05888_amd``). It draws random numbers, lays out the
acquisition geometry and synthesizes echoes from the forward model of
Eq. 1 (Sec. II-A): a point-scatterer scene, range-compressed, at complex
baseband. It never backprojects: interpolation of echoes, carrier-phase
re-application and accumulation over pixels live only in the oracle and in the
HIP kernels, which share no code.
"""
from .scenario import Scenario, Grid, make_config, CONFIG_IDS, subset_indices, receiver_velocity, receiver_track, dpc_track
from .echo import synthesize_echo, add_noise, quantize_echo, dequantize_echo

__all__ = [
    "Scenario", "Grid", "make_config", "CONFIG_IDS", "subset_indices", "receiver_velocity", "receiver_track", "dpc_track",
    "synthesize_echo", "add_noise", "quantize_echo", "dequantize_echo",
]
