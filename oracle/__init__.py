"""FP64 CPU oracle for the radar echo-synthesis hot path (test infrastructure only).

Plain, slow, obviously correct NumPy float64 implementation of what the GPU path
computes: scene state per chirp, single-bounce visibility, the closed-form
physical-optics triangle integral, the coherent facet sum over frequency x
virtual channel x chirp, the beat signal, the range and Doppler FFTs and the RDM.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU library and the GPU library
never calls it. Every function cites the passage of the paper (section, equation
or table) it follows; where the paper is silent the docstring names the reading.
"""
from .constants import C0
from .waveform import derived, range_axis, velocity_axis, table2_row
from .geometry import world_triangles, facet_frames, point_positions
from .facet_integral import (phi, phi_sinc, phi_series, phi_vertex, facet_integral,
                             gordon_integral, quadrature_integral)
from .visibility import segment_occluded, visibility
from .echo import synthesize, facet_terms
from .rdm import beat, range_fft, doppler_fft, rdm, rdm_from_echo, rdm_loss

__all__ = [
    "C0", "derived", "range_axis", "velocity_axis", "table2_row", "world_triangles",
    "facet_frames", "point_positions", "phi", "phi_sinc", "phi_series", "phi_vertex",
    "facet_integral", "gordon_integral", "quadrature_integral", "segment_occluded",
    "visibility", "synthesize", "facet_terms", "beat", "range_fft", "doppler_fft",
    "rdm", "rdm_from_echo", "rdm_loss",
]
