"""FP64 CPU oracle for time-domain backprojection (TDBP).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here. The
product path (``paper_2101_05888_amd``) never imports this package and fails
loudly when its HIP library is missing.

The oracle is a plain, slow, obviously correct NumPy transcription of the
backprojection sum that inverts Eq. 1 (Sec. II-A), with the beam gate of
Sec. II-C evaluated per term, and of its gradient with respect to the
navigation and the sound speed, and of its linear adjoint with respect to the
echo (reprojection), and of the dynamic range compression applied to the
image for display (Eqs. 11-12) and of the time-varying gain and spectral
whitening applied to the echoes (Eqs. 9-10) and of the range compression
that produces them (the matched filter with Eq. 1's waveform q), and of the
time-delay estimation between consecutive pings that feeds the DPC motion
estimate (Sec. II-D). It shares no code with the HIP path.
"""
from .tdbp import (pixel_points, backproject, backproject_image, gated_term_count,
                   gated_term_count_rows, vjp, vjp_segment_bound, reproject, sharpness,
                   sharpness_cotangent, sinc_kernel, SINC_HALF, motion_delay, track_delay, track_position,
                   refracted_leg)
from .metrics import rel_l2, phase_error_mrad
from .drc import drc
from .tvg import tvg
from .whiten import whiten
from .rangec import range_compress
from . import dpc

__all__ = ["pixel_points", "backproject", "backproject_image", "gated_term_count",
           "gated_term_count_rows", "vjp", "vjp_segment_bound", "reproject", "sharpness",
           "sharpness_cotangent", "sinc_kernel", "SINC_HALF", "motion_delay", "track_delay", "track_position",
           "refracted_leg",
           "rel_l2", "phase_error_mrad", "drc", "tvg", "whiten", "range_compress", "dpc"]
