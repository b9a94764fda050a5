"""Seeded synthetic compressed time frames (inputs only).

This module draws compressed-frame streams with the shapes of Pb-Pb running.
It never decodes a stream: residuals are measured codes minus the prediction
of a float64 geometric shadow of the track model, which keeps the streams
valid decoder input.  Both the GPU library's tests and benchmarks and the CPU
oracle consume its frames.  See synth.frames.  synth.phys draws physical
clusters (positions as doubles, grouped by track), the encoder's input.
"""
from .frames import WORKLOADS, FrameSpec, batch_specs, make_frame, make_frames, spec_for  # noqa: F401
from .phys import make_phys, phys_sizes  # noqa: F401
