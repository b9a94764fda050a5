"""Seeded synthetic compressed time frames (inputs only).

This module draws compressed-frame streams with the shapes of Pb-Pb running;
it holds none of the decoding arithmetic.  Both the GPU library's tests and
benchmarks and the CPU oracle consume its frames.  See synth.frames.
"""
from .frames import WORKLOADS, FrameSpec, batch_specs, make_frame, spec_for  # noqa: F401
