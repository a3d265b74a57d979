"""Seeded synthetic video clips with ground truth.

This module only produces inputs (luma planes) and the truth they were built
from; it holds none of the measure engine's arithmetic.  Both the GPU path's
tests and the CPU oracle consume its frames.

Content recipe (shapes and effects of the paper's workloads, Sec. IV, which
uses private broadcast material):
  * background: uniform noise blurred by a periodic Gaussian (sigma scaled by
    2**L so it looks alike at the working level), mapped to [lo, hi];
  * a frame is a toroidal crop at an offset that moves by the shot's pan;
  * opaque textured rectangles with their own velocities;
  * transitions: hardcuts and K-frame linear dissolves;
  * sampling: progressive, interlaced TFF/BFF (fields half a frame apart) and
    3:2 pulldown (24p source, 5-frame cadence);
  * effects in order: compose, dissolve, flicker, flash, noise, clip.
"""
from .gen import (  # noqa: F401
    ClipSpec,
    ShotSpec,
    Renderer,
    make_c1,
    make_c2,
    make_mix_clip,
    make_c5,
    render,
    MIX_FORMATS,
)
