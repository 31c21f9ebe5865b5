"""Seeded synthetic inputs shared by the HIP path, its tests and the CPU oracle.

This module holds no arithmetic of the adaptive-sampling method itself (no density,
normalisation, sampling, scatter or filtering).  It only makes inputs:

* procedural HDR scenes (Gaussian blobs + hard-edged star polygons, lognormal(0,1)
  intensities) with albedo / normal / depth auxiliary buffers,
* camera clips with global rotation + translation and the exact backward motion
  vectors (screen-edge disocclusions included),
* per-pixel pools of noisy "rendered" samples, truth * (1 + n) with
  n = lognormal(0, 0.8) - E[lognormal(0, 0.8)]  (zero-mean multiplicative noise with
  firefly tails), standing in for the paper's pre-rendered path-traced samples
  (Sec. 3, last paragraph: samples are pre-rendered and combined into any budget),
* seeded random-init network weights (Kaiming-uniform),
* a blue-noise threshold texture by void-and-cluster (the table of u the sampling step can
  draw from instead of Philox).

Everything is NumPy and addressed by integer seeds, so the same call gives the same
arrays on any machine.
"""
from .scene import (make_scene, render_view, make_frame, make_clip, camera_motion,
                    sample_pool, FrameData)
from .weights import (density_cnn_spec, unet_spec, small_kernel_cnn_spec, init_weights,
                      kernel_channels)

__all__ = [
    "make_scene", "render_view", "make_frame", "make_clip", "camera_motion", "sample_pool",
    "FrameData", "density_cnn_spec", "unet_spec", "small_kernel_cnn_spec", "init_weights",
    "kernel_channels",
]
from .bluenoise import void_and_cluster, blue_noise_thresholds
