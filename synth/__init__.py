"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds only input generation: Gaussian parameter sets, cameras,
surface point clouds, target images, bundle-adjustment tracks and ray-cast
greyscale views with exact depth (multi-view stereo inputs).  It holds
none of the splatting arithmetic (no projection, binning, compositing,
gradients or seeding) and none of the bundle adjustment's (the tracks'
measurements come from a pinhole projection written in the generator for
that purpose alone); both the oracle and the HIP path consume what it
produces.

Canonical parameter layout (one float32 row per scalar field, N columns):

    rows 0..2    mean x, y, z
    rows 3..5    log-scale (three axes)
    rows 6..9    rotation quaternion (w, x, y, z), not necessarily unit
    row  10      opacity logit
    rows 11..    spherical-harmonic colour coefficients, coefficient-major:
                 row 11 + 3*k + ch holds coefficient k = l*l + l + m of
                 channel ch, k < (D+1)^2 for SH degree D.

Cameras are dicts with width, height, fx, fy, cx, cy and a float32 3x4
world-to-camera matrix [R|t] (OpenCV axes: x right, y down, z forward).
Images are float32 planar [3, H, W].

Every generator draws from numpy.random.default_rng(seed) in the order its
docstring states, so the same seed gives the same arrays on any machine.
"""

from .gen import (  # noqa: F401
    param_rows,
    sh_coeffs,
    make_camera,
    look_at_camera,
    ring_cameras,
    cfg1_inputs,
    random_gaussians,
    Scene,
    spheres_planes_scene,
    sample_surface,
    surface_gaussians,
    noisy_cloud,
    random_image,
    random_normal,
    ba_tracks,
    textured_views,
)
