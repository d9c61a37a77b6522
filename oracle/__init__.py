"""Plain FP64 CPU oracle for differentiable tile-based Gaussian splatting.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
CPU-baseline leg may import this package.  The product path (the HIP library
and its Python binding) never imports, calls or links anything here, and this
package never imports the product path.  The two share no code; the only
common module is `synth`, which generates seeded inputs and holds none of the
method's arithmetic.

What it computes (PocketGS, arXiv 2601.17354, Sec. "Hardware-Aligned
Differentiable Splatting Optimization", and the 3D Gaussian Splatting
conventions that section inherits):

  projection.py  EWA projection of 3D Gaussians to 2D conics, radius, tile
                 rectangle, depth and view-dependent colour (inherited; the
                 paper does not restate it).
  binning.py     tile binning, (tile, depth) keys and their stable order; the
                 sort yields the permutation pi of the index-mapping subsection.
  render.py      per-pixel front-to-back compositing, the replay trace
                 S = {id, C_in, alpha} with per-pixel counts, and the backward
                 of the compositing recursion (equation "backward_chain")
                 in both the cached form and the recompute-T form.
  loss.py        L1 and SSIM losses and their image gradients.
  adam.py        Adam on the canonical layout.
  seed.py        KNN local statistics and disc-like covariance seeding (Sec.
                 "Prior-Conditioned Gaussian Parameterization").
  sh.py          real spherical-harmonic basis used for colour.
  mlp.py         the learned seeding network (bfloat16 products, float32
                 accumulation emulated) and its loss and targets.
  ba.py          robust bundle adjustment (Sec. "GPU-Native Global BA"):
                 Huber reprojection objective, gauge, damped normal equations.
  mvs.py         single-reference Census / plane-sweep / SGM stereo with the
                 depth range, reference score, confidence filter and fusion
                 (Sec. "Single-Reference Cost-Volume MVS").

Everything is float64.  Decisions that turn floating point into integers
(culling, radius, tile rectangle, depth key, alpha skip, termination) are
taken on float64 values; every such decision also reports how close it came
to its threshold so a test can treat a near-tie as either outcome.
"""
