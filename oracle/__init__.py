"""FP64 CPU oracle for the differentiable RGB + depth + 16-d feature rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (``paper_2511_16144_amd``)
imports, links or calls anything here; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.
It shares no code with the HIP path; the two meet only through the seeded
input generators in ``scenes/``.

What it computes (paper: Sec. III-B.1 renders the Gaussians
Theta = {p, q, s, alpha, c, f} with the usual 3DGS rasterizer into an
RGB image and a feature map; Sec. III-B.3, Eq. (1) adds the rendered depth
used by the L1 depth loss and optimises Theta through the renderer):

  * ``raster_fp64``  -- the plain per-pixel definition, vectorised over pixel
    blocks in torch float64, with the gradient taken by torch.autograd;
  * ``brute``        -- a second, pure-Python (``math`` module) per-pixel
    brute force for tiny scenes, used to pin ``raster_fp64`` (forward) and,
    through central finite differences, its autodiff gradient;
  * ``loss_fp64``    -- the mapping loss of Eq. (1) downstream of the
    renderer, with its D-SSIM term (Gaussian-window SSIM, zero padding), and
    its gradient with respect to the rendered images by torch.autograd;
  * ``decoder_fp64`` -- the feature-distillation loss of Eq. (2) through a
    1x1-convolution decoder, with its gradients (feature map, weights, bias);
  * ``prune_fp64``   -- language-guided pruning, Eq. (4): K nearest
    neighbours, distance and feature-similarity thresholds, and the geometric
    criteria.

The paper gives no rasterizer formulas; the readings taken where it is silent
(colour model, depth definition, cut-offs, termination, pose perturbation...)
are listed in ``Settings`` and in the module docstrings.  Paper-side parity is
unpinned (the paper prints no per-pixel value); every pin comes from closed
forms, invariants, brute force and finite differences (see ``tests/``).
"""
from .raster_fp64 import (Settings, project_view, composite, render, vjp,
                          l1_upstream, l1_loss, loss_and_grads)

__all__ = ["Settings", "project_view", "composite", "render", "vjp",
           "l1_upstream", "l1_loss", "loss_and_grads"]
