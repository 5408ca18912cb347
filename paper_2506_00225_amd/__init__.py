"""MI355X-native semantic Gaussian rasterizer and candidate-view scorer.

The hot path (projection, tile binning with an on-device radix sort,
front-to-back compositing of colour / depth / silhouette / sparse top-k
semantics, its backward pass, and batched view scoring) runs in the HIP
library libsgr.so behind the C ABI of include/sgr.h; this package only
marshals arguments and takes device memory and streams from PyTorch.
"""
from . import _lib, autotune
from ._lib import SgrError
from .rasterizer import (FusedAdam, Frame, Gaussians, camera_array, loss_config, make_config, mapping_loss_grad,
                         render, score_maps, topk_select, topk_update)

__all__ = ["FusedAdam", "Frame", "Gaussians", "SgrError", "autotune", "camera_array", "loss_config", "make_config",
           "mapping_loss_grad", "render", "score_maps", "topk_select", "topk_update", "_lib"]
