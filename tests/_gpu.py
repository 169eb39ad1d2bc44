"""GPU test helpers: skip cleanly without a GPU, convert scenes to device arrays."""
import numpy as np
import pytest
import torch

import paper_2605_13600_amd as P


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_device(scene_gaussians, scene_views):
    return P.gaussians_to_device(scene_gaussians), P.views_to_device(scene_views)
