"""Host-side argument checks of the torch binding (no GPU needed): every
tensor's dtype, shape, layout and size is checked against the frame before
anything reaches the library, and a wrong one raises ValueError."""
import numpy as np
import pytest
import torch

from paper_2506_00225_amd import Gaussians, make_config, scenes
from paper_2506_00225_amd.rasterizer import Frame


def _gaussians(n=10, k=3):
    sc = scenes.tiny_scene(n=n, k=k)
    f = lambda a: torch.from_numpy(a).float().contiguous()
    return Gaussians(f(sc.means), f(sc.scales), f(sc.quats), f(sc.opacity), f(sc.rgb), f(sc.sem_val),
                     torch.from_numpy(sc.sem_idx).contiguous())


def _frame(n=10, k=3, V=2):
    """A Frame with its bookkeeping but no device workspace."""
    fr = Frame.__new__(Frame)
    fr.n, fr.V, fr.cfg = n, V, make_config(16, k)
    fr.device = torch.device("cuda")
    fr.pix = [64, 32][:V]
    fr.pix_off = list(np.cumsum([0] + fr.pix))
    fr.generation = 0
    return fr


@pytest.mark.parametrize("name,bad,msg", [
    ("means", torch.zeros(10, 4), "shape"),
    ("quats", torch.zeros(10, 3), "shape"),
    ("opacity", torch.zeros(10, 1), "shape"),
    ("sem_val", torch.zeros(10, 4), "shape"),
    ("sem_idx", torch.zeros(10, 3, dtype=torch.int32), "uint8"),
    ("rgb", torch.zeros(10, 3, dtype=torch.float64), "float32"),
    ("scales", torch.zeros(3, 10).t(), "contiguous"),
])
def test_gaussians_shape_dtype_layout_checked(name, bad, msg):
    g = _gaussians()
    setattr(g, name, bad)
    with pytest.raises(ValueError, match=msg):
        g.validate()


def test_gaussians_checked_against_the_frame():
    """A frame's k and n decide the shapes: a top-k list shorter than the
    config's k (the library would read past it) is rejected."""
    g = _gaussians(n=10, k=3)
    with pytest.raises(ValueError, match="shape"):
        g.validate(n=10, k=4)
    with pytest.raises(ValueError, match="shape"):
        g.validate(n=11, k=3)
    with pytest.raises(ValueError, match="CUDA"):  # everything else right: host tensors are refused last
        g.validate(n=10, k=3, device="cuda")


def test_map_and_gradient_tensors_checked():
    fr = _frame()
    P = fr.pix_off[-1]
    with pytest.raises(ValueError, match="elements"):
        fr._view_ptrs(torch.zeros(P - 1), 1, 4, name="depth")
    with pytest.raises(ValueError, match="elements"):
        fr._view_ptrs(torch.zeros(P, 2), 3, 4, name="rgb")
    with pytest.raises(ValueError, match="int32"):
        fr._view_ptrs(torch.zeros(P), 1, 4, name="n_contrib", dtype=torch.int32)
    with pytest.raises(ValueError, match="contiguous"):
        fr._view_ptrs(torch.zeros(3, P).t(), 3, 4, name="rgb")
    with pytest.raises(ValueError, match="CUDA"):
        fr._view_ptrs(torch.zeros(P, 3), 3, 4, name="rgb")
    with pytest.raises(ValueError, match="grad sil: .* elements"):
        fr._map_grads({"sil": torch.zeros(P - 5)})
    with pytest.raises(ValueError, match="grad sem: .* elements"):
        fr._map_grads({"sem": torch.zeros(P, 15)})


def test_gradient_outputs_checked():
    g = _gaussians()
    with pytest.raises(ValueError, match="gradient sem_val"):
        Frame._grads(g, {"sem_val": torch.zeros(10, 2)})
    with pytest.raises(ValueError, match="gradient means"):
        Frame._grads(g, {"means": torch.zeros(10, 3, dtype=torch.float64)})


def test_device_without_index_means_the_current_device():
    """A frame made for "cuda" compares equal to tensors on the current
    device (a bare "cuda" device differs from "cuda:0" in torch)."""
    from paper_2506_00225_amd.rasterizer import _device
    d = _device("cuda")
    assert d.type == "cuda" and d.index is not None
    assert _device("cuda:0") == torch.device("cuda", 0)
    assert _device("cpu") == torch.device("cpu")
