"""The mapping-step helpers (loss gradient, fused Adam) against plain PyTorch
fp32 references of the same operations, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2506_00225_amd import FusedAdam, mapping_loss_grad

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _torch_loss(maps, t_rgb, t_depth, label, w):
    P = maps["depth"].shape[0]
    m = (maps["sil"] > w[4]).float().detach()
    l_d = (m * (maps["depth"] - t_depth).abs()).sum() * w[0]
    l_c = (m[:, None] * (maps["rgb"] - t_rgb).abs()).sum() * w[1]
    l_s = (maps["sil"] - 1).abs().sum() * w[2]
    pl = maps["sem"].gather(1, label.long()[:, None])[:, 0]
    l_ce = -torch.log(pl.clamp_min(1e-6)).sum() * w[3]
    return (l_d + l_c + l_s + l_ce) / P


@pytest.mark.parametrize("P,C", [(1000, 16), (4099, 102)])
def test_mapping_loss_grad_matches_torch(P, C):
    print("[case] loss grad", P, C, flush=True)
    g = torch.Generator().manual_seed(P)
    dev = "cuda"
    maps = {"rgb": torch.rand(P, 3, generator=g), "depth": torch.rand(P, generator=g) * 5,
            "sil": torch.rand(P, generator=g) * 0.02 + 0.98, "sem": torch.rand(P, C, generator=g) / C}
    maps["sem"][::7, :] = 0.0  # exercises the 1e-6 floor, where the gradient is zero
    t_rgb, t_depth = torch.rand(P, 3, generator=g), torch.rand(P, generator=g) * 5
    label = torch.randint(0, C, (P,), generator=g, dtype=torch.int32)
    w = (1.0, 0.5, 1.0, 1.0, 0.99)
    ref = {k: v.clone().requires_grad_(True) for k, v in maps.items()}
    _torch_loss(ref, t_rgb, t_depth, label, w).backward()
    got = mapping_loss_grad({k: v.to(dev) for k, v in maps.items()}, t_rgb.to(dev), t_depth.to(dev), label.to(dev), C,
                            weights=w)
    torch.cuda.synchronize()
    for k in ("rgb", "depth", "sil", "sem"):
        assert torch.allclose(got[k].cpu(), ref[k].grad, rtol=1e-5, atol=1e-9), k


def test_fused_adam_matches_torch_adam_with_clamps():
    print("[case] fused adam", flush=True)
    g = torch.Generator().manual_seed(0)
    ps = [torch.randn(1000, 3, generator=g), torch.rand(777, generator=g), torch.rand(500, 16, generator=g),
          torch.randn(1001, generator=g)]
    bounds = [(-float("inf"), float("inf")), (1e-4, 0.9999), (0.0, float("inf")), (-1.0, 1.0)]
    ref = [p.clone() for p in ps]
    dev = [p.cuda() for p in ps[:3]]
    # the last parameter starts 4 bytes into its allocation: the kernel's
    # element-wise path (16-byte vectors need aligned arrays)
    holder = torch.empty(1002, device="cuda")
    holder[1:].copy_(ps[3])
    dev.append(holder[1:])
    assert dev[3].data_ptr() % 16 != 0
    grads = [torch.zeros_like(p) for p in dev]
    opt = FusedAdam([(p, gr, lo, hi) for p, gr, (lo, hi) in zip(dev, grads, bounds)], lr=1e-2)
    topt = torch.optim.Adam(ref, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(5):
        gs = [torch.randn(p.shape, generator=g) for p in ps]
        for r, gg in zip(ref, gs):
            r.grad = gg.clone()
        topt.step()
        with torch.no_grad():
            for r, (lo, hi) in zip(ref, bounds):
                r.clamp_(lo, hi)
        for d, gg in zip(grads, gs):
            d.copy_(gg)
        opt.step()
    torch.cuda.synchronize()
    for d, r in zip(dev, ref):
        assert torch.allclose(d.cpu(), r, rtol=1e-5, atol=1e-6)
