"""What the trained density buys (Sec. 7, the "Ours Uniform" rows): the shipped C4 weights on
16 held-out procedural clips at 0.25 spp, each clip rendered with the same sample pools by the
learned path (sampler + kernel network) and by uniform sampling with its own trained kernel
network.  The paired per-clip PSNR difference must be positive with 95 % confidence (Student-t
interval over the clips), and both must beat the fixed-kernel fallback."""
import os

import pytest
import torch

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2602_08642_amd", "weights", "c4_trained.npz")


def test_learned_density_beats_uniform_at_equal_spp():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import evaluate
    res = evaluate.compare_trained(WEIGHTS, budgets=(0.25,))
    print(res)
    g = res["paired_gain_vs_uniform"]
    assert g["clips"] == 16
    assert g["ci95_db"][0] > 0.0, g
    assert res["paired_gain_vs_fallback"]["ci95_db"][0] > 0.0
    assert res["uniform"]["psnr"] > res["fallback"]["psnr"]
