"""Parity at the benchmark's full sizes, in the launch configurations bench.py times: the 1080p
U-Net (bf16 as in C3, fp32 as in C2, and bf16 with the 4K configuration's four heads of
67/58/58/49 logits), the fused sampler CNN at 1080p and the gathering pyramids of C3, of the
paper configuration and of the 3840x2160 configuration (bf16 logits, temporal term), each
against the FP64 oracle over the whole frame, element by element.  Networks are checked
stage-wise (every layer on the GPU's input of that layer) and end to end per head, as
tests/_nets.py describes."""
import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import filt as ofilt
from oracle import unet as ounet
from tests import _nets
from tests._tol import assert_mag_close

pytestmark = pytest.mark.gpu
DEV = "cuda"
H, W = 1080, 1920


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


# end-to-end tolerances per head: normwise (the stated relative error against FP64) and
# element by element relative to abs(r) + rms(r)
E2E = {torch.bfloat16: (2e-2, 6e-2), torch.float32: (1e-5, 1e-4)}
LAYER_TOL = {torch.bfloat16: 2e-2, torch.float32: 1e-5}


def _wq(w, dtype):
    return {k: (torch.tensor(a).to(dtype).double(), torch.tensor(b).double()) for k, (a, b) in w.items()}


@pytest.mark.parametrize("dtype,heads", [
    (torch.bfloat16, [43, 34, 25]),          # C3
    (torch.float32, [34, 34, 25]),           # C2
    (torch.bfloat16, [67, 58, 58, 49]),      # the 4K configuration's heads
])
def test_unet_1080p_matches_oracle(ops, dtype, heads):
    spec = procgen.unet_spec(16, heads)
    w = procgen.init_weights(spec, 21)
    net = ops.Net(spec, w, dtype, DEV)
    x = torch.rand(1, H, W, 16, generator=torch.Generator().manual_seed(4))
    x[..., 15] = 0
    xd = x.to(DEV).to(dtype)
    logits = ops.kernel_predict(net, xd, heads, dtype)
    rec, chain = _nets.unet_chain(ops, net, xd, heads, dtype)
    what = f"unet 1080p {str(dtype)[6:]} {heads}"
    for l, K in enumerate(heads):
        if dtype == torch.bfloat16:
            assert torch.equal(logits[l][..., :K], chain[l][..., :K]), l
        else:   # the fused heads sum the 1x1 product in another order
            assert_mag_close(logits[l][..., :K].cpu(), chain[l][..., :K].cpu(),
                             chain[l][..., :K].abs().cpu() + float(chain[l][..., :K].abs().mean()),
                             1e-6, what=f"{what} fused vs chain head {l}")
    wq = _wq(w, dtype)
    _nets.check_layers(rec, wq, {l["name"]: l["relu"] for l in spec}, LAYER_TOL[dtype], what)
    del rec, chain
    ref = ounet.unet_forward(x.to(dtype).double(), wq, len(heads))
    _nets.check_end_to_end([t.cpu() for t in logits], ref, heads, *E2E[dtype], what=what)


@pytest.mark.parametrize("cin,dtype", [(16, torch.bfloat16), (8, torch.float32)])
def test_sampler_1080p_matches_oracle(ops, cin, dtype):
    spec = procgen.density_cnn_spec(cin)
    w = procgen.init_weights(spec, 22)
    net = ops.Net(spec, w, dtype, DEV)
    x = torch.rand(1, H, W, cin, generator=torch.Generator().manual_seed(5))
    xd = x.to(DEV).to(dtype)
    z, s = ops.density_predict(net, xd, 0.25)
    rec, zc = _nets.sampler_chain(ops, net, xd)
    what = f"sampler 1080p {str(dtype)[6:]}"
    # the fused kernel sums K in another order than the layer chain (bf16: an intermediate may
    # round one ulp apart)
    tol = 2.0 ** -6 if dtype == torch.bfloat16 else 1e-5
    assert_mag_close(z.cpu(), zc.cpu(), zc.abs().cpu() + float(zc.abs().mean()), tol,
                     what=f"{what} fused vs chain")
    wq = _wq(w, dtype)
    _nets.check_layers(rec, wq, {l["name"]: l["relu"] for l in spec}, LAYER_TOL[dtype], what)
    layers = [(wq[l["name"]][0], wq[l["name"]][1], l["relu"]) for l in spec]
    zr = odens.cnn_forward(x.to(dtype).double(), layers)[..., 0]
    _nets.check_end_to_end([z.cpu()], [zr], [0], *E2E[dtype], what=what)
    # the normalisation on the GPU's z: s > 0, so relative to s itself
    sr = odens.normalise(z.double().cpu(), 0.25)
    assert_mag_close(s.cpu(), sr, sr, 1e-5, what="normalisation 1080p")


@pytest.mark.parametrize("case", [
    # C3 reconstruction: 3 levels, kd 5x5, ku 3x3, kt 3x3, bf16 logits, warped history
    (1080, 1920, 3, 5, 3, 3),
    # the paper's reconstruction (App. A) on 1080p padded to 1088 rows: 5 levels, kd 5x5,
    # the printed 2x2 ku, kt 5x5
    (1088, 1920, 5, 5, 2, 5),
    # the 3840x2160 configuration: 4 levels, kd 7x7, ku 3x3, kt 3x3 (67-way softmax at level 0)
    (2160, 3840, 4, 7, 3, 3),
])
def test_denoise_pyramid_fullsize(ops, case):
    H, W, levels, KD, KU, KT = case
    g = torch.Generator().manual_seed(23)
    Ls = [torch.randn(1, H >> l, W >> l, 4, generator=g) * 2.0 for l in range(levels)]
    for t in Ls:
        t[..., 3] = 0
    Ks = procgen.kernel_channels(levels, KD, KU, KT, True)
    logits = []
    for l in range(levels):
        ks = ops.round_kstride(Ks[l], torch.bfloat16)
        z = torch.randn(1, H >> l, W >> l, ks, generator=g) * 2.0
        z[..., Ks[l]:] = 0.0
        logits.append(z.to(torch.bfloat16))
    prev = torch.randn(1, H, W, 4, generator=g)
    prev[..., 3] = 0
    mv = torch.rand(1, H, W, 2, generator=g) * 24 - 12
    out = ops.denoise_pyramid([t.to(DEV) for t in Ls], [t.to(DEV) for t in logits], KD, KU, KT,
                              prev.to(DEV), mv.to(DEV))
    L64 = [t.double() for t in Ls]
    z64 = [t.double() for t in logits]
    ref = ofilt.denoise_pyramid(L64, z64, KD, KU, KT, prev.double(), mv.double())[0]
    mag = ofilt.denoise_magnitude(L64, z64, KD, KU, KT, prev.double(), mv.double())[0]
    assert_mag_close(out[..., :3], ref[..., :3], mag[..., :3], 1e-5, what=str(case))
    assert torch.all(out[..., 3] == 0)
