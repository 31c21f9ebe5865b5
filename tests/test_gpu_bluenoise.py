"""Blue-noise u (Sec. 6.3): the mask, the s-normalised scatter and its backward with u read from
a void-and-cluster threshold texture tiled with a per-image, per-frame toroidal offset, against
the oracle (the mask bit for bit)."""
import math

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import sampling as osamp
from tests._tol import assert_mag_close
from tests.test_gpu_backward import _np, assert_grad_close

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


@pytest.fixture(scope="module")
def tex64():
    return procgen.blue_noise_thresholds(64)


def _s_map(N, H, W, B, seed):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(N, H, W)) * 2.0
    return odens.normalise(torch.tensor(z), B).numpy().astype(np.float32)


@pytest.mark.parametrize("shape,T", [((1, 128, 128), 64), ((2, 37, 53), 64), ((1, 1080, 1920), 64),
                                     ((3, 20, 31), 7), ((1, 5, 9), 1)])
def test_mask_texture_bit_exact(ops, tex64, shape, T):
    tex = tex64 if T == 64 else procgen.blue_noise_thresholds(T, seed=T)
    s = _s_map(*shape, 0.25, sum(shape))
    for frame in (0, 5):
        r = ops.sample_mask(torch.tensor(s, device=DEV), 31, frame, want_p=True,
                            u_tex=torch.tensor(tex, device=DEV))
        m = osamp.mask(s, 31, frame, u_tex=tex)
        assert np.array_equal(r["count"].cpu().numpy(), m["count"])
        assert int(r["total"].item()) == m["total"]
        cap = r["capacity"]
        assert np.array_equal(r["sample_pixel"][:min(cap, m["total"])].cpu().numpy(),
                              m["sample_pixel"][:cap])


def test_mask_texture_stratified_on_gpu(ops, tex64):
    """Constant p: every 64 x 64 window takes exactly ceil(p T^2 - 1/2) holdouts."""
    N, H, W, T = 2, 200, 264, 64
    for k, p in ((0, 0.25), (1, 0.125 + 2.0 ** -12)):
        s = torch.full((N, H, W), k + p, dtype=torch.float32, device=DEV)
        c = ops.sample_mask(s, 8, 3, u_tex=torch.tensor(tex64, device=DEV))["count"].cpu().numpy()
        want = T * T * k + math.ceil(p * T * T - 0.5)
        for n in range(N):
            for y0, x0 in ((0, 0), (17, 101), (H - T, W - T)):
                assert int(c[n, y0:y0 + T, x0:x0 + T].astype(np.int64).sum()) == want


def test_mask_texture_argument_checks(ops, tex64):
    from paper_2602_08642_amd import _lib as L
    s = torch.full((1, 8, 8), 0.5, device=DEV)
    r = ops.sample_mask(s, 1, 0)   # buffers
    lib = L.load()
    ws = torch.empty(lib.aps_sample_mask_workspace_size(1, 8, 8), dtype=torch.uint8, device=DEV)
    t = torch.tensor(tex64, device=DEV)
    for bad in (0, 5000):
        assert lib.aps_sample_mask_ex(ops._p(s), 1, 8, 8, 1, 0, ops._p(t), bad, L.APS_ROUND_STOCHASTIC,
                                      ops._p(r["count"]), ops._p(r["pixel_offset"]), ops._p(r["sample_pixel"]),
                                      r["capacity"], ops._p(r["total"]), None, ops._p(ws), ws.numel(),
                                      None, ops._stream()) == L.APS_ERR_ARG
    assert lib.aps_sample_mask_ex(ops._p(s), 1, 8, 8, 1, 0, None, 0, 3, ops._p(r["count"]),
                                  ops._p(r["pixel_offset"]), ops._p(r["sample_pixel"]), r["capacity"],
                                  ops._p(r["total"]), None, ops._p(ws), ws.numel(), None,
                                  ops._stream()) == L.APS_ERR_ARG
    with pytest.raises(ValueError):
        ops.sample_mask(s, 1, 0, u_tex=t[:, :32].contiguous())


@pytest.mark.parametrize("mode", ["hard", "relaxed"])
def test_scatter_texture_matches_oracle(ops, tex64, mode):
    N, H, W, levels, seed, frame = 2, 48, 40, 3, 13, 4
    s = _s_map(N, H, W, 0.5, 3)
    t = torch.tensor(tex64, device=DEV)
    st = torch.tensor(s, device=DEV)
    r = ops.sample_mask(st, seed, frame, u_tex=t)
    total = int(r["total"].item())
    rng = np.random.default_rng(4)
    smp = torch.tensor(rng.normal(1.0, 0.7, size=(r["capacity"], 4)).astype(np.float32), device=DEV)
    Ls = ops.scatter_samples(st, r["count"], r["pixel_offset"], smp, levels, mode, 10.0, seed, frame,
                             u_tex=t)
    sn = smp[:total].cpu().numpy()
    ref = osamp.scatter(s.astype(np.float64), r["count"].cpu().numpy(), sn, seed, frame, mode, 10.0,
                        u_tex=tex64)
    mag = osamp.scatter(s.astype(np.float64), r["count"].cpu().numpy(), np.abs(sn), seed, frame, mode,
                        10.0, u_tex=tex64)
    for l, (a, b) in enumerate(zip(osamp.pyramid(ref, levels), osamp.pyramid(mag, levels))):
        assert_mag_close(Ls[l], a, b, 1e-5, what=f"{mode} level {l}")
    if mode == "relaxed":
        # the Philox u would weight the holdouts differently
        Lp = ops.scatter_samples(st, r["count"], r["pixel_offset"], smp, levels, mode, 10.0, seed, frame)
        assert not torch.equal(Lp[0], Ls[0])


def test_scatter_backward_texture(ops, tex64):
    N, H, W, levels, seed, frame = 2, 16, 24, 3, 21, 3
    s = _s_map(N, H, W, 0.5, 5)
    t = torch.tensor(tex64, device=DEV)
    st = torch.tensor(s, device=DEV)
    r = ops.sample_mask(st, seed, frame, u_tex=t)
    total = int(r["total"].item())
    rng = np.random.default_rng(5)
    smp = torch.tensor(rng.normal(size=(r["capacity"], 4)).astype(np.float32), device=DEV)
    gL = [torch.tensor(rng.normal(size=(N, H >> l, W >> l, 4)).astype(np.float32), device=DEV)
          for l in range(levels)]
    gs = ops.scatter_samples_bwd(st, r["count"], r["pixel_offset"], smp, gL, "relaxed", 10.0, seed,
                                 frame, u_tex=t)
    s64 = torch.tensor(s.astype(np.float64), requires_grad=True)
    L0 = osamp.scatter(s64, r["count"].cpu().numpy(), smp[:total].cpu().numpy(), seed, frame,
                       "relaxed", 10.0, u_tex=tex64)
    pyr = osamp.pyramid(L0, levels)
    sum(((p * torch.tensor(_np(g))).sum()) for p, g in zip(pyr, gL)).backward()
    assert_grad_close(gs, s64.grad, 1e-4, "relaxed, texture u")
