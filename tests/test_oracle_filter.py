"""Pins of the oracle's joint softmax, gathers, upsampling, warp and reconstruction."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.special
import torch

from oracle import filt

NEG = -1e30


def _edge_shift(img, dy, dx):
    """numpy edge-padded shift: out[y, x] = img[clamp(y+dy), clamp(x+dx)]."""
    N, H, W, C = img.shape
    r = max(abs(dy), abs(dx), 1)
    p = np.pad(img, ((0, 0), (r, r), (r, r), (0, 0)), mode="edge")
    return p[:, r + dy:r + dy + H, r + dx:r + dx + W]


def test_joint_softmax_matches_library():
    z = torch.randn(2, 3, 4, 34, dtype=torch.float64) * 3
    ws = filt.joint_softmax(z, [25, 9])
    ref = scipy.special.softmax(z.numpy(), axis=-1)
    assert np.allclose(torch.cat(ws, -1).numpy(), ref, rtol=1e-13)
    assert torch.allclose(sum(w.sum(-1) for w in ws), torch.ones(2, 3, 4, dtype=torch.float64))


@pytest.mark.parametrize("K", [3, 5, 7])
def test_gather_zero_logits_is_box_filter(K):
    img = torch.randn(1, 11, 13, 4, dtype=torch.float64)
    w = torch.softmax(torch.zeros(1, 11, 13, K * K, dtype=torch.float64), -1)
    ours = filt.gather(img, w, K).numpy()
    ref = ndi.uniform_filter(img.numpy(), size=(1, K, K, 1), mode="nearest")
    assert np.allclose(ours, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("tap", [(0, 0), (1, -2), (-2, 2), (2, 1)])
def test_gather_one_hot_is_clamped_shift(tap):
    dy, dx = tap
    K = 5
    img = torch.randn(2, 6, 9, 4, dtype=torch.float64)
    z = torch.full((2, 6, 9, K * K), NEG, dtype=torch.float64)
    z[..., (dy + 2) * K + (dx + 2)] = 0.0
    (w,) = filt.joint_softmax(z, [K * K])
    out = filt.gather(img, w, K)
    assert np.array_equal(out.numpy(), _edge_shift(img.numpy(), dy, dx))


def test_upsample_zero_logits_ku3():
    coarse = torch.randn(1, 5, 7, 4, dtype=torch.float64)
    w = torch.full((1, 10, 14, 9), 1.0 / 9, dtype=torch.float64)
    ours = filt.upsample(coarse, w, 3, 10, 14).numpy()
    box = ndi.uniform_filter(coarse.numpy(), size=(1, 3, 3, 1), mode="nearest")
    ref = np.repeat(np.repeat(box, 2, axis=1), 2, axis=2)
    assert np.allclose(ours, ref, rtol=1e-12, atol=1e-12)


def test_upsample_one_hot_taps():
    coarse = torch.randn(1, 4, 5, 4, dtype=torch.float64)
    c = coarse.numpy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            w = torch.zeros(1, 8, 10, 9, dtype=torch.float64)
            w[..., (dy + 1) * 3 + (dx + 1)] = 1.0
            out = filt.upsample(coarse, w, 3, 8, 10).numpy()
            for y in range(8):
                for x in range(10):
                    yy = min(max(y // 2 + dy, 0), 3)
                    xx = min(max(x // 2 + dx, 0), 4)
                    assert np.array_equal(out[0, y, x], c[0, yy, xx])
    # printed 2x2 form: tap (i, j) reads (floor((x+i)/2), floor((y+j)/2))
    for j in (0, 1):
        for i in (0, 1):
            w = torch.zeros(1, 8, 10, 4, dtype=torch.float64)
            w[..., j * 2 + i] = 1.0
            out = filt.upsample(coarse, w, 2, 8, 10).numpy()
            for y in range(8):
                for x in range(10):
                    assert np.array_equal(out[0, y, x], c[0, min((y + j) // 2, 3), min((x + i) // 2, 4)])


def test_warp_pins():
    prev = torch.randn(2, 9, 12, 4, dtype=torch.float64)
    zero = torch.zeros(2, 9, 12, 2, dtype=torch.float64)
    assert torch.equal(filt.warp(prev, zero), prev)
    mv = torch.zeros(2, 9, 12, 2, dtype=torch.float64)
    mv[..., 0] = 3.0
    mv[..., 1] = -2.0
    assert np.array_equal(filt.warp(prev, mv).numpy(), _edge_shift(prev.numpy(), -2, 3))
    rng = np.random.default_rng(0)
    mv = torch.tensor(rng.uniform(-4, 4, (2, 9, 12, 2)).astype(np.float32), dtype=torch.float64)
    ours = filt.warp(prev, mv).numpy()
    P = prev.numpy()
    yy, xx = np.meshgrid(np.arange(9), np.arange(12), indexing="ij")
    for n in range(2):
        for c in range(4):
            ref = ndi.map_coordinates(P[n, ..., c], [yy + mv[n, ..., 1].numpy(), xx + mv[n, ..., 0].numpy()],
                                      order=1, mode="nearest")
            assert np.allclose(ours[n, ..., c], ref, rtol=1e-12, atol=1e-12)


def _rand_levels(N, H, W, levels, seed=0):
    g = torch.Generator().manual_seed(seed)
    return [torch.randn(N, H >> l, W >> l, 4, generator=g, dtype=torch.float64) for l in range(levels)]


def test_reconstruction_preserves_constant():
    """Joint normalisation (App. A): constant levels and history give that constant."""
    KD, KU, KT, levels = 5, 3, 3, 3
    N, H, W = 1, 16, 20
    L = [torch.full((N, H >> l, W >> l, 4), 2.5, dtype=torch.float64) for l in range(levels)]
    g = torch.Generator().manual_seed(1)
    logits = [torch.randn(N, H >> l, W >> l, 60, generator=g, dtype=torch.float64) * 2 for l in range(levels)]
    prev = torch.full((N, H, W, 4), 2.5, dtype=torch.float64)
    mv = torch.randn(N, H, W, 2, generator=g, dtype=torch.float64) * 3
    out = filt.denoise_pyramid(L, logits, KD, KU, KT, prev, mv)
    for o in out:
        assert torch.allclose(o, torch.full_like(o, 2.5), rtol=1e-13)


def test_reconstruction_block_selection():
    """One-hot logits select one source: kd centre -> L^0, ku centre -> parent of Lhat^1,
    kt centre -> warped history."""
    KD, KU, KT, levels = 5, 3, 3, 2
    N, H, W = 1, 8, 10
    L = _rand_levels(N, H, W, levels)
    g = torch.Generator().manual_seed(3)
    prev = torch.randn(N, H, W, 4, generator=g, dtype=torch.float64)
    mv = torch.randn(N, H, W, 2, generator=g, dtype=torch.float64)
    K0 = KD * KD + KU * KU + KT * KT
    coarse_logits = torch.full((N, H // 2, W // 2, KD * KD), NEG, dtype=torch.float64)
    coarse_logits[..., 12] = 0
    for which, off in (("kd", 12), ("ku", KD * KD + 4), ("kt", KD * KD + KU * KU + 4)):
        z0 = torch.full((N, H, W, K0), NEG, dtype=torch.float64)
        z0[..., off] = 0
        out = filt.denoise_pyramid(L, [z0, coarse_logits], KD, KU, KT, prev, mv)[0]
        if which == "kd":
            assert torch.equal(out, L[0])
        elif which == "ku":
            assert torch.equal(out, L[1].repeat_interleave(2, 1).repeat_interleave(2, 2))
        else:
            assert torch.equal(out, filt.warp(prev, mv))


def test_first_frame_excludes_temporal():
    KD, KU, KT, levels = 5, 3, 3, 2
    L = _rand_levels(1, 8, 8, levels)
    z = [torch.randn(1, 8, 8, 43, dtype=torch.float64), torch.randn(1, 4, 4, 25, dtype=torch.float64)]
    a = filt.denoise_pyramid(L, z, KD, KU, KT)[0]
    z2 = [z[0][..., :34], z[1]]
    b = filt.denoise_pyramid(L, z2, KD, KU, KT)[0]
    assert torch.equal(a, b)


def test_demodulation_pins():
    """d = 1 at z = 0 (identity); a constant z scales the filter input and output by inverse
    factors, so a linear reconstruction is unchanged; levels are block means; |z| is clamped."""
    from oracle import demod
    g = torch.Generator().manual_seed(3)
    N, H, W, levels, KD, KU, KT = 1, 16, 24, 3, 5, 3, 3
    L = [torch.randn(N, H >> l, W >> l, 4, generator=g, dtype=torch.float64) for l in range(levels)]
    for t in L:
        t[..., 3] = 0
    Ks = [KD * KD + (KU * KU if l < levels - 1 else 0) for l in range(levels)]
    z = [torch.randn(N, H >> l, W >> l, Ks[l], generator=g, dtype=torch.float64) for l in range(levels)]
    # identity at z = 0
    zero = torch.zeros(N, H, W, 3, dtype=torch.float64)
    Ld = demod.demodulate(L[0], zero, levels)
    assert torch.equal(Ld[0], L[0])
    # levels are the block means of level 0
    pool = lambda x: torch.nn.functional.avg_pool2d(x.permute(0, 3, 1, 2), 2).permute(0, 2, 3, 1)
    assert torch.allclose(Ld[1], pool(Ld[0]), rtol=1e-14, atol=1e-15)
    assert torch.allclose(Ld[2], pool(pool(Ld[0])), rtol=1e-14, atol=1e-15)
    # a constant map: out = d * F(L / d) = F(L) for the linear pyramid
    c = torch.full((N, H, W, 3), 0.7, dtype=torch.float64)
    pyr = demod.demodulate(L[0], c, levels)
    ref = filt.denoise_pyramid(demod.demodulate(L[0], zero, levels), z, KD, KU, KT)[0]
    out = demod.remodulate(filt.denoise_pyramid(pyr, z, KD, KU, KT)[0], c)
    assert torch.allclose(out, ref, rtol=1e-12, atol=1e-12)
    # per-pixel: the map divides exactly where it is predicted
    zz = torch.clamp(torch.randn(N, H, W, 3, generator=g, dtype=torch.float64), -3, 3) * 2   # inside the clamp
    Ld = demod.demodulate(L[0], zz, 1)[0]
    assert torch.allclose(Ld[..., :3] * torch.exp(zz), L[0][..., :3], rtol=1e-13)
    assert torch.equal(demod.demod_map(torch.tensor([-20.0, 20.0], dtype=torch.float64)),
                       torch.exp(torch.tensor([-8.0, 8.0], dtype=torch.float64)))
