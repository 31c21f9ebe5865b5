"""Pins of the oracle's networks (against torch.nn layers), TMO and gradients (FD)."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import procgen
from oracle import density, filt, sampling, tmo, unet


def _nchw_conv(x, wb, k):
    w, b = wb
    return Fn.conv2d(x, w.permute(0, 3, 1, 2), b, padding=k // 2)


def test_unet_matches_torch_layers():
    heads = procgen.kernel_channels(3, 5, 3, 3, True)
    spec = procgen.unet_spec(16, heads, widths=(8, 8, 16, 16))
    wts = unet.to_torch(procgen.init_weights(spec, 3))
    x = torch.randn(2, 16, 24, 16, dtype=torch.float64)
    ours = unet.unet_forward(x, wts, 3)
    # the same architecture built from library layers in NCHW
    r = lambda t, n: Fn.relu(_nchw_conv(t, wts[n], 3))
    up = lambda t: Fn.interpolate(t, scale_factor=2, mode="nearest")
    pool = lambda t: Fn.avg_pool2d(t, 2)
    xc = x.permute(0, 3, 1, 2)
    e0 = r(r(xc, "enc0a"), "enc0b")
    e1 = r(r(pool(e0), "enc1a"), "enc1b")
    e2 = r(r(pool(e1), "enc2a"), "enc2b")
    e3 = r(r(pool(e2), "bota"), "botb")
    d2 = r(r(torch.cat([up(e3), e2], 1), "dec2a"), "dec2b")
    d1 = r(r(torch.cat([up(d2), e1], 1), "dec1a"), "dec1b")
    d0 = r(r(torch.cat([up(d1), e0], 1), "dec0a"), "dec0b")
    for l, f in enumerate([d0, d1, d2]):
        ref = _nchw_conv(f, wts[f"head{l}"], 1).permute(0, 2, 3, 1)
        assert ours[l].shape == ref.shape
        assert torch.allclose(ours[l], ref, rtol=1e-11, atol=1e-12)


def test_unet_five_heads_matches_torch_layers():
    """The five-level pyramid's head 4 is a 1x1 conv on the 2x2-pooled bottleneck; heads 0-3
    are those of the four-head network."""
    heads = procgen.kernel_channels(5, 5, 2, 5, True)
    assert heads == [54, 29, 29, 29, 25]                      # App. A: 25 + 4 + 25 at l = 0
    spec = procgen.unet_spec(16, heads, widths=(8, 8, 16, 16))
    wts = unet.to_torch(procgen.init_weights(spec, 4))
    x = torch.randn(1, 32, 48, 16, dtype=torch.float64)
    ours = unet.unet_forward(x, wts, 5)
    four = unet.unet_forward(x, wts, 4)
    for l in range(4):
        assert torch.equal(ours[l], four[l])
    r = lambda t, n: Fn.relu(_nchw_conv(t, wts[n], 3))
    pool = lambda t: Fn.avg_pool2d(t, 2)
    xc = x.permute(0, 3, 1, 2)
    e0 = r(r(xc, "enc0a"), "enc0b")
    e1 = r(r(pool(e0), "enc1a"), "enc1b")
    e2 = r(r(pool(e1), "enc2a"), "enc2b")
    e3 = r(r(pool(e2), "bota"), "botb")
    ref = _nchw_conv(pool(e3), wts["head4"], 1).permute(0, 2, 3, 1)
    assert ours[4].shape == (1, 2, 3, 25)
    assert torch.allclose(ours[4], ref, rtol=1e-11, atol=1e-12)


def test_density_quarter_pins():
    """Quarter-resolution density: the budget sum over the full frame, block constancy, the
    uniform floor, the 2x2 block mean as the CNN input, and a constant CNN giving s = B."""
    spec = procgen.density_cnn_spec(8)
    wts = unet.to_torch(procgen.init_weights(spec, 6))
    layers = [(wts[l["name"]][0], wts[l["name"]][1], l["relu"]) for l in spec]
    g = torch.Generator().manual_seed(7)
    x = torch.randn(2, 12, 20, 8, generator=g, dtype=torch.float64)
    B = 0.25
    zq, s = density.density_quarter(x, layers, B)
    assert zq.shape == (2, 6, 10) and s.shape == (2, 12, 20)
    for n in range(2):
        assert abs(float(s[n].sum()) - 12 * 20 * B) < 1e-10        # sum(s) = Npx * B
    assert torch.equal(s[:, 0::2, 0::2], s[:, 1::2, 1::2])
    assert torch.equal(s[:, 0::2, 0::2], s[:, 0::2, 1::2])
    assert torch.equal(s[:, 0::2, 0::2], s[:, 1::2, 0::2])
    assert float(s.min()) >= B / 8 - 1e-15
    # features constant on 2x2 blocks: the block mean is the block's value
    xb = x[:, 0::2, 0::2].repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)
    zqb, _ = density.density_quarter(xb, layers, B)
    assert torch.allclose(zqb, density.cnn_forward(x[:, 0::2, 0::2], layers)[..., 0], rtol=1e-12, atol=1e-12)
    # a hand-checked block mean
    t = torch.arange(16, dtype=torch.float64).reshape(1, 4, 4, 1)
    assert density.block_mean2(t)[0, :, :, 0].tolist() == [[2.5, 4.5], [10.5, 12.5]]
    # zero weights: z is the bias everywhere, the softmax is uniform and s = B exactly
    flat = [(torch.zeros_like(w), torch.full_like(b, 0.3), relu) for w, b, relu in layers]
    _, s0 = density.density_quarter(x, flat, B)
    assert torch.allclose(s0, torch.full_like(s0, B), rtol=0, atol=1e-15)


def test_density_cnn_matches_torch_layers():
    spec = procgen.density_cnn_spec(8)
    wts = unet.to_torch(procgen.init_weights(spec, 5))
    x = torch.randn(1, 12, 10, 8, dtype=torch.float64)
    layers = [(wts[l["name"]][0], wts[l["name"]][1], l["relu"]) for l in spec]
    ours = density.cnn_forward(x, layers)
    t = x.permute(0, 3, 1, 2)
    t = Fn.relu(_nchw_conv(t, wts["d0"], 3))
    t = Fn.relu(_nchw_conv(t, wts["d1"], 3))
    t = _nchw_conv(t, wts["d2"], 3)
    assert torch.allclose(ours, t.permute(0, 2, 3, 1), rtol=1e-11, atol=1e-12)


def test_tmo_curve_properties():
    x = torch.linspace(-6, 6, 20001, dtype=torch.float64)
    for s, h in ((0.1, 0.9), (0.5, 0.5), (0.9, 0.1), (0.3, 0.7)):
        t = tmo.tau(x, s, h)
        assert torch.all((t > 0) & (t <= 1))
        inner = x.abs() <= 3                  # away from binary64 saturation of the tails
        assert torch.all((t[inner] > 0) & (t[inner] < 1))
        assert torch.all(t[1:] >= t[:-1])
        assert abs(float(tmo.tau(torch.tensor(0.0, dtype=torch.float64), s, h)) - 0.5) < 1e-15
        for x0 in (s - 1.0, 1.0 - h):        # C1 joins
            xl = torch.tensor(x0 - 1e-9, dtype=torch.float64, requires_grad=True)
            xr = torch.tensor(x0 + 1e-9, dtype=torch.float64, requires_grad=True)
            tl, tr = tmo.tau(xl, s, h), tmo.tau(xr, s, h)
            assert abs(float(tl) - float(tr)) < 1e-8
            gl = torch.autograd.grad(tl, xl)[0]
            gr = torch.autograd.grad(tr, xr)[0]
            assert abs(float(gl) - 0.5) < 1e-8 and abs(float(gr) - 0.5) < 1e-8
        xg = x.clone().requires_grad_(True)
        g = torch.autograd.grad(tmo.tau(xg, s, h).sum(), xg)[0]
        assert torch.all(g > 0) and torch.all(g <= 0.5 + 1e-15)   # 0 < d tau / d log L <= 1/2
    # s, h -> 1: the curve approaches a logistic in x (Reinhard in log space): symmetric about 0
    t = tmo.tau(x, 0.999999, 0.999999)
    assert torch.allclose(t + torch.flip(t, [0]), torch.ones_like(t), atol=1e-5)


def test_srgb_known_values():
    v = torch.tensor([0.0, 0.0031308, 0.5, 1.0], dtype=torch.float64)
    out = tmo.srgb(v).numpy()
    ref = [0.0, 0.0031308 * 12.92, 1.055 * 0.5 ** (1 / 2.4) - 0.055, 1.0]
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-15)
    assert abs(out[2] - 0.7353569830524495) < 1e-12


def test_loss_reduces_to_l1_without_history():
    a = torch.rand(1, 4, 4, 3, dtype=torch.float64)
    b = torch.rand(1, 4, 4, 3, dtype=torch.float64)
    assert torch.allclose(tmo.frame_loss(a, b), (a - b).abs().mean())
    # identical history differences: only the spatial term remains when it dominates
    lt_zero = tmo.frame_loss(a, b, a, b)
    assert torch.allclose(lt_zero, torch.maximum(1.25 * torch.zeros_like(a), (a - b).abs()).mean())


# ---------------------------------------------------------------- gradient pins (FD)

def test_relaxed_scatter_gradient_fd():
    rng = np.random.default_rng(4)
    s0 = rng.uniform(0.05, 2.5, (1, 4, 5)).astype(np.float32)
    seed, frame, lam = 11, 0, 10.0
    r = sampling.mask(s0, seed, frame)
    smp = torch.tensor(rng.normal(size=(r["total"], 4)))
    u = r["u"].reshape(-1)
    s64 = s0.astype(np.float64).reshape(-1)
    p = s64 - np.floor(s64)
    # keep away from kinks: ramp ends (u = p, u = p - p/lambda) and integers
    ok = (np.abs(u - p) > 1e-3) & (np.abs(u - (p - p / lam)) > 1e-3) & (p > 1e-3) & (p < 1 - 1e-3)
    s = torch.tensor(s0.astype(np.float64), requires_grad=True)
    f = lambda s_: sampling.scatter(s_, r["count"], smp, seed, frame, "relaxed", lam)[..., :3].reshape(-1, 3)
    J = torch.autograd.functional.jacobian(f, s)          # [npx, 3, 1, 4, 5]
    eps = 1e-6
    for i in np.nonzero(ok)[0]:
        sp = s.detach().clone().reshape(-1)
        sm = sp.clone()
        sp[i] += eps
        sm[i] -= eps
        fd = (f(sp.reshape(s.shape)) - f(sm.reshape(s.shape)))[i] / (2 * eps)
        an = J.reshape(20, 3, 20)[i, :, i]
        assert torch.allclose(an, fd, rtol=1e-6, atol=1e-8)


def test_filter_gradients_fd():
    KD, KU, KT, levels = 3, 3, 3, 2
    g = torch.Generator().manual_seed(7)
    N, H, W = 1, 6, 6
    L = [torch.randn(N, H >> l, W >> l, 4, generator=g, dtype=torch.float64, requires_grad=True) for l in range(levels)]
    z = [torch.randn(N, H, W, 27, generator=g, dtype=torch.float64, requires_grad=True),
         torch.randn(N, H // 2, W // 2, 9, generator=g, dtype=torch.float64, requires_grad=True)]
    prev = torch.randn(N, H, W, 4, generator=g, dtype=torch.float64, requires_grad=True)
    mv = (torch.rand(N, H, W, 2, generator=g, dtype=torch.float64) * 3 - 1.5)
    mv = torch.where((mv - mv.round()).abs() < 0.05, mv + 0.1, mv)     # off the bilinear cell edges
    f = lambda L0, L1, z0, z1, pv: filt.denoise_pyramid([L0, L1], [z0, z1], KD, KU, KT, pv, mv)[0]
    assert torch.autograd.gradcheck(f, (L[0], L[1], z[0], z[1], prev), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_normalise_and_conv_gradients_fd():
    g = torch.Generator().manual_seed(8)
    z = torch.randn(2, 3, 4, generator=g, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: density.normalise(t, 0.25), (z,), eps=1e-6, atol=1e-8)
    x = torch.randn(1, 5, 4, 3, generator=g, dtype=torch.float64, requires_grad=True)
    w = torch.randn(2, 3, 3, 3, generator=g, dtype=torch.float64, requires_grad=True)
    b = torch.randn(2, generator=g, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(density.conv2d_nhwc, (x, w, b), eps=1e-6, atol=1e-8)


def _srgb_decode(I):
    """IEC 61966-2-1 decoding (the inverse of the encoding the tonemapper ends with)."""
    I = np.asarray(I, dtype=np.float64)
    return np.where(I <= 0.04045, I / 12.92, ((I + 0.055) / 1.055) ** 2.4)


def _radiance_with_logs(v):
    """A pixel whose channels have log(L + 1e-4) = v (the tonemapper's log with its epsilon)."""
    L = torch.zeros(1, 1, 1, 4, dtype=torch.float64)
    L[0, 0, 0, :3] = torch.tensor(np.exp(np.asarray(v, dtype=np.float64)) - 1e-4)
    return L


@pytest.mark.parametrize("case", [
    # log-RGB (1, 2, 3), mean 2; saturation 1.5 -> (0.5, 2, 3.5); exposure -2.25, contrast 0.2
    # -> x = 0.2 (sat + k) = (-0.35, -0.05, 0.25), all on the linear part for s = 0.4, h = 0.6
    # (toe below -0.6, shoulder from 0.4): tau = (1 + x) / 2 = (0.325, 0.475, 0.625).
    # Reading x = alpha sat + k would give (-2.15, -1.85, -1.55) (toe); saturating about the
    # linear mean (log 10.064 = 2.309) would move every channel.
    ((1.0, 2.0, 3.0), dict(k=-2.25, alpha=0.2, beta=1.5, s=0.4, h=0.6), (0.325, 0.475, 0.625)),
    # log-RGB (-1, -0.25, 0.125), saturation 1, exposure 0.25, contrast 2 -> x = (-1.5, 0, 0.75);
    # s = h = 0.5: toe 0.25 exp((x + 0.5) / 0.5) = 0.25 e^-2, line 0.5, shoulder
    # 1 - 0.25 exp(-(x - 0.5) / 0.5) = 1 - 0.25 e^-0.5
    ((-1.0, -0.25, 0.125), dict(k=0.25, alpha=2.0, beta=1.0, s=0.5, h=0.5),
     (0.033833820809153176, 0.5, 0.8483673350718416)),
    # saturation 0 collapses every channel onto the log-RGB mean (-0.5): x = 0.5 (-0.5 + 0.3)
    # = -0.1 on the line for s = h = 0.3 -> 0.45 in every channel
    ((-2.0, 0.0, 0.5), dict(k=0.3, alpha=0.5, beta=0.0, s=0.3, h=0.3), (0.45, 0.45, 0.45)),
])
def test_tonemap_hand_values(case):
    """The composition of Sec. 5, I = sRGB(tau(alpha (sat_beta(log L) + k))) with saturation
    about the per-pixel log-RGB mean, on hand-evaluated pixels; sRGB undone with the standard
    decoding, so the pin does not reuse the tonemapper's own encoding."""
    logs, prm, want_tau = case
    I = tmo.tonemap(_radiance_with_logs(logs), prm)[0, 0, 0].numpy()
    assert np.allclose(_srgb_decode(I), want_tau, rtol=0, atol=1e-12), (_srgb_decode(I), want_tau)


def test_tmo_loss_gradient_fd():
    g = torch.Generator().manual_seed(9)
    L = (torch.rand(1, 4, 4, 4, generator=g, dtype=torch.float64) * 3 + 0.05).requires_grad_(True)
    ref = torch.rand(1, 4, 4, 4, generator=g, dtype=torch.float64) * 3 + 0.05
    prm = dict(k=0.1, alpha=0.4, beta=1.1, s=0.4, h=0.6)
    f = lambda t: tmo.frame_loss(tmo.tonemap(t, prm), tmo.tonemap(ref, prm))
    assert torch.autograd.gradcheck(f, (L,), eps=1e-7, atol=1e-6)


def test_adamw_matches_torch_optimizer():
    from oracle import optim
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=50)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=1e-2, betas=(0.8, 0.985), eps=1e-8, weight_decay=0.02)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        g = rng.normal(size=50)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = optim.adamw_step(p, g, m, v, t, 1e-2)
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_feature_pins():
    from oracle import features as of
    v = torch.tensor([-3.0, -0.5, 0.0, 0.25, 10.0], dtype=torch.float64)
    assert torch.allclose(of.slog1p(v), torch.tensor(np.sign(v.numpy()) * np.log1p(np.abs(v.numpy()))))
    L = torch.rand(1, 3, 4, 4, dtype=torch.float64) * 5
    prm = dict(k=0.0, alpha=0.4, beta=1.0, s=0.5, h=0.5)
    assert torch.allclose(of.tonemap_eval(L[..., :3]), tmo.tonemap(L, prm), rtol=1e-14)
    aux = torch.rand(1, 3, 4, 8, dtype=torch.float64)
    L0 = torch.randn(1, 3, 4, 4, dtype=torch.float64)
    s = torch.rand(1, 3, 4, dtype=torch.float64)
    f = of.kernel_features(aux, L0, s)
    assert f.shape == (1, 3, 4, 16)
    assert torch.equal(f[..., :7], aux[..., :7]) and torch.equal(f[..., 10], s)
    assert torch.all(f[..., 11:] == 0)
    mv = torch.zeros(1, 3, 4, 2, dtype=torch.float64)
    mv[0, 0, 0] = torch.tensor([-0.6, 0.0])     # leaves the frame at the left edge
    f2 = of.kernel_features(aux, L0, s, L0, mv)
    assert f2[0, 0, 0, 14] == 0 and f2[0, 1, 1, 14] == 1
    assert torch.allclose(f2[0, 1, 1, 11:14], of.slog1p(L0[0, 1, 1, :3]))
