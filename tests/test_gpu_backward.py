"""Backward parity of the hand-written HIP gradients against the FP64 oracle's gradients
(torch autograd of the oracle's forward definitions, themselves pinned by finite differences
in test_oracle_*.py).

Gradient tolerance: a gradient entry is a sum of many products; its binary32 evaluation is
accurate relative to the sum of their magnitudes, which the entry's own size can understate
when terms cancel.  Elementwise |g - r| <= tol * (|r| + rms(r)) with tol 1e-4 for float32
paths and 2e-2 where bf16 storage rounds the operands.
"""
import math
import zlib

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import features as ofeat
from oracle import filt as ofilt
from oracle import optim as oopt
from oracle import sampling as osamp
from oracle import tmo as otmo
from oracle import unet as ounet

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


def _np(t):
    return t.detach().float().cpu().double().numpy()


def assert_grad_close(g, r, tol, what=""):
    g, r = _np(g), np.asarray(r.detach().cpu().numpy() if torch.is_tensor(r) else r, dtype=np.float64)
    rms = float(np.sqrt(np.mean(r * r))) + 1e-30
    err = np.abs(g - r)
    bound = tol * (np.abs(r) + rms)
    bad = err > bound
    if bad.any():
        i = np.argmax(err / bound)
        raise AssertionError(f"{what}: {bad.sum()}/{bad.size} exceed; worst err {err.flat[i]:.3e} "
                             f"ref {r.flat[i]:.3e} rms {rms:.3e}; normwise "
                             f"{np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300):.2e}")


def _seed(*a):
    return zlib.crc32(repr(a).encode())


# ------------------------------------------------------------------ filter backward

@pytest.mark.parametrize("cfg", [
    (1, 32, 48, 3, 5, 3, 3, True, torch.float32),
    (2, 24, 40, 2, 5, 3, 3, False, torch.float32),
    (1, 32, 32, 4, 7, 3, 3, True, torch.float32),
    (1, 32, 48, 4, 7, 3, 3, True, torch.bfloat16),
    (1, 16, 24, 2, 5, 2, 5, True, torch.float32),
    (1, 24, 32, 3, 3, 3, 3, True, torch.bfloat16),
])
def test_denoise_pyramid_backward(ops, cfg):
    N, H, W, levels, KD, KU, KT, temporal, ldt = cfg
    g = torch.Generator().manual_seed(_seed(cfg))
    Ks = procgen.kernel_channels(levels, KD, KU, KT, temporal)
    Ls = [torch.randn(N, H >> l, W >> l, 4, generator=g) for l in range(levels)]
    for t in Ls:
        t[..., 3] = 0
    logits = []
    for l in range(levels):
        z = torch.randn(N, H >> l, W >> l, ops.round_kstride(Ks[l], ldt), generator=g) * 1.5
        z[..., Ks[l]:] = 0
        logits.append(z.to(ldt))
    prev = mv = None
    if temporal:
        prev = torch.randn(N, H, W, 4, generator=g)
        prev[..., 3] = 0
        mv = torch.rand(N, H, W, 2, generator=g) * 10 - 5
    gout = torch.randn(N, H, W, 4, generator=g)
    gout[..., 3] = 0
    d = lambda t: None if t is None else t.to(DEV)
    glog, gL, gprev = ops.denoise_pyramid_bwd([d(t) for t in Ls], [d(t) for t in logits], KD, KU, KT,
                                              d(prev), d(mv), d(gout), grad_dtype=torch.float32)
    L64 = [t.double().requires_grad_(True) for t in Ls]
    z64 = [t.double().requires_grad_(True) for t in logits]
    p64 = prev.double().requires_grad_(True) if temporal else None
    out = ofilt.denoise_pyramid(L64, z64, KD, KU, KT, p64, mv.double() if temporal else None)[0]
    (out * gout.double()).sum().backward()
    for l in range(levels):
        assert_grad_close(glog[l][..., :Ks[l]], z64[l].grad[..., :Ks[l]], 1e-4, f"dlogits[{l}]")
        assert torch.all(glog[l][..., Ks[l]:] == 0)
        assert_grad_close(gL[l][..., :3], L64[l].grad[..., :3], 1e-4, f"dL[{l}]")
    if temporal:
        assert_grad_close(gprev[..., :3], p64.grad[..., :3], 1e-4, "dprev")


# ------------------------------------------------------------------ scatter / normalisation

@pytest.mark.parametrize("mode", ["hard", "relaxed"])
def test_scatter_backward(ops, mode):
    N, H, W, levels, seed, frame = 2, 16, 24, 3, 21, 3
    rng = np.random.default_rng(5)
    z = rng.normal(size=(N, H, W)) * 2
    s = odens.normalise(torch.tensor(z), 0.5).numpy().astype(np.float32)
    st = torch.tensor(s, device=DEV)
    r = ops.sample_mask(st, seed, frame)
    total = int(r["total"].item())
    smp = torch.tensor(rng.normal(size=(r["capacity"], 4)).astype(np.float32), device=DEV)
    gL = [torch.tensor(rng.normal(size=(N, H >> l, W >> l, 4)).astype(np.float32), device=DEV)
          for l in range(levels)]
    gs = ops.scatter_samples_bwd(st, r["count"], r["pixel_offset"], smp, gL, mode, 10.0, seed, frame)
    s64 = torch.tensor(s.astype(np.float64), requires_grad=True)
    L0 = osamp.scatter(s64, r["count"].cpu().numpy(), smp[:total].cpu().numpy(), seed, frame, mode, 10.0)
    pyr = osamp.pyramid(L0, levels)
    sum(((p * torch.tensor(_np(g))).sum()) for p, g in zip(pyr, gL)).backward()
    assert_grad_close(gs, s64.grad, 1e-4, mode)
    # accumulate mode adds
    gs2 = ops.scatter_samples_bwd(st, r["count"], r["pixel_offset"], smp, gL, mode, 10.0, seed,
                                  frame, grad_s=gs.clone())
    assert torch.allclose(gs2, 2 * gs)


def test_normalize_backward(ops):
    rng = np.random.default_rng(6)
    z = (rng.normal(size=(2, 20, 30)) * 2).astype(np.float32)
    g = rng.normal(size=z.shape).astype(np.float32)
    gz = ops.normalize_density_bwd(torch.tensor(z, device=DEV), 0.25, torch.tensor(g, device=DEV))
    z64 = torch.tensor(z.astype(np.float64), requires_grad=True)
    (odens.normalise(z64, 0.25) * torch.tensor(g.astype(np.float64))).sum().backward()
    assert_grad_close(gz, z64.grad, 1e-4)


@pytest.mark.parametrize("kind", ["sampler", "kernel"])
def test_features_backward(ops, kind):
    rng = np.random.default_rng(7)
    N, H, W = 1, 12, 20
    aux = torch.tensor(rng.random((N, H, W, 8)).astype(np.float32))
    L0 = torch.tensor(rng.normal(size=(N, H, W, 4)).astype(np.float32) * 3)
    L0[..., 3] = 0
    s = torch.tensor(rng.random((N, H, W)).astype(np.float32) + 0.1)
    prev = torch.tensor(rng.random((N, H, W, 4)).astype(np.float32) * 4)
    prev[..., 3] = 0
    mv = torch.tensor((rng.random((N, H, W, 2)) * 6 - 3).astype(np.float32))
    C = 16
    f = ops.assemble_features(kind, aux.to(DEV), L0.to(DEV), s.to(DEV), prev.to(DEV), mv.to(DEV), C)
    gf = torch.tensor(rng.normal(size=(N, H, W, C)).astype(np.float32))
    gL0 = torch.zeros(N, H, W, 4, device=DEV)
    gs = torch.zeros(N, H, W, device=DEV)
    gp = torch.zeros(N, H, W, 4, device=DEV)
    ops.assemble_features_bwd(kind, gf.to(DEV), L0.to(DEV), prev.to(DEV), mv.to(DEV), gL0, gs, gp)
    L64 = L0.double().requires_grad_(True)
    s64 = s.double().requires_grad_(True)
    p64 = prev.double().requires_grad_(True)
    if kind == "sampler":
        ref = ofeat.sampler_features(aux.double(), p64, mv.double(), C)
    else:
        ref = ofeat.kernel_features(aux.double(), L64, s64, p64, mv.double(), C)
    assert np.allclose(_np(f), ref.detach().numpy(), rtol=1e-5, atol=1e-6)
    (ref * gf.double()).sum().backward()
    if kind == "kernel":
        assert_grad_close(gL0[..., :3], L64.grad[..., :3], 1e-4, "dL0")
        assert_grad_close(gs, s64.grad, 1e-4, "ds")
    assert_grad_close(gp[..., :3], p64.grad[..., :3], 1e-4, "dprev")


# ------------------------------------------------------------------ convolutions

@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("cfg", [
    ("direct", 1, 20, 36, 16, 0, 32, 3, True),
    ("direct", 2, 16, 24, 32, 0, 34, 1, False),
    ("pool2", 1, 12, 20, 32, 0, 64, 3, True),
    ("up2cat", 1, 16, 24, 64, 32, 32, 3, True),
    ("direct", 1, 18, 30, 16, 0, 1, 3, False),
    ("pool2", 1, 4, 6, 32, 0, 25, 1, False),          # the five-level pyramid's coarsest head
])
def test_conv_backward(ops, cfg, dtype):
    mode, N, H, W, Cx, C2, Cout, k, relu = cfg
    g = torch.Generator().manual_seed(_seed(cfg))
    if mode == "pool2":
        x = torch.randn(N, 2 * H, 2 * W, Cx, generator=g)
    elif mode == "up2cat":
        x = torch.randn(N, H // 2, W // 2, Cx, generator=g)
    else:
        x = torch.randn(N, H, W, Cx, generator=g)
    x2 = torch.randn(N, H, W, C2, generator=g) if C2 else None
    cin = Cx + C2
    w = torch.randn(Cout, k, k, cin, generator=g) / math.sqrt(k * k * cin)
    b = torch.randn(Cout, generator=g) * 0.1
    spec = dict(name="l", cin=cin, cout=Cout, k=k, relu=relu)
    net = ops.Net([spec], {"l": (w.numpy(), b.numpy())}, dtype=dtype, device=DEV)
    _, pk, bias = net.layer("l")
    pkT = ops.pack_dgrad(spec, net.master["l"][0], dtype)
    xd = x.to(DEV).to(dtype)
    x2d = x2.to(DEV).to(dtype) if x2 is not None else None
    ldy = Cout if relu else (Cout + 7) // 8 * 8
    y = ops.conv2d(xd, spec, pk, bias, mode, x2d, ldy=ldy)
    gy = torch.randn(N, H, W, ldy, generator=g)
    gy[..., Cout:] = 0
    dx, dx2, dw, db = ops.conv2d_bwd(xd, x2d, mode, spec, pkT, gy.to(DEV).to(dtype), y if relu else None)
    # oracle on the values the GPU saw (bf16-rounded operands widened exactly)
    x64 = xd.double().cpu().requires_grad_(True)
    x264 = x2d.double().cpu().requires_grad_(True) if x2 is not None else None
    w64 = (net.master["l"][0].to(dtype).double().cpu()).requires_grad_(True)
    b64 = b.double().requires_grad_(True)
    if mode == "pool2":
        xin = ounet.avgpool2(x64)
    elif mode == "up2cat":
        xin = torch.cat([ounet.up2(x64), x264], -1)
    else:
        xin = x64
    yr = odens.conv2d_nhwc(xin, w64, b64)
    gyr = gy[..., :Cout].to(dtype).double()
    if relu:
        # the ReLU decision is taken on the GPU's forward output by both sides
        gyr = gyr * (y[..., :Cout].double().cpu() > 0)
    (yr * gyr).sum().backward()
    tol = 1e-4 if dtype == torch.float32 else 2e-2
    assert_grad_close(dx, x64.grad, tol, f"dx {cfg}")
    if x2 is not None:
        assert_grad_close(dx2, x264.grad, tol, f"dx2 {cfg}")
    assert_grad_close(dw, w64.grad, tol, f"dw {cfg}")
    assert_grad_close(db, b64.grad, tol, f"db {cfg}")


# ------------------------------------------------------------------ loss and optimiser

@pytest.mark.parametrize("temporal", [False, True])
def test_tmo_loss_and_gradients(ops, temporal):
    rng = np.random.default_rng(8)
    N, H, W = 2, 14, 18
    mk = lambda: torch.tensor(np.concatenate([rng.lognormal(0, 1, (N, H, W, 3)) - 0.1,
                                              np.zeros((N, H, W, 1))], -1).astype(np.float32))
    out, ref, pout, pref = mk(), mk(), mk(), mk()
    mv = torch.tensor((rng.random((N, H, W, 2)) * 8 - 4).astype(np.float32))
    params = torch.tensor(np.array([[0.2, 0.4, 1.1, 0.3, 0.7], [-0.3, 0.5, 0.9, 0.6, 0.2]], np.float32))
    d = lambda t: t.to(DEV)
    loss, gout, gprev = ops.tmo_loss(d(out), d(ref), d(params), d(pout) if temporal else None,
                                     d(pref) if temporal else None, d(mv) if temporal else None)
    o64 = out.double().requires_grad_(True)
    p64 = pout.double().requires_grad_(True)
    tot = 0.0
    for n in range(N):
        prm = dict(zip(["k", "alpha", "beta", "s", "h"], params[n].double().tolist()))
        I = otmo.tonemap(o64[n:n + 1], prm)
        Ir = otmo.tonemap(ref[n:n + 1].double(), prm)
        if temporal:
            Ip = ofilt.warp(otmo.tonemap(p64[n:n + 1], prm), mv[n:n + 1].double())
            Ipr = ofilt.warp(otmo.tonemap(pref[n:n + 1].double(), prm), mv[n:n + 1].double())
            valid = ofeat.valid_from_mv(mv[n:n + 1].double())
            tot = tot + otmo.frame_loss(I, Ir, Ip, Ipr, valid) / N
        else:
            tot = tot + otmo.frame_loss(I, Ir) / N
    tot.backward()
    assert abs(float(loss.item()) - float(tot)) <= 1e-5 * abs(float(tot))
    assert_grad_close(gout[..., :3], o64.grad[..., :3], 1e-4, "dout")
    if temporal:
        assert_grad_close(gprev[..., :3], p64.grad[..., :3], 1e-4, "dprev")


def test_adamw_step(ops):
    rng = np.random.default_rng(9)
    p = rng.normal(size=1000).astype(np.float32).astype(np.float64)
    m = np.zeros(1000)
    v = np.zeros(1000)
    pd = torch.tensor(p.astype(np.float32), device=DEV)
    md = torch.zeros(1000, device=DEV)
    vd = torch.zeros(1000, device=DEV)
    for t in range(1, 4):
        g = rng.normal(size=1000).astype(np.float32)
        ops.adamw_step(pd, md, vd, torch.tensor(g, device=DEV), 1e-3, t)
        p, m, v = oopt.adamw_step(p, g, m, v, t, 1e-3)
    assert np.allclose(_np(pd), p, rtol=1e-5, atol=1e-7)
    ss = ops.sumsq(pd)
    assert abs(float(ss.item()) - float((p ** 2).sum())) <= 1e-5 * float((p ** 2).sum())
