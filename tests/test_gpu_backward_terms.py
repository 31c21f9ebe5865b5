"""Backward entry points of the standalone terms against the FP64 oracle's autograd:
aps_reproject_bwd (App. A eq. app-recon-full), aps_upsample_bwd (eq. app-upsample) and
aps_density_predict_bwd (Sec. 3, Overview: sampler network + budget normalisation).

Tolerances as in test_gpu_backward.py: elementwise |g - r| <= tol (|r| + rms(r)), tol 1e-4 for
float32 paths and 2e-2 where bf16 storage rounds operands or gradients.  The density chain is
checked stage-wise: the oracle's normalisation backward runs at the GPU's z, and both sides
take the ReLU decisions of the GPU's activations (a bf16 activation near zero may round to the
other side of the kink)."""
import math
import zlib

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import filt as ofilt
from tests.test_gpu_backward import assert_grad_close

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


def _seed(*a):
    return zlib.crc32(repr(a).encode())


def _logits(ops, N, H, W, K, ldt, g, scale=1.5):
    z = torch.randn(N, H, W, ops.round_kstride(K, ldt), generator=g) * scale
    z[..., K:] = 0
    return z.to(ldt)


def _tol(ldt, gdt):
    return 2e-2 if gdt == torch.bfloat16 else 1e-4


@pytest.mark.parametrize("cfg", [
    # N, H, W, KD, KU, KT, has_upsample, logit dtype, gradient dtype
    (1, 48, 64, 5, 3, 3, True, torch.float32, torch.float32),
    (2, 30, 44, 7, 3, 3, False, torch.float32, torch.float32),
    (1, 32, 48, 5, 2, 5, True, torch.bfloat16, torch.float32),
    (1, 40, 72, 7, 3, 3, True, torch.bfloat16, torch.bfloat16),
])
def test_reproject_backward(ops, cfg):
    N, H, W, KD, KU, KT, hu, ldt, gdt = cfg
    g = torch.Generator().manual_seed(_seed(cfg))
    sizes = [KD * KD] + ([KU * KU] if hu else []) + [KT * KT]
    K = sum(sizes)
    z0 = _logits(ops, N, H, W, K, ldt, g)
    prev = torch.randn(N, H, W, 4, generator=g)
    prev[..., 3] = 0
    mv = torch.rand(N, H, W, 2, generator=g) * 12 - 6
    gacc = torch.randn(N, H, W, 4, generator=g)
    gacc[..., 3] = 0
    glog, gprev = ops.reproject_bwd(prev.to(DEV), mv.to(DEV), z0.to(DEV), KD, KU, KT, hu,
                                    gacc.to(DEV), grad_dtype=gdt)
    z64 = z0.double().requires_grad_(True)
    p64 = prev.double().requires_grad_(True)
    w = ofilt.joint_softmax(z64, sizes)
    T = ofilt.gather(ofilt.warp(p64, mv.double()), w[-1], KT)
    (T * gacc.double()).sum().backward()
    tol = _tol(ldt, gdt)
    assert_grad_close(glog[..., :K], z64.grad[..., :K], tol, f"dlogits {cfg}")
    assert torch.all(glog[..., K:].float() == 0)
    assert_grad_close(gprev[..., :3], p64.grad[..., :3], 1e-4, f"dprev {cfg}")
    # grad_prev accumulates: a second call adds the same amount
    g2 = gprev.clone()
    from paper_2602_08642_amd import _lib
    lib = _lib.load()
    import ctypes as C
    nb = lib.aps_reproject_bwd_workspace_size(N, H, W, KD, KU, KT, int(hu))
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    zd, pd, md, gd = z0.to(DEV), prev.to(DEV), mv.to(DEV), gacc.to(DEV)
    gl2 = torch.empty_like(glog)
    P = lambda t: C.c_void_p(t.data_ptr())
    rc = lib.aps_reproject_bwd(P(pd), P(md), P(zd), ops._dt(ldt), zd.shape[-1], KD, KU, KT, int(hu),
                               N, H, W, P(gd), P(gl2), ops._dt(gdt), gl2.shape[-1], P(g2), P(ws), nb,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    assert torch.equal(gl2, glog)
    assert torch.allclose(g2, 2 * gprev, rtol=1e-6, atol=1e-6 * float(gprev.abs().max()))


@pytest.mark.parametrize("cfg", [
    # N, H, W, KD, KU, KT, has_temporal, logit dtype, gradient dtype
    (1, 48, 64, 5, 3, 3, True, torch.float32, torch.float32),
    (2, 26, 38, 5, 3, 3, False, torch.float32, torch.float32),
    (1, 32, 48, 5, 2, 5, True, torch.float32, torch.float32),
    (1, 34, 50, 7, 3, 3, False, torch.bfloat16, torch.bfloat16),
])
def test_upsample_backward(ops, cfg):
    N, H, W, KD, KU, KT, ht, ldt, gdt = cfg
    g = torch.Generator().manual_seed(_seed(cfg))
    sizes = [KD * KD, KU * KU] + ([KT * KT] if ht else [])
    K = sum(sizes)
    z = _logits(ops, N, H, W, K, ldt, g)
    coarse = torch.randn(N, H // 2, W // 2, 4, generator=g)
    coarse[..., 3] = 0
    gacc = torch.randn(N, H, W, 4, generator=g)
    gacc[..., 3] = 0
    glog, gc = ops.upsample_bwd(coarse.to(DEV), z.to(DEV), KD, KU, KT, ht, gacc.to(DEV),
                                grad_dtype=gdt)
    z64 = z.double().requires_grad_(True)
    c64 = coarse.double().requires_grad_(True)
    w = ofilt.joint_softmax(z64, sizes)
    U = ofilt.upsample(c64, w[1], KU, H, W)
    (U * gacc.double()).sum().backward()
    tol = _tol(ldt, gdt)
    assert_grad_close(glog[..., :K], z64.grad[..., :K], tol, f"dlogits {cfg}")
    assert torch.all(glog[..., K:].float() == 0)
    assert_grad_close(gc[..., :3], c64.grad[..., :3], 1e-4, f"dcoarse {cfg}")
    assert torch.all(gc[..., 3] == 0)


def test_term_backwards_are_zero_sum_in_the_logits(ops):
    """The joint softmax is shift invariant: each pixel's logit gradient sums to zero."""
    N, H, W = 1, 24, 32
    g = torch.Generator().manual_seed(3)
    z = _logits(ops, N, H, W, 43, torch.float32, g)
    prev = torch.randn(N, H, W, 4, generator=g)
    mv = torch.rand(N, H, W, 2, generator=g) * 4 - 2
    gacc = torch.randn(N, H, W, 4, generator=g)
    gl, _ = ops.reproject_bwd(prev.to(DEV), mv.to(DEV), z.to(DEV), 5, 3, 3, True, gacc.to(DEV))
    s = gl[..., :43].double().sum(-1)
    assert float(s.abs().max()) < 1e-5 * float(gl.abs().max())


@pytest.mark.parametrize("cfg", [
    # N, H, W, C, dtype, budget
    (1, 40, 56, 8, torch.float32, 0.25),
    (2, 36, 52, 16, torch.float32, 0.5),
    (1, 48, 64, 16, torch.bfloat16, 0.25),
])
def test_density_predict_backward(ops, cfg):
    N, H, W, C, dt, B = cfg
    spec = procgen.density_cnn_spec(C)
    wts = procgen.init_weights(spec, _seed(cfg) % 1000)
    net = ops.Net(spec, wts, dt, DEV)
    g = torch.Generator().manual_seed(_seed(cfg))
    feat = torch.rand(N, H, W, C, generator=g).to(DEV).to(dt)
    gs = torch.randn(N, H, W, generator=g)
    grads, gfeat = ops.density_predict_bwd(net, feat, B, gs.to(DEV))
    # the GPU's activations of the same layers (the entry point recomputes exactly these)
    acts = [feat]
    for i, l in enumerate(spec):
        sp, pk, b = net.layer(l["name"])
        last = i == len(spec) - 1
        acts.append(ops.conv2d(acts[-1], sp, pk, b, out_dtype=torch.float32 if last else None,
                               ldy=1 if last else None))
    zg = acts[-1].view(N, H, W)
    # oracle, stage-wise: the normalisation backward at the GPU's z ...
    z64 = zg.double().cpu().requires_grad_(True)
    (odens.normalise(z64, B) * gs.double()).sum().backward()
    gz = z64.grad
    # ... and the conv chain with the GPU's ReLU decisions
    x = feat.double().cpu().requires_grad_(True)
    h = x
    wb = []
    for i, l in enumerate(spec):
        w64 = torch.tensor(wts[l["name"]][0]).to(dt).double().requires_grad_(True)
        b64 = torch.tensor(wts[l["name"]][1], dtype=torch.float64).requires_grad_(True)
        wb.append((w64, b64))
        h = odens.conv2d_nhwc(h, w64, b64)
        if l["relu"]:
            h = h * (acts[i + 1].double().cpu() > 0)
    (h[..., 0] * gz).sum().backward()
    tol = 1e-4 if dt == torch.float32 else 2e-2
    for i, l in enumerate(spec):
        dw, db = grads[l["name"]]
        w64, b64 = wb[i]
        assert_grad_close(dw, w64.grad, tol, f"dw {l['name']} {cfg}")
        if i < len(spec) - 1:
            assert_grad_close(db, b64.grad, tol, f"db {l['name']} {cfg}")
        else:
            # softmax shift invariance: the output bias has an exactly zero gradient
            assert float(b64.grad.abs().max()) < 1e-9 * float(w64.grad.norm())
            assert float(db.abs().max()) <= 1e-3 * float(w64.grad.norm())
    assert_grad_close(gfeat, x.grad, tol, f"dfeat {cfg}")
