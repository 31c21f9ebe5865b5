"""End-to-end gradients of one frame (both networks) against the FP64 oracle, and a short
training run on procedural clips."""
import dataclasses
import os

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import features as ofeat
from oracle import filt as ofilt
from oracle import sampling as osamp
from oracle import tmo as otmo
from oracle import unet as ounet

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _small_cfg():
    from paper_2602_08642_amd import pipeline
    return dataclasses.replace(pipeline.CONFIGS["c4"], H=32, W=32, net_dtype=torch.float32,
                               logit_dtype=torch.float32, widths=(8, 16, 16, 16))


@pytest.mark.parametrize("demod,latents", [(False, 0), (True, 0), (True, 4)])
def test_frame_gradients_match_oracle(demod, latents):
    """With latents the frame takes the previous frame's latents (a leaf with a gradient) and its
    own latents enter the loss through a fixed random weighting, so the gradient reaches the
    latent head channels and both networks through the warped latent inputs."""
    from paper_2602_08642_amd import autograd as ag
    from paper_2602_08642_amd import ops, pipeline, train
    cfg = dataclasses.replace(_small_cfg(), demod=demod, latents=latents)
    N, H, W = 2, cfg.H, cfg.W
    dspec, kspec = pipeline.density_spec(cfg), pipeline.kernel_spec(cfg)
    dw = procgen.init_weights(dspec, 3)
    kw = procgen.init_weights(kspec, 4)
    cb = train.make_clips([500, 501], H, W, 2, DEV)
    gen = torch.Generator(device=DEV).manual_seed(0)
    dnet = train.TrainNet(dspec, dw, torch.float32, DEV)
    knet = train.TrainNet(kspec, kw, torch.float32, DEV)
    prev = cb.ref[0].clone()                       # a history frame (constant input)
    mv = cb.mv[1]
    pool = train.sample_pool(cb.ref[1], gen)
    seed, frame = 77, 1
    g = torch.Generator().manual_seed(9)
    lat_in = torch.randn(N, H, W, 4, generator=g)
    wlat = torch.randn(N, H, W, 4, generator=g) * 1e-3
    lat_d = lat_in.to(DEV).requires_grad_(True) if latents else None
    out, s, lat_out = train.frame_forward(dnet, knet, cfg, cb.aux[1], prev, mv, pool, seed, frame,
                                          "relaxed", lat=lat_d, want_latent=True)
    loss = ag.TMOLoss.apply(out, None, cb.ref[1], None, None, cb.params)
    if latents:
        loss = loss + (lat_out * wlat.to(DEV)).sum()
    loss.backward()

    # oracle: the same frame in FP64 with the GPU's s-derived mask and samples
    cap = int(N * H * W * (cfg.budget + 1)) + 1024
    req = ops.sample_mask(s.detach(), seed, frame, capacity=cap)
    total = int(req["total"].item())
    smp = ops.fixture_render(pool, req["count"], req["pixel_offset"], cap)[:total].cpu().numpy()
    tw = lambda wd: {k: (torch.tensor(w, dtype=torch.float64, requires_grad=True),
                         torch.tensor(b, dtype=torch.float64, requires_grad=True)) for k, (w, b) in wd.items()}
    dwt, kwt = tw(dw), tw(kw)
    aux = cb.aux[1].double().cpu()
    p64, m64 = prev.double().cpu(), mv.double().cpu()
    l64 = lat_in.double().requires_grad_(True) if latents else None
    fs = ofeat.sampler_features(aux, p64, m64, cfg.sampler_cin, lat=l64)
    z = odens.cnn_forward(fs, [(dwt[l["name"]][0], dwt[l["name"]][1], l["relu"]) for l in dspec])[..., 0]
    s64 = odens.normalise(z, cfg.budget)
    assert np.allclose(s64.detach().numpy(), s.detach().cpu().numpy(), rtol=1e-4)
    L0 = osamp.scatter(s64, req["count"].cpu().numpy(), smp, seed, frame, "relaxed", 10.0)
    Ls = osamp.pyramid(L0, cfg.levels)
    fk = ofeat.kernel_features(aux, L0, s64, p64, m64, cfg.kernel_cin, lat=l64)
    logits = ounet.unet_forward(fk, kwt, cfg.levels)
    if demod:   # learned demodulation: the filter sees L0 / d, its output is multiplied by d
        from oracle import demod as odemod
        k0 = cfg.filter_channels()[0]
        zd = logits[0][..., k0:k0 + 3]
        o64 = odemod.remodulate(ofilt.denoise_pyramid(odemod.demodulate(L0, zd, cfg.levels), logits,
                                                      cfg.KD, cfg.KU, cfg.KT, p64, m64)[0], zd)
    else:
        o64 = ofilt.denoise_pyramid(Ls, logits, cfg.KD, cfg.KU, cfg.KT, p64, m64)[0]
    ltot = 0
    for n in range(N):
        prm = dict(zip(["k", "alpha", "beta", "s", "h"], cb.params[n].double().cpu().tolist()))
        ltot = ltot + otmo.frame_loss(otmo.tonemap(o64[n:n + 1], prm),
                                      otmo.tonemap(cb.ref[1][n:n + 1].double().cpu(), prm)) / N
    if latents:
        k1 = cfg.filter_channels()[0] + 3
        ltot = ltot + (logits[0][..., k1:k1 + 4] * wlat.double()).sum()
    ltot.backward()
    assert abs(float(loss.item()) - float(ltot)) < 1e-4 * abs(float(ltot))
    if latents:
        ref_g = l64.grad
        rel = float((lat_d.grad.double().cpu() - ref_g).norm() / ref_g.norm())
        assert rel < 2e-3, ("latent input gradient", rel)
    worst = 0.0
    for net, ref in ((knet, kwt), (dnet, dwt)):
        for name, lr in net.layers.items():
            wscale = float(ref[name][0].grad.norm())
            for g, r in ((lr.w.grad, ref[name][0].grad), (lr.b.grad, ref[name][1].grad)):
                gn, rn = g.double().cpu(), r
                # floor: a gradient that vanishes exactly is compared on its layer's scale
                rel = float((gn - rn).norm() / max(float(rn.norm()), 1e-3 * wscale, 1e-30))
                worst = max(worst, rel)
                assert rel < 2e-3, (name, rel)
    # the budget softmax is shift invariant: the sampler's output bias gets no gradient
    assert float(dwt["d2"][1].grad.abs().max()) < 1e-10
    assert float(dnet.layers["d2"].b.grad.abs().max()) < 1e-4 * float(dwt["d2"][0].grad.norm())
    print(f"worst normwise parameter-gradient error {worst:.2e}")


def test_training_reduces_loss():
    from paper_2602_08642_amd import pipeline, train
    cfg = dataclasses.replace(pipeline.CONFIGS["c4"], H=64, W=64)
    tc = train.TrainConfig(steps=40, batch=2, frames=3, lr=2e-3, n_train_clips=4, log_every=100)
    _, _, hist = train.train(cfg, tc, DEV, log=lambda *a: None)
    first = np.mean([h["loss"] for h in hist[:8]])
    last = np.mean([h["loss"] for h in hist[-8:]])
    assert all(np.isfinite(h["loss"]) for h in hist)
    assert last < first, (first, last)


@pytest.mark.parametrize("estimator", ["straight_through", "gumbel", "dasr"])
def test_training_steps_with_each_estimator(estimator):
    """Two training steps with each compared estimator of the sampling step run through and give
    finite losses and gradients (their kernels are checked against the oracle elsewhere)."""
    from paper_2602_08642_amd import pipeline, train
    cfg = dataclasses.replace(pipeline.CONFIGS["c4"], H=32, W=32)
    dnet, knet, hist = train.train(cfg, train.TrainConfig(steps=2, batch=2, frames=2, n_train_clips=2,
                                                          estimator=estimator, log_every=1),
                                   DEV, log=lambda m: None)
    assert all(np.isfinite(h["loss"]) for h in hist)
    ev = train.evaluate(cfg, dnet, knet, [10000], 2, DEV, mode="dasr" if estimator == "dasr" else "hard")
    assert np.isfinite(ev["psnr"])


def test_training_steps_with_demodulation_and_latents():
    """Training through learned demodulation and the recurrent latents: the latents of frame t feed
    frame t+1 inside the two-frame window and the run gives finite losses; the evaluation then
    carries them across its frames."""
    from paper_2602_08642_amd import pipeline, train
    cfg = dataclasses.replace(pipeline.CONFIGS["c4"], H=32, W=32, demod=True, latents=4)
    dnet, knet, hist = train.train(cfg, train.TrainConfig(steps=3, batch=2, frames=3, n_train_clips=2,
                                                          log_every=1), DEV, log=lambda m: None)
    assert all(np.isfinite(h["loss"]) for h in hist)
    for name, lr in knet.layers.items():
        assert torch.isfinite(lr.w).all(), name
    ev = train.evaluate(cfg, dnet, knet, [10000], 3, DEV)
    assert np.isfinite(ev["psnr"])


def test_checkpoint_resume_continues_the_run():
    """Trainer.save / load keep the masters, the AdamW moments, the step count and the sample
    generator: the loaded state equals the saved one bit for bit, and the resumed run's next step
    has the uninterrupted run's budget and loss (up to the float atomics of the warp transposes,
    whose summation order is not fixed)."""
    import tempfile

    from paper_2602_08642_amd import pipeline, train
    cfg = dataclasses.replace(pipeline.CONFIGS["c4"], H=64, W=64)
    tc = train.TrainConfig(steps=4, batch=2, frames=2, n_train_clips=2, log_every=100)
    a = train.Trainer(cfg, tc, DEV)
    a.step()
    a.step()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ckpt.npz")
        a.save(path)
        saved = a.state_dict()
        ra = a.step()
        b = train.Trainer(cfg, tc, DEV)
        b.load(path)
        loaded = b.state_dict()
        assert sorted(loaded) == sorted(saved)
        for k in saved:
            assert np.array_equal(loaded[k], saved[k]), k
        rb = b.step()
    assert rb["step"] == ra["step"] == 3 and rb["budget"] == ra["budget"]
    assert abs(rb["loss"] - ra["loss"]) <= 1e-4 * abs(ra["loss"])
