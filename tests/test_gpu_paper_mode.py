"""The paper's own reconstruction (App. A: five levels, 5x5 kd at every level, the printed 2x2
ku, 5x5 kt and a 54-way softmax at level 0) with the quarter-resolution density map (Sec. 7),
stage by stage against the FP64 oracle on the inputs the GPU saw."""
import dataclasses

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import filt as ofilt
from oracle import sampling as osamp
from oracle import unet as ounet
from tests import _nets
from tests._tol import assert_mag_close, rel_norm
from tests.test_gpu_backward import assert_grad_close

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


def _bf16_feature_close(got, ref, what):
    """bf16 network inputs are the float32 evaluation (within 1e-5 relative + 1e-6 of the
    oracle, checked in float32 by the feature tests) rounded to nearest even, whose error is at
    most half an ulp, 2^-8 of the value at the bottom of its binade: the bound is
    (2^-8 + 1e-5) abs(r) + 1e-6.  Channel by channel worst cases are printed."""
    got, ref = got.double().cpu(), ref.double()
    err = (got - ref).abs()
    rel = 2.0 ** -8 + 1e-5
    bound = rel * ref.abs() + 1e-6
    for c in range(ref.shape[-1]):
        print(f"FEATURES {what} ch{c}: max err {float(err[..., c].max()):.3e}  max err/bound "
              f"{float((err[..., c] / bound[..., c]).max()):.3f}")
    assert_mag_close(got, ref, ref.abs() + 1e-6 / rel, rel, what=what)


def _q(w, dtype):
    return {k: (torch.tensor(a).to(dtype).double(), torch.tensor(b).double()) for k, (a, b) in w.items()}


E2E = {torch.bfloat16: (2e-2, 6e-2), torch.float32: (1e-5, 1e-4)}
LAYER_TOL = {torch.bfloat16: 2e-2, torch.float32: 1e-5}


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_five_head_unet_matches_oracle(ops, dtype):
    heads = procgen.kernel_channels(5, 5, 2, 5, True)
    spec = procgen.unet_spec(16, heads)
    w = procgen.init_weights(spec, 31)
    net = ops.Net(spec, w, dtype, DEV)
    x = torch.randn(2, 48, 64, 16, generator=torch.Generator().manual_seed(3))
    x[..., 15] = 0
    xd = x.to(DEV).to(dtype)
    logits = ops.kernel_predict(net, xd, heads, dtype)
    assert logits[4].shape[1:3] == (3, 4)
    rec, chain = _nets.unet_chain(ops, net, xd, heads, dtype)
    what = f"five-head unet {str(dtype)[6:]}"
    for l, K in enumerate(heads):
        c = chain[l][..., :K].cpu()
        if dtype == torch.bfloat16:
            assert torch.equal(logits[l][..., :K].cpu(), c), l
        else:
            assert_mag_close(logits[l][..., :K].cpu(), c, c.abs() + float(c.abs().mean()), 1e-6,
                             what=f"{what} fused vs chain head {l}")
    _nets.check_layers(rec, _q(w, dtype), {l["name"]: l["relu"] for l in spec}, LAYER_TOL[dtype], what)
    ref = ounet.unet_forward(x.to(dtype).double(), _q(w, dtype), 5)
    _nets.check_end_to_end([t.cpu() for t in logits], ref, heads, *E2E[dtype], what=what)


def test_five_heads_need_sixteen(ops):
    from paper_2602_08642_amd import _lib as L
    heads = procgen.kernel_channels(5, 5, 2, 5, True)
    spec = procgen.unet_spec(16, heads)
    net = ops.Net(spec, procgen.init_weights(spec, 1), torch.float32, DEV)
    x = torch.zeros(1, 40, 64, 16, device=DEV)          # 40 = 8 * 5: fine for 4 heads only
    with pytest.raises(L.ApsError):
        ops.kernel_predict(net, x, heads, torch.float32)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("shape", [(1, 2, 2, 4), (2, 14, 22, 16), (1, 64, 96, 8)])
def test_avgpool2_and_upsample_exact(ops, dtype, shape):
    g = torch.Generator().manual_seed(sum(shape))
    x = (torch.randn(*shape, generator=g) * 3).to(dtype)
    y = ops.avgpool2(x.to(DEV)).cpu()
    xf = x.float()
    exp = ((xf[:, 0::2, 0::2] + xf[:, 0::2, 1::2]) + (xf[:, 1::2, 0::2] + xf[:, 1::2, 1::2])) * 0.25
    assert torch.equal(y, exp.to(dtype))
    sq = torch.randn(shape[0], shape[1] // 2, shape[2] // 2, generator=g)
    s = ops.upsample_nearest2(sq.to(DEV)).cpu()
    assert torch.equal(s, sq.repeat_interleave(2, 1).repeat_interleave(2, 2))


def test_avgpool2_shape_errors(ops):
    from paper_2602_08642_amd import _lib as L
    lib = L.load()
    x = torch.zeros(1, 6, 8, 8, device=DEV)
    y = torch.zeros(1, 3, 4, 8, device=DEV)
    assert lib.aps_avgpool2(ops._p(x), 1, 5, 8, 8, L.APS_F32, ops._p(y), ops._stream()) == L.APS_ERR_SHAPE
    assert lib.aps_avgpool2(ops._p(x), 1, 6, 8, 6, L.APS_F32, ops._p(y), ops._stream()) == L.APS_ERR_SHAPE
    assert lib.aps_avgpool2(ops._p(x), 0, 6, 8, 8, L.APS_F32, None, ops._stream()) == L.APS_OK


@pytest.mark.parametrize("cin,dtype", [(16, torch.bfloat16), (8, torch.float32)])
def test_density_quarter_matches_oracle(ops, cin, dtype):
    spec = procgen.density_cnn_spec(cin)
    w = procgen.init_weights(spec, 32)
    net = ops.Net(spec, w, dtype, DEV)
    N, H, W, B = 2, 40, 72, 0.25
    x = torch.rand(N, H, W, cin, generator=torch.Generator().manual_seed(9)).to(dtype)
    xq = ops.avgpool2(x.to(DEV))
    zq, sq = ops.density_predict(net, xq, B)
    s = ops.upsample_nearest2(sq)
    rec, _ = _nets.sampler_chain(ops, net, xq)
    what = f"quarter density {str(dtype)[6:]}"
    _nets.check_layers(rec, _q(w, dtype), {l["name"]: l["relu"] for l in spec}, LAYER_TOL[dtype], what)
    layers = [(torch.tensor(w[l["name"]][0]).to(dtype).double(), torch.tensor(w[l["name"]][1], dtype=torch.float64),
               l["relu"]) for l in spec]
    zr, sr = odens.density_quarter(x.double(), layers, B)
    _nets.check_end_to_end([zq.cpu()], [zr], [0], *E2E[dtype], what=what)
    # normalisation and block replication on the GPU's logits
    s_exp = odens.normalise(zq.double().cpu(), B).repeat_interleave(2, 1).repeat_interleave(2, 2)
    assert_mag_close(s.cpu(), s_exp, s_exp, 1e-5, what="quarter normalisation")
    for n in range(N):
        assert abs(float(s[n].double().sum()) - H * W * B) < 1e-3
    assert rel_norm(s.cpu(), sr) < 10 * E2E[dtype][0]


@pytest.mark.parametrize("cfg", [
    (1, 64, 96, torch.bfloat16),
    (2, 32, 48, torch.float32),
])
def test_five_level_pyramid_matches_oracle(ops, cfg):
    from tests.test_gpu_stages import _rand_inputs
    N, H, W, ldt = cfg
    Ls, logits, prev, mv = _rand_inputs(N, H, W, 5, 5, 2, 5, True, 41, ldt)
    assert [t.shape[-1] for t in logits] == [56, 32, 32, 32, 32] if ldt == torch.bfloat16 else True
    out = ops.denoise_pyramid([t.to(DEV) for t in Ls], [t.to(DEV) for t in logits], 5, 2, 5,
                              prev.to(DEV), mv.to(DEV))
    L64 = [t.double() for t in Ls]
    z64 = [t.double() for t in logits]
    ref = ofilt.denoise_pyramid(L64, z64, 5, 2, 5, prev.double(), mv.double())[0]
    mag = ofilt.denoise_magnitude(L64, z64, 5, 2, 5, prev.double(), mv.double())[0]
    assert_mag_close(out[..., :3], ref[..., :3], mag[..., :3], 1e-5, what=str(cfg))
    assert torch.all(out[..., 3] == 0)


def test_five_level_pyramid_backward(ops):
    N, H, W, levels = 1, 32, 48, 5
    g = torch.Generator().manual_seed(43)
    Ks = procgen.kernel_channels(levels, 5, 2, 5, True)
    Ls = [torch.randn(N, H >> l, W >> l, 4, generator=g) for l in range(levels)]
    for t in Ls:
        t[..., 3] = 0
    logits = []
    for l in range(levels):
        z = torch.randn(N, H >> l, W >> l, ops.round_kstride(Ks[l], torch.float32), generator=g) * 1.5
        z[..., Ks[l]:] = 0
        logits.append(z)
    prev = torch.randn(N, H, W, 4, generator=g)
    prev[..., 3] = 0
    mv = torch.rand(N, H, W, 2, generator=g) * 10 - 5
    gout = torch.randn(N, H, W, 4, generator=g)
    gout[..., 3] = 0
    d = lambda t: t.to(DEV)
    glog, gL, gprev = ops.denoise_pyramid_bwd([d(t) for t in Ls], [d(t) for t in logits], 5, 2, 5,
                                              d(prev), d(mv), d(gout), grad_dtype=torch.float32)
    L64 = [t.double().requires_grad_(True) for t in Ls]
    z64 = [t.double().requires_grad_(True) for t in logits]
    p64 = prev.double().requires_grad_(True)
    out = ofilt.denoise_pyramid(L64, z64, 5, 2, 5, p64, mv.double())[0]
    (out * gout.double()).sum().backward()
    for l in range(levels):
        assert_grad_close(glog[l][..., :Ks[l]], z64[l].grad[..., :Ks[l]], 1e-4, f"dlogits[{l}]")
        assert_grad_close(gL[l][..., :3], L64[l].grad[..., :3], 1e-4, f"dL[{l}]")
    assert_grad_close(gprev[..., :3], p64.grad[..., :3], 1e-4, "dprev")


@pytest.mark.parametrize("mode", ["hard", "relaxed"])
def test_scatter_five_levels(ops, mode):
    from tests.test_gpu_stages import _scatter_case
    _scatter_case(ops, 1, 64, 96, 5, mode)


def test_paper_mode_frame(ops):
    """One temporal frame of the paper configuration (reduced to 64x96), random-init networks:
    quarter-resolution density, blue-noise mask, render stand-in, scatter into 5 levels,
    five-head U-Net, learned demodulation around the 5-level 5/2/5 pyramid with the warped
    previous output."""
    from paper_2602_08642_amd import pipeline
    cfg = dataclasses.replace(pipeline.CONFIGS["paper"], H=64, W=96)
    assert cfg.filter_channels() == [54, 29, 29, 29, 25]
    assert cfg.head_channels() == [61, 29, 29, 29, 25]          # + demodulation map (3) + latents (4)
    assert cfg.kernel_cin == 24 and cfg.sampler_cin == 16
    dspec, kspec = pipeline.density_spec(cfg), pipeline.kernel_spec(cfg)
    dw, kw = procgen.init_weights(dspec, 51), procgen.init_weights(kspec, 52)
    r = pipeline.FrameRenderer(cfg, dw, kw, device=DEV)
    seed, t = 77, 1
    clip = procgen.make_clip(seed, cfg.H, cfg.W, 3)
    fr = clip[t]
    aux = torch.tensor(fr.aux[None], device=DEV)
    prev = torch.zeros(1, cfg.H, cfg.W, 4)
    prev[..., :3] = torch.tensor(clip[0].truth)
    prev = prev.to(DEV)
    mv = torch.tensor(fr.mv[None], device=DEV)
    dt = cfg.net_dtype
    # density at a quarter of the pixels
    s = r.density(aux, prev, mv)
    feat = ops.assemble_features("sampler", aux, prev=prev, mv=mv, C_out=cfg.sampler_cin, dtype=dt)
    zq, sq = ops.density_predict(r.dnet, ops.avgpool2(feat), cfg.budget)
    assert torch.equal(s, ops.upsample_nearest2(sq))
    layers = [(torch.tensor(dw[l["name"]][0]).to(dt).double(), torch.tensor(dw[l["name"]][1], dtype=torch.float64),
               l["relu"]) for l in dspec]
    zr, _ = odens.density_quarter(feat.double().cpu(), layers, cfg.budget)
    _nets.check_end_to_end([zq.cpu()], [zr], [0], *E2E[dt], what="paper frame density")
    assert abs(float(s.double().sum()) - cfg.H * cfg.W * cfg.budget) < 1e-3
    # mask (bit-exact on the GPU's s) and the render stand-in
    req = r.request(s, seed, t)
    assert r.u_tex is not None                        # the paper configuration dithers with blue noise
    tex = r.u_tex.cpu().numpy()
    assert np.array_equal(tex, procgen.blue_noise_thresholds(64))
    mo = osamp.mask(s.cpu().numpy(), seed, t, u_tex=tex)
    assert np.array_equal(req["count"].cpu().numpy(), mo["count"])
    pool = torch.tensor(procgen.sample_pool(fr.truth, seed, t, 8), device=DEV)
    smp = ops.fixture_render(pool, req["count"], req["pixel_offset"], req["capacity"])
    out, Ls, logits = r.reconstruct(aux, s, req, smp, seed, t, prev, mv)
    total = int(req["total"].item())
    L0r = osamp.scatter(s.double().cpu(), mo["count"], smp[:total].cpu().numpy(), seed, t, u_tex=tex)
    for l, ref in enumerate(osamp.pyramid(L0r, cfg.levels)):
        assert torch.allclose(Ls[l].double().cpu(), ref, rtol=1e-5, atol=1e-5), l
    # five-head U-Net on the GPU's features
    kf = ops.assemble_features("kernel", aux, Ls[0], s, prev, mv, cfg.kernel_cin, dt)
    zref = ounet.unet_forward(kf.double().cpu(), _q(kw, dt), 5)
    for l, K in enumerate(cfg.head_channels()):
        assert logits[l].shape[1:3] == (cfg.H >> l, cfg.W >> l)
    _nets.check_end_to_end([t.cpu() for t in logits], zref, cfg.head_channels(), *E2E[dt],
                           what="paper frame unet")
    # learned demodulation around the 5-level pyramid, on the GPU's logits
    from oracle import demod as odemod
    z64 = [t.double().cpu() for t in logits]
    zd = z64[0][..., 54:57]
    Ld = odemod.demodulate(Ls[0].double().cpu(), zd, 5)
    Lda = odemod.demodulate(Ls[0].double().cpu().abs(), zd, 5)
    ref = odemod.remodulate(ofilt.denoise_pyramid(Ld, z64, 5, 2, 5, prev.double().cpu(), mv.double().cpu())[0], zd)
    mag = odemod.remodulate(ofilt.denoise_magnitude(Lda, z64, 5, 2, 5, prev.double().cpu(), mv.double().cpu())[0], zd)
    assert_mag_close(out[..., :3], ref[..., :3], mag[..., :3], 1e-5, what="paper frame")
    # the recurrent latents of this frame are the level-0 head's four channels after the map
    assert torch.equal(r.latent, logits[0][..., 57:61].float())
    # next frame: both networks see them warped along the new motion vectors
    from oracle import features as ofeat
    fr2 = clip[2]
    aux2 = torch.tensor(fr2.aux[None], device=DEV)
    mv2 = torch.tensor(fr2.mv[None], device=DEV)
    lat1 = r.latent.clone()
    fs = ops.assemble_features("sampler", aux2, prev=out, mv=mv2, C_out=16, dtype=dt, lat=r._lat(out))
    fs_ref = ofeat.sampler_features(aux2.double().cpu(), out.double().cpu(), mv2.double().cpu(), 16,
                                    lat=lat1.double().cpu())
    _bf16_feature_close(fs, fs_ref, "sampler features")
    s2 = r.density(aux2, out, mv2)
    zq2, sq2 = ops.density_predict(r.dnet, ops.avgpool2(fs), cfg.budget)
    assert torch.equal(s2, ops.upsample_nearest2(sq2))
    req2 = r.request(s2, seed, 2)
    smp2 = ops.fixture_render(torch.tensor(procgen.sample_pool(fr2.truth, seed, 2, 8), device=DEV),
                              req2["count"], req2["pixel_offset"], req2["capacity"])
    out2, Ls2, logits2 = r.reconstruct(aux2, s2, req2, smp2, seed, 2, out, mv2, history=r.history)
    kf2 = ops.assemble_features("kernel", aux2, Ls2[0], s2, out, mv2, 24, dt, lat=lat1)
    kf2_ref = ofeat.kernel_features(aux2.double().cpu(), Ls2[0].double().cpu(), s2.double().cpu(),
                                    out.double().cpu(), mv2.double().cpu(), 24, lat=lat1.double().cpu())
    _bf16_feature_close(kf2, kf2_ref, "kernel features")
    assert torch.isfinite(out2).all() and not torch.equal(r.latent, lat1)
