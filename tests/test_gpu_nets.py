"""Network parity: the kernel-predictor U-Net and the sampler CNN through their C ABI entry
points against the FP64 oracle, and the fused conv + 1x1 head against separate launches."""
import math

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import unet as ounet
from tests import _nets
from tests._tol import assert_mag_close

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


E2E = {torch.bfloat16: (2e-2, 6e-2), torch.float32: (1e-5, 1e-4)}
LAYER_TOL = {torch.bfloat16: 2e-2, torch.float32: 1e-5}


def _wq(w, dtype):
    return {k: (torch.tensor(a).to(dtype).double(), torch.tensor(b).double()) for k, (a, b) in w.items()}


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("heads", [[43, 34, 25], [67, 58, 58, 49]])
def test_unet_matches_oracle(ops, dtype, heads):
    """Stage-wise and end to end (tests/_nets.py), and the fused entry point against the chain
    of single-layer calls: bit for bit in bf16, to float32 rounding in fp32 (the fused heads sum
    the 1x1 product in another order)."""
    spec = procgen.unet_spec(16, heads)
    w = procgen.init_weights(spec, 11)
    net = ops.Net(spec, w, dtype, DEV)
    g = torch.Generator().manual_seed(1)
    x = torch.randn(2, 48, 64, 16, generator=g)
    x[..., 15] = 0
    xd = x.to(DEV).to(dtype)
    logits = ops.kernel_predict(net, xd, heads, dtype)
    rec, chain = _nets.unet_chain(ops, net, xd, heads, dtype)
    what = f"unet {str(dtype)[6:]} {heads}"
    for l, K in enumerate(heads):
        if dtype == torch.bfloat16:
            assert torch.equal(logits[l][..., :K], chain[l][..., :K]), l
        else:
            c = chain[l][..., :K].cpu()
            assert_mag_close(logits[l][..., :K].cpu(), c, c.abs() + float(c.abs().mean()), 1e-6,
                             what=f"{what} fused vs chain head {l}")
    wq = _wq(w, dtype)
    _nets.check_layers(rec, wq, {l["name"]: l["relu"] for l in spec}, LAYER_TOL[dtype], what)
    ref = ounet.unet_forward(x.to(dtype).double(), wq, len(heads))
    _nets.check_end_to_end([t.cpu() for t in logits], ref, heads, *E2E[dtype], what=what)


@pytest.mark.parametrize("cin", [64, 32])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("cout,K", [(32, 34), (32, 43), (64, 34), (64, 58), (32, 67), (64, 67), (32, 80)])
def test_fused_head_bit_identical(ops, dtype, cout, K, cin):
    """aps_conv2d_fwd_head: logits equal the separate 1x1 head on the stored layer output, and the
    main output equals the plain layer, bit for bit (bf16 with 32 inputs and outputs: the row
    sweep with its head, four and five head m-tiles, 72 columns = two bands and a ragged one)."""
    from paper_2602_08642_amd import _lib as L
    g = torch.Generator().manual_seed(cout * 100 + K + cin)
    N, H, W = 1, 40, 72
    x = torch.randn(N, H, W, cin, generator=g).to(DEV).to(dtype)
    sa = dict(name="a", cin=cin, cout=cout, k=3, relu=True)
    sh = dict(name="h", cin=cout, cout=K, k=1, relu=False)
    wa = (torch.randn(cout, 3, 3, cin, generator=g) / math.sqrt(9 * cin)).numpy()
    wh = (torch.randn(K, 1, 1, cout, generator=g) / math.sqrt(cout)).numpy()
    net = ops.Net([sa, sh], {"a": (wa, np.random.default_rng(0).normal(size=cout).astype(np.float32) * 0.1),
                             "h": (wh, np.random.default_rng(1).normal(size=K).astype(np.float32) * 0.1)},
                  dtype, DEV)
    _, pa, ba = net.layer("a")
    _, ph, bh = net.layer("h")
    ks = ops.round_kstride(K, dtype)
    y = ops.conv2d(x, sa, pa, ba)
    ref = ops.conv2d(y, sh, ph, bh, ldy=ks)
    fused = torch.full((N, H, W, ks), 7.0, dtype=dtype, device=DEV)
    ymain = torch.empty_like(y)
    dt = L.APS_F32 if dtype == torch.float32 else L.APS_BF16
    L.check(L.load().aps_conv2d_fwd_head(ops._p(x), None, N, H, W, cin, 0, L.APS_CONV_DIRECT, ops._p(pa),
                                         ops._p(ba), cout, 1, ops._p(ph), ops._p(bh), K, dt,
                                         ops._p(ymain), cout, ops._p(fused), ks, ops._stream()), "fused")
    assert torch.equal(fused[..., :K], ref[..., :K])
    assert torch.equal(ymain, y)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
@pytest.mark.parametrize("relu", [True, False])
@pytest.mark.parametrize("cin,cout", [(16, 32), (32, 32), (32, 64), (64, 64)])
@pytest.mark.parametrize("N,H,W", [(1, 1, 5), (2, 23, 37), (1, 67, 131), (3, 40, 72), (1, 130, 66)])
def test_row_sweep_conv(ops, cin, cout, relu, N, H, W, dtype):
    """The 3x3 layers with 16 or 32 inputs and 32 or 64 outputs (the row-sweep kernels; 64 -> 64
    runs the tiled kernel on both sides, a control): against the FP64 oracle convolution of the
    same inputs (2e-2 of the layer magnitude in bf16, 1e-5 in fp32, as every layer), and bit for
    bit against the tiled kernel, whose main output the fused-head entry point writes (same taps,
    same order).  The shapes cut bands of 32 columns and segments of rows raggedly, include a
    one-row image, and for even sizes also the pooled copy."""
    from paper_2602_08642_amd import _lib as L
    g = torch.Generator().manual_seed(N * 1000 + H * W + cin + cout + relu)
    K = 34
    x = torch.randn(N, H, W, cin, generator=g).to(DEV).to(dtype)
    sa = dict(name="a", cin=cin, cout=cout, k=3, relu=relu)
    sh = dict(name="h", cin=cout, cout=K, k=1, relu=False)
    wa = torch.randn(cout, 3, 3, cin, generator=g) / math.sqrt(9 * cin)
    ba = torch.randn(cout, generator=g) * 0.1
    wh = (torch.randn(K, 1, 1, cout, generator=g) / math.sqrt(cout)).numpy()
    net = ops.Net([sa, sh], {"a": (wa.numpy(), ba.numpy()),
                             "h": (wh, np.zeros(K, np.float32))}, dtype, DEV)
    _, pa, bb = net.layer("a")
    _, ph, bh = net.layer("h")
    y = ops.conv2d(x, sa, pa, bb)
    wq = wa.to(dtype).double()
    ref = odens.conv2d_nhwc(x.double().cpu(), wq, ba.double())
    mag = odens.conv2d_nhwc(x.double().cpu().abs(), wq.abs(), ba.double().abs())
    if relu:
        ref = torch.relu(ref)
    tol = 2e-2 if dtype == torch.bfloat16 else 1e-5
    assert_mag_close(y.double().cpu(), ref, mag, tol, what=f"row sweep {dtype} {cin} {N}x{H}x{W}")
    ks = ops.round_kstride(K, dtype)
    dt = L.APS_BF16 if dtype == torch.bfloat16 else L.APS_F32
    ymain = torch.empty_like(y)
    logits = torch.empty((N, H, W, ks), dtype=dtype, device=DEV)
    L.check(L.load().aps_conv2d_fwd_head(ops._p(x), None, N, H, W, cin, 0, L.APS_CONV_DIRECT, ops._p(pa),
                                         ops._p(bb), cout, int(relu), ops._p(ph), ops._p(bh), K, dt,
                                         ops._p(ymain), cout, ops._p(logits), ks, ops._stream()), "head")
    assert torch.equal(ymain, y)
    if H % 2 == 0 and W % 2 == 0:
        y2 = torch.empty_like(y)
        pooled = torch.full((N, H // 2, W // 2, cout), 3.0, dtype=dtype, device=DEV)
        L.check(L.load().aps_conv2d_fwd_pool(ops._p(x), None, N, H, W, cin, 0, L.APS_CONV_DIRECT,
                                             ops._p(pa), ops._p(bb), cout, int(relu), dt,
                                             ops._p(y2), ops._p(pooled), ops._stream()), "fwd_pool")
        assert torch.equal(y2, y)
        q = y.float().cpu()
        exp = ((q[:, 0::2, 0::2] + q[:, 0::2, 1::2]) + (q[:, 1::2, 0::2] + q[:, 1::2, 1::2])) * 0.25
        assert torch.equal(pooled.cpu(), exp.to(dtype))


@pytest.mark.parametrize("cin", [8, 16])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_sampler_cnn_matches_oracle(ops, cin, dtype):
    spec = procgen.density_cnn_spec(cin)
    w = procgen.init_weights(spec, 5)
    net = ops.Net(spec, w, dtype, DEV)
    g = torch.Generator().manual_seed(2 + cin)
    x = torch.rand(2, 40, 56, cin, generator=g)
    xd = x.to(DEV).to(dtype)
    z, s = ops.density_predict(net, xd, 0.25)
    rec, _ = _nets.sampler_chain(ops, net, xd)
    wq = _wq(w, dtype)
    what = f"sampler {cin} {str(dtype)[6:]}"
    _nets.check_layers(rec, wq, {l["name"]: l["relu"] for l in spec}, LAYER_TOL[dtype], what)
    layers = [(wq[l["name"]][0], wq[l["name"]][1], l["relu"]) for l in spec]
    zr = odens.cnn_forward(x.to(dtype).double(), layers)[..., 0]
    _nets.check_end_to_end([z.cpu()], [zr], [0], *E2E[dtype], what=what)
    sr = odens.normalise(z.double().cpu(), 0.25)
    assert_mag_close(s.cpu(), sr, sr, 1e-5, what="normalisation")


@pytest.mark.parametrize("cin", [8, 16])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("H,W", [(40, 56), (23, 37), (1, 5), (16, 52), (67, 131)])
def test_fused_sampler_equals_layer_by_layer(ops, cin, dtype, H, W):
    """The one-kernel sampler CNN gives the layer-by-layer result, including ragged bands and
    one-row images.  Both round the intermediates to the storage type, but they sum K in other
    orders (bf16: per kernel row in the row sweep, runs of four (tap, group) pairs in the tiled
    layers; fp32: the 16 -> 1 layer on the vector ALU), so an intermediate may round one ulp
    apart: bf16 within 2^-6 of the output scale, fp32 within 1e-5."""
    spec = procgen.density_cnn_spec(cin)
    w = procgen.init_weights(spec, 9)
    net = ops.Net(spec, w, dtype, DEV)
    g = torch.Generator().manual_seed(H * W + cin)
    x = (torch.rand(3, H, W, cin, generator=g) * 2 - 0.5).to(DEV).to(dtype)
    z, _ = ops.density_predict(net, x, 0.25)
    h = x
    for l in spec[:2]:
        ls, pk, b = net.layer(l["name"])
        h = ops.conv2d(h, ls, pk, b)
    ls, pk, b = net.layer(spec[2]["name"])
    zr = ops.conv2d(h, ls, pk, b, out_dtype=torch.float32)[..., 0]
    tol = 2.0 ** -6 if dtype == torch.bfloat16 else 1e-5
    scale = float(zr.abs().max())
    assert torch.allclose(z, zr, rtol=tol, atol=tol * scale), float((z - zr).abs().max()) / scale


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
@pytest.mark.parametrize("cin,cout,H,W", [(32, 32, 40, 72), (64, 64, 24, 48), (128, 128, 16, 32),
                                          (32, 64, 8, 16)])
def test_pooled_output_equals_pool2_transform(ops, cin, cout, H, W, dtype):
    """aps_conv2d_fwd_pool: y equals the plain conv, pooled equals the 2x2 mean of y taken in
    the POOL2 transform's order, and the next layer reading pooled equals the POOL2 route,
    all bit for bit."""
    from paper_2602_08642_amd import _lib as L
    g = torch.Generator().manual_seed(cin + cout + H)
    N = 2
    x = torch.randn(N, H, W, cin, generator=g).to(DEV).to(dtype)
    sa = dict(name="a", cin=cin, cout=cout, k=3, relu=True)
    wa = (torch.randn(cout, 3, 3, cin, generator=g) / math.sqrt(9 * cin)).numpy()
    ba = (torch.randn(cout, generator=g) * 0.1).numpy()
    net = ops.Net([sa], {"a": (wa, ba)}, dtype, DEV)
    _, pa, bb = net.layer("a")
    ref = ops.conv2d(x, sa, pa, bb)
    y = torch.empty_like(ref)
    pooled = torch.full((N, H // 2, W // 2, cout), 3.0, dtype=dtype, device=DEV)
    L.check(L.load().aps_conv2d_fwd_pool(ops._p(x), None, N, H, W, cin, 0, L.APS_CONV_DIRECT,
                                         ops._p(pa), ops._p(bb), cout, 1,
                                         L.APS_BF16 if dtype == torch.bfloat16 else L.APS_F32, ops._p(y),
                                         ops._p(pooled), ops._stream()), "fwd_pool")
    assert torch.equal(y, ref)
    q = ref.float().cpu()
    exp = ((q[:, 0::2, 0::2] + q[:, 0::2, 1::2]) + (q[:, 1::2, 0::2] + q[:, 1::2, 1::2])) * 0.25
    assert torch.equal(pooled.cpu(), exp.to(dtype))
    # and the next layer reading it directly equals the POOL2 route
    sb = dict(name="b", cin=cout, cout=cout, k=3, relu=True)
    wb = (torch.randn(cout, 3, 3, cout, generator=g) / math.sqrt(9 * cout)).numpy()
    net2 = ops.Net([sb], {"b": (wb, np.zeros(cout, np.float32))}, dtype, DEV)
    _, pb, b2 = net2.layer("b")
    assert torch.equal(ops.conv2d(pooled, sb, pb, b2), ops.conv2d(y, sb, pb, b2, mode="pool2"))


@pytest.mark.parametrize("N,H,W", [(1, 64, 96), (2, 40, 56), (1, 24, 8)])
def test_kernel_predict_equals_layer_chain(ops, N, H, W):
    """kernel_predict (pooled copies written by the producing layers, heads 0 and 1 fused into
    the last 3x3 conv of their level) gives the logits of the plain layer-by-layer chain of
    aps_conv2d_fwd calls (pool2 / up2cat input transforms, separate 1x1 heads) bit for bit."""
    heads = [43, 34, 25]
    spec = procgen.unet_spec(16, heads)
    w = procgen.init_weights(spec, 31)
    net = ops.Net(spec, w, torch.bfloat16, DEV)
    g = torch.Generator().manual_seed(H + W)
    x = torch.randn(N, H, W, 16, generator=g).to(DEV).to(torch.bfloat16)
    logits = ops.kernel_predict(net, x, heads, torch.bfloat16)

    def conv(name, inp, mode="direct", x2=None, ldy=None):
        ls, pk, b = net.layer(name)
        return ops.conv2d(inp, ls, pk, b, mode=mode, x2=x2, ldy=ldy)
    e0 = conv("enc0b", conv("enc0a", x))
    e1 = conv("enc1b", conv("enc1a", e0, "pool2"))
    e2 = conv("enc2b", conv("enc2a", e1, "pool2"))
    e3 = conv("botb", conv("bota", e2, "pool2"))
    d2 = conv("dec2b", conv("dec2a", e3, "up2cat", e2))
    d1 = conv("dec1b", conv("dec1a", d2, "up2cat", e1))
    d0 = conv("dec0b", conv("dec0a", d1, "up2cat", e0))
    for l, (f, K) in enumerate(zip([d0, d1, d2], heads)):
        ref = conv(f"head{l}", f, ldy=ops.round_kstride(K, torch.bfloat16))
        assert torch.equal(logits[l][..., :K], ref[..., :K]), l


@pytest.mark.parametrize("dtype,odt,tol", [(torch.bfloat16, torch.bfloat16, 2e-2),
                                           (torch.bfloat16, torch.float32, 1e-2),
                                           (torch.float32, torch.float32, 1e-5)])
@pytest.mark.parametrize("cin,cout,mode", [(32, 25, "direct"), (256, 64, "direct"), (40, 34, "direct"),
                                           (256, 29, "pool2"), (128, 61, "pool2"), (32, 67, "direct"),
                                           (64, 80, "pool2")])
def test_conv1x1_matches_oracle(ops, dtype, odt, tol, cin, cout, mode):
    """The 1x1 (logit head) convolution against the FP64 oracle: a pixel count that fills no
    whole wave (2 x 7 x 9), input channels that end inside a 32-channel chunk (40), up to 256
    channels, the 2x2-pool input transform, and outputs into a padded row stride."""
    from oracle import density as odens
    from oracle import unet as ounet
    g = torch.Generator().manual_seed(cin * 7 + cout)
    N, H, W = 2, 7, 9
    xin = torch.randn(N, 2 * H if mode == "pool2" else H, 2 * W if mode == "pool2" else W, cin, generator=g)
    w = torch.randn(cout, 1, 1, cin, generator=g) / math.sqrt(cin)
    b = torch.randn(cout, generator=g) * 0.1
    sp = dict(name="h", cin=cin, cout=cout, k=1, relu=False)
    net = ops.Net([sp], {"h": (w.numpy(), b.numpy())}, dtype, DEV)
    _, pk, bb = net.layer("h")
    ld = ops.round_kstride(cout, odt)
    y = ops.conv2d(xin.to(DEV).to(dtype), sp, pk, bb, mode=mode, out_dtype=odt, ldy=ld)
    assert y.shape == (N, H, W, ld)
    x64 = xin.to(dtype).double()
    if mode == "pool2":   # the kernel rounds the pooled input to the storage type
        x64 = ounet.avgpool2(x64).to(dtype).double()
    w64 = w.to(dtype).double()
    ref = odens.conv2d_nhwc(x64, w64, b.double())
    mag = odens.conv2d_nhwc(x64.abs(), w64.abs(), b.double().abs())
    got = y[..., :cout].double().cpu()
    assert_mag_close(got, ref, mag, tol, what=f"1x1 {cin}->{cout} {mode}")
