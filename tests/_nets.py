"""Network parity helpers: the U-Net and the sampler CNN as chains of single-layer library calls,
each layer checked against the FP64 oracle convolution on the inputs the GPU gave it.

Why stage-wise.  A whole-network magnitude (the network evaluated on absolute inputs and
parameters) bounds the error rigorously but grows by the layers' absolute gains (about 10^20
for the 14-layer U-Net with Kaiming-uniform weights), so an elementwise check against it says
nothing.  Instead (1) the fused entry point (aps_kernel_predict / aps_density_predict) is
compared bit for bit, or to a few float32 ulps where a fused kernel sums in another order,
with the chain of aps_conv2d_fwd calls; (2) every layer of that chain is compared element by
element with the oracle convolution of the GPU's own input of that layer, relative to that
layer's magnitude sum abs(w) abs(x) + abs(b) (tol 2e-2 in bf16, 1e-5 in float32, as the
single-layer tests); (3) the end-to-end outputs are compared with the whole FP64 oracle network
per head: normwise, and element by element relative to abs(r) + rms(r) of the head."""
import numpy as np
import torch

from oracle import density as odens
from oracle import unet as ounet
from tests._tol import assert_mag_close, to_np


def _layer(ops, net, name, inp, mode="direct", x2=None, out_dtype=None, ldy=None):
    ls, pk, b = net.layer(name)
    return ops.conv2d(inp, ls, pk, b, mode=mode, x2=x2, out_dtype=out_dtype, ldy=ldy)


def unet_chain(ops, net, x, heads, logit_dtype):
    """Layer-by-layer U-Net on the GPU. -> (records [(name, mode, x, x2, y)], logits)."""
    rec = []

    def conv(name, inp, mode="direct", x2=None, out_dtype=None, ldy=None):
        y = _layer(ops, net, name, inp, mode, x2, out_dtype, ldy)
        rec.append((name, mode, inp, x2, y))
        return y
    e0 = conv("enc0b", conv("enc0a", x))
    e1 = conv("enc1b", conv("enc1a", e0, "pool2"))
    e2 = conv("enc2b", conv("enc2a", e1, "pool2"))
    e3 = conv("botb", conv("bota", e2, "pool2"))
    d2 = conv("dec2b", conv("dec2a", e3, "up2cat", e2))
    d1 = conv("dec1b", conv("dec1a", d2, "up2cat", e1))
    d0 = conv("dec0b", conv("dec0a", d1, "up2cat", e0))
    feats = [(d0, "direct"), (d1, "direct"), (d2, "direct"), (e3, "direct"), (e3, "pool2")]
    logits = []
    for l, K in enumerate(heads):
        f, mode = feats[l]
        logits.append(conv(f"head{l}", f, mode, out_dtype=logit_dtype,
                           ldy=ops.round_kstride(K, logit_dtype)))
    return rec, logits


def sampler_chain(ops, net, x):
    rec = []
    h = x
    for i, name in enumerate(["d0", "d1", "d2"]):
        last = i == 2
        y = _layer(ops, net, name, h, out_dtype=torch.float32 if last else None, ldy=1 if last else None)
        rec.append((name, "direct", h, None, y))
        h = y
    return rec, h[..., 0]


def check_layers(records, wq, relu, tol, what):
    """Each layer against the oracle convolution of its GPU input, elementwise relative to the
    layer's magnitude; prints the worst ratio per layer."""
    worst = 0.0
    for name, mode, x, x2, y in records:
        w, b = wq[name]
        x64 = x.double().cpu()
        if mode == "pool2":
            x64 = ounet.avgpool2(x64)
        elif mode == "up2cat":
            x64 = torch.cat([ounet.up2(x64), x2.double().cpu()], -1)
        cout = w.shape[0]
        ref = odens.conv2d_nhwc(x64, w, b)
        if relu[name]:
            ref = torch.relu(ref)
        mag = odens.conv2d_nhwc(x64.abs(), w.abs(), b.abs())
        got = y[..., :cout].double().cpu()
        assert_mag_close(got, ref, mag, tol, what=f"{what} layer {name}")
        r = float((to_np(got - ref).__abs__() / (to_np(mag) + 1e-30)).max())
        worst = max(worst, r)
        print(f"LAYER {what} {name}: max|y-r|/mag {r:.3e}")
        del ref, mag, x64
    return worst


def check_end_to_end(outputs, refs, heads, tol_norm, tol_elem, what):
    """Per head: normwise relative error <= tol_norm and, element by element,
    abs(y - r) <= tol_elem (abs(r) + rms(r)); prints both figures."""
    res = []
    for l, K in enumerate(heads):
        y = to_np(outputs[l][..., :K]) if K else to_np(outputs[l])
        r = to_np(refs[l])
        rms = float(np.sqrt(np.mean(r * r)))
        ratio = float((np.abs(y - r) / (np.abs(r) + rms)).max())
        norm = float(np.linalg.norm(y - r) / max(np.linalg.norm(r), 1e-300))
        print(f"PRECISION {what} head{l} K={K}: normwise {norm:.3e}  max|y-r|/(|r|+rms) {ratio:.3e}")
        assert norm <= tol_norm, (what, l, norm)
        assert ratio <= tol_elem, (what, l, ratio)
        res.append((norm, ratio))
    return res
