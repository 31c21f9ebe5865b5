"""Network layer specifications and seeded random-init weights (inputs only).

Weights are stored OHWI: w[cout, ky, kx, cin] (ky, kx in 0..k-1, tap offset = k - k//2),
bias[cout].  Kaiming-uniform init (bound sqrt(6 / fan_in)) scaled by a per-layer gain.
"""
from __future__ import annotations

import numpy as np


def kernel_channels(levels: int, KD: int, KU: int, KT: int, temporal: bool):
    """Logit channels per pyramid level: KD^2, + KU^2 below the coarsest, + KT^2 at level 0."""
    out = []
    for l in range(levels):
        k = KD * KD
        if l < levels - 1:
            k += KU * KU
        if l == 0 and temporal:
            k += KT * KT
        out.append(k)
    return out


def density_cnn_spec(cin: int = 8, width: int = 16):
    """Sampler CNN: three 3x3 convs, cin -> 16 -> 16 -> 1, ReLU between."""
    return [dict(name="d0", cin=cin, cout=width, k=3, relu=True, gain=1.0),
            dict(name="d1", cin=width, cout=width, k=3, relu=True, gain=1.0),
            dict(name="d2", cin=width, cout=1, k=3, relu=False, gain=0.5)]


def small_kernel_cnn_spec(cin: int = 16, width: int = 16, kout: int = 25):
    """Single-level kernel predictor: three 3x3 convs, cin -> 16 -> 16 -> kout logits."""
    return [dict(name="k0", cin=cin, cout=width, k=3, relu=True, gain=1.0),
            dict(name="k1", cin=width, cout=width, k=3, relu=True, gain=1.0),
            dict(name="k2", cin=width, cout=kout, k=3, relu=False, gain=0.3)]


def unet_spec(cin: int, head_channels, widths=(32, 64, 128, 256)):
    """4-level U-Net: two 3x3 conv+ReLU per level, 2x2 average-pool down, nearest-2x up and
    concat [upsampled, skip], 1x1 logit heads at decoder levels 0 .. len(head_channels)-1.
    The head of the bottom level (3) reads the bottleneck output; a fifth head (level 4, for
    the five-level pyramid) reads the 2x2 average pool of the bottleneck output."""
    c0, c1, c2, c3 = widths
    s = [
        dict(name="enc0a", cin=cin, cout=c0, k=3, relu=True, gain=1.0),
        dict(name="enc0b", cin=c0, cout=c0, k=3, relu=True, gain=1.0),
        dict(name="enc1a", cin=c0, cout=c1, k=3, relu=True, gain=1.0),
        dict(name="enc1b", cin=c1, cout=c1, k=3, relu=True, gain=1.0),
        dict(name="enc2a", cin=c1, cout=c2, k=3, relu=True, gain=1.0),
        dict(name="enc2b", cin=c2, cout=c2, k=3, relu=True, gain=1.0),
        dict(name="bota", cin=c2, cout=c3, k=3, relu=True, gain=1.0),
        dict(name="botb", cin=c3, cout=c3, k=3, relu=True, gain=1.0),
        dict(name="dec2a", cin=c3 + c2, cout=c2, k=3, relu=True, gain=1.0),
        dict(name="dec2b", cin=c2, cout=c2, k=3, relu=True, gain=1.0),
        dict(name="dec1a", cin=c2 + c1, cout=c1, k=3, relu=True, gain=1.0),
        dict(name="dec1b", cin=c1, cout=c1, k=3, relu=True, gain=1.0),
        dict(name="dec0a", cin=c1 + c0, cout=c0, k=3, relu=True, gain=1.0),
        dict(name="dec0b", cin=c0, cout=c0, k=3, relu=True, gain=1.0),
    ]
    feat_c = [c0, c1, c2, c3, c3]
    for l, K in enumerate(head_channels):
        s.append(dict(name=f"head{l}", cin=feat_c[l], cout=K, k=1, relu=False, gain=0.1))
    return s


def init_weights(spec, seed: int):
    """{name: (w[cout, k, k, cin] float32, b[cout] float32)} from a seeded generator."""
    rng = np.random.default_rng([int(seed), 0x3E1C47])
    out = {}
    for layer in spec:
        fan_in = layer["cin"] * layer["k"] * layer["k"]
        bound = layer["gain"] * np.sqrt(6.0 / fan_in)
        w = rng.uniform(-bound, bound, (layer["cout"], layer["k"], layer["k"], layer["cin"]))
        b = rng.uniform(-1.0, 1.0, layer["cout"]) * (0.1 * layer["gain"] / np.sqrt(fan_in))
        out[layer["name"]] = (w.astype(np.float32), b.astype(np.float32))
    return out
