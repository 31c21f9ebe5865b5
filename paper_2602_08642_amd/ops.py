"""Torch-tensor wrappers of the libaps C ABI.

Each function checks shapes and dtypes, allocates its outputs with torch (device memory
only), and calls the library on the current HIP stream.  All arithmetic of the path runs
in the library's kernels; nothing here computes on the data.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L

_BF16, _F32 = torch.bfloat16, torch.float32


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(torch_dtype):
    if torch_dtype == _F32:
        return L.APS_F32
    if torch_dtype == _BF16:
        return L.APS_BF16
    raise TypeError(f"unsupported dtype {torch_dtype}")


def _tdt(aps_dtype):
    return _F32 if aps_dtype == L.APS_F32 else _BF16


def _need(t, name, dtype=None, dev=True):
    if t is None:
        raise ValueError(f"{name} is required")
    if dev and not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t


class _Workspace:
    """Per-device scratch buffer that only grows (no allocation once warm)."""

    def __init__(self):
        self.buf = {}

    def get(self, nbytes: int, device):
        key = (device.index if device.index is not None else torch.cuda.current_device())
        b = self.buf.get(key)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
            self.buf[key] = b
        return b


WS = _Workspace()


def _status_tensor(device):
    return torch.zeros(1, dtype=torch.int32, device=device)


# ------------------------------------------------------------------ density (a1, a2)

def normalize_density(z, budget: float, uniform_frac: float = 1.0 / 8.0, status=None):
    _need(z, "z", _F32)
    N, H, W = z.shape
    s = torch.empty_like(z)
    lib = L.load()
    nb = lib.aps_normalize_workspace_size(N, H, W)
    ws = WS.get(nb, z.device)
    L.check(lib.aps_normalize_density(_p(z), N, H, W, budget, uniform_frac, _p(s), _p(ws), nb,
                                      _p(status), _stream()), "normalize_density")
    return s


# ------------------------------------------------------------------ mask (a3)

def _tex(u_tex):
    """(pointer, side) of an optional square float32 device texture of thresholds."""
    if u_tex is None:
        return None, 0
    _need(u_tex, "u_tex", _F32)
    if u_tex.dim() != 2 or u_tex.shape[0] != u_tex.shape[1]:
        raise ValueError("u_tex must be a square [T, T] float32 texture")
    return _p(u_tex), u_tex.shape[0]


_ROUNDING = {"stochastic": L.APS_ROUND_STOCHASTIC, "holdout": L.APS_ROUND_HOLDOUT,
             "deterministic": L.APS_ROUND_DETERMINISTIC}
_MODES = {"hard": L.APS_HARD, "relaxed": L.APS_RELAXED, "straight_through": L.APS_STRAIGHT_THROUGH,
          "gumbel": L.APS_GUMBEL, "dasr": L.APS_DASR}
# the mask rounding each scatter mode reads
MODE_ROUNDING = {"hard": "stochastic", "relaxed": "stochastic", "straight_through": "holdout",
                 "gumbel": "holdout", "dasr": "deterministic"}


def sample_mask(s, seed: int, frame: int, capacity: int | None = None, want_p=False, status=None,
                u_tex=None, rounding: str = "stochastic"):
    _need(s, "s", _F32)
    N, H, W = s.shape
    dev = s.device
    npix = N * H * W
    if capacity is None:
        capacity = npix * 2
    count = torch.empty((N, H, W), dtype=torch.uint8, device=dev)
    poff = torch.empty((N, H, W), dtype=torch.int32, device=dev)
    spix = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    total = torch.empty(1, dtype=torch.int32, device=dev)
    p = torch.empty_like(s) if want_p else None
    lib = L.load()
    nb = lib.aps_sample_mask_workspace_size(N, H, W)
    ws = WS.get(nb, dev)
    tp, T = _tex(u_tex)
    L.check(lib.aps_sample_mask_ex(_p(s), N, H, W, seed, frame, tp, T, _ROUNDING[rounding], _p(count),
                                   _p(poff), _p(spix), capacity, _p(total), _p(p), _p(ws), nb,
                                   _p(status), _stream()),
            "sample_mask")
    return dict(count=count, pixel_offset=poff, sample_pixel=spix, total=total, p=p,
                capacity=capacity)


def sample_mask_noalloc(s, seed: int, frame: int, capacity: int | None = None, want_p=False,
                        status=None, u_tex=None, rounding: str = "stochastic"):
    """sample_mask through the entry point that takes no workspace (the library's static
    scratch; at most 2^25 pixels)."""
    _need(s, "s", _F32)
    N, H, W = s.shape
    dev = s.device
    if capacity is None:
        capacity = N * H * W * 2
    count = torch.empty((N, H, W), dtype=torch.uint8, device=dev)
    poff = torch.empty((N, H, W), dtype=torch.int32, device=dev)
    spix = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    total = torch.empty(1, dtype=torch.int32, device=dev)
    p = torch.empty_like(s) if want_p else None
    tp, T = _tex(u_tex)
    L.check(L.load().aps_sample_mask_noalloc(_p(s), N, H, W, seed, frame, tp, T, _ROUNDING[rounding],
                                             _p(count), _p(poff), _p(spix), capacity, _p(total),
                                             _p(p), _p(status), _stream()),
            "sample_mask_noalloc")
    return dict(count=count, pixel_offset=poff, sample_pixel=spix, total=total, p=p,
                capacity=capacity)


def fixture_render(pool, count, pixel_offset, capacity: int):
    _need(pool, "pool", _F32)
    N, H, W = count.shape
    J = pool.shape[-2]
    out = torch.empty((max(capacity, 1), 4), dtype=_F32, device=pool.device)
    L.check(L.load().aps_fixture_render(_p(pool), J, _p(count), _p(pixel_offset), N, H, W,
                                        capacity, _p(out), _stream()), "fixture_render")
    return out


# ------------------------------------------------------------------ scatter (a4)

def scatter_samples(s, count, pixel_offset, samples, levels: int, mode: str = "hard",
                    lam: float = 10.0, seed: int = 0, frame: int = 0, u_tex=None, tau: float = 0.5):
    """mode: hard, relaxed (lam), straight_through, gumbel (tau) or dasr; the mask must have been
    drawn with MODE_ROUNDING[mode]."""
    _need(s, "s", _F32)
    _need(samples, "samples", _F32)
    N, H, W = s.shape
    Ls = [torch.empty((N, H >> l, W >> l, 4), dtype=_F32, device=s.device) for l in range(levels)]
    arr = (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in Ls])
    m = _MODES[mode]
    tp, T = _tex(u_tex)
    L.check(L.load().aps_scatter_samples_ex(_p(s), _p(count), _p(pixel_offset), _p(samples),
                                            samples.shape[0], N, H, W, levels, m,
                                            tau if mode == "gumbel" else lam, seed, frame,
                                            tp, T, arr, _stream()),
            "scatter_samples")
    return Ls


def assemble_features(kind: str, aux, L0=None, s=None, prev=None, mv=None, C_out: int = 16,
                      dtype=_F32, lat=None):
    """lat: the previous frame's recurrent latents [N,H,W,4] (warped and appended)."""
    _need(aux, "aux", _F32)
    if lat is not None:
        _need(lat, "lat", _F32)
    N, H, W, _ = aux.shape
    out = torch.empty((N, H, W, C_out), dtype=dtype, device=aux.device)
    k = L.APS_FEAT_SAMPLER if kind == "sampler" else L.APS_FEAT_KERNEL
    L.check(L.load().aps_assemble_features_ex(k, _p(aux), _p(L0), _p(s), _p(prev), _p(mv), _p(lat),
                                              N, H, W, C_out, _dt(dtype), _p(out), _stream()),
            "assemble_features")
    return out


# ------------------------------------------------------------------ networks (a1, a5)

class Net:
    """Device weights of a conv network: fp32 OHWI masters, packed copies and the layer table.

    spec: list of dicts (name, cin, cout, k, relu); weights: {name: (w[cout,k,k,cin], b[cout])}.
    """

    def __init__(self, spec, weights, dtype=_F32, device="cuda"):
        self.spec = [dict(l) for l in spec]
        self.dtype = dtype
        self.device = torch.device(device)
        self.master = {}
        for l in self.spec:
            w, b = weights[l["name"]]
            self.master[l["name"]] = (torch.as_tensor(w, dtype=_F32).to(self.device).contiguous(),
                                      torch.as_tensor(b, dtype=_F32).to(self.device).contiguous())
        self.packed = {}
        self.repack()

    def repack(self):
        lib = L.load()
        desc = L.NetDesc()
        desc.n_layers = len(self.spec)
        desc.dtype = _dt(self.dtype)
        for i, l in enumerate(self.spec):
            w, b = self.master[l["name"]]
            n = lib.aps_conv_packed_elems(l["cout"], l["k"], l["cin"])
            pk = self.packed.get(l["name"])
            if pk is None or pk.numel() != n:
                pk = torch.empty(n, dtype=self.dtype, device=self.device)
                self.packed[l["name"]] = pk
            L.check(lib.aps_conv_pack_weights(_p(w), l["cout"], l["k"], l["cin"], desc.dtype, _p(pk),
                                              _stream()), "pack_weights")
            desc.layer[i] = L.ConvLayer(pk.data_ptr(), b.data_ptr(), l["cin"], l["cout"], l["k"],
                                        int(l["relu"]))
        self.desc = desc

    def layer(self, name):
        i = [l["name"] for l in self.spec].index(name)
        return self.spec[i], self.packed[name], self.master[name][1]


def conv2d(x, layer_spec, packed, bias, mode: str = "direct", x2=None, out_dtype=None,
           ldy: int | None = None, out=None):
    """One conv layer through aps_conv2d_fwd (mode: direct | pool2 | up2cat)."""
    _need(x, "x")
    N = x.shape[0]
    if mode == "direct":
        H, W, Cx = x.shape[1], x.shape[2], x.shape[3]
        m, C2 = L.APS_CONV_DIRECT, 0
    elif mode == "pool2":
        H, W, Cx = x.shape[1] // 2, x.shape[2] // 2, x.shape[3]
        m, C2 = L.APS_CONV_POOL2, 0
    elif mode == "up2cat":
        _need(x2, "x2", x.dtype)
        H, W, Cx, C2 = x2.shape[1], x2.shape[2], x.shape[3], x2.shape[3]
        m = L.APS_CONV_UP2_CAT
    else:
        raise ValueError(mode)
    out_dtype = out_dtype or x.dtype
    cout = layer_spec["cout"]
    ldy = ldy or cout
    if out is None:
        out = torch.empty((N, H, W, ldy), dtype=out_dtype, device=x.device)
    L.check(L.load().aps_conv2d_fwd(_p(x), _p(x2), N, H, W, Cx, C2, m, _p(packed), _p(bias), cout,
                                    layer_spec["k"], int(layer_spec["relu"]), _dt(x.dtype), _p(out),
                                    ldy, _dt(out_dtype), _stream()), "conv2d")
    return out


def density_predict(net: Net, feat, budget: float, uniform_frac: float = 1.0 / 8.0, status=None):
    _need(feat, "feat", net.dtype)
    N, H, W, Cf = feat.shape
    z = torch.empty((N, H, W), dtype=_F32, device=feat.device)
    s = torch.empty((N, H, W), dtype=_F32, device=feat.device)
    lib = L.load()
    width = max(l["cout"] for l in net.spec[:2])
    nb = lib.aps_density_predict_workspace_size(N, H, W, width, _dt(net.dtype))
    ws = WS.get(nb, feat.device)
    L.check(lib.aps_density_predict(C.byref(net.desc), _p(feat), N, H, W, Cf, budget, uniform_frac,
                                    _p(z), _p(s), _p(ws), nb, _p(status), _stream()),
            "density_predict")
    return z, s


def avgpool2(x):
    """[N,H,W,C] -> [N,H/2,W/2,C] 2x2 block means (quarter-resolution sampler input)."""
    _need(x, "x")
    N, H, W, Cx = x.shape
    y = torch.empty((N, H // 2, W // 2, Cx), dtype=x.dtype, device=x.device)
    L.check(L.load().aps_avgpool2(_p(x), N, H, W, Cx, _dt(x.dtype), _p(y), _stream()), "avgpool2")
    return y


def upsample_nearest2(s_q):
    """[N,Hq,Wq] float32 -> [N,2Hq,2Wq]: every pixel takes its 2x2 block's value."""
    _need(s_q, "s_q", _F32)
    N, Hq, Wq = s_q.shape
    s = torch.empty((N, 2 * Hq, 2 * Wq), dtype=_F32, device=s_q.device)
    L.check(L.load().aps_upsample_nearest2(_p(s_q), N, Hq, Wq, _p(s), _stream()), "upsample_nearest2")
    return s


def demodulate(L0, z0, z_offset: int, levels: int):
    """Learned demodulation: pyramid of L0 / exp(z), z = z0[..., z_offset:z_offset+3]."""
    _need(L0, "L0", _F32)
    _need(z0, "z0")
    N, H, W, _ = L0.shape
    Ld = [torch.empty((N, H >> l, W >> l, 4), dtype=_F32, device=L0.device) for l in range(levels)]
    arr = (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in Ld])
    L.check(L.load().aps_demodulate(_p(L0), _p(z0), _dt(z0.dtype), z0.shape[-1], z_offset, N, H, W,
                                    levels, arr, _stream()), "demodulate")
    return Ld


def remodulate(x, z0, z_offset: int, out=None, lat_offset: int = -1, lat_out=None):
    """out = x * exp(z); with lat_out, also copies z0[..., lat_offset:lat_offset+4] (latents)."""
    _need(x, "x", _F32)
    _need(z0, "z0")
    N, H, W, _ = x.shape
    out = torch.empty_like(x) if out is None else out
    if lat_out is not None:
        _need(lat_out, "lat_out", _F32)
    L.check(L.load().aps_remodulate(_p(x), _p(z0), _dt(z0.dtype), z0.shape[-1], z_offset, lat_offset,
                                    N, H, W, _p(out), _p(lat_out), _stream()), "remodulate")
    return out


def demodulate_bwd(L0, z0, z_offset: int, grad_Ld, grad_L0=None, grad_z=None):
    """-> (grad_L0 [N,H,W,4], grad_z [N,H,W,3]); given buffers are accumulated into."""
    _need(L0, "L0", _F32)
    N, H, W, _ = L0.shape
    acc = grad_L0 is not None
    if acc != (grad_z is not None):
        raise ValueError("pass both gradient buffers to accumulate, or neither")
    grad_L0 = torch.empty_like(L0) if grad_L0 is None else grad_L0
    grad_z = torch.empty((N, H, W, 3), dtype=_F32, device=L0.device) if grad_z is None else grad_z
    arr = (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in grad_Ld])
    L.check(L.load().aps_demodulate_bwd(_p(L0), _p(z0), _dt(z0.dtype), z0.shape[-1], z_offset, N, H, W,
                                        len(grad_Ld), arr, _p(grad_L0), _p(grad_z), int(acc), _stream()),
            "demodulate_bwd")
    return grad_L0, grad_z


def remodulate_bwd(x, z0, z_offset: int, grad_out, grad_in=None, grad_z=None):
    _need(x, "x", _F32)
    N, H, W, _ = x.shape
    acc = grad_in is not None
    if acc != (grad_z is not None):
        raise ValueError("pass both gradient buffers to accumulate, or neither")
    grad_in = torch.empty_like(x) if grad_in is None else grad_in
    grad_z = torch.empty((N, H, W, 3), dtype=_F32, device=x.device) if grad_z is None else grad_z
    L.check(L.load().aps_remodulate_bwd(_p(x), _p(z0), _dt(z0.dtype), z0.shape[-1], z_offset, N, H, W,
                                        _p(grad_out), _p(grad_in), _p(grad_z), int(acc), _stream()),
            "remodulate_bwd")
    return grad_in, grad_z


def round_kstride(K: int, dtype) -> int:
    v = 8 if dtype == _BF16 else 4
    return (K + v - 1) // v * v


def kernel_predict(net: Net, feat, head_channels, logit_dtype=_F32, side_offset=None):
    """-> logits (list per level); with side_offset, (logits, side): side [N,H,W,4] holds
    logits[0][..., side_offset:side_offset+3] and a 0 (the compact demodulation map, written
    by the fused level-0 head)."""
    _need(feat, "feat", net.dtype)
    N, H, W, Cf = feat.shape
    n = len(head_channels)
    ks = [round_kstride(k, logit_dtype) for k in head_channels]
    logits = [torch.empty((N, H >> l, W >> l, ks[l]), dtype=logit_dtype, device=feat.device)
              for l in range(n)]
    lib = L.load()
    nb = lib.aps_kernel_predict_workspace_size(C.byref(net.desc), N, H, W)
    ws = WS.get(nb, feat.device)
    arr = (C.c_void_p * 5)(*[t.data_ptr() for t in logits])
    karr = (C.c_int * 5)(*ks)
    if side_offset is None:
        L.check(lib.aps_kernel_predict(C.byref(net.desc), _p(feat), N, H, W, Cf, n, arr,
                                       _dt(logit_dtype), karr, _p(ws), nb, _stream()), "kernel_predict")
        return logits
    side = torch.empty((N, H, W, 4), dtype=logit_dtype, device=feat.device)
    L.check(lib.aps_kernel_predict_ex(C.byref(net.desc), _p(feat), N, H, W, Cf, n, arr,
                                      _dt(logit_dtype), karr, _p(side), int(side_offset), _p(ws), nb,
                                      _stream()), "kernel_predict")
    return logits, side


# ------------------------------------------------------------------ reconstruction (a6-a9)

def denoise_pyramid(Ls, logits, KD: int, KU: int, KT: int, prev=None, mv=None, demod_offset: int = -1,
                    lat_offset: int = -1, out_demod=None, lat_out=None):
    """With demod_offset >= 0 (Ls demodulated): out is remodulated in the level-0 kernel, the
    reconstruction before it goes to out_demod, and with lat_out the latents are copied."""
    levels = len(Ls)
    L0 = _need(Ls[0], "L0", _F32)
    N, H, W, _ = L0.shape
    ldt = logits[0].dtype
    for t in logits:
        _need(t, "logits", ldt)
    out = torch.empty_like(L0)
    lib = L.load()
    nb = lib.aps_denoise_pyramid_workspace_size(N, H, W, levels)
    ws = WS.get(nb, L0.device)
    la = (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in Ls])
    za = (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in logits])
    ka = (C.c_int * L.APS_MAX_LEVELS)(*[t.shape[-1] for t in logits])
    L.check(lib.aps_denoise_pyramid_ex(la, za, _dt(ldt), ka, levels, KD, KU, KT, _p(prev), _p(mv),
                                       N, H, W, demod_offset, lat_offset, _p(out), _p(out_demod),
                                       _p(lat_out), _p(ws), nb, _stream()), "denoise_pyramid")
    return out


def reproject(prev, mv, logits0, KD, KU, KT, has_upsample: bool, accum=None):
    _need(prev, "prev", _F32)
    N, H, W, _ = prev.shape
    accum = torch.zeros_like(prev) if accum is None else accum
    L.check(L.load().aps_reproject(_p(prev), _p(mv), _p(logits0), _dt(logits0.dtype),
                                   logits0.shape[-1], KD, KU, KT, int(has_upsample), N, H, W,
                                   _p(accum), _stream()), "reproject")
    return accum


def upsample(coarse, logits, KD, KU, KT, has_temporal: bool, accum=None):
    _need(coarse, "coarse", _F32)
    N, Hc, Wc, _ = coarse.shape
    H, W = logits.shape[1], logits.shape[2]
    accum = torch.zeros((N, H, W, 4), dtype=_F32, device=coarse.device) if accum is None else accum
    L.check(L.load().aps_upsample(_p(coarse), _p(logits), _dt(logits.dtype), logits.shape[-1], KD,
                                  KU, KT, int(has_temporal), N, H, W, _p(accum), _stream()),
            "upsample")
    return accum


# ------------------------------------------------------------------ backward (a10)

def reproject_bwd(prev, mv, logits0, KD, KU, KT, has_upsample: bool, grad_accum, grad_dtype=None,
                  want_prev: bool = True):
    """-> (grad_logits0 [same shape as logits0], grad_prev or None) of the reproject term."""
    _need(prev, "prev", _F32)
    _need(grad_accum, "grad_accum", _F32)
    N, H, W, _ = prev.shape
    gdt = grad_dtype or logits0.dtype
    glog = torch.empty(logits0.shape, dtype=gdt, device=prev.device)
    gprev = torch.zeros_like(prev) if want_prev else None
    lib = L.load()
    nb = lib.aps_reproject_bwd_workspace_size(N, H, W, KD, KU, KT, int(has_upsample))
    ws = WS.get(nb, prev.device)
    L.check(lib.aps_reproject_bwd(_p(prev), _p(mv), _p(logits0), _dt(logits0.dtype), logits0.shape[-1],
                                  KD, KU, KT, int(has_upsample), N, H, W, _p(grad_accum), _p(glog),
                                  _dt(gdt), glog.shape[-1], _p(gprev), _p(ws), nb, _stream()),
            "reproject_bwd")
    return glog, gprev


def upsample_bwd(coarse, logits, KD, KU, KT, has_temporal: bool, grad_accum, grad_dtype=None):
    """-> (grad_logits [same shape as logits], grad_coarse) of the upsampling term."""
    _need(coarse, "coarse", _F32)
    _need(grad_accum, "grad_accum", _F32)
    N, H, W = logits.shape[0], logits.shape[1], logits.shape[2]
    gdt = grad_dtype or logits.dtype
    glog = torch.empty(logits.shape, dtype=gdt, device=coarse.device)
    gc = torch.empty_like(coarse)
    lib = L.load()
    nb = lib.aps_upsample_bwd_workspace_size(N, H, W, KD, KU, KT, int(has_temporal))
    ws = WS.get(nb, coarse.device)
    L.check(lib.aps_upsample_bwd(_p(coarse), _p(logits), _dt(logits.dtype), logits.shape[-1], KD, KU,
                                 KT, int(has_temporal), N, H, W, _p(grad_accum), _p(glog), _dt(gdt),
                                 glog.shape[-1], _p(gc), _p(ws), nb, _stream()), "upsample_bwd")
    return glog, gc


def density_predict_bwd(net: Net, feat, budget: float, grad_s, uniform_frac: float = 1.0 / 8.0,
                        want_feat: bool = True):
    """-> ({layer name: (dw [cout,k,k,cin] f32, db [cout] f32)}, grad_feat or None)."""
    _need(feat, "feat", net.dtype)
    _need(grad_s, "grad_s", _F32)
    N, H, W, Cf = feat.shape
    names = [l["name"] for l in net.spec]
    pk = [pack_dgrad(l, net.master[l["name"]][0], net.dtype) for l in net.spec]
    gw = [torch.empty((l["cout"], l["k"], l["k"], l["cin"]), dtype=_F32, device=feat.device)
          for l in net.spec]
    gb = [torch.empty(l["cout"], dtype=_F32, device=feat.device) for l in net.spec]
    gf = torch.empty_like(feat) if want_feat else None
    lib = L.load()
    nb = lib.aps_density_predict_bwd_workspace_size(C.byref(net.desc), N, H, W)
    ws = WS.get(nb, feat.device)
    arr = lambda ts: (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
    L.check(lib.aps_density_predict_bwd(C.byref(net.desc), arr(pk), _p(feat), N, H, W, Cf, budget,
                                        uniform_frac, _p(grad_s), arr(gw), arr(gb), _p(gf), _p(ws), nb,
                                        _stream()), "density_predict_bwd")
    return {n: (w, b) for n, w, b in zip(names, gw, gb)}, gf


def denoise_pyramid_bwd(Ls, logits, KD: int, KU: int, KT: int, prev, mv, grad_out,
                        grad_dtype=None, want_prev: bool = True):
    """-> (grad_logits list [same shape as logits], grad_L list, grad_prev or None)."""
    levels = len(Ls)
    L0 = _need(Ls[0], "L0", _F32)
    _need(grad_out, "grad_out", _F32)
    N, H, W, _ = L0.shape
    ldt = logits[0].dtype
    gdt = grad_dtype or ldt
    glog = [torch.empty(t.shape, dtype=gdt, device=t.device) for t in logits]
    gL = [torch.empty_like(t) for t in Ls]
    gprev = torch.zeros_like(prev) if (prev is not None and want_prev) else None
    lib = L.load()
    nb = lib.aps_denoise_pyramid_bwd_workspace_size(N, H, W, levels, KD, KU, KT, int(prev is not None))
    ws = WS.get(nb, L0.device)
    arr = lambda ts: (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in ts])
    ka = (C.c_int * L.APS_MAX_LEVELS)(*[t.shape[-1] for t in logits])
    L.check(lib.aps_denoise_pyramid_bwd(arr(Ls), arr(logits), _dt(ldt), ka, levels, KD, KU, KT,
                                        _p(prev), _p(mv), N, H, W, _p(grad_out), arr(glog),
                                        _dt(gdt), ka, arr(gL), _p(gprev), _p(ws), nb, _stream()),
            "denoise_pyramid_bwd")
    return glog, gL, gprev


def scatter_samples_bwd(s, count, pixel_offset, samples, grad_L, mode="relaxed", lam=10.0,
                        seed=0, frame=0, grad_s=None, u_tex=None, tau: float = 0.5, L_ref=None):
    _need(s, "s", _F32)
    N, H, W = s.shape
    acc = grad_s is not None
    if grad_s is None:
        grad_s = torch.empty_like(s)
    arr = (C.c_void_p * L.APS_MAX_LEVELS)(*[t.data_ptr() for t in grad_L])
    m = _MODES[mode]
    tp, T = _tex(u_tex)
    if L_ref is not None:
        _need(L_ref, "L_ref", _F32)
    L.check(L.load().aps_scatter_samples_bwd_ex(_p(s), _p(count), _p(pixel_offset), _p(samples),
                                                samples.shape[0], N, H, W, len(grad_L), m,
                                                tau if mode == "gumbel" else lam, seed, frame, tp, T,
                                                _p(L_ref), arr, _p(grad_s), int(acc), _stream()),
            "scatter_samples_bwd")
    return grad_s


def normalize_density_bwd(z, budget, grad_s, uniform_frac=1.0 / 8.0):
    _need(z, "z", _F32)
    _need(grad_s, "grad_s", _F32)
    N, H, W = z.shape
    gz = torch.empty_like(z)
    lib = L.load()
    nb = lib.aps_normalize_bwd_workspace_size(N, H, W)
    ws = WS.get(nb, z.device)
    L.check(lib.aps_normalize_density_bwd(_p(z), N, H, W, budget, uniform_frac, _p(grad_s),
                                          _p(gz), _p(ws), nb, _stream()), "normalize_density_bwd")
    return gz


def assemble_features_bwd(kind, grad_feat, L0=None, prev=None, mv=None, grad_L0=None,
                          grad_s=None, grad_prev=None, has_lat=False, grad_lat=None):
    _need(grad_feat, "grad_feat")
    N, H, W, Cf = grad_feat.shape
    k = L.APS_FEAT_SAMPLER if kind == "sampler" else L.APS_FEAT_KERNEL
    L.check(L.load().aps_assemble_features_bwd_ex(k, _p(L0), _p(prev), _p(mv), int(has_lat), N, H, W,
                                                  Cf, _dt(grad_feat.dtype), _p(grad_feat), _p(grad_L0),
                                                  _p(grad_s), _p(grad_prev), _p(grad_lat), _stream()),
            "assemble_features_bwd")


def copy_channels(src, dst_dtype, dst_ld, C_copy=None):
    """[..., src_ld] -> [..., dst_ld] in dst_dtype, first C_copy channels copied, rest zero."""
    _need(src, "src")
    src_ld = src.shape[-1]
    C_copy = src_ld if C_copy is None else C_copy
    npix = src.numel() // src_ld
    out = torch.empty(tuple(src.shape[:-1]) + (dst_ld,), dtype=dst_dtype, device=src.device)
    L.check(L.load().aps_copy_channels(_p(src), _dt(src.dtype), src_ld, _p(out), _dt(dst_dtype),
                                       dst_ld, npix, C_copy, _stream()), "copy_channels")
    return out


def scale_by(x, scale):
    _need(x, "x", _F32)
    _need(scale, "scale", _F32)
    L.check(L.load().aps_scale_by(_p(x), x.numel(), _p(scale), _stream()), "scale_by")
    return x


def pack_dgrad(layer_spec, w_master, dtype):
    lib = L.load()
    n = lib.aps_conv_packed_elems(layer_spec["cin"], layer_spec["k"], layer_spec["cout"])
    pk = torch.empty(n, dtype=dtype, device=w_master.device)
    L.check(lib.aps_conv_pack_weights_dgrad(_p(w_master), layer_spec["cout"], layer_spec["k"],
                                            layer_spec["cin"], _dt(dtype), _p(pk), _stream()),
            "pack_weights_dgrad")
    return pk


def conv2d_bwd(x, x2, mode, layer_spec, packed_T, dy, ymask=None, need_dx=True, need_dx2=True):
    """Gradients of one conv layer.  dy [N,H,W,ldy] in the net dtype; ymask = the layer's
    post-ReLU output (None without ReLU).  -> (dx, dx2, dw [cout,k,k,cin] f32, db [cout] f32)."""
    _need(dy, "dy", x.dtype)
    N, H, W, ldy = dy.shape
    cout, cin, k = layer_spec["cout"], layer_spec["cin"], layer_spec["k"]
    Cx = x.shape[-1]
    C2 = x2.shape[-1] if x2 is not None else 0
    m = {"direct": L.APS_CONV_DIRECT, "pool2": L.APS_CONV_POOL2, "up2cat": L.APS_CONV_UP2_CAT}[mode]
    lib = L.load()
    dx = dx2 = None
    if need_dx or (need_dx2 and x2 is not None):
        dX = torch.empty((N, H, W, cin), dtype=x.dtype, device=x.device)
        L.check(lib.aps_conv2d_bwd_data(_p(dy), _p(ymask), ldy, N, H, W, cout, _p(packed_T), k, cin,
                                        _dt(x.dtype), _p(dX), _stream()), "conv2d_bwd_data")
        if mode == "direct":
            dx = dX
        else:
            dx = torch.empty_like(x)
            dx2 = torch.empty_like(x2) if x2 is not None else None
            L.check(lib.aps_conv_input_grad(m, _p(dX), N, H, W, Cx, C2, _dt(x.dtype), _p(dx), 0,
                                            _p(dx2), 0, _stream()), "conv_input_grad")
    dw = torch.empty((cout, k, k, cin), dtype=_F32, device=x.device)
    db = torch.empty(cout, dtype=_F32, device=x.device)
    nb = lib.aps_conv2d_bwd_weight_workspace_size(N, H, W, Cx, C2, cout, k)
    ws = WS.get(nb, x.device)
    L.check(lib.aps_conv2d_bwd_weight(_p(x), _p(x2), m, N, H, W, Cx, C2, _p(dy), _p(ymask), ldy,
                                      cout, k, _dt(x.dtype), _p(dw), _p(db), _p(ws), nb, _stream()),
            "conv2d_bwd_weight")
    return dx, dx2, dw, db


# ------------------------------------------------------------------ training (a11)

def tmo_loss(out, ref, params, prev_out=None, prev_ref=None, mv=None, want_prev=True):
    """-> (loss [1] device, grad_out, grad_prev or None); params [N,5] (k, alpha, beta, s, h)."""
    _need(out, "out", _F32)
    _need(ref, "ref", _F32)
    _need(params, "params", _F32)
    N, H, W, _ = out.shape
    loss = torch.empty(1, dtype=_F32, device=out.device)
    gout = torch.empty_like(out)
    gprev = torch.zeros_like(out) if (prev_out is not None and want_prev) else None
    lib = L.load()
    nb = lib.aps_tmo_loss_workspace_size(N, H, W)
    ws = WS.get(nb, out.device)
    L.check(lib.aps_tmo_loss(_p(out), _p(ref), _p(prev_out), _p(prev_ref), _p(mv), _p(params), N, H,
                             W, _p(loss), _p(gout), _p(gprev), _p(ws), nb, _stream()), "tmo_loss")
    return loss, gout, gprev


def adamw_step(param, m, v, grad, lr, step, beta1=0.8, beta2=0.985, eps=1e-8, weight_decay=0.02,
               grad_scale=1.0):
    for t, nm in ((param, "param"), (m, "m"), (v, "v"), (grad, "grad")):
        _need(t, nm, _F32)
    L.check(L.load().aps_adamw_step(_p(param), _p(m), _p(v), _p(grad), param.numel(), lr, beta1,
                                    beta2, eps, weight_decay, step, grad_scale, _stream()),
            "adamw_step")


def sumsq(x, out=None):
    """Sum of squares of x into a device scalar (out: an existing 1-element float32 slot)."""
    _need(x, "x", _F32)
    if out is None:
        out = torch.empty(1, dtype=_F32, device=x.device)
    lib = L.load()
    nb = lib.aps_sumsq_workspace_size(x.numel())
    ws = WS.get(nb, x.device)
    L.check(lib.aps_sumsq(_p(x), x.numel(), _p(out), _p(ws), nb, _stream()), "sumsq")
    return out
