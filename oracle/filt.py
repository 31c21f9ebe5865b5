"""Gathering pyramidal filter, FP64 (App. A).

Logit channel order per pixel and level: [kd (KD^2) | ku (KU^2) if l < L-1 |
kt (KT^2) if l == 0 and the temporal term is on].  Within each block the taps run
row-major over (dy, dx), each in [-r, r]: channel (dy + r) * K + (dx + r) weights the
value at (x + dx, y + dy) (eq. app-gather indexes kappa_ij at (x+i, y+j)).
Every gather clamps coordinates to the image edge.
"""
import torch

F64 = torch.float64


def joint_softmax(logits, sizes):
    """Softmax over the concatenated kernels of one level (eqs. app-softmax-mid/full).

    logits [N, H, W, >= sum(sizes)] -> list of weight blocks [N, H, W, size_i]; sums to 1.
    """
    k = sum(sizes)
    z = logits[..., :k]
    w = torch.softmax(z, dim=-1)
    out, o = [], 0
    for n in sizes:
        out.append(w[..., o:o + n])
        o += n
    return out


def _shift(img, dy, dx):
    """out[y, x] = img[clamp(y + dy), clamp(x + dx)]."""
    N, H, W, C = img.shape
    ys = torch.clamp(torch.arange(H) + dy, 0, H - 1)
    xs = torch.clamp(torch.arange(W) + dx, 0, W - 1)
    return img[:, ys][:, :, xs]


def gather(img, w, K: int):
    """G(img, w)[x, y] = sum_{dy, dx in [-r, r]} w[(dy+r)K + (dx+r)] * img[x+dx, y+dy] (eq. app-gather)."""
    r = K // 2
    out = torch.zeros_like(img)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out = out + w[..., (dy + r) * K + (dx + r)].unsqueeze(-1) * _shift(img, dy, dx)
    return out


def upsample(coarse, w, KU: int, H: int, W: int):
    """U(coarse, w) at the fine resolution H x W (eq. app-upsample).

    KU = 3: 3x3 taps around the parent (floor(x/2), floor(y/2)).
    KU = 2: the printed form, taps at (floor((x+i)/2), floor((y+j)/2)), i, j in {0, 1},
    channel j*2 + i.
    """
    N, Hc, Wc, C = coarse.shape
    yy = torch.arange(H)
    xx = torch.arange(W)
    out = torch.zeros(N, H, W, C, dtype=coarse.dtype)
    if KU == 2:
        taps = [((y_off, x_off), y_off * 2 + x_off) for y_off in (0, 1) for x_off in (0, 1)]
        for (j, i), ch in taps:
            ys = torch.clamp((yy + j) // 2, 0, Hc - 1)
            xs = torch.clamp((xx + i) // 2, 0, Wc - 1)
            out = out + w[..., ch].unsqueeze(-1) * coarse[:, ys][:, :, xs]
        return out
    r = KU // 2
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            ys = torch.clamp(yy // 2 + dy, 0, Hc - 1)
            xs = torch.clamp(xx // 2 + dx, 0, Wc - 1)
            out = out + w[..., (dy + r) * KU + (dx + r)].unsqueeze(-1) * coarse[:, ys][:, :, xs]
    return out


def warp(prev, mv):
    """W(prev)[x, y] = bilinear sample of prev at (x + mv_x, y + mv_y), index coordinates,
    both bilinear taps clamped to the edge (App. A, eq. app-recon-full: W_t warps the
    previous output along the motion vectors).

    prev [N, H, W, C]; mv [N, H, W, 2] with (dx, dy).
    """
    N, H, W, C = prev.shape
    mv = torch.as_tensor(mv, dtype=F64)
    py = torch.arange(H, dtype=F64).reshape(1, H, 1) + mv[..., 1]
    px = torch.arange(W, dtype=F64).reshape(1, 1, W) + mv[..., 0]
    y0 = torch.floor(py)
    x0 = torch.floor(px)
    fy = (py - y0).unsqueeze(-1)
    fx = (px - x0).unsqueeze(-1)
    y0 = y0.long()
    x0 = x0.long()
    n = torch.arange(N).reshape(N, 1, 1)

    def tap(yi, xi):
        return prev[n, torch.clamp(yi, 0, H - 1), torch.clamp(xi, 0, W - 1)]

    return ((1 - fy) * ((1 - fx) * tap(y0, x0) + fx * tap(y0, x0 + 1))
            + fy * ((1 - fx) * tap(y0 + 1, x0) + fx * tap(y0 + 1, x0 + 1)))


def level_sizes(l: int, levels: int, KD: int, KU: int, KT: int, temporal: bool):
    sizes = [KD * KD]
    if l < levels - 1:
        sizes.append(KU * KU)
    if l == 0 and temporal:
        sizes.append(KT * KT)
    return sizes


def denoise_pyramid(L, logits, KD: int, KU: int, KT: int, prev=None, mv=None):
    """Coarse-to-fine reconstruction (eqs. app-recon-coarse/mid/full).

    L: list of levels [N, H/2^l, W/2^l, C];  logits: list of [N, H_l, W_l, >= K_l].
    prev, mv: previous HDR output and motion vectors; None = no temporal term (first frame).
    Returns the list of reconstructed levels [Lhat^0, ..., Lhat^{L-1}].
    """
    levels = len(L)
    temporal = prev is not None
    out = [None] * levels
    for l in range(levels - 1, -1, -1):
        N, H, W, C = L[l].shape
        sizes = level_sizes(l, levels, KD, KU, KT, temporal)
        ws = joint_softmax(logits[l], sizes)
        y = gather(L[l], ws[0], KD)
        if l < levels - 1:
            y = y + upsample(out[l + 1], ws[1], KU, H, W)
        if l == 0 and temporal:
            y = y + gather(warp(prev, mv), ws[-1], KT)
        out[l] = y
    return out


def denoise_magnitude(L, logits, KD, KU, KT, prev=None, mv=None):
    """The same reconstruction applied to |values|: sum_k w_k |v_k| per output, the
    magnitude a floating-point evaluation of the weighted sums is accurate relative to."""
    absL = [x.abs() for x in L]
    absprev = prev.abs() if prev is not None else None
    levels = len(L)
    temporal = prev is not None
    out = [None] * levels
    for l in range(levels - 1, -1, -1):
        N, H, W, C = L[l].shape
        ws = joint_softmax(logits[l], level_sizes(l, levels, KD, KU, KT, temporal))
        y = gather(absL[l], ws[0], KD)
        if l < levels - 1:
            y = y + upsample(out[l + 1], ws[1], KU, H, W)
        if l == 0 and temporal:
            y = y + gather(warp(absprev, mv), ws[-1], KT)
        out[l] = y
    return out
