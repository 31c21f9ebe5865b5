"""Stochastic rounding, s-normalised scatter and the average-pooling pyramid.

* Sec. 4.2, eq. holdout: floor(s_i) samples always; one extra (the holdout) iff
  u_i < p_i, p_i = s_i - floor(s_i).
* Sec. 4.2, eq. stoch_rnoisy: L_noisy_i = (sum of the floor(s_i) samples + H_i) / s_i.
* Sec. 4.3, eqs. relaxed_holdout and h_factor: in training H_i = r_i * h * ramp with a
  clipped linear ramp of slope lambda/p and h = 2 lambda / (2 lambda - 1).  The paper
  writes the ramp as clamp(lambda/p * (u + p - 1), 0, 1), which is non-zero iff
  u > 1 - p; this implementation uses the mirrored variate u -> 1 - u (equally uniform), giving
  clamp(lambda * (p - u) / p, 0, 1), non-zero iff u < p, so the relaxed forward takes
  exactly the samples of the hard mask drawn from the same u.
* App. A, eq. app-pyramid: level l is the mean of L_noisy over 2^l x 2^l blocks.
* u: Philox (one counter per pixel), or a blue-noise threshold texture (Sec. 6.3 uses
  blue-noise dithering) tiled over the frame with a toroidal offset per image and frame:
  u[n, y, x] = tex[(y + oy) mod T, (x + ox) mod T], (ox, oy) = (word0, word1) mod T of
  Philox with counter (n, frame, 2, 0).

Counts, offsets and the compact list are exact integer results.
"""
import numpy as np
import torch

from .philox import philox4x32_10, uniform24

BLOCK = 256          # pixels per block of the per-block exclusive offsets
COUNT_MAX = 255      # counts are stored as uint8


def pixel_index(N, H, W):
    return np.arange(N * H * W, dtype=np.uint64).reshape(N, H, W)


STREAM_TEX_OFFSET = 2


def tex_offsets(seed: int, n: int, frame: int, T: int):
    """(ox, oy) of image n at this frame: Philox words 0 and 1 of counter (n, frame, 2, 0) mod T."""
    seed = int(seed)
    w = philox4x32_10(np.uint64(n), np.uint64(frame), np.uint64(STREAM_TEX_OFFSET), np.uint64(0),
                      seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return int(w[0]) % T, int(w[1]) % T


def u_values(N, H, W, seed: int, frame: int, u_tex=None):
    """u [N, H, W] float64: Philox per pixel, or the tiled texture with per-image offsets."""
    if u_tex is None:
        return uniform24(seed, pixel_index(N, H, W), frame)
    tex = np.asarray(u_tex, dtype=np.float32).astype(np.float64)
    T = tex.shape[0]
    assert tex.shape == (T, T)
    u = np.empty((N, H, W))
    for n in range(N):
        ox, oy = tex_offsets(seed, n, frame, T)
        rows = (np.arange(H) + oy) % T          # texture row of each image row
        cols = (np.arange(W) + ox) % T          # texture column of each image column
        u[n] = tex[np.ix_(rows, cols)]
    return u


def mask(s32, seed: int, frame: int, u_tex=None, rounding: str = "stochastic"):
    """s32: float32 [N, H, W] densities; u_tex: optional float32 [T, T] threshold texture.
    rounding: "stochastic" count = floor(s) + [u < p] (eq. holdout); "holdout" floor(s) + [p > 0]
    (the holdout requested wherever it exists, for the straight-through and Gumbel-Softmax
    estimators); "deterministic" round(s) = floor(s + 1/2) (Sec. 4.1 eq. kuz_fw, DASR).

    Returns dict(count uint8 [N,H,W], p float64 [N,H,W] (exact), u float64, take bool,
    block_offset int64 [ceil(Npix/256)+1] (exclusive; last entry = total),
    sample_pixel int64 [total] (global pixel index, ascending), total int, overflow bool).
    """
    s = np.asarray(s32, dtype=np.float32).astype(np.float64)   # exact widening
    N, H, W = s.shape
    fl = np.floor(s)
    p = s - fl                                                 # exact
    u = u_values(N, H, W, seed, frame, u_tex)
    if rounding == "stochastic":
        take = u < p
    elif rounding == "holdout":
        take = p > 0
    elif rounding == "deterministic":
        take = np.floor(s + 0.5) > fl
    else:
        raise ValueError(rounding)
    cnt = fl + take
    overflow = bool((cnt > COUNT_MAX).any())
    count = np.minimum(cnt, COUNT_MAX).astype(np.int64)
    flat = count.reshape(-1)
    nblk = (flat.size + BLOCK - 1) // BLOCK
    padded = np.zeros(nblk * BLOCK, np.int64)
    padded[:flat.size] = flat
    bsum = padded.reshape(nblk, BLOCK).sum(1)
    block_offset = np.concatenate([[0], np.cumsum(bsum)])
    sample_pixel = np.repeat(np.arange(flat.size, dtype=np.int64), flat)
    return dict(count=count.astype(np.uint8), p=p, u=u, take=take,
                block_offset=block_offset, sample_pixel=sample_pixel,
                total=int(flat.sum()), overflow=overflow)


def h_factor(lam: float) -> float:
    """Sec. 4.3, eq. h_factor."""
    return 2.0 * lam / (2.0 * lam - 1.0)


def relaxed_ramp(p, u, lam: float):
    """clamp(lambda * (p - u) / p, 0, 1) for p > 0, and 0 where p == 0 (mirrored u)."""
    p = torch.as_tensor(p, dtype=torch.float64)
    u = torch.as_tensor(u, dtype=torch.float64)
    safe = torch.where(p > 0, p, torch.ones_like(p))
    r = torch.clamp(lam * (p - u) / safe, 0.0, 1.0)
    return torch.where(p > 0, r, torch.zeros_like(r))


def scatter(s, count, samples, seed: int, frame: int, mode: str = "hard", lam: float = 10.0,
            u_tex=None):
    """Sec. 4.2 eq. stoch_rnoisy (hard) / Sec. 4.3 eq. relaxed_holdout (relaxed): L_noisy [N, H, W, 4] (channel 3 = 0) from samples delivered in request order.

    s: [N, H, W] densities (torch float64 for autograd, or numpy; the floor and the
       fractional part are taken from its value);
    count: uint8 [N, H, W] from `mask`;  samples: [total, 4] in pixel order.
    """
    s = torch.as_tensor(s, dtype=torch.float64)
    N, H, W = s.shape
    cnt = np.asarray(count).reshape(-1).astype(np.int64)
    smp = torch.as_tensor(np.asarray(samples), dtype=torch.float64)
    sf = s.reshape(-1)
    fl = np.floor(sf.detach().numpy())
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    pix_of = np.repeat(np.arange(cnt.size), cnt)            # owning pixel of each sample
    j = np.arange(cnt.sum()) - start[pix_of]               # index within the pixel
    is_base = j < fl[pix_of]
    base = torch.zeros(cnt.size, 4, dtype=torch.float64)
    base = base.index_add(0, torch.as_tensor(pix_of[is_base]), smp[torch.as_tensor(is_base)])
    hold_idx = np.nonzero(~is_base)[0]
    hold = torch.zeros(cnt.size, 4, dtype=torch.float64)
    if hold_idx.size:
        hold = hold.index_add(0, torch.as_tensor(pix_of[hold_idx]), smp[torch.as_tensor(hold_idx)])
    if mode == "hard":
        H_i = hold
    elif mode == "relaxed":
        p = sf - torch.as_tensor(fl)                           # gradient of p w.r.t. s is 1
        u = torch.as_tensor(u_values(N, H, W, seed, frame, u_tex).reshape(-1))
        H_i = hold * (h_factor(lam) * relaxed_ramp(p, u, lam))[:, None]
    else:
        raise ValueError(mode)
    # s > 0 always holds for normalised densities (s >= B/8); a zero density has no
    # samples and its estimate is defined as 0.
    pos = sf > 0
    L = torch.where(pos[:, None], (base + H_i) / torch.where(pos, sf, torch.ones_like(sf))[:, None],
                    torch.zeros_like(base))
    L = torch.cat([L[:, :3], torch.zeros_like(L[:, 3:])], 1)
    return L.reshape(N, H, W, 4)


def pyramid(L0, levels: int):
    """[L^0, ..., L^{levels-1}]; L^l = mean of L^0 over each 2^l x 2^l block (eq. app-pyramid)."""
    L0 = torch.as_tensor(L0, dtype=torch.float64)
    N, H, W, C = L0.shape
    out = [L0]
    for l in range(1, levels):
        b = 2 ** l
        assert H % b == 0 and W % b == 0, "pyramid sizes must divide by 2^(levels-1)"
        out.append(L0.reshape(N, H // b, b, W // b, b, C).mean(dim=(2, 4)))
    return out
