"""Bias of the sampling step's gradient estimators against the exact gradient of the expected
loss (the paper's gradient-comparison figure, Sec. 4.3, in numbers).  Not a pytest module: run
`python -m tests.estimator_bias [--draws M]` on a GPU; it prints one JSON line.

Setup: a 16x16 image (a smooth HDR field with a bright patch), a smooth density s in [0.05, 1.55]
(so the holdout decides most pixels), per-draw sample pools truth * (1 + n) from procgen, a fixed
5x5 box reconstruction and the mean squared error to the truth.  Every draw is one image of a
batch (Philox u differs per image).  The estimators' gradients come from the library's scatter
kernels (mask, renderer stand-in, scatter forward and backward on the GPU); the loss gradient
and the reference come from the FP64 oracle: for each draw, the exact per-draw gradient
(holdout flips plus the fixed-indicator gradient, `oracle.estimators.exact_grad_draw`), whose
mean over draws converges to the gradient of the expected loss.  Reported per estimator: the
relative distance of its mean gradient from the reference mean, the cosine, and the bias with
the Monte Carlo noise of the per-draw differences taken out.
"""
import argparse
import json
import math

import numpy as np
import torch

import procgen
from oracle import estimators as est
from oracle import filt as ofilt
from oracle import sampling as osamp

F64 = torch.float64
H = W = 16
P = H * W


def setup():
    yy, xx = torch.meshgrid(torch.arange(H, dtype=F64), torch.arange(W, dtype=F64), indexing="ij")
    truth = torch.stack([1 + torch.sin(xx / 3), 1 + torch.cos(yy / 4), 0.5 + 0.1 * xx], -1)
    truth[(xx > 9) & (yy < 6)] *= 6.0
    s = (0.6 + 0.5 * torch.sin(xx / 5 + yy / 7)) * 1.2 + 0.05
    return truth, s.float().double()


def loss_fn(truth):
    w25 = None

    def loss(L):                     # L [..., P, 3] -> per-batch MSE of the 5x5 box reconstruction
        nonlocal w25
        lead = L.shape[:-2]
        img = L.reshape(-1, H, W, 3)
        if w25 is None or w25.shape[0] != img.shape[0]:
            w25 = torch.full((img.shape[0], H, W, 25), 1.0 / 25, dtype=F64)
        out = ofilt.gather(img, w25, 5)
        return ((out - truth) ** 2).sum((-3, -2, -1)).reshape(lead) / P
    return loss


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--draws", type=int, default=4096)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--seed", type=int, default=2602)
    a = ap.parse_args()
    from paper_2602_08642_amd import ops
    dev = "cuda"
    truth, s = setup()
    loss = loss_fn(truth)
    modes = {"relaxed (ours, lambda 10)": ("relaxed", {}), "straight-through": ("straight_through", {}),
             "gumbel-softmax tau 0.5": ("gumbel", {"tau": 0.5}), "gumbel-softmax tau 0.1": ("gumbel", {"tau": 0.1}),
             "DASR surrogate": ("dasr", {})}
    acc = {k: torch.zeros(P, dtype=F64) for k in modes}
    dsq = {k: torch.zeros(P, dtype=F64) for k in modes}
    ref = torch.zeros(P, dtype=F64)
    M = 0
    fl = torch.floor(s).reshape(-1).long()
    Lref = torch.zeros(a.batch, H, W, 4, dtype=torch.float32)
    Lref[..., :3] = truth.float()
    Lref = Lref.to(dev)
    st = s.float().expand(a.batch, H, W).contiguous().to(dev)
    for bi in range(a.draws // a.batch):
        N = a.batch
        frame = bi
        pools = np.concatenate([procgen.sample_pool(truth.numpy(), a.seed, frame * N + n, 8) for n in range(N)])
        pool_d = torch.tensor(pools, device=dev)
        rgb = torch.tensor(pools[..., :3], dtype=F64).reshape(N, P, 8, 3)
        u = torch.tensor(osamp.u_values(N, H, W, a.seed, frame)).reshape(N, P)
        # the reference: exact per-draw gradients on the same samples and u
        exact = []
        for n in range(N):
            b = torch.stack([rgb[n, i, :fl[i]].sum(0) for i in range(P)])
            r = torch.stack([rgb[n, i, fl[i]] for i in range(P)])
            exact.append(est.exact_grad_draw(s.reshape(-1), b, r, u[n], loss))
        exact = torch.stack(exact)
        ref += exact.sum(0)
        for k, (mode, kw) in modes.items():
            req = ops.sample_mask(st, a.seed, frame, rounding=ops.MODE_ROUNDING[mode])
            smp = ops.fixture_render(pool_d, req["count"], req["pixel_offset"], req["capacity"])
            (L0,) = ops.scatter_samples(st, req["count"], req["pixel_offset"], smp, 1, mode, 10.0,
                                        a.seed, frame, **kw)
            Lc = L0.cpu().double()[..., :3].reshape(N, P, 3).requires_grad_(True)
            (gL,) = torch.autograd.grad(loss(Lc).sum(), Lc)
            g4 = torch.zeros(N, H, W, 4, dtype=torch.float32)
            g4[..., :3] = gL.reshape(N, H, W, 3).float()
            gs = ops.scatter_samples_bwd(st, req["count"], req["pixel_offset"], smp, [g4.to(dev)], mode,
                                         10.0, a.seed, frame, L_ref=Lref, **kw)
            g = gs.cpu().double().reshape(N, P)
            acc[k] += g.sum(0)
            dsq[k] += ((g - exact) ** 2).sum(0)
        M += N
    refm = ref / M
    out = {"draws": M, "image": f"{W}x{H}", "loss": "MSE of a 5x5 box reconstruction to the truth",
           "reference": "exact per-draw gradient (holdout flips + fixed-indicator gradient), mean over draws",
           "estimators": {}}
    for k in modes:
        mk = acc[k] / M
        d = mk - refm
        var = dsq[k] / M - d ** 2                    # per-pixel variance of the per-draw differences
        noise2 = float(var.sum()) / (M - 1)
        bias2 = float((d ** 2).sum()) - noise2
        nref = float(refm.norm())
        out["estimators"][k] = {"rel_distance": round(float(d.norm()) / nref, 4),
                                "cosine": round(float(mk @ refm) / float(mk.norm()) / nref, 4),
                                "bias_without_noise": round(math.sqrt(max(bias2, 0.0)) / nref, 4),
                                "noise": round(math.sqrt(noise2) / nref, 4)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
