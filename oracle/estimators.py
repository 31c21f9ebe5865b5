"""Gradient estimators of the sampling step, FP64 (torch CPU autograd).

Per pixel i (RGB rows): the density s_i, p_i = s_i - floor(s_i), the sum b_i of the floor(s_i)
samples that are always taken, the holdout sample r_i and the uniform u_i.

* hard (Sec. 4.2, eqs. holdout, stoch_rnoisy): L = (b + r [u < p]) / s.  Its gradient through
  the indicator is zero; only the normalisation by s is differentiable.
* relaxed (Sec. 4.3, eqs. relaxed_holdout, h_factor; u mirrored as in `sampling`):
  L = (b + r h clamp(lambda (p - u) / p, 0, 1)) / s.
* straight-through (Sec. 4.3, comparison figure; Bengio et al. 2013): the hard forward, with
  d[u < p]/dp taken as 1 in the backward pass (where p > 0: an integer s has no holdout).
* Gumbel-Softmax (Sec. 4.3; the binary concrete relaxation of Jang et al. / Maddison et al.):
  the indicator replaced by sigmoid((logit p - logit u) / tau), which tends to [u < p] as
  tau -> 0 (logistic noise -logit u; the same mirrored u).
* DASR (Sec. 4.1, eqs. kuz_fw, kuz_grad; Kuznetsov et al. 2018): deterministic rounding,
  L = mean of round(s) samples for s >= 1/2 and 0 below, with the surrogate gradient
  dL/ds = (L_ref - L) / round(s) for s >= 1/2 and L_ref below (L_ref: the reference radiance).

The reference for the comparison is the exact gradient of the expected loss of the stochastic
(hard) forward.  For one draw of u, an unbiased sample of it is
  g_i = loss(I_i = 1) - loss(I_i = 0) + d loss / d s_i with every indicator held fixed,
the first term by flipping pixel i's holdout (Sec. 4.2: "computing this gradient exactly
requires edge sampling of each discontinuity"); its expectation over u is the gradient of
E[loss], which `expected_grad_enum` computes by enumerating every mask of a tiny image.
"""
import itertools

import torch

from .sampling import h_factor, relaxed_ramp

F64 = torch.float64


def _split(s):
    fl = torch.floor(s.detach())
    return fl, s - fl            # p carries the gradient of s (dp/ds = 1)


def L_hard(s, b, r, u):
    _, p = _split(s)
    I = (u < p.detach()).to(F64)
    return (b + r * I[:, None]) / s[:, None]


def L_relaxed(s, b, r, u, lam: float = 10.0):
    _, p = _split(s)
    w = h_factor(lam) * relaxed_ramp(p, u, lam)
    return (b + r * w[:, None]) / s[:, None]


def L_straight_through(s, b, r, u):
    _, p = _split(s)
    # value [u < p], slope 1 where a holdout exists (p > 0)
    I = (u < p.detach()).to(F64) + (p - p.detach()) * (p.detach() > 0).to(F64)
    return (b + r * I[:, None]) / s[:, None]


def L_gumbel(s, b, r, u, tau: float = 0.5):
    _, p = _split(s)
    logit = lambda x: torch.log(x) - torch.log1p(-x)
    pos = p > 0
    pc = torch.where(pos, p, torch.full_like(p, 0.5))
    I = torch.where(pos, torch.sigmoid((logit(pc) - logit(torch.clamp(u, 1e-300, 1.0))) / tau),
                    torch.zeros_like(p))
    return (b + r * I[:, None]) / s[:, None]


class _DASR(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, pool, L_ref):
        n = torch.where(s >= 0.5, torch.floor(s + 0.5), torch.zeros_like(s))
        L = torch.zeros(s.shape[0], pool.shape[2], dtype=F64)
        for i in range(s.shape[0]):
            k = int(n[i])
            if k > 0:
                L[i] = pool[i, :k].sum(0) / k
        ctx.save_for_backward(s, n, L, L_ref)
        return L

    @staticmethod
    def backward(ctx, gL):
        s, n, L, L_ref = ctx.saved_tensors
        dLds = torch.where((s >= 0.5)[:, None], (L_ref - L) / torch.clamp(n, min=1.0)[:, None], L_ref)
        return (gL * dLds).sum(1), None, None


def L_dasr(s, pool, L_ref):
    """pool [P, J, 3] with J >= max round(s); L_ref [P, 3]."""
    return _DASR.apply(s, pool, L_ref)


def exact_grad_draw(s, b, r, u, loss):
    """Unbiased sample (for this u) of grad_s E_u[loss(L_hard)]: holdout flips plus the
    gradient with every indicator fixed.  loss maps L [P, 3] (or a batch [B, P, 3]) to a
    scalar (per batch element)."""
    s = s.detach()
    fl, p = _split(s)
    I = (u < p).to(F64)
    P = s.shape[0]
    # flips: batch row i has pixel i's indicator set to 1 (first half) or 0 (second half)
    I1 = I.repeat(P, 1)
    I1[torch.arange(P), torch.arange(P)] = 1.0
    I0 = I.repeat(P, 1)
    I0[torch.arange(P), torch.arange(P)] = 0.0
    L1 = (b[None] + r[None] * I1[..., None]) / s[None, :, None]
    L0 = (b[None] + r[None] * I0[..., None]) / s[None, :, None]
    flip = loss(L1) - loss(L0)
    sv = s.clone().requires_grad_(True)
    fixed = loss((b + r * I[:, None]) / sv[:, None])
    (g_norm,) = torch.autograd.grad(fixed, sv)
    return flip + g_norm


def expected_grad_enum(s, b, r, loss):
    """grad_s of E[loss] over every mask outcome (2^P of them; tiny P only)."""
    sv = s.detach().clone().requires_grad_(True)
    fl = torch.floor(sv.detach())
    p = sv - fl
    P = s.shape[0]
    E = torch.zeros((), dtype=F64)
    for bits in itertools.product((0.0, 1.0), repeat=P):
        I = torch.tensor(bits, dtype=F64)
        prob = torch.prod(torch.where(I > 0, p, 1.0 - p))
        E = E + prob * loss((b + r * I[:, None]) / sv[:, None])
    (g,) = torch.autograd.grad(E, sv)
    return g
