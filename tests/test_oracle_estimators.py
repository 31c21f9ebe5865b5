"""Pins of the gradient-estimator oracle (straight-through, Gumbel-Softmax, DASR, relaxed) and of
the exact expected gradient it is compared against."""
import itertools

import numpy as np
import torch

from oracle import estimators as est

F64 = torch.float64


def _problem(P, seed):
    g = torch.Generator().manual_seed(seed)
    s = torch.rand(P, generator=g, dtype=F64) * 2.2 + 0.15
    b = torch.randn(P, 3, generator=g, dtype=F64) * torch.floor(s)[:, None]
    r = torch.rand(P, 3, generator=g, dtype=F64) * 3.0
    M = torch.randn(P, P, generator=g, dtype=F64) / P ** 0.5      # a non-local linear "filter"
    t = torch.randn(P, 3, generator=g, dtype=F64)
    loss = lambda L: (((M @ L) - t) ** 2).sum((-2, -1)) + 0.1 * (L ** 3).sum((-2, -1))
    return s, b, r, loss


def test_exact_draw_gradient_is_unbiased_by_enumeration():
    """E over every mask outcome of the per-draw flip gradient = grad of E[loss] (exact)."""
    P = 7
    s, b, r, loss = _problem(P, 1)
    p = s - torch.floor(s)
    mean = torch.zeros(P, dtype=F64)
    for bits in itertools.product((0, 1), repeat=P):
        I = torch.tensor(bits, dtype=torch.bool)
        u = torch.where(I, p / 2, (1 + p) / 2)            # a u that gives this outcome
        prob = torch.prod(torch.where(I, p, 1 - p))
        mean = mean + prob * est.exact_grad_draw(s, b, r, u, loss)
    ref = est.expected_grad_enum(s, b, r, loss)
    assert torch.allclose(mean, ref, rtol=1e-10, atol=1e-12)


def test_expected_gradient_matches_finite_differences():
    P = 6
    s, b, r, loss = _problem(P, 2)
    g = est.expected_grad_enum(s, b, r, loss)

    def E(sv):
        p = sv - torch.floor(sv)
        tot = 0.0
        for bits in itertools.product((0.0, 1.0), repeat=P):
            I = torch.tensor(bits, dtype=F64)
            tot += float(torch.prod(torch.where(I > 0, p, 1 - p)) * loss((b + r * I[:, None]) / sv[:, None]))
        return tot

    for i in range(P):
        e = torch.zeros(P, dtype=F64)
        e[i] = 1e-6
        fd = (E(s + e) - E(s - e)) / 2e-6
        assert abs(fd - float(g[i])) <= 1e-6 * (1 + abs(fd))


def test_straight_through_forward_and_slope():
    P = 9
    s, b, r, _ = _problem(P, 3)
    u = torch.rand(P, generator=torch.Generator().manual_seed(4), dtype=F64)
    sv = s.clone().requires_grad_(True)
    L = est.L_straight_through(sv, b, r, u)
    assert torch.equal(L.detach(), est.L_hard(s, b, r, u))
    gL = torch.randn(P, 3, dtype=F64)
    (g,) = torch.autograd.grad((L * gL).sum(), sv)
    assert torch.allclose(g, ((r - L.detach()) * gL).sum(1) / s, rtol=1e-12)   # dI/dp := 1


def test_gumbel_tends_to_hard_and_relaxed_to_hard():
    P = 64
    s, b, r, _ = _problem(P, 5)
    p = s - torch.floor(s)
    u = torch.rand(P, generator=torch.Generator().manual_seed(6), dtype=F64)
    keep = (u - p).abs() > 1e-3                         # away from the step
    hard = est.L_hard(s, b, r, u)
    assert torch.allclose(est.L_gumbel(s, b, r, u, 1e-4)[keep], hard[keep], rtol=1e-9, atol=1e-9)
    assert torch.allclose(est.L_relaxed(s, b, r, u, 1e7)[keep], hard[keep], rtol=1e-5, atol=1e-6)


def test_dasr_forward_and_surrogate_by_hand():
    s = torch.tensor([0.3, 0.7, 1.4, 2.6], dtype=F64, requires_grad=True)
    pool = torch.arange(4 * 3 * 3, dtype=F64).reshape(4, 3, 3)
    Lref = torch.full((4, 3), 10.0, dtype=F64)
    L = est.L_dasr(s, pool, Lref)
    exp = torch.stack([torch.zeros(3), pool[1, 0], pool[2, 0], pool[3].mean(0)])
    assert torch.equal(L.detach(), exp)
    (g,) = torch.autograd.grad(L.sum(), s)
    # s < 1/2: L_ref; otherwise (L_ref - L) / round(s), summed over RGB
    want = torch.tensor([30.0, (30.0 - float(pool[1, 0].sum())) / 1, (30.0 - float(pool[2, 0].sum())) / 1,
                         (30.0 - float(pool[3].mean(0).sum())) / 3], dtype=F64)
    assert torch.allclose(g, want, rtol=1e-12)
