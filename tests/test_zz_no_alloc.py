"""The no-allocation mask entry point (aps_sample_mask_noalloc, static device scratch) against
the workspace entry point aps_sample_mask_ex on the same inputs: counts, offsets, the sample
list, the total and p bit for bit, on two calls in a row (the second smaller, ragged, with
the blue-noise texture and the holdout rounding), then a third with the first's shape."""
import ctypes as C

import numpy as np
import pytest
import torch

import procgen

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


def _density(N, H, W, seed):
    g = torch.Generator().manual_seed(seed)
    s = torch.rand(N, H, W, generator=g) * 3.0
    s.view(-1)[::97] = torch.floor(s.view(-1)[::97])     # integer densities never add a sample
    s.view(-1)[5::211] = 0.0
    return s.to(DEV)


def _noalloc_via_abi(ops, s, seed, frame, u_tex, rounding, capacity):
    """The raw C-ABI call (ctypes), outputs allocated here."""
    from paper_2602_08642_amd import _lib
    N, H, W = s.shape
    count = torch.empty((N, H, W), dtype=torch.uint8, device=DEV)
    poff = torch.empty((N, H, W), dtype=torch.int32, device=DEV)
    spix = torch.empty(capacity, dtype=torch.int32, device=DEV)
    total = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    p = torch.empty_like(s)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    tp = ptr(u_tex) if u_tex is not None else None
    T = u_tex.shape[0] if u_tex is not None else 0
    rc = _lib.load().aps_sample_mask_noalloc(
        ptr(s), N, H, W, seed, frame, tp, T, rounding, ptr(count), ptr(poff), ptr(spix), capacity,
        ptr(total), ptr(p), ptr(status), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, _lib.load().aps_status_string(rc)
    return dict(count=count, pixel_offset=poff, sample_pixel=spix, total=total, p=p, status=status)


def _compare(ops, s, seed, frame, u_tex=None, rounding="stochastic"):
    from paper_2602_08642_amd import _lib
    N, H, W = s.shape
    cap = 2 * N * H * W
    rmode = {"stochastic": _lib.APS_ROUND_STOCHASTIC, "holdout": _lib.APS_ROUND_HOLDOUT}[rounding]
    got = _noalloc_via_abi(ops, s, seed, frame, u_tex, rmode, cap)
    ref = ops.sample_mask(s, seed, frame, capacity=cap, want_p=True, u_tex=u_tex, rounding=rounding)
    torch.cuda.synchronize()
    total = int(ref["total"].item())
    assert int(got["total"].item()) == total
    assert total > 0
    for k in ("count", "pixel_offset", "p"):
        assert torch.equal(got[k], ref[k]), k
    assert torch.equal(got["sample_pixel"][:total], ref["sample_pixel"][:total])
    assert int(got["status"].item()) == 0
    return total


def test_noalloc_mask_matches_workspace_mask(ops):
    # 1: two 540x960 images (Philox u, stochastic rounding)
    t1 = _compare(ops, _density(2, 540, 960, 1), seed=9, frame=3)
    # 2: smaller and ragged (97 x 133, not a multiple of the 256-pixel blocks), blue-noise u,
    #    the holdout always requested; the static array still holds the first call's sums
    tex = torch.tensor(procgen.blue_noise_thresholds(64), device=DEV)
    t2 = _compare(ops, _density(1, 97, 133, 2), seed=10, frame=4, u_tex=tex, rounding="holdout")
    # 3: the first shape again, other densities
    t3 = _compare(ops, _density(2, 540, 960, 3), seed=11, frame=5)
    assert t2 < t1 and t3 > t2


def test_noalloc_mask_ops_binding_and_empty(ops):
    s = _density(1, 64, 80, 4)
    a = ops.sample_mask_noalloc(s, 3, 1, want_p=True)
    b = ops.sample_mask(s, 3, 1, want_p=True)
    torch.cuda.synchronize()
    n = int(b["total"].item())
    assert int(a["total"].item()) == n
    assert torch.equal(a["count"], b["count"]) and torch.equal(a["p"], b["p"])
    assert torch.equal(a["sample_pixel"][:n], b["sample_pixel"][:n])
    e = ops.sample_mask_noalloc(torch.empty((0, 8, 8), dtype=torch.float32, device=DEV), 3, 1)
    assert int(e["total"].item()) == 0
