"""Pins of the oracle's RNG, density normalisation, mask, scatter and pyramid."""
import math
import os

import numpy as np
import pytest
import scipy.special
import torch

from oracle import density, philox, sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[0:4], v[4], v[5])
        assert [int(x) for x in out] == v[6:10]


def test_uniform24_exact_and_uniform():
    u = philox.uniform24(12345, np.arange(200000, dtype=np.uint64), 3)
    assert u.min() >= 0.0 and u.max() <= 1.0 - 2.0 ** -24
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))          # exact 24-bit values
    assert np.all(u.astype(np.float32).astype(np.float64) == u)   # exact in binary32
    hist = np.histogram(u, bins=20, range=(0, 1))[0]
    chi2 = ((hist - 10000.0) ** 2 / 10000.0).sum()
    assert chi2 < 50.0                                             # 19 dof; p < 1e-4
    u2 = philox.uniform24(12346, np.arange(10, dtype=np.uint64), 3)
    assert not np.array_equal(u[:10], u2)
    u3 = philox.uniform24(12345, np.arange(10, dtype=np.uint64), 4)
    assert not np.array_equal(u[:10], u3)


def test_uniform24_uses_the_four_words_of_a_block():
    """Pixels 4q .. 4q+3 take words 0..3 of the Philox block with counter (q, frame, 0, 0),
    the same block the KAT-pinned generator gives for that counter."""
    seed, frame = 0x0123456789ABCDEF, 7
    for q in (0, 1, 12345, 2 ** 29 + 3):
        words = philox.philox4x32_10(q, frame, 0, 0, seed & 0xFFFFFFFF, seed >> 32)
        for k in range(4):
            u = philox.uniform24(seed, np.array([4 * q + k], np.uint64), frame)[0]
            assert u == (int(words[k]) >> 8) * 2.0 ** -24


def test_conv_matches_library():
    g = torch.Generator().manual_seed(0)
    x = torch.randn(2, 9, 7, 5, generator=g, dtype=torch.float64)
    w = torch.randn(6, 3, 3, 5, generator=g, dtype=torch.float64)
    b = torch.randn(6, generator=g, dtype=torch.float64)
    ours = density.conv2d_nhwc(x, w, b)
    ref = torch.nn.functional.conv2d(x.permute(0, 3, 1, 2), w.permute(0, 3, 1, 2), b, padding=1)
    assert torch.allclose(ours, ref.permute(0, 2, 3, 1), rtol=1e-12, atol=1e-12)
    w1 = torch.randn(4, 1, 1, 5, generator=g, dtype=torch.float64)
    ours1 = density.conv2d_nhwc(x, w1, b[:4])
    ref1 = torch.nn.functional.conv2d(x.permute(0, 3, 1, 2), w1.permute(0, 3, 1, 2), b[:4])
    assert torch.allclose(ours1, ref1.permute(0, 2, 3, 1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("B", [0.25, 0.125, 1.5])
def test_normalise_budget(B):
    z = torch.randn(3, 16, 24, dtype=torch.float64) * 2.0
    s = density.normalise(z, B)
    npx = 16 * 24
    assert torch.allclose(s.sum(dim=(1, 2)), torch.full((3,), npx * B, dtype=torch.float64), rtol=1e-12)
    assert (s >= B / 8 * (1 - 1e-15)).all()
    sm = scipy.special.softmax(z.numpy().reshape(3, -1), axis=1).reshape(3, 16, 24)
    assert np.allclose(s.numpy(), B / 8 + 7 * B / 8 * npx * sm, rtol=1e-13)
    # a constant logit map gives the uniform density B
    assert torch.allclose(density.normalise(torch.zeros(1, 4, 4, dtype=torch.float64), B),
                          torch.full((1, 4, 4), B, dtype=torch.float64))


def _tiny_s(seed=0, shape=(2, 5, 7)):
    rng = np.random.default_rng(seed)
    s = rng.exponential(0.6, shape).astype(np.float32)
    s.flat[::5] = np.maximum(np.round(s.flat[::5]), 1.0)   # some exact integers (p = 0)
    s.flat[1] = 0.0                                        # a zero density: no sample, L = 0
    return s


def test_mask_brute_force():
    s = _tiny_s()
    N, H, W = s.shape
    r = sampling.mask(s, seed=99, frame=2)
    cnt = np.zeros_like(s, dtype=np.int64)
    for n in range(N):
        for y in range(H):
            for x in range(W):
                pix = n * H * W + y * W + x
                sv = float(s[n, y, x])
                fl = math.floor(sv)
                u = philox.uniform24(99, np.array([pix], np.uint64), 2)[0]
                cnt[n, y, x] = fl + (1 if u < sv - fl else 0)
    assert np.array_equal(r["count"].astype(np.int64), cnt)
    assert r["total"] == cnt.sum()
    assert np.array_equal(r["sample_pixel"], np.repeat(np.arange(cnt.size), cnt.reshape(-1)))
    # integer densities never add the extra sample
    ints = s == np.floor(s)
    assert np.array_equal(r["count"][ints].astype(np.float32), s[ints])


def test_mask_block_offsets_and_reproducible():
    s = np.full((1, 40, 33), 0.7, np.float32)
    r1 = sampling.mask(s, seed=5, frame=0)
    r2 = sampling.mask(s, seed=5, frame=0)
    assert np.array_equal(r1["count"], r2["count"])
    flat = r1["count"].reshape(-1).astype(np.int64)
    for b in range(len(r1["block_offset"]) - 1):
        assert r1["block_offset"][b] == flat[: b * 256].sum()
    assert r1["block_offset"][-1] == r1["total"]
    r3 = sampling.mask(s, seed=6, frame=0)
    assert not np.array_equal(r1["count"], r3["count"])


def test_mask_expected_count_equals_budget():
    rng = np.random.default_rng(1)
    z = torch.tensor(rng.normal(size=(1, 32, 32)) * 1.5)
    B = 0.25
    s = density.normalise(z, B).numpy().astype(np.float32)
    totals = np.array([sampling.mask(s, seed=k, frame=0)["total"] for k in range(256)])
    p = s - np.floor(s)
    expect = float(s.astype(np.float64).sum())
    sigma = math.sqrt((p * (1 - p)).sum() / 256)
    assert abs(expect - 32 * 32 * B) < 1e-3
    assert abs(totals.mean() - expect) < 4 * sigma


def test_ramp_expectation_closed_form():
    """E_u[h * ramp] = p (eq. h_factor) and E_u[(h*ramp)^2] = h^2 p (1 - 2/(3 lambda))."""
    u = (np.arange(2_000_000) + 0.5) / 2_000_000
    for lam in (1.0, 4.0, 10.0):
        h = sampling.h_factor(lam)
        for p in (0.05, 0.3, 0.9):
            r = sampling.relaxed_ramp(np.full_like(u, p), u, lam).numpy()
            assert abs((h * r).mean() - p) < 2e-6
            assert abs(((h * r) ** 2).mean() - h * h * p * (1 - 2 / (3 * lam))) < 2e-6
    # a steep ramp is the hard step away from the threshold
    p = np.full(1000, 0.4)
    uu = np.linspace(0, 1, 1000)
    r = sampling.relaxed_ramp(p, uu, 1e9).numpy()
    far = np.abs(uu - 0.4) > 1e-6
    assert np.array_equal(r[far] > 0.5, (uu < p)[far])


def _samples_for(r, value_fn):
    return np.stack([value_fn(int(pix), j) for pix, j in
                     zip(r["sample_pixel"], _local_index(r))]) if r["total"] else np.zeros((0, 4))


def _local_index(r):
    cnt = r["count"].reshape(-1).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    return np.arange(r["total"]) - start[r["sample_pixel"]]


def test_scatter_brute_force_and_constant():
    s = _tiny_s(3)
    N, H, W = s.shape
    seed, frame, lam = 7, 1, 10.0
    r = sampling.mask(s, seed, frame)
    rng = np.random.default_rng(2)
    smp = rng.normal(size=(r["total"], 4))
    smp[:, 3] = 0
    for mode in ("hard", "relaxed"):
        L = sampling.scatter(s.astype(np.float64), r["count"], smp, seed, frame, mode, lam).numpy()
        # literal per-pixel loop
        k = 0
        for pix in range(N * H * W):
            sv = float(s.reshape(-1)[pix])
            fl = math.floor(sv)
            c = int(r["count"].reshape(-1)[pix])
            acc = np.zeros(3)
            for j in range(c):
                if j < fl:
                    acc += smp[k + j, :3]
                else:
                    p = sv - fl
                    u = philox.uniform24(seed, np.array([pix], np.uint64), frame)[0]
                    wgt = 1.0 if mode == "hard" else (2 * lam / (2 * lam - 1)) * min(max(lam * (p - u) / p, 0.0), 1.0)
                    acc += wgt * smp[k + j, :3]
            k += c
            n, rem = divmod(pix, H * W)
            y, x = divmod(rem, W)
            want = acc / sv if sv > 0 else np.zeros(3)
            assert np.allclose(L[n, y, x, :3], want, rtol=1e-12, atol=1e-12)
            assert L[n, y, x, 3] == 0
    # integer densities and constant samples reproduce the constant exactly
    si = np.full((1, 4, 4), 2.0, np.float32)
    ri = sampling.mask(si, 0, 0)
    Lc = sampling.scatter(si.astype(np.float64), ri["count"], np.full((ri["total"], 4), 3.0), 0, 0)
    assert torch.all(Lc[..., :3] == 3.0)


def test_scatter_unbiased_monte_carlo():
    """E_u[L_noisy] = E[sample] (Sec. 4.2): constant samples c give mean c over seeds."""
    s = np.array([[[0.1, 0.3, 0.55, 1.25, 2.7, 0.02]]], np.float32)
    c = 2.0
    for mode in ("hard", "relaxed"):
        acc = np.zeros(s.shape)
        n = 4000
        for seed in range(n):
            r = sampling.mask(s, seed, 0)
            L = sampling.scatter(s.astype(np.float64), r["count"], np.full((r["total"], 4), c), seed, 0, mode)
            acc += L[..., 0].numpy()
        mean = acc / n
        p = s - np.floor(s)
        # per-pixel variance of L = c^2 * Var[holdout weight] / s^2
        sd = c * np.sqrt(p * (1 - p) * (1.04 if mode == "relaxed" else 1.0) + 1e-12) / s / math.sqrt(n)
        assert np.all(np.abs(mean - c) < 5 * sd + 1e-12), (mode, mean)


def test_pyramid_matches_avg_pool():
    x = torch.randn(2, 16, 24, 4, dtype=torch.float64)
    pyr = sampling.pyramid(x, 4)
    for l in range(4):
        ref = torch.nn.functional.avg_pool2d(x.permute(0, 3, 1, 2), 2 ** l).permute(0, 2, 3, 1)
        assert torch.allclose(pyr[l], ref, rtol=1e-13, atol=1e-14)
    c = torch.full((1, 8, 8, 4), 1.7, dtype=torch.float64)
    assert all(torch.allclose(p, torch.full_like(p, 1.7)) for p in sampling.pyramid(c, 3))


# ------------------------------------------------------------------ blue-noise u

def test_blue_noise_texture_properties():
    import procgen
    T = 64
    r = procgen.void_and_cluster(T)
    assert sorted(r.ravel().tolist()) == list(range(T * T))
    u = procgen.blue_noise_thresholds(T)
    assert np.array_equal(u.astype(np.float64), (r + 0.5) / (T * T))     # exact in binary32
    # blue: the lowest frequencies carry almost no power (white noise: about 1/12 * T^2 each)
    F = np.abs(np.fft.fft2(u - u.mean())) ** 2
    low = [(0, 1), (1, 0), (1, 1), (0, 2), (2, 0), (1, 2), (2, 1), (2, 2)]
    assert sum(F[a, b] for a, b in low) < 1e-3 * len(low) * T * T / 12
    # well spread: the sparsest 1/16 of the thresholds keeps every pair >= 2 px apart (torus)
    pts = np.argwhere(r < T * T // 16)
    d = np.abs(pts[:, None, :] - pts[None, :, :])
    d = np.minimum(d, T - d)
    dist = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(dist, 99)
    assert dist.min() >= 2.0


def test_mask_texture_stratification():
    """For constant p every T x T window of u holds each threshold once, so it takes exactly
    ceil(p T^2 - 1/2) holdouts: the blue-noise mask is stratified, not just unbiased."""
    import procgen
    T = 16
    tex = procgen.blue_noise_thresholds(T, seed=3)
    N, H, W = 2, 40, 52
    for k, p in ((0, 0.25), (1, 0.3), (2, 0.8125)):
        s = np.full((N, H, W), k + p, np.float32)
        m = sampling.mask(s, 99, 5, u_tex=tex)
        c = m["count"].astype(np.int64)
        want = T * T * k + math.ceil(p * T * T - 0.5)
        for n in range(N):
            for y0, x0 in ((0, 0), (3, 7), (H - T, W - T), (11, 30)):
                assert int(c[n, y0:y0 + T, x0:x0 + T].sum()) == want


def test_mask_texture_lookup_orientation():
    """Rows of u are rows of the texture, cyclically shifted: a transposed or mirrored lookup
    fails; offsets change with the frame and the image."""
    import procgen
    T = 16
    tex = procgen.blue_noise_thresholds(T, seed=4).astype(np.float64)
    u = sampling.u_values(2, 24, 40, 7, 9, tex)
    for n in range(2):
        shifts = []
        for y in range(24):
            row = u[n, y, :T]
            hits = [(ty, sh) for ty in range(T) for sh in range(T) if np.array_equal(np.roll(tex[ty], -sh), row)]
            assert len(hits) == 1
            shifts.append(hits[0])
        oy, ox = shifts[0]
        assert all(h == ((oy + y) % T, ox) for y, h in enumerate(shifts))
        # x continues past the tile: column T + x repeats column x
        assert np.array_equal(u[n, :, T:2 * T], u[n, :, :T])
    offs = {sampling.tex_offsets(7, n, f, T) for n in range(2) for f in range(16)}
    assert len(offs) >= 20


def test_scatter_texture_relaxed_limit_is_hard():
    """With texture u the relaxed holdout weight is h * ramp with the same u: as lambda grows it
    tends to the hard holdout of the mask drawn from that u."""
    import procgen
    T = 16
    tex = procgen.blue_noise_thresholds(T, seed=5)
    rng = np.random.default_rng(3)
    N, H, W = 1, 20, 24
    s = (rng.random((N, H, W)) * 2.5 + 0.05).astype(np.float32)
    m = sampling.mask(s, 21, 2, u_tex=tex)
    smp = rng.normal(1.0, 0.5, (m["total"], 4))
    hard = sampling.scatter(s.astype(np.float64), m["count"], smp, 21, 2, "hard", u_tex=tex)
    rel = sampling.scatter(s.astype(np.float64), m["count"], smp, 21, 2, "relaxed", 1e7, u_tex=tex)
    assert torch.allclose(rel, hard, rtol=1e-5, atol=1e-6)
    # and the Philox u would have given another mask
    assert not np.array_equal(sampling.mask(s, 21, 2)["count"], m["count"])


def test_mask_rounding_variants():
    s = np.array([[[0.0, 0.3, 0.5, 0.75, 1.0, 1.49999, 1.5, 2.2, 3.999]]], np.float32)
    m_h = sampling.mask(s, 1, 0, rounding="holdout")["count"][0, 0].tolist()
    m_d = sampling.mask(s, 1, 0, rounding="deterministic")["count"][0, 0].tolist()
    assert m_h == [0, 1, 1, 1, 1, 2, 2, 3, 4]                 # floor(s) + [p > 0]
    assert m_d == [0, 0, 1, 1, 1, 1, 2, 2, 4]                 # round half up: floor(s + 1/2)
    st = sampling.mask(s, 1, 0)
    fl = np.floor(s.astype(np.float64))
    assert np.array_equal(st["count"], (fl + (st["u"] < s - fl)).astype(np.uint8))
