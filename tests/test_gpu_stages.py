"""Stage-wise parity of the HIP path (through the C ABI) against the FP64 oracle.

Every stage consumes the same inputs on both sides; the oracle takes the GPU's float32
inputs of that stage, widened exactly to float64.
"""
import math
import zlib

import numpy as np
import pytest
import torch

import procgen
from oracle import density as odens
from oracle import filt as ofilt
from oracle import sampling as osamp
from tests._tol import assert_mag_close, rel_norm, to_np

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2602_08642_amd import ops as o
    return o


def _s_map(N, H, W, B, seed, scale=1.5):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(N, H, W)) * scale
    s = odens.normalise(torch.tensor(z), B).numpy().astype(np.float32)
    return s


# ------------------------------------------------------------------ a2 normalisation

@pytest.mark.parametrize("shape,B", [((1, 128, 128), 0.25), ((2, 45, 67), 0.125), ((1, 1080, 1920), 0.25)])
def test_normalize_matches_oracle(ops, shape, B):
    rng = np.random.default_rng(1)
    z = (rng.normal(size=shape) * 2.0).astype(np.float32)
    s = ops.normalize_density(torch.tensor(z, device=DEV), B)
    ref = odens.normalise(torch.tensor(z, dtype=torch.float64), B)
    assert_mag_close(s, ref, ref, 1e-5, what="normalise")
    npx = shape[1] * shape[2]
    sums = to_np(s).reshape(shape[0], -1).sum(1)
    assert np.allclose(sums, npx * B, rtol=1e-5)
    s2 = ops.normalize_density(torch.tensor(z, device=DEV), B)
    assert torch.equal(s, s2)                                  # deterministic


# ------------------------------------------------------------------ a3 mask, bit-exact

def _check_mask(ops, s, seed, frame):
    cap = int(np.floor(s.astype(np.float64)).sum()) + s.size + 16
    r = ops.sample_mask(torch.tensor(s, device=DEV), seed, frame, capacity=cap, want_p=True)
    o = osamp.mask(s, seed, frame)
    assert np.array_equal(r["count"].cpu().numpy(), o["count"])
    total = int(r["total"].item())
    assert total == o["total"]
    assert np.array_equal(r["sample_pixel"][:total].cpu().numpy().astype(np.int64), o["sample_pixel"])
    cnt = o["count"].reshape(-1).astype(np.int64)
    excl = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    assert np.array_equal(r["pixel_offset"].cpu().numpy().reshape(-1), excl)
    assert np.array_equal(r["p"].cpu().numpy().astype(np.float64), o["p"])
    return r


@pytest.mark.parametrize("shape", [(1, 128, 128), (2, 37, 53), (1, 1080, 1920)])
def test_mask_bit_exact(ops, shape):
    s = _s_map(*shape, 0.25, seed=3)
    s.flat[::97] = np.floor(s.flat[::97]) + 1.0       # exact integers: p = 0
    s.flat[5] = 0.0
    s.flat[7] = 3.999999761581421                       # just below an integer
    s.flat[11] = 7.5
    _check_mask(ops, s, seed=0x1234_5678_9ABC, frame=5)


def test_mask_reproducible_and_seeded(ops):
    s = torch.tensor(_s_map(1, 64, 96, 0.25, seed=4), device=DEV)
    a = ops.sample_mask(s, 7, 0)
    b = ops.sample_mask(s, 7, 0)
    c = ops.sample_mask(s, 8, 0)
    n = int(a["total"].item())
    assert n == int(b["total"].item())
    assert torch.equal(a["count"], b["count"])
    assert torch.equal(a["sample_pixel"][:n], b["sample_pixel"][:n])
    assert torch.equal(a["pixel_offset"], b["pixel_offset"])
    assert not torch.equal(a["count"], c["count"])


def test_mask_fixed_p_u_edge_cases(ops):
    # p exactly representable; u values cover [0, 1); strict < at every threshold
    s = np.array([[[0.0, 0.5, 1.0, 1.5, 2.0 ** -24, 1 - 2.0 ** -24, 254.0, 254.5]]], np.float32)
    _check_mask(ops, s, seed=99, frame=1)


def test_mask_capacity_and_status(ops):
    s = torch.full((1, 16, 16), 1.5, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    r = ops.sample_mask(s, 1, 0, capacity=100, status=st)
    torch.cuda.synchronize()
    assert int(r["total"].item()) > 100
    assert int(st.item()) & 4
    s2 = torch.full((1, 4, 4), 300.0, device=DEV)
    st.zero_()
    r2 = ops.sample_mask(s2, 1, 0, capacity=16 * 256, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) & 1
    assert int(r2["count"].max().item()) == 255


def test_mask_empty(ops):
    r = ops.sample_mask(torch.zeros((0, 8, 8), device=DEV), 1, 0, capacity=0)
    assert int(r["total"].item()) == 0
    L = ops.scatter_samples(torch.zeros((0, 8, 8), device=DEV), r["count"], r["pixel_offset"],
                            torch.zeros((1, 4), device=DEV), 2)
    assert L[0].shape == (0, 8, 8, 4)


def test_expected_count_is_budget(ops):
    s = torch.tensor(_s_map(1, 256, 256, 0.25, seed=9), device=DEV)
    tot = np.array([int(ops.sample_mask(s, k, 0)["total"].item()) for k in range(64)])
    sn = to_np(s)
    p = sn - np.floor(sn)
    sigma = math.sqrt((p * (1 - p)).sum() / 64)
    assert abs(tot.mean() - sn.sum()) < 4 * sigma
    assert abs(sn.sum() - 256 * 256 * 0.25) < 1.0


# ------------------------------------------------------------------ a4 scatter + pyramid

def _scatter_case(ops, N, H, W, levels, mode, seed=5, frame=2):
    s = _s_map(N, H, W, 0.25, seed=seed, scale=2.0)
    truth = np.stack([procgen.render_view(procgen.make_scene(seed + n, H, W))[0] for n in range(N)])
    pool = np.stack([procgen.sample_pool(truth[n], seed, frame, 8) for n in range(N)]).reshape(N * H * W, 8, 4)
    st = torch.tensor(s, device=DEV)
    r = ops.sample_mask(st, seed, frame)
    cap = r["capacity"]
    smp = ops.fixture_render(torch.tensor(pool, device=DEV), r["count"], r["pixel_offset"], cap)
    total = int(r["total"].item())
    # the renderer stand-in hands out pool[i][j mod J] in request order
    cnt = r["count"].cpu().numpy().reshape(-1).astype(np.int64)
    pix = np.repeat(np.arange(cnt.size), cnt)
    j = np.arange(total) - np.concatenate([[0], np.cumsum(cnt)[:-1]])[pix]
    assert np.array_equal(smp[:total].cpu().numpy(), pool[pix, j % 8])
    Ls = ops.scatter_samples(st, r["count"], r["pixel_offset"], smp, levels, mode, 10.0, seed, frame)
    smp_np = smp[:total].cpu().numpy()
    ref0 = osamp.scatter(s.astype(np.float64), r["count"].cpu().numpy(), smp_np, seed, frame, mode, 10.0)
    mag0 = osamp.scatter(s.astype(np.float64), r["count"].cpu().numpy(), np.abs(smp_np), seed, frame, mode, 10.0)
    refs = osamp.pyramid(ref0, levels)
    mags = osamp.pyramid(mag0, levels)
    for l in range(levels):
        assert_mag_close(Ls[l], refs[l], mags[l], 1e-5, what=f"{mode} level {l}")


@pytest.mark.parametrize("mode", ["hard", "relaxed"])
def test_scatter_pyramid_c1(ops, mode):
    _scatter_case(ops, 1, 128, 128, 1, mode)


@pytest.mark.parametrize("mode", ["hard", "relaxed"])
def test_scatter_pyramid_ragged(ops, mode):
    _scatter_case(ops, 2, 72, 40, 3, mode)          # 16x16 tiles, ragged in y and x


def test_scatter_pyramid_1080p(ops):
    _scatter_case(ops, 1, 1080, 1920, 3, "hard")


# ------------------------------------------------------------------ a6-a9 reconstruction

def _rand_inputs(N, H, W, levels, KD, KU, KT, temporal, seed, ldtype):
    g = torch.Generator().manual_seed(seed)
    Ls = [torch.randn(N, H >> l, W >> l, 4, generator=g) * 2.0 for l in range(levels)]
    for t in Ls:
        t[..., 3] = 0
    Ks = procgen.kernel_channels(levels, KD, KU, KT, temporal)
    logits = []
    from paper_2602_08642_amd.ops import round_kstride
    for l in range(levels):
        ks = round_kstride(Ks[l], ldtype)
        z = torch.randn(N, H >> l, W >> l, ks, generator=g) * 2.0
        z[..., Ks[l]:] = 0.0
        logits.append(z.to(ldtype))
    prev = mv = None
    if temporal:
        prev = torch.randn(N, H, W, 4, generator=g)
        prev[..., 3] = 0
        mv = (torch.rand(N, H, W, 2, generator=g) * 16 - 8)
        mv[0, :3, :3] = torch.tensor([-0.25, 0.75])   # negative fractional parts
    return Ls, logits, prev, mv


@pytest.mark.parametrize("cfg", [
    # (N, H, W, levels, KD, KU, KT, temporal, logit dtype)
    (1, 128, 128, 1, 5, 3, 3, False, torch.float32),
    (1, 72, 80, 3, 5, 3, 3, False, torch.float32),
    (2, 64, 96, 3, 5, 3, 3, True, torch.float32),
    (1, 64, 96, 3, 5, 3, 3, True, torch.bfloat16),
    (1, 48, 80, 4, 7, 3, 3, True, torch.float32),
    (1, 48, 80, 4, 7, 3, 3, True, torch.bfloat16),    # C5's level kernels: bf16 logits, 67-way softmax
    (1, 48, 64, 4, 5, 2, 5, True, torch.float32),
    (1, 40, 56, 2, 3, 3, 3, True, torch.bfloat16),
])
def test_denoise_pyramid_matches_oracle(ops, cfg):
    N, H, W, levels, KD, KU, KT, temporal, ldt = cfg
    Ls, logits, prev, mv = _rand_inputs(N, H, W, levels, KD, KU, KT, temporal, 11, ldt)
    out = ops.denoise_pyramid([t.to(DEV) for t in Ls], [t.to(DEV) for t in logits], KD, KU, KT,
                              prev.to(DEV) if temporal else None, mv.to(DEV) if temporal else None)
    L64 = [t.double() for t in Ls]
    z64 = [t.double() for t in logits]
    p64 = prev.double() if temporal else None
    m64 = mv.double() if temporal else None
    ref = ofilt.denoise_pyramid(L64, z64, KD, KU, KT, p64, m64)[0]
    mag = ofilt.denoise_magnitude(L64, z64, KD, KU, KT, p64, m64)[0]
    assert_mag_close(out[..., :3], ref[..., :3], mag[..., :3], 1e-5, what=str(cfg))
    assert torch.all(out[..., 3] == 0)


def test_denoise_pyramid_1080p_c2(ops):
    Ls, logits, _, _ = _rand_inputs(1, 1080, 1920, 3, 5, 3, 3, False, 12, torch.float32)
    out = ops.denoise_pyramid([t.to(DEV) for t in Ls], [t.to(DEV) for t in logits], 5, 3, 3)
    # sampled rows (top, bottom, interior) through the full oracle on row bands
    L64 = [t.double() for t in Ls]
    z64 = [t.double() for t in logits]
    ref = ofilt.denoise_pyramid(L64, z64, 5, 3, 3)[0]
    mag = ofilt.denoise_magnitude(L64, z64, 5, 3, 3)[0]
    assert_mag_close(out[..., :3], ref[..., :3], mag[..., :3], 1e-5, what="1080p")


def test_filter_invariants(ops):
    """Constant image preserved; one-hot centre logits pass data through bit-exactly."""
    N, H, W, levels, KD, KU, KT = 1, 64, 64, 3, 5, 3, 3
    Ls, logits, prev, mv = _rand_inputs(N, H, W, levels, KD, KU, KT, True, 13, torch.float32)
    const = [torch.full_like(t, 1.75) for t in Ls]
    for t in const:
        t[..., 3] = 0
    pc = torch.full_like(prev, 1.75)
    pc[..., 3] = 0
    out = ops.denoise_pyramid([t.to(DEV) for t in const], [t.to(DEV) for t in logits], KD, KU, KT,
                              pc.to(DEV), mv.to(DEV))
    assert torch.allclose(out[..., :3].cpu(), torch.full((N, H, W, 3), 1.75), rtol=2e-6)
    Ks = procgen.kernel_channels(levels, KD, KU, KT, False)
    onehot = []
    for l in range(levels):
        z = torch.full((N, H >> l, W >> l, (Ks[l] + 3) // 4 * 4), -1e30)
        z[..., 12] = 0.0
        onehot.append(z.to(DEV))
    out = ops.denoise_pyramid([t.to(DEV) for t in Ls], onehot, KD, KU, KT)
    assert torch.equal(out.cpu(), Ls[0])


def test_reproject_and_upsample_entry_points(ops):
    N, H, W, KD, KU, KT = 1, 48, 64, 5, 3, 3
    Ls, logits, prev, mv = _rand_inputs(N, H, W, 2, KD, KU, KT, True, 14, torch.float32)
    z0 = logits[0]
    T = ops.reproject(prev.to(DEV), mv.to(DEV), z0.to(DEV), KD, KU, KT, True)
    U = ops.upsample(Ls[1].to(DEV), z0.to(DEV), KD, KU, KT, True)
    w = ofilt.joint_softmax(z0.double(), [25, 9, 9])
    refT = ofilt.gather(ofilt.warp(prev.double(), mv.double()), w[2], KT)
    magT = ofilt.gather(ofilt.warp(prev.double().abs(), mv.double()), w[2], KT)
    refU = ofilt.upsample(Ls[1].double(), w[1], KU, H, W)
    magU = ofilt.upsample(Ls[1].double().abs(), w[1], KU, H, W)
    assert_mag_close(T[..., :3], refT[..., :3], magT[..., :3], 1e-5, what="reproject")
    assert_mag_close(U[..., :3], refU[..., :3], magU[..., :3], 1e-5, what="upsample")


# ------------------------------------------------------------------ a1/a5 convolutions

def _conv_ref(x, w, b, relu):
    y = odens.conv2d_nhwc(x, w, b)
    mag = odens.conv2d_nhwc(x.abs(), w.abs(), b.abs())
    return (torch.relu(y) if relu else y), mag


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("cfg", [
    # (mode, N, H, W, Cx, C2, Cout, k)
    ("direct", 1, 37, 45, 8, 0, 16, 3),
    ("direct", 2, 32, 48, 16, 0, 32, 3),
    ("direct", 1, 20, 36, 32, 0, 1, 3),
    ("direct", 1, 24, 40, 64, 0, 25, 3),
    ("direct", 1, 16, 32, 128, 0, 256, 3),
    ("pool2", 1, 18, 20, 32, 0, 64, 3),
    ("up2cat", 1, 24, 40, 64, 32, 32, 3),
    ("up2cat", 1, 16, 16, 256, 128, 128, 3),
    ("direct", 1, 36, 44, 32, 0, 34, 1),
    ("direct", 1, 18, 22, 256, 0, 49, 1),
])
def test_conv_matches_oracle(ops, cfg, dtype):
    mode, N, H, W, Cx, C2, Cout, k = cfg
    g = torch.Generator().manual_seed(zlib.crc32(repr(cfg).encode()))
    if mode == "pool2":
        x = torch.randn(N, 2 * H, 2 * W, Cx, generator=g)
        xin = x.double().reshape(N, H, 2, W, 2, Cx).mean(dim=(2, 4))
        x2 = None
    elif mode == "up2cat":
        x = torch.randn(N, H // 2, W // 2, Cx, generator=g)
        x2 = torch.randn(N, H, W, C2, generator=g)
        xin = torch.cat([x.double().repeat_interleave(2, 1).repeat_interleave(2, 2), x2.double()], -1)
    else:
        x = torch.randn(N, H, W, Cx, generator=g)
        xin = x.double()
        x2 = None
    cin = Cx + C2
    w = torch.randn(Cout, k, k, cin, generator=g) / math.sqrt(k * k * cin)
    b = torch.randn(Cout, generator=g) * 0.1
    spec = dict(name="l", cin=cin, cout=Cout, k=k, relu=True)
    net = ops.Net([spec], {"l": (w.numpy(), b.numpy())}, dtype=dtype, device=DEV)
    _, pk, bias = net.layer("l")
    xd = x.to(DEV).to(dtype)
    x2d = x2.to(DEV).to(dtype) if x2 is not None else None
    ldy = (Cout + 3) // 4 * 4 if Cout > 1 else 1
    y = ops.conv2d(xd, spec, pk, bias, mode, x2d, out_dtype=torch.float32, ldy=ldy) if dtype == torch.bfloat16 \
        else ops.conv2d(xd, spec, pk, bias, mode, x2d, ldy=ldy)
    ref, mag = _conv_ref(xin, w.double(), b.double(), True)
    tol = 1e-5 if dtype == torch.float32 else 2e-2
    assert_mag_close(y[..., :Cout], ref, mag, tol, what=f"{cfg} {dtype}")
    if ldy > Cout:
        assert torch.all(y[..., Cout:] == 0)


@pytest.mark.parametrize("shape", [(1, 2160, 3840), (2, 2160, 3840)])
def test_mask_offsets_at_4k(ops, shape):
    """The scan of the per-block counts at 4K: one frame (32 block sums per scan thread, the
    register path) and two frames (64 per thread, the loop path).  pixel_offset is the exclusive
    prefix sum of the counts, total their sum, and the compacted pixel list names each pixel as
    often as its count, in order."""
    g = torch.Generator(device="cuda").manual_seed(11)
    s = (torch.rand(shape, generator=g, device="cuda") * 0.5).contiguous()
    r = ops.sample_mask(s, seed=77, frame=3)
    cnt = r["count"].reshape(-1).to(torch.int64)
    incl = torch.cumsum(cnt, 0)
    assert int(r["total"].item()) == int(incl[-1].item())
    assert torch.equal(r["pixel_offset"].reshape(-1).to(torch.int64), incl - cnt)
    total = int(r["total"].item())
    want = torch.repeat_interleave(torch.arange(cnt.numel(), device="cuda"), cnt)
    assert torch.equal(r["sample_pixel"][:total].to(torch.int64), want)
