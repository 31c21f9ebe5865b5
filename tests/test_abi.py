"""CPU checks of the C ABI: the library builds, loads, and exports every declared symbol."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aps.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(aps_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2602_08642_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2602_08642_amd import build
        build.build()
    return _lib.load()


def test_header_declares_entry_points():
    names = _declared()
    for must in ["aps_density_predict", "aps_sample_mask", "aps_scatter_samples", "aps_reproject",
                 "aps_upsample", "aps_denoise_pyramid", "aps_kernel_predict", "aps_normalize_density"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2602_08642_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    # every declared symbol has a binding signature, and vice versa
    assert set(_lib.SIGNATURES) == set(_declared())


def test_host_side_validation_without_gpu(lib):
    """Argument checks run on the host and return before any HIP call."""
    assert lib.aps_version() == 10000
    assert lib.aps_status_string(0) == b"ok"
    # NULL inputs
    assert lib.aps_sample_mask(None, 1, 4, 4, 0, 0, None, None, None, 0, None, None, None, 0, None, None) == 1
    # unsupported kernel size for packing
    assert lib.aps_conv_pack_weights(1, 4, 5, 4, 0, 1, None) == 3
    assert lib.aps_conv_packed_elems(16, 3, 32) == 4 * 9 * 1 * 512
    # pyramid sizes must divide by 2^(levels-1)
    arr = (__import__("ctypes").c_void_p * 5)(1, 1, 1, 1, 1)
    assert lib.aps_scatter_samples(1, 1, 1, 1, 10, 1, 6, 8, 3, 0, 10.0, 0, 0, arr, None) == 2
    # workspace too small
    assert lib.aps_normalize_density(1, 1, 8, 8, 0.25, 0.125, 1, 1, 1, None, None) == 4
    # relaxed mode needs lambda >= 1
    assert lib.aps_scatter_samples(1, 1, 1, 1, 10, 1, 8, 8, 1, 1, 0.5, 0, 0, arr, None) == 6
    # the no-allocation mask rejects problems beyond its static scratch (2^25 pixels) before
    # any HIP call
    assert lib.aps_sample_mask_noalloc(1, 5, 2160, 3840, 0, 0, None, 0, 0, 1, 1, 1, 10, 1, None,
                                       None, None) == 7
    assert lib.aps_status_string(7).startswith(b"problem larger")
