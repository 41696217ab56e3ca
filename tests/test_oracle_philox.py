"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11) and of the
uniform action draw that random playouts use (Sec. 6 random policy).

Pins: the known-answer vectors published with the Random123 library by the
authors of Philox; rocRAND's independent host implementation; and
uniformity of the multiply-shift reduction.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ref

# Known-answer vectors for Philox4x32 with 10 rounds, as distributed with
# Random123 (the reference implementation of Salmon et al., SC'11):
# (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    assert tuple(int(x) for x in ref.philox(ctr, key)) == out


def _rocrand_pin(tmp_path_factory):
    gxx = shutil.which("g++")
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if gxx is None or not os.path.exists(hdr):
        pytest.skip("rocRAND headers or g++ not available")
    d = tmp_path_factory.mktemp("rocrand_pin")
    so = str(d / "pin.so")
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_pin.cpp")
    subprocess.check_call([gxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-fPIC",
                           "-shared", "-o", so, src])
    L = ctypes.CDLL(so)
    L.pin_philox.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
    L.pin_philox.restype = None
    return L


def test_philox_matches_rocrand(tmp_path_factory):
    """rocRAND keys with the seed and puts (offset/4) in counter words 0-1
    and the subsequence in words 2-3.  The playout counter is
    (ply/4, game_id lo, game_id hi, 0), i.e. offset/4 = ply/4 + (gid_lo << 32)
    and subsequence = gid_hi."""
    L = _rocrand_pin(tmp_path_factory)
    rng = np.random.default_rng(7)
    out = np.zeros(4, np.uint32)
    for _ in range(300):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        gid = int(rng.integers(0, 2**30)) | (int(rng.integers(0, 2**31)) << 32)
        ply = int(rng.integers(0, 400))
        gid_lo, gid_hi = gid & 0xFFFFFFFF, gid >> 32
        L.pin_philox(seed, gid_hi, 4 * ((ply >> 2) | (gid_lo << 32)),
                     out.ctypes.data_as(ctypes.c_void_p))
        key = (seed & 0xFFFFFFFF, seed >> 32)
        mine = ref.philox((ply >> 2, gid_lo, gid_hi, 0), key)
        assert list(out) == list(mine)
        assert ref.draw(seed, gid, ply) == int(out[ply & 3])


def test_draw_is_uniform():
    """Chi-square of the 32-bit words reduced to [0, n) by multiply-shift."""
    n_bins = 7
    counts = np.zeros(n_bins, np.int64)
    total = 0
    for gid in range(2000):
        for ply in range(40):
            w = ref.draw(12345, gid, ply)
            counts[(w * n_bins) >> 32] += 1
            total += 1
    exp = total / n_bins
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 6 degrees of freedom: P(chi2 > 22.46) = 0.001
    assert chi2 < 22.46, (counts, chi2)


def test_draw_word_layout():
    """One 10-round block serves four consecutive plies (word ply % 4)."""
    seed, gid = 0x0123456789ABCDEF, 42
    for ply in range(0, 16):
        blk = ref.philox((ply >> 2, gid, 0, 0), (seed & 0xFFFFFFFF, seed >> 32))
        assert ref.draw(seed, gid, ply) == int(blk[ply & 3])
