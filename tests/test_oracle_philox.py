"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

# Known-answer vectors published with the generator's reference implementation
# (counter words, key words -> output words).
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_known_answers(ctr, key, expect):
    out = philox.philox4x32_10(ctr, key)
    assert tuple(int(x) for x in out) == expect


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2**32, size=(4, 257), dtype=np.uint64)
    k = rng.integers(0, 2**32, size=(2,), dtype=np.uint64)
    vec = philox.philox4x32_10(tuple(c), tuple(k))
    for j in range(0, 257, 37):
        one = philox.philox4x32_10(tuple(int(x) for x in c[:, j]), (int(k[0]), int(k[1])))
        assert [int(v[j]) for v in vec] == [int(x) for x in one]


def test_mode_words_parity_and_key():
    # Even and odd iz share one Philox call: words (x0, x1) and (x2, x3).
    seed = (7 << 32) | 11
    x = philox.philox4x32_10((3, 5, 9, 0), (11, 7))
    a0, b0 = philox.mode_words(seed, 9, 5, 6)
    a1, b1 = philox.mode_words(seed, 9, 5, 7)
    assert (int(a0), int(b0), int(a1), int(b1)) == tuple(int(v) for v in x)


_ROCRAND_SRC = r"""
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main() {
  unsigned long long seeds[3] = {0ull, 0x123456789abcdefull, 0xffffffffffffffffull};
  unsigned int ctrs[4][4] = {{0,0,0,0},{1,2,3,4},{0xfffffffeu,7,0x80000000u,0},{12345,0,77,1}};
  for (int s = 0; s < 3; ++s) for (int c = 0; c < 4; ++c) {
    unsigned long long off = ((unsigned long long)ctrs[c][1] << 32) | ctrs[c][0];
    unsigned long long sub = ((unsigned long long)ctrs[c][3] << 32) | ctrs[c][2];
    rocrand_device::philox4x32_10_engine e(seeds[s], sub, off * 4ull);
    uint4 r = e.next4();
    printf("%llu %u %u %u %u %u %u %u %u\n", seeds[s], ctrs[c][0], ctrs[c][1], ctrs[c][2], ctrs[c][3], r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_against_rocrand_host_engine(tmp_path):
    """rocRAND's Philox engine (compiled from its headers for the host) as a black box."""
    src = tmp_path / "p.cpp"
    src.write_text(_ROCRAND_SRC)
    exe = tmp_path / "p"
    r = subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include", "-O1", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND host probe: " + r.stderr[-400:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    lines = [list(map(int, ln.split())) for ln in out.strip().splitlines()]
    assert len(lines) == 12
    for v in lines:
        seed, c, expect = v[0], v[1:5], v[5:9]
        got = philox.philox4x32_10(tuple(c), philox.seed_key(seed))
        assert [int(g) for g in got] == expect
