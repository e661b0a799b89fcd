"""Pins of the oracle's counter-based generator (Philox4xW-10, Salmon et al.
SC'11), which replaces the paper's MT19937 (Sec. 2 step 5) so that every
particle-step owns its draws."""
import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox4x64_matches_numpy(ora):
    # numpy's Philox is the 4x64-10 instance of the same construction; it
    # advances the counter by one before producing each block.
    rng = np.random.default_rng(1234)
    for _ in range(200):
        key = rng.integers(0, 2**64, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        expect = bg.random_raw(4)
        nxt = ctr.copy()
        nxt[0] = nxt[0] + np.uint64(1)
        got = ora.philox4x64_10(nxt, key)
        assert np.array_equal(got, expect)


def test_philox_weyl_constants_from_their_definition():
    # The key increments are floor(2^W * (golden ratio - 1)) and
    # floor(2^W * (sqrt(3) - 1)); recompute them with exact integers and
    # compare with the constants in the source.
    src = open(os.path.join(os.path.dirname(HERE), "oracle", "philox.c")).read()
    consts = {int(h, 16) for h in re.findall(r"0x([0-9A-Fa-f]+)u", src)}

    def golden(w):
        # (sqrt(5) - 1) / 2 * 2^w
        return (math.isqrt(5 << (2 * w)) - (1 << w)) >> 1

    def sqrt3m1(w):
        return math.isqrt(3 << (2 * w)) - (1 << w)

    for w in (32, 64):
        assert golden(w) in consts, hex(golden(w))
        assert sqrt3m1(w) in consts, hex(sqrt3m1(w))


def _rocrand_kat(lines):
    exe = os.path.join("/tmp", "pic_rocrand_kat_%d" % os.getpid())
    src = os.path.join(HERE, "rocrand_philox_kat.cpp")
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND known-answer source")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe, src], check=True,
                   capture_output=True)
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout
    os.remove(exe)
    return [list(map(int, l.split())) for l in out.strip().splitlines()]


def test_philox4x32_matches_rocrand(ora):
    # rocRAND ships an independently written Philox4x32-10 (host-callable);
    # its blocks are the known answers for the 32-bit instance.
    rng = np.random.default_rng(99)
    # rocRAND addresses counter words 0-1 as a 64-bit offset of 4-word
    # blocks, so word 1 stays below 2^30 here to keep 4*offset in range.
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 2**30 - 1, 0xFFFFFFFF,
                                  0xFFFFFFFF)]
    for _ in range(64):
        c = [int(v) for v in rng.integers(0, 2**32, size=6, dtype=np.uint64)]
        c[3] %= 2**30
        cases.append(tuple(c))
    # the layout the simulation uses: key (seed, run), ctr (step, slot, 16*sp+p, 0)
    for step in (0, 1, 12345, 2**31 + 7):
        for slot in (0, 5, 1_000_000):
            for sp, pur in ((0, 0), (0, 3), (1, 0), (1, 2)):
                cases.append((7, 3, step, slot, 16 * sp + pur, 0))
    lines = [" ".join(str(v) for v in c) for c in cases]
    ref = _rocrand_kat(lines)
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        got = ora.philox4x32_10(c[2:], c[:2])
        assert list(map(int, got)) == r, c


def test_uniform_map_and_chi2(ora):
    # u = (r + 1/2) 2^-32 lies strictly inside (0, 1) for every u32 and the
    # words are uniform: chi^2 over 256 bins of 4 x 20000 words.
    lo = (0 + 0.5) * 2.0**-32
    hi = (0xFFFFFFFF + 0.5) * 2.0**-32
    assert 0.0 < lo and hi < 1.0 and hi == 1.0 - 2.0**-33
    words = []
    for slot in range(20000):
        words.extend(ora.philox4x32_10([17, slot, 1, 0], [5, 6]))
    words = np.array(words, dtype=np.uint64)
    u = (words.astype(np.float64) + 0.5) * 2.0**-32
    h, _ = np.histogram(u, bins=256, range=(0, 1))
    e = u.size / 256
    chi2 = ((h - e) ** 2 / e).sum()
    # 255 dof: mean 255, sd ~22.6; 99.99% quantile ~ 345
    assert 170 < chi2 < 345, chi2
    # no correlation between adjacent slots' first words
    a = u[0::4]
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 0.03
