"""Pins for the oracle's noise stream: Philox4x32-10, the uniform map and
Box-Muller. The paper fixes only the zero mean and 2 D dt covariance of the
random displacement (Eq. 1); the generator is a design choice pinned here
against AMD's rocRAND implementation and against the normal distribution."""
import os
import random
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import ora

HERE = os.path.dirname(os.path.abspath(__file__))


def philox_py(ctr, key):
    """Third, pure-Python Philox4x32-10 (Salmon et al., SC'11)."""
    c = list(ctr)
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
    return tuple(c)


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rref")
    subprocess.check_call([hipcc, "-O1", "-o", exe,
                           os.path.join(HERE, "golden", "rocrand_philox_ref.cpp")])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_ref):
    rng = random.Random(7)
    cases = [((0, 0, 0, 0), (0, 0)),
             ((0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF))]
    for _ in range(300):
        cases.append(((rng.getrandbits(32), rng.getrandbits(30), rng.getrandbits(32),
                       rng.getrandbits(32)), (rng.getrandbits(32), rng.getrandbits(32))))
    # the counter layouts the library uses: (step, bead, replica, tag<<24|group)
    for step in (0, 1, 99, 12345):
        for bead in (0, 1, 999):
            cases.append(((step, bead, 5, (2 << 24) | 17), (4, 0)))
    inp = "\n".join(" ".join("%x" % v for v in c + k) for c, k in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (c, k), line in zip(cases, out):
        ref = tuple(int(x, 16) for x in line.split())
        assert ora.philox(c, k) == ref, (c, k)


def test_philox_three_implementations_agree():
    rng = random.Random(11)
    for _ in range(500):
        c = tuple(rng.getrandbits(32) for _ in range(4))
        k = (rng.getrandbits(32), rng.getrandbits(32))
        assert ora.philox(c, k) == philox_py(c, k)


def test_uniform_map_exact_values():
    assert ora.uniform(0) == 2.0 ** -24
    assert ora.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert ora.uniform(0x80000000) == 0.5 + 2.0 ** -24
    assert ora.uniform(0x1FF) == 2.0 ** -24          # low 9 bits ignored
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2 ** 32, size=2000, dtype=np.uint64):
        u = ora.uniform(int(x))
        assert 0.0 < u < 1.0
        m = u * 2.0 ** 24
        assert m == int(m) and int(m) % 2 == 1          # odd multiple of 2^-24
        assert np.float32(u) == u                        # exact in binary32


def test_event_uniform_exact_values():
    # two words -> an odd multiple of 2^-53 from the top 52 bits of hi:lo
    assert ora.uniform53(0, 0) == 2.0 ** -53
    assert ora.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert ora.uniform53(0x80000000, 0) == 0.5 + 2.0 ** -53
    assert ora.uniform53(0, 0xFFF) == 2.0 ** -53               # low 12 bits ignored
    assert ora.uniform53(0, 0x1000) == 3.0 * 2.0 ** -53
    assert ora.uniform53(1, 0) == (2.0 * 2 ** 20 + 1) * 2.0 ** -53
    rng = np.random.default_rng(4)
    prev = 0.0
    for w in np.sort(rng.integers(0, 2 ** 64, size=2000, dtype=np.uint64)):
        u = ora.uniform53(int(w) >> 32, int(w) & 0xFFFFFFFF)
        assert 0.0 < u < 1.0 and u >= prev
        assert (u * 2.0 ** 53) % 2 == 1                       # odd multiple of 2^-53
        prev = u
    # a probability far below the one-word grid (2^-24 ~ 6e-8) is resolved:
    # the fraction of 64-bit words mapped below p is p to within 2^-52
    p = 1.3e-9
    m_below = np.ceil(p * 2.0 ** 52 - 0.5)
    assert abs(m_below / 2.0 ** 52 - p) <= 2.0 ** -52


def test_philox_words_uniform_chi2():
    counts = np.zeros((4, 64))
    for i in range(20000):
        w = ora.philox((i, 3, 7, 1), (123, 456))
        for a in range(4):
            counts[a, w[a] >> 26] += 1
    for a in range(4):
        p = stats.chisquare(counts[a]).pvalue
        assert p > 1e-4, (a, p)


def test_box_muller_special_cases():
    # u0 with -2 ln u0 = 1 is not on the grid; check the structure instead:
    # xi_x^2 + xi_y^2 = -2 ln u0 and atan2(xi_y, xi_x) = 2 pi u1 (mod 2 pi)
    rng = np.random.default_rng(3)
    for _ in range(200):
        w = [int(v) for v in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        xi = ora.normals(w)
        u = [ora.uniform(v) for v in w]
        assert np.isclose(xi[0] ** 2 + xi[1] ** 2, -2.0 * np.log(u[0]), rtol=1e-12)
        ang = np.arctan2(xi[1], xi[0]) % (2 * np.pi)
        assert np.isclose(np.cos(ang - 2 * np.pi * u[1]), 1.0, atol=1e-12)
        assert np.isclose(abs(xi[2]), np.sqrt(-2.0 * np.log(u[2])) * abs(np.cos(2 * np.pi * u[3])),
                          rtol=1e-12)
    # u1 = 1/4 + 2^-24 puts the pair almost on the y axis
    w = [0x80000000, 0x40000000, 0x80000000, 0x00000000]
    xi = ora.normals(w)
    assert abs(xi[0]) < 1e-6 and xi[1] > 0


def test_noise_is_standard_normal():
    xs = np.array([ora.noise(9, step, bead, 3, 0, 2) for step in range(400) for bead in range(50)])
    for a in range(3):
        col = xs[:, a]
        assert stats.kstest(col, "norm").pvalue > 1e-4
        assert abs(col.mean()) < 5 / np.sqrt(len(col))
        assert abs(col.var() - 1.0) < 5 * np.sqrt(2.0 / len(col))
    c = np.corrcoef(xs.T)
    assert np.max(np.abs(c - np.eye(3))) < 5 / np.sqrt(len(xs))


def test_noise_streams_differ_by_every_counter_word():
    base = ora.noise(5, 10, 20, 30, 0, 40)
    for args in [(6, 10, 20, 30, 0, 40), (5, 11, 20, 30, 0, 40), (5, 10, 21, 30, 0, 40),
                 (5, 10, 20, 31, 0, 40), (5, 10, 20, 30, 1, 40), (5, 10, 20, 30, 0, 41)]:
        assert not np.allclose(ora.noise(*args), base)


def _fourth_normal_py(words):
    # r1 sin(2 pi u3) from the word map and Box-Muller written out with math
    import math
    u2 = ((words[2] >> 9) + 0.5) * 2.0 ** -23
    u3 = ((words[3] >> 9) + 0.5) * 2.0 ** -23
    return math.sqrt(-2.0 * math.log(u2)) * math.sin(2.0 * math.pi * u3)


def test_noise_map_one_definition():
    # map 1: steps 4m..4m+2 keep the first three normals of their own block;
    # step 4m+3 takes the fourth normals of the blocks of steps 4m, 4m+1, 4m+2
    seed = 0x0123456789ABCDEF
    key = (seed & 0xFFFFFFFF, seed >> 32)
    rng = np.random.default_rng(5)
    for _ in range(200):
        m = int(rng.integers(0, 2 ** 28))
        bead, rep, grp = (int(v) for v in rng.integers(0, 1000, size=3))
        tag = int(rng.integers(0, 2))
        for r in range(3):
            a = ora.noise(seed, 4 * m + r, bead, rep, tag, grp, noise_map=1)
            assert np.array_equal(a, ora.noise(seed, 4 * m + r, bead, rep, tag, grp))
        got = ora.noise(seed, 4 * m + 3, bead, rep, tag, grp, noise_map=1)
        ref = [_fourth_normal_py(philox_py((4 * m + q, bead, rep, (tag << 24) | grp), key)) for q in range(3)]
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
        # the fourth normal is the one normals() leaves out
        w = ora.philox((4 * m, bead, rep, (tag << 24) | grp), key)
        four = ora.normals4(w)
        assert np.array_equal(four[:3], ora.normals(w))
        assert np.isclose(four[3], ref[0], rtol=1e-13, atol=1e-13)


def _four_normals_py(words):
    # Box-Muller of both pairs, from the word map written out with math
    import math
    u = [((w >> 9) + 0.5) * 2.0 ** -23 for w in words]
    r0 = math.sqrt(-2.0 * math.log(u[0]))
    r1 = math.sqrt(-2.0 * math.log(u[2]))
    return [r0 * math.cos(2.0 * math.pi * u[1]), r0 * math.sin(2.0 * math.pi * u[1]),
            r1 * math.cos(2.0 * math.pi * u[3]), r1 * math.sin(2.0 * math.pi * u[3])]


def test_noise_map_two_definition():
    # map 2: bead 4q + r takes normal r of the blocks with bead word 3q + c as
    # its component c; the step word is the step itself (no carry over steps)
    seed = 0x0F1E2D3C4B5A6978
    key = (seed & 0xFFFFFFFF, seed >> 32)
    rng = np.random.default_rng(8)
    for _ in range(200):
        step = int(rng.integers(0, 2 ** 32))
        q, r = int(rng.integers(0, 256)), int(rng.integers(0, 4))
        rep, grp = (int(v) for v in rng.integers(0, 1000, size=2))
        tag = int(rng.integers(0, 2))
        got = ora.noise(seed, step, 4 * q + r, rep, tag, grp, noise_map=2)
        ref = [_four_normals_py(philox_py((step, 3 * q + c, rep, (tag << 24) | grp), key))[r] for c in range(3)]
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_noise_map_two_uses_each_normal_once():
    # the 12 normals of a group's three blocks go to 12 distinct (bead, component)
    # slots, and neighbouring groups draw from disjoint blocks: over a chain of
    # 40 beads every normal of blocks 0..29 is used exactly once
    seed, step, rep, tag, grp = 77, 5, 9, 0, 3
    key = (seed & 0xFFFFFFFF, seed >> 32)
    pool = np.array([_four_normals_py(philox_py((step, b, rep, (tag << 24) | grp), key)) for b in range(30)])
    used = np.array([ora.noise(seed, step, j, rep, tag, grp, noise_map=2) for j in range(40)])
    assert np.allclose(np.sort(used.ravel()), np.sort(pool.ravel()), rtol=1e-13, atol=1e-13)
    assert len(np.unique(np.round(used.ravel(), 12))) == 120


def test_noise_map_two_is_standard_and_uncorrelated():
    xs = np.array([ora.noise(13, step, bead, 2, 0, 1, noise_map=2) for step in range(300) for bead in range(40)])
    for a in range(3):
        col = xs[:, a]
        assert stats.kstest(col, "norm").pvalue > 1e-4
        assert abs(col.mean()) < 5 / np.sqrt(len(col))
        assert abs(col.var() - 1.0) < 5 * np.sqrt(2.0 / len(col))
    c = np.corrcoef(xs.T)
    assert np.max(np.abs(c - np.eye(3))) < 5 / np.sqrt(len(xs))
    # beads 4q and 4q + 1 share their radii (one Box-Muller pair per block and
    # component): their normals are still uncorrelated
    x = xs.reshape(300, 40, 3)
    a, b = x[:, 0::4, :].ravel(), x[:, 1::4, :].ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(len(a))
    assert abs(np.corrcoef(a ** 2, b ** 2)[0, 1]) < 5 / np.sqrt(len(a))


def test_fourth_normals_are_standard_and_independent_of_the_third():
    # (r1 cos 2 pi u3, r1 sin 2 pi u3) is a Box-Muller pair: both N(0,1),
    # uncorrelated, and their squares sum to r1^2 ~ Exp(mean 2)
    key = (11, 22)
    n = 40000
    third, fourth = np.empty(n), np.empty(n)
    for i in range(n):
        four = ora.normals4(ora.philox((i, 7, 3, 0), key))
        third[i], fourth[i] = four[2], four[3]
    assert stats.kstest(fourth, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(third, fourth)[0, 1]) < 4.5 / np.sqrt(n)
    assert stats.kstest(third ** 2 + fourth ** 2, "expon", args=(0, 2.0)).pvalue > 1e-3
