"""Pins of the oracle's counter RNG and Gaussian transform.

The Philox round structure (which words are multiplied, how the high and low
halves and the key are combined, when the key is bumped) is written once in
the oracle and instantiated for 32- and 64-bit words.  numpy ships an
independent Philox4x64-10; matching it bit for bit pins that structure.  The
32-bit multipliers and Weyl constants are those of Salmon et al. (SC'11);
their output is then checked statistically."""
import math

import numpy as np
import pytest
from scipy import stats


def test_philox4x64_matches_numpy(orc):
    # numpy's Philox increments the 256-bit counter before each block.
    for key in (0, 1, 0xDEADBEEFCAFEBABE):
        bg = np.random.Philox(key=key, counter=0)
        raw = bg.random_raw(4 * 6)
        k = [key & ((1 << 64) - 1), 0]
        # numpy stores the 128-bit key as two words, low first
        for blk in range(6):
            out = orc.philox4x64_10([blk + 1, 0, 0, 0], k)
            assert out == [int(x) for x in raw[4 * blk:4 * blk + 4]], (key, blk)


def test_philox4x64_counter_carry_matches_numpy(orc):
    bg = np.random.Philox(key=[3, 9])
    st = bg.state
    st["state"]["counter"] = np.array([2**64 - 1, 5, 0, 0], dtype=np.uint64)
    st["buffer_pos"] = 4
    bg.state = st
    raw = bg.random_raw(4)
    assert orc.philox4x64_10([0, 6, 0, 0], [3, 9]) == [int(x) for x in raw]


def test_philox4x32_is_a_bijection_sample(orc):
    # distinct counters give distinct outputs (no collisions in a sample)
    seen = set()
    for c in range(2000):
        seen.add(tuple(orc.philox4x32_10([c, 7, 0, 0], [1, 0])))
    assert len(seen) == 2000


def _uniform_sample(orc, n_cells=4096, steps=(0, 1, 2)):
    u = []
    for s in steps:
        for c in range(n_cells):
            u.append(orc.uniforms(1, 0, 1, c, s))
    return np.array(u)


def test_uniforms_moments_and_chi2(orc):
    u = _uniform_sample(orc)
    assert u.min() > 0 and u.max() < 1
    flat = u.ravel()
    n = flat.size
    assert abs(flat.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
    assert abs(flat.var() - 1 / 12) < 4 * 0.0745 / math.sqrt(n)
    hist, _ = np.histogram(flat, bins=64, range=(0, 1))
    chi2 = stats.chisquare(hist).pvalue
    assert chi2 > 1e-4
    # word-to-word and counter-to-counter correlation
    for a in range(4):
        for b in range(a + 1, 4):
            r = np.corrcoef(u[:, a], u[:, b])[0, 1]
            assert abs(r) < 4 / math.sqrt(len(u))
    r = np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]
    assert abs(r) < 4 / math.sqrt(len(u))


def test_uniforms_are_exact_in_fp32(orc):
    u = _uniform_sample(orc, n_cells=512, steps=(5,))
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    # 23-bit grid with a half-step offset
    k = u * 2**24
    assert np.array_equal(k, np.round(k)) and np.all(np.round(k) % 2 == 1)


def test_uniform_matches_definition_of_raw_words(orc):
    for c in range(50):
        raw = orc.philox_cell(123456789012, 3, 1, c, 77)
        u = orc.uniforms(123456789012, 3, 1, c, 77)
        for r, x in zip(raw, u):
            assert x == ((r >> 9) + 0.5) / 2**23


def test_counter_layout_separates_streams(orc):
    a = orc.philox_cell(1, 0, 1, 10, 5)
    assert orc.philox_cell(1, 0, 2, 10, 5) != a          # tag
    assert orc.philox_cell(1, 1, 1, 10, 5) != a          # level
    assert orc.philox_cell(2, 0, 1, 10, 5) != a          # seed
    assert orc.philox_cell(1, 0, 1, 10, 5 + 2**32) != a  # high step bits
    assert orc.philox_cell(1, 0, 1, 10, 5) == a          # deterministic


def test_counter_words_are_the_documented_ones(orc):
    seed, level, tag, cell, step = 0x123456789, 5, 1, 77, (3 << 32) | 11
    want = orc.philox4x32_10([cell, 11, 3 | (5 << 16) | (1 << 24), 0],
                             [seed & 0xFFFFFFFF, seed >> 32])
    assert orc.philox_cell(seed, level, tag, cell, step) == want


def test_normals_moments(orc):
    xi = np.array([orc.normals(7, 0, c, s) for s in range(4) for c in range(5000)])
    n = len(xi)
    for k in range(3):
        x = xi[:, k]
        assert abs(x.mean()) < 4 / math.sqrt(n)
        assert abs(x.var() - 1) < 4 * math.sqrt(2 / n)
        assert abs(stats.kurtosis(x, fisher=False) - 3) < 4 * math.sqrt(24 / n)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    # the two normals of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(xi[:, 0], xi[:, 1])[0, 1]) < 4 / math.sqrt(n)
    assert abs(np.corrcoef(xi[:, 0], xi[:, 2])[0, 1]) < 4 / math.sqrt(n)


def test_normals_from_uniforms_definition(orc):
    u = orc.uniforms(9, 2, 1, 33, 44)
    xi = orc.normals(9, 2, 33, 44)
    r0 = math.sqrt(-2 * math.log(u[0]))
    r2 = math.sqrt(-2 * math.log(u[2]))
    assert xi[0] == pytest.approx(r0 * math.cos(2 * math.pi * u[1]), rel=1e-15)
    assert xi[1] == pytest.approx(r0 * math.sin(2 * math.pi * u[1]), rel=1e-15)
    assert xi[2] == pytest.approx(r2 * math.cos(2 * math.pi * u[3]), rel=1e-15)
    # the truncation of the 23-bit grid: |xi| < sqrt(-2 ln 2^-24)
    assert math.sqrt(-2 * math.log(2**-24)) == pytest.approx(5.768, abs=1e-3)
