"""Pins of the oracle's noise source: Philox4x32-10 (Salmon, Moraes, Dror and
Shaw, SC'11) and the Box-Muller normals built on it.  No published
known-answer vector is available here, so the generator is pinned by
inverting its round function from the published definition, by bijectivity,
bit balance and avalanche, and the normals by their moments and distribution.
CPU only."""
import numpy as np
import pytest
from scipy import stats

import oracle as O

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def _inverse_philox(out, key):
    """Undo 10 Philox4x32 rounds: each round's low product words are outputs
    1 and 3, so the multiplied inputs follow from the modular inverses of the
    odd multipliers; the high words then unmask the other two inputs."""
    inv0, inv1 = pow(M0, -1, 1 << 32), pow(M1, -1, 1 << 32)
    y = [int(v) for v in out]
    keys = []
    k0, k1 = int(key[0]), int(key[1])
    for r in range(10):
        keys.append((k0, k1))
        k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
    for r in reversed(range(10)):
        k0, k1 = keys[r]
        x2 = (y[1] * inv1) & MASK
        x0 = (y[3] * inv0) & MASK
        hi1 = (M1 * x2) >> 32
        hi0 = (M0 * x0) >> 32
        x1 = y[0] ^ hi1 ^ k0
        x3 = y[2] ^ hi0 ^ k1
        y = [x0, x1, x2, x3]
    return y


def test_philox_inverts_to_counter():
    rng = np.random.default_rng(0)
    for _ in range(200):
        ctr = rng.integers(0, 1 << 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 1 << 32, 2, dtype=np.uint64).astype(np.uint32)
        out = O.philox4x32_10(ctr, key)
        assert _inverse_philox(out, key) == [int(v) for v in ctr]
    # edge counters and keys
    for ctr, key in [([0, 0, 0, 0], [0, 0]), ([MASK] * 4, [MASK, MASK]), ([1, 0, 0, 0], [0, 1])]:
        out = O.philox4x32_10(ctr, key)
        assert _inverse_philox(out, key) == ctr


def _words(n, key=(1, 0), step=0):
    return np.array([O.philox4x32_10([s, step, 0, 0], key) for s in range(n)], dtype=np.uint64)


def test_philox_bit_balance_and_distinct_outputs():
    w = _words(20000)
    rows = {tuple(r) for r in w.tolist()}
    assert len(rows) == len(w)
    bits = ((w[:, :, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(float)
    p = bits.mean(axis=0)
    sigma = np.sqrt(0.25 / len(w))
    assert np.abs(p - 0.5).max() < 5.5 * sigma
    # top byte of every word uniform over 256 bins
    for j in range(4):
        hist = np.bincount((w[:, j] >> 24).astype(int), minlength=256)
        chi2 = ((hist - len(w) / 256) ** 2 / (len(w) / 256)).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4


def test_philox_avalanche():
    rng = np.random.default_rng(1)
    flips = []
    for _ in range(400):
        ctr = rng.integers(0, 1 << 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 1 << 32, 2, dtype=np.uint64).astype(np.uint32)
        a = O.philox4x32_10(ctr, key)
        ctr2 = ctr.copy()
        word, bit = rng.integers(0, 4), rng.integers(0, 32)
        ctr2[word] ^= np.uint32(1 << int(bit))
        b = O.philox4x32_10(ctr2, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    flips = np.array(flips)
    # 128 output bits, each flips with probability 1/2
    assert abs(flips.mean() - 64) < 5 * np.sqrt(32 / len(flips))
    assert flips.min() > 30


@pytest.mark.parametrize("q,first", [(9, 3), (27, 4)])
def test_normals_distribution(q, first):
    samples = []
    for s in range(6000 if q == 27 else 20000):
        eta = O.normals(q, 12345, 3, s % 7, s)
        assert np.all(eta[:first] == 0.0)
        samples.append(eta[first:])
    x = np.array(samples)
    flat = x.ravel()
    n = flat.size
    assert abs(flat.mean()) < 5 / np.sqrt(n)
    assert abs(flat.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(flat, fisher=False) - 3) < 5 * np.sqrt(24 / n)
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    # every mode is standard normal and the modes are uncorrelated
    assert np.abs(x.mean(axis=0)).max() < 5 / np.sqrt(len(x))
    corr = np.corrcoef(x.T)
    assert np.abs(corr - np.eye(q - first)).max() < 5 / np.sqrt(len(x))


def test_normals_keyed_by_all_counter_fields():
    base = O.normals(27, 7, 0, 0, 0)
    for args in [(8, 0, 0, 0), (7, 1, 0, 0), (7, 0, 1, 0), (7, 0, 0, 1), (7 + (1 << 32), 0, 0, 0)]:
        other = O.normals(27, *args)
        assert np.abs(other[4:] - base[4:]).min() > 0.0
    assert np.array_equal(O.normals(27, 7, 0, 0, 0), base)


def test_normals_finite_at_extreme_words():
    """u1 is never 0, so eta stays finite; this holds for any Philox word."""
    # the largest magnitude the transform can produce: u1 = 2^-24
    assert np.sqrt(-2 * np.log(2.0 ** -24)) < 6.0
    eta = np.array([O.normals(9, s, 0, 0, 0) for s in range(2000)])
    assert np.all(np.isfinite(eta)) and np.abs(eta).max() < 6.0


def _normals_from_definition(q, seed, replica, step, site):
    """eta of the stated mapping, evaluated here from Philox words: normal
    n = v - first of pair p = n // 2 takes block p // 2, words 2 (p % 2) and
    2 (p % 2) + 1 as (a, b); u1 = ((a >> 8) + 1) 2^-24, u2 = (b >> 8) 2^-24,
    r = sqrt(-2 ln u1), cosine for even n; counter (site, step mod 2^32,
    replica, block + 2^8 floor(step / 2^32))."""
    first = 3 if q == 9 else 4
    key = [seed & MASK, seed >> 32]
    eta = np.zeros(q)
    for v in range(first, q):
        n = v - first
        p = n // 2
        blk = p // 2
        ctr = [site, step & MASK, replica, blk + ((step >> 32) << 8)]
        w = O.philox4x32_10(ctr, key)
        a, b = int(w[2 * (p % 2)]), int(w[2 * (p % 2) + 1])
        u1 = ((a >> 8) + 1) * 2.0 ** -24
        u2 = (b >> 8) * 2.0 ** -24
        r = np.sqrt(-2.0 * np.log(u1))
        eta[v] = r * (np.cos(2 * np.pi * u2) if n % 2 == 0 else np.sin(2 * np.pi * u2))
    return eta


@pytest.mark.parametrize("q", [9, 19, 27])
@pytest.mark.parametrize("step", [0, 5, (1 << 32) - 1, 1 << 32, (1 << 32) + 7, (1 << 40) + 3, (1 << 56) - 1])
def test_normals_follow_the_stated_mapping(q, step):
    """The counter layout, word selection and Box-Muller transform stated for
    the noise, including the steps of 2^32 and beyond (whose counters carry
    the high step bits next to the block index)."""
    seed, replica = (1 << 33) + 77, 5
    for site in (0, 1, 4095, (1 << 32) - 1):
        got = O.normals(q, seed, replica, step, site)
        ref = _normals_from_definition(q, seed, replica, step, site)
        assert np.abs(got - ref).max() < 1e-14


def test_normals_of_steps_2_to_the_32_apart_differ():
    """The paper's normals are independent at every step: steps t and
    t + 2^32 (and t + 2^40) draw different normals, where a 32-bit step
    word would repeat them."""
    for t in (0, 3, 1000):
        base = O.normals(27, 9, 1, t, 17)
        for far in (t + (1 << 32), t + (1 << 40)):
            other = O.normals(27, 9, 1, far, 17)
            assert np.abs(other[4:] - base[4:]).min() > 0.0
