"""Pins of the oracle's Philox4x64-10 generator.

The generator is the published Philox4x64-10 (Salmon, Moraes, Dror & Shaw,
SC'11).  numpy ships an independent implementation of the same generator
(numpy.random.Philox, 4x64, 10 rounds); its first raw output block at counter
c is the block of counter c+1, so the oracle is compared with it bit for bit.
"""
import numpy as np
import pytest

from oracle import su3ref


def _numpy_block(ctr, key):
    c = [int(x) for x in ctr]
    # numpy increments the 256-bit counter before generating: start one below
    borrow = 1
    for i in range(4):
        v = c[i] - borrow
        borrow = 1 if v < 0 else 0
        c[i] = v % (1 << 64)
    bg = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64),
                         counter=np.array(c, dtype=np.uint64))
    return np.array([bg.random_raw() for _ in range(4)], dtype=np.uint64)


def test_philox_matches_numpy_on_structured_counters():
    # the counters the method uses: (link id, sweep, subgroup<<32 | attempt, tag)
    for seed in (0, 1, 12345, 2**63 + 7):
        for ctr in ([0, 0, 0, 0], [17, 3, (2 << 32) | 1, 0], [4 * 16**4 - 1, 31, 0, 1],
                    [123456, 0, 2, 2], [2**40, 2**33, 2**32, 0]):
            got = su3ref.philox4x64(ctr, [seed, 0])
            ref = _numpy_block(ctr, [seed, 0])
            assert np.array_equal(got, ref), (seed, ctr)


def test_philox_matches_numpy_on_random_counters_and_keys():
    rng = np.random.default_rng(2024)
    for _ in range(300):
        ctr = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**64, size=2, dtype=np.uint64)
        assert np.array_equal(su3ref.philox4x64(ctr, key), _numpy_block(ctr, key))


def test_philox_counter_carry_edge():
    # all-ones words exercise the numpy-side borrow and the full 64-bit range
    ctr = [2**64 - 1, 2**64 - 1, 5, 9]
    assert np.array_equal(su3ref.philox4x64(ctr, [3, 4]), _numpy_block(ctr, [3, 4]))


@pytest.mark.parametrize("word", [0, 1, 2, 3])
def test_philox_output_bits_uniform(word):
    # each output bit of consecutive counters is a fair coin (5 sigma)
    n = 4000
    outs = np.array([su3ref.philox4x64([i, 7, 0, 0], [1, 0])[word] for i in range(n)], dtype=np.uint64)
    bits = ((outs[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.float64)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n))
