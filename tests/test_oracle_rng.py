"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11) against rocRAND's."""
import numpy as np
import pytest

import oracle
from tests import exact

pytestmark = pytest.mark.skipif(exact.build_philox_pin(force=False) is None,
                                reason="rocRAND headers not installed")


def _grid(n=2000, seed=11):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # edge counters and keys: all zero, all ones, and the counter shapes the chain uses
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    ctr[2] = [7, 3, 123456, 0]          # (sweep, phase, pair>>1, sweep_hi)
    ctr[3] = [0, 0x200, 4095, 0]        # init domain
    ctr[4] = [99, 0x100, 2, 1]          # schedule domain, sweep beyond 2^32
    return ctr, key


def test_philox_matches_rocrand_on_grid():
    ctr, key = _grid()
    ref = exact.rocrand_philox(ctr, key)
    got = np.stack([oracle.philox(c, k) for c, k in zip(ctr, key)])
    assert np.array_equal(got, ref)


def test_philox_is_a_permutation_sample_and_sensitive_to_every_input_word():
    base_c = np.array([5, 6, 7, 8], dtype=np.uint32)
    base_k = np.array([9, 10], dtype=np.uint32)
    y0 = oracle.philox(base_c, base_k)
    for w in range(4):
        c = base_c.copy()
        c[w] ^= 1
        assert not np.array_equal(oracle.philox(c, base_k), y0)
    for w in range(2):
        k = base_k.copy()
        k[w] ^= 1
        assert not np.array_equal(oracle.philox(base_c, k), y0)


def test_philox_output_bits_are_balanced():
    # 4096 consecutive counters: each of the 128 output bits is set about half the time
    outs = np.stack([oracle.philox([i, 0, 0, 0], [1, 2]) for i in range(4096)])
    bits = np.unpackbits(outs.view(np.uint8), axis=1)
    frac = bits.mean(axis=0)
    # binomial sd = sqrt(0.25/4096) = 0.0078; 5 sd
    assert np.all(np.abs(frac - 0.5) < 0.04)
