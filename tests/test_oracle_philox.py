"""Pins for the oracle's random-number contract.

The Philox4x32-10 blocks are checked against PyTorch's header-only Philox
engine (ATen/core/PhiloxRNGEngine.h, compiled here with g++) -- a library
implementation independent of the oracle.  The uniform mapping is checked
for exactness (odd multiples of 2^-24) and for uniformity (KS test).
"""
import numpy as np
import pytest
import scipy.stats


def test_philox_matches_pytorch_engine(orc, torch_philox):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0), (2**64 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1),
             (0x299F31D0A4093822, 0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2**63)), *[int(v) for v in rng.integers(0, 2**32, 4)]))
    for seed, c0, c1, c2, c3 in cases:
        got = orc.philox_bulk(1, c0, c1, c2, c3, seed)[0]
        ref = torch_philox(seed, c0, c1, c2, c3)
        assert np.array_equal(got, ref), (seed, c0, c1, c2, c3, got, ref)


def test_philox_bulk_counter_layout(orc, torch_philox):
    blk = orc.philox_bulk(64, 1000, 5, 7, 9, 12345)
    for i in (0, 1, 31, 63):
        assert np.array_equal(blk[i], torch_philox(12345, 1000 + i, 5, 7, 9))


def test_uniform24_exact_and_open_interval(orc):
    w = np.array([0, 1, 511, 512, 2**32 - 1, 2**31], np.uint32)
    u = orc.uniform24(w)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 2.0 ** -24
    assert u[3] == 3 * 2.0 ** -24
    assert u[4] == 1.0 - 2.0 ** -24
    assert np.all((u > 0) & (u < 1))
    # exact in float32
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    for x in w:
        assert orc.lib().orc_uniform24(int(x)) == orc.uniform24(np.array([x]))[0]


def test_uniforms_pass_ks(orc):
    blk = orc.philox_bulk(1 << 18, 0, 3, 1, 2, 0)
    u = orc.uniform24(blk.reshape(-1))
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3
    # word columns are independent streams too
    for c in range(4):
        assert scipy.stats.kstest(orc.uniform24(blk[:, c]), "uniform").pvalue > 1e-4
