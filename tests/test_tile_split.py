"""Host logic of the persistent launch's tile cut (no GPU): every human's
units are covered exactly, only the sizes the launch shape allows occur, and
the remainder after whole rounds of big tiles is spread over the CUs one tile
per CU at a time."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def cap():
    from paper_2603_01122_amd import capred
    if not hasattr(capred, "tile_split"):
        pytest.skip("library built without the batched plan")
    return capred


SIZES = {4: (4, 2, 1), 2: (2, 1, 0), 1: (1, 0, 0)}


def test_units_are_covered_exactly(cap):
    r = np.random.default_rng(0)
    for _ in range(400):
        n = int(r.integers(1, 40))
        P = int(r.choice([1, 2, 4]))
        C = int(r.integers(1, 300))
        R = C * int(r.integers(1, 5))
        units = r.integers(0, 3000, size=n)
        cnt = cap.tile_split(units, P, R, C)
        assert np.all(cnt >= 0)
        sz = np.array(SIZES[P])
        assert np.array_equal(cnt @ sz, units)
        assert np.all(cnt[:, sz == 0] == 0)


def test_tail_spreads_over_the_cus(cap):
    """Units in whole big tiles per human (no forced small tiles): after the
    whole rounds, the remainder Ur (mod 4 C) takes at most one tile per CU."""
    r = np.random.default_rng(1)
    for _ in range(200):
        C = int(r.integers(8, 300))
        R = 2 * C
        units = 4 * r.integers(1, 200, size=int(r.integers(1, 30)))
        U = int(units.sum())
        cnt = cap.tile_split(units, 4, R, C)
        tiles = int(cnt.sum())
        rounds = U // (4 * R)
        Ur = U - 4 * R * rounds
        full_cu_rounds = (Ur - 1) // (4 * C) if Ur else 0   # one big tile per CU each
        tail = tiles - R * rounds - C * full_cu_rounds
        assert 0 <= tail <= C, (U, C, tail)
        # a remainder of at most one unit per CU is cut to single units
        if 0 < Ur - 4 * C * full_cu_rounds <= C:
            assert cnt[:, 2].sum() == Ur - 4 * C * full_cu_rounds


def test_sixteen_human_workload_cut(cap):
    """The 16-human serving workload at 512 threads x 4 on 256 CUs x 2 blocks:
    3053 units = 2 rounds of 512 big tiles + 1005 units.  The policy asks for
    247 more big tiles, 8 halves and 1 quarter (256 tiles, one per CU); the
    humans' own remainders already bring 10 halves and 9 quarters, so no big
    tile is split: 756 big tiles, 10 halves, 9 quarters."""
    from paper_2603_01122_amd import scenes
    units = np.array([-(-h.N // 512) for h in scenes.config3().humans])
    assert units.sum() == 3053
    assert int(((units % 4) // 2).sum()) == 10 and int((units % 2).sum()) == 9
    cnt = cap.tile_split(units, 4, 512, 256)
    assert tuple(cnt.sum(0)) == (756, 10, 9)
    # with room for the targets (every human a multiple of 4 units) the cut is
    # exactly the policy's: 2 rounds + 247 big, 8 halves, 1 quarter
    units4 = 4 * (units // 4)
    units4[0] += 3053 - units4.sum() - (3053 - units4.sum()) % 4
    U = int(units4.sum())
    cnt4 = cap.tile_split(units4, 4, 512, 256)
    Ur = U - 4 * 512 * (U // 2048)
    big = (Ur - 512 + 1) // 2
    half = (Ur - 4 * big) // 2
    quarter = Ur - 4 * big - 2 * half
    assert tuple(cnt4.sum(0)) == (512 * (U // 2048) + big, half, quarter)


def test_invalid_arguments(cap):
    with pytest.raises(cap.CapError):
        cap.tile_split([4, 4], 3, 16, 8)
    with pytest.raises(cap.CapError):
        cap.tile_split([4, -1], 4, 16, 8)
    with pytest.raises(cap.CapError):
        cap.tile_split([4], 4, 0, 8)
