"""Pins of the oracle's Gaussian-smoothed occupancy and multi-human union
(Sec. III-B smoothing before emplacement; Sec. IV-B point-wise max union).

* smoothing equals SciPy's Gaussian filter (separable, zero padding, the same
  truncated and renormalised kernel) on random, ragged and border-heavy grids;
* sigma -> infinity with radius 1 is the 3x3 box average (closed form 1/9);
* radius 0 is count / N exactly;
* mass inside the grid is conserved when nothing lies within r of the border;
  a corner delta keeps exactly the mass of the kernel's in-grid quadrant;
* transposing the input transposes the output (catches swapped axes);
* selected cells equal the full computation at those cells;
* the union equals NumPy's element-wise maximum and is attained by one input.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi


def scipy_smooth(counts, N, sigma, radius):
    out = np.empty(counts.shape, np.float64)
    for t in range(counts.shape[0]):
        out[t] = ndi.gaussian_filter(counts[t].astype(np.float64) / N, sigma, mode="constant",
                                     cval=0.0, truncate=radius / sigma)
    return out


@pytest.mark.parametrize("shape,sigma,radius", [((3, 40, 33), 1.0, 3), ((2, 17, 64), 0.7, 2),
                                                ((1, 9, 7), 2.5, 8), ((2, 64, 64), 1.3, 4)])
def test_smooth_equals_scipy_gaussian_filter(orc, shape, sigma, radius):
    r = np.random.default_rng(int(sigma * 10) + radius)
    c = r.integers(0, 200, shape).astype(np.uint32)
    c[:, 0, :] = r.integers(1000, 2000, shape[2])       # heavy border rows
    c[:, :, -1] = r.integers(1000, 2000, shape[1])
    N = int(c.reshape(shape[0], -1).sum(1).max()) + 5
    got = orc.smooth(c, N, sigma, radius)
    ref = scipy_smooth(c, N, sigma, radius)
    assert np.max(np.abs(got - ref)) <= 1e-15 * max(1.0, np.abs(ref).max()) * 50


def test_smooth_box_limit(orc):
    c = np.zeros((1, 9, 9), np.uint32)
    c[0, 4, 4] = 90
    got = orc.smooth(c, 90, 1e6, 1)[0]
    box = np.zeros((9, 9))
    box[3:6, 3:6] = 1.0 / 9.0
    assert np.max(np.abs(got - box)) <= 1e-12


def test_smooth_radius_zero_is_identity(orc):
    r = np.random.default_rng(1)
    c = r.integers(0, 1 << 20, (4, 11, 13)).astype(np.uint32)
    N = 3 << 20
    assert np.array_equal(orc.smooth(c, N, 1.0, 0), c.astype(np.float64) / N)


def test_smooth_mass(orc):
    r = np.random.default_rng(2)
    c = np.zeros((2, 30, 40), np.uint32)
    c[:, 5:25, 5:35] = r.integers(0, 100, (2, 20, 30))
    N = 100000
    got = orc.smooth(c, N, 1.2, 5)
    assert np.allclose(got.reshape(2, -1).sum(1), c.reshape(2, -1).sum(1) / N, rtol=0,
                       atol=1e-14)
    # a delta in the corner keeps the in-grid quadrant of the kernel: for a
    # separable kernel that is (sum_{d>=0} w1(d))^2 with w1 the normalised 1-D kernel
    d = np.zeros((1, 20, 20), np.uint32)
    d[0, 0, 0] = 7
    got = orc.smooth(d, 7, 1.2, 5)
    one = np.zeros((1, 20, 20), np.uint32)
    one[0, 10, 10] = 7
    full = orc.smooth(one, 7, 1.2, 5)[0]
    row = full[10]                      # = w1(dx) * w1(0)
    col = full[:, 10]
    w1 = row / np.sqrt(full[10, 10])    # normalised 1-D kernel values
    assert np.isclose(w1.sum(), 1.0, atol=1e-14)
    quad = w1[10:16].sum() ** 2
    assert np.isclose(got.sum(), quad, rtol=1e-13)
    assert np.allclose(row, col, rtol=0, atol=1e-16)


def test_smooth_transpose_and_cells(orc):
    r = np.random.default_rng(3)
    c = r.integers(0, 50, (3, 21, 34)).astype(np.uint32)
    a = orc.smooth(c, 5000, 1.7, 4)
    b = orc.smooth(np.ascontiguousarray(c.transpose(0, 2, 1)), 5000, 1.7, 4)
    assert np.allclose(a, b.transpose(0, 2, 1), rtol=1e-14, atol=0)
    cells = r.integers(0, c.size, 500)
    assert np.array_equal(orc.smooth(c, 5000, 1.7, 4, cells=cells), a.reshape(-1)[cells])


def test_smooth_rejects(orc):
    c = np.zeros((1, 4, 4), np.uint32)
    with pytest.raises(ValueError):
        orc.smooth(c, 0, 1.0, 1)
    with pytest.raises(ValueError):
        orc.smooth(c, 1, 0.0, 1)
    with pytest.raises(ValueError):
        orc.smooth(c, 1, 1.0, 1, cells=[16])


def test_union_max(orc):
    r = np.random.default_rng(4)
    g = [r.random((5, 7, 9)).astype(np.float32) for _ in range(6)]
    g[2][0] = 0.0
    u = orc.union_max(g)
    assert np.array_equal(u, np.maximum.reduce(g))
    assert np.all(np.any(np.stack(g) == u[None], axis=0))
    assert np.array_equal(orc.union_max(g[:1]), g[0])
