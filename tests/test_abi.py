"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function declared in include/capred.h, and rejects invalid arguments
with CAP_E_INVALID before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cap():
    from paper_2603_01122_amd import capred
    return capred


def declared_functions():
    src = open(os.path.join(ROOT, "include", "capred.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cap_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(cap):
    names = declared_functions()
    assert len(names) >= 20
    lib = C.CDLL(cap.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(cap.EXPORTED) >= set(names)


def test_abi_version(cap):
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "capred.h")).read()
    assert cap.abi_version() == int(re.search(r"#define CAP_ABI_VERSION (\d+)", hdr).group(1))


def _model(K=8, B=2, G=2, beta=None):
    beta = np.ones(B, np.float32) if beta is None else np.asarray(beta, np.float32)
    return C_model_keep(K, beta, np.zeros((G, 2), np.float32))


class C_model_keep:
    def __init__(self, K, beta, goals, speed=1.0, dt=0.1):
        from paper_2603_01122_amd import capred
        self.m = capred.Model(K, speed, dt, beta, goals)
        self.c = self.m.c()


@pytest.mark.parametrize("K,B,G,beta,msg", [
    (1, 2, 2, None, "K"), (33, 2, 2, None, "K"), (8, 0, 2, None, "B"), (8, 17, 2, None, "B"),
    (8, 2, 0, None, "G"), (8, 2, 65, None, "G"), (8, 16, 40, None, "G * B"),
    (8, 2, 2, [1.0, 0.0], "beta"), (8, 2, 2, [1.0, float("nan")], "beta")])
def test_invalid_models_rejected(cap, K, B, G, beta, msg):
    mk = _model(K, B, G, beta)
    rc = cap._lib.cap_belief_update(C.byref(mk.c), C.c_void_p(8), 1, C.c_void_p(8), None, None)
    assert rc == cap.CAP_E_INVALID
    assert msg in cap._lib.cap_last_error().decode()


def test_invalid_predict_arguments(cap):
    mk = _model()
    z = (C.c_double * 2)(1.0, 1.0)
    good = cap.grid_c((0, 0, 0.1, 16, 16))
    p = C.c_void_p(256)
    f = cap._lib.cap_predict_occupancy
    cases = [
        dict(grid=cap.grid_c((0, 0, 0.0, 16, 16))),
        dict(grid=cap.grid_c((0, 0, 0.1, 0, 16))),
        dict(grid=cap.grid_c((0, 0, 0.1, 16, 20000))),
        dict(N=0), dict(N=(1 << 30) + 1), dict(H=0), dict(H=5000), dict(cycle=0x7FFFFFFF),
        dict(belief=None), dict(counts=None),
        dict(grid=cap.grid_c((0, 0, 1e-9, 16, 16))),      # step < 2 lattice units? no: huge
        dict(z=(C.c_double * 2)(1e12, 0.0)),
    ]
    for c in cases:
        rc = f(C.byref(mk.c), C.byref(c.get("grid", good)), c.get("z", z), c.get("belief", p),
               c.get("N", 100), c.get("H", 10), 0, 0, c.get("cycle", 0), c.get("counts", p), None,
               None, None, None)
        assert rc == cap.CAP_E_INVALID, (c, cap._lib.cap_last_error())


def test_tiny_step_rejected(cap):
    from paper_2603_01122_amd import capred
    m = capred.Model(8, 1e-9, 1e-3, [1.0], [[0.0, 0.0]])
    mc = m.c()
    z = (C.c_double * 2)(0.0, 0.0)
    g = capred.grid_c((0, 0, 0.1, 8, 8))
    p = C.c_void_p(256)
    rc = capred._lib.cap_predict_occupancy(C.byref(mc), C.byref(g), z, p, 10, 2, 0, 0, 0, p, None,
                                           None, None, None)
    assert rc == capred.CAP_E_INVALID and "lattice" in capred._lib.cap_last_error().decode()


def test_invalid_loglik_and_workspace(cap):
    f = cap._lib.cap_loglik_backward
    p = C.c_void_p(256)
    need = cap._lib.cap_loglik_backward_workspace(10, 3, 4, 0)
    assert need == 10 * 3 * 6 * 8
    rc = f(8, 1.0, 0.1, p, p, 10, 5, p, 3, p, 4, 0, p, p, p, p, need - 1, None)
    assert rc == cap.CAP_E_WORKSPACE
    rc = f(8, 1.0, 0.1, p, p, 10, 5, p, 3, p, 0, 0, p, p, p, p, need, None)
    assert rc == cap.CAP_E_INVALID
    rc = cap._lib.cap_loglik(1, 1.0, 0.1, p, p, 10, 5, p, 3, p, 4, 0, p, None)
    assert rc == cap.CAP_E_INVALID
    # N * G above 2^25 (one wave per (track, goal) at most must keep int thread indices)
    rc = cap._lib.cap_loglik(8, 1.0, 0.1, p, p, (1 << 22) + 1, 5, p, 8, p, 4, 0, p, None)
    assert rc == cap.CAP_E_INVALID and b"2^25" in cap._lib.cap_last_error()
    rc = f(8, 1.0, 0.1, p, p, (1 << 22) + 1, 5, p, 8, p, 4, 0, p, p, p, p, 1 << 40, None)
    assert rc == cap.CAP_E_INVALID
    rc = cap._lib.cap_normalize(p, 10, 0, p, None)
    assert rc == cap.CAP_E_INVALID
    rc = cap._lib.cap_philox_blocks(-1, 0, 0, 0, 0, 0, p, None)
    assert rc == cap.CAP_E_INVALID
    rc = cap._lib.cap_simulate_tracks(8, 1.0, 0, None, 0.1, 0, 0, 0.0, 4, 10, p, p, p, 0, 0, p, p,
                                      None)
    assert rc == cap.CAP_E_INVALID


def test_invalid_control_sets(cap):
    """Multi-speed control sets are validated on the host before any launch."""
    p = C.c_void_p(256)
    grid = cap.grid_c((0.0, 0.0, 0.1, 16, 16))
    z0 = (C.c_double * 2)(0.8, 0.8)

    def predict(m):
        return cap._lib.cap_predict_occupancy(C.byref(m.c()), C.byref(grid), z0, p, 100, 5, 0, 0,
                                              0, p, p, None, None, None)
    beta, goals = np.ones(2, np.float32), np.array([[1.0, 1.0]], np.float32)
    cases = [
        (cap.Model(16, 1.0, 0.1, beta, goals, speeds=np.full(9, 0.5)), cap.CAP_E_INVALID),
        (cap.Model(16, 1.0, 0.1, beta, goals, speeds=[0.5, 0.0]), cap.CAP_E_INVALID),
        (cap.Model(32, 1.0, 0.1, beta, goals, speeds=[0.3, 0.6, 0.9, 1.2, 1.5]), cap.CAP_E_INVALID),
        (cap.Model(16, 1.0, 0.1, beta, goals, speeds=[0.5, 1.0], speed_mask=0b100),
         cap.CAP_E_INVALID),
        (cap.Model(12, 1.0, 0.1, beta, goals, speeds=[0.5, 1.0]), cap.CAP_E_UNSUPPORTED),
    ]
    for m, want in cases:
        assert predict(m) == want, cap._lib.cap_last_error().decode()
    assert cap._lib.cap_simulate_tracks(16, 1.0, 2, (C.c_double * 2)(0.5, -1.0), 0.1, 0, 0, 0.1,
                                        4, 10, p, p, p, 0, 0, p, p, None) == cap.CAP_E_INVALID


def test_invalid_mppi(cap):
    """MPPI arguments are validated on the host before any launch."""
    p = C.c_void_p(256)
    z = (C.c_double * 4)(0, 0, 1, 0)
    grid = cap.grid_c((0.0, 0.0, 0.1, 16, 16))

    def cost(tau):
        return cap.cap_mppi_cost((C.c_double * 4)(3, 3, 10, 0), (C.c_double * 4)(0.6, 0.6, 2, 0),
                                 (C.c_double * 2)(2, 1), 1000.0, 0.1, 0.0, tau)
    f = cap._lib.cap_mppi_step
    assert f(z, z, 4, 0.1, 8, p, p, p, 3, C.byref(grid), C.byref(cost(0.0)), p, None) == \
        cap.CAP_E_INVALID
    assert f(z, z, 0, 0.1, 8, p, p, None, 0, None, C.byref(cost(1.0)), p, None) == \
        cap.CAP_E_INVALID
    assert f(z, z, 4, 0.1, 8, p, C.c_void_p(264), None, 0, None, C.byref(cost(1.0)), p,
             None) == cap.CAP_E_INVALID                                   # misaligned delta
    assert f(z, z, 4, 0.1, 8, p, p, p, 3, None, C.byref(cost(1.0)), p, None) == \
        cap.CAP_E_INVALID                                                 # occupancy, no grid


def test_invalid_probe_arguments(cap):
    """The measurement probes validate their arguments before any launch."""
    p = C.c_void_p(256)
    f = cap._lib.cap_probe_global_atomic
    assert f(1, 1, None, 10, None) == cap.CAP_E_INVALID          # no buffer
    assert f(1, 1, p, 5, None) == cap.CAP_E_INVALID              # below 2^6 words
    assert f(1, 1, p, 31, None) == cap.CAP_E_INVALID             # above 2^30 words
    assert f(0, 1, p, 10, None) == cap.CAP_E_INVALID
    assert f(1, 0, p, 10, None) == cap.CAP_E_INVALID
    assert cap._lib.cap_probe(7, 1, 1, p, None) == cap.CAP_E_INVALID
    assert cap._lib.cap_probe(0, 1, 1, None, None) == cap.CAP_E_INVALID
