"""The FP64 oracle pinned against references outside itself (CPU only)."""

import dataclasses

import numpy as np
import pytest

import pins
from gee_workloads import powerlaw_10m, random_small_graph, sbm_dense, sbm_small
from oracle import oracle as orc


@pytest.fixture(scope="module")
def lib():
    return orc.load()


def test_brute_force(lib):
    pins.pin_brute_force(lib)


def test_hand_worked(lib):
    pins.pin_hand_worked(lib)


def test_closed_forms(lib):
    pins.pin_closed_forms(lib)


def test_directed_degrees(lib):
    pins.pin_directed_degrees(lib)


def test_scipy_route_directed_degrees(lib):
    gs = []
    for seed in range(3):
        g = random_small_graph(seed, N=150, E=1200, K=4, weighted=True, sym=False)
        for d, c in ((False, False), (True, False), (True, True)):
            gs.append(dataclasses.replace(g.with_options(d, True, c, name=f"io{seed}{d}{c}"), deg_io=True))
    pins.pin_scipy_route(lib, gs)


def test_laplacian_symmetric(lib):
    pins.pin_laplacian_symmetric(lib)


def test_degrees(lib):
    pins.pin_degrees(lib)


def test_scipy_route_small(lib):
    gs = []
    for seed in range(4):
        for sym in (True, False):
            g = random_small_graph(seed, N=200, E=1500, K=5, weighted=bool(seed % 2), sym=sym)
            for d, l, c in pins.FLAG_COMBOS:
                gs.append(g.with_options(d, l, c, name=f"rand{seed}_{sym}_{d}{l}{c}"))
    pins.pin_scipy_route(lib, gs)


def test_scipy_route_sbm_small(lib):
    pins.pin_scipy_route(lib, [sbm_small("off"), sbm_small("all")])


@pytest.mark.slow
def test_scipy_route_sbm_dense(lib):
    pins.pin_scipy_route(lib, [sbm_dense()])


def test_scipy_route_powerlaw_scaled(lib):
    # the power-law recipe at 1/20 of the edges: hubs, weights, unknown labels, K = 50
    g = powerlaw_10m(N=60_000, E=500_000, K=50, dmax=5_000.0)
    pins.pin_scipy_route(lib, [g, g.with_options(False, False, False, name="pl_off")])


def test_invariants_random(lib):
    for seed in range(3):
        for sym in (True, False):
            g = random_small_graph(seed, N=300, E=2000, K=6, weighted=True, sym=sym)
            pins.pin_invariants(lib, g)


def test_invariants_sbm(lib):
    pins.pin_invariants(lib, sbm_small("off"))


def test_sbm_statistics(lib):
    pins.pin_sbm_statistics(lib, sbm_small("off"), 0.13, 0.10)


def test_error_codes(lib):
    s = np.array([0, 1], np.int32)
    d = np.array([1, 2], np.int32)
    lab = np.array([0, 1, 0], np.int32)
    with pytest.raises(orc.OracleError) as e:
        orc.embed(s, d, None, 3, np.array([0, 2, 0], np.int32), 2, lib=lib)
    assert e.value.code == -2
    with pytest.raises(orc.OracleError) as e:
        orc.embed(s, np.array([1, 3], np.int32), None, 3, lab, 2, lib=lib)
    assert e.value.code == -3
    with pytest.raises(orc.OracleError) as e:
        orc.embed(s, d, np.array([1.0, np.nan], np.float32), 3, lab, 2, lib=lib)
    assert e.value.code == -4
    with pytest.raises(orc.OracleError) as e:
        orc.embed(s, d, None, 3, lab, 0, lib=lib)
    assert e.value.code == -1
