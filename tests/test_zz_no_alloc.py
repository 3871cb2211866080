"""gee_embed_noalloc through the C ABI (needs an MI355X): the entry point that allocates
nothing and uses the library's fixed scratch. Two calls in a row, the second on a smaller
graph, each bitwise equal to gee_embed_ws with a caller workspace (the same kernels and
schedule) and within the oracle bar; a request beyond the scratch is refused on the host."""

import ctypes

import pytest
import torch

from gee_workloads import powerlaw_10m
from gee_workloads.configs import random_small_graph, sbm_small
from oracle import embed_graph as or_embed_graph
from paper_2406_03726_amd import _lib

from gpu_util import DEV, assert_close, flags, graph_tensors

pytestmark = pytest.mark.gpu

GEE_ERR_SCRATCH = -10


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(lib, g):
    s, d, w, lab = graph_tensors(g)
    Z = torch.full((g.N, g.K), float("nan"), dtype=torch.float32, device=DEV)
    rc = lib.gee_embed_noalloc(_p(s), _p(d), _p(w), g.E, g.N, _p(lab), g.K, flags(g), _p(Z), _stream())
    assert rc == 0, lib.gee_status_string(rc)
    return Z


def _with_workspace(lib, g):
    s, d, w, lab = graph_tensors(g)
    Z = torch.full((g.N, g.K), float("nan"), dtype=torch.float32, device=DEV)
    nb = lib.gee_embed_workspace_bytes(g.E, g.N, g.K, flags(g), int(w is not None), None)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    rc = lib.gee_embed_ws(_p(s), _p(d), _p(w), g.E, g.N, _p(lab), g.K, flags(g), _p(Z), None, _p(ws), nb,
                          _stream())
    assert rc == 0, lib.gee_status_string(rc)
    return Z


def test_noalloc_matches_the_workspace_entry_point():
    lib = _lib.load()
    assert lib.gee_init() == 0
    big = powerlaw_10m(N=200_000, E=2_000_000, K=50, dmax=20_000.0)  # hubs, weights, unknown labels
    small = sbm_small("all")
    tiny = random_small_graph(9, N=700, E=5000, K=70).with_options(True, True, False)
    for g in (big, small, tiny):
        print(f"[gpu-test] noalloc N={g.N} E={g.E} K={g.K}", flush=True)
        lib.gee_get_data_errors(_stream(), ctypes.byref(ctypes.c_uint32()))
        Za = _noalloc(lib, g)
        Zw = _with_workspace(lib, g)
        torch.cuda.synchronize()
        bits = ctypes.c_uint32(1)
        assert lib.gee_get_data_errors(_stream(), ctypes.byref(bits)) == 0 and bits.value == 0
        assert torch.equal(Za, Zw)
        assert_close(Za, or_embed_graph(g), f"noalloc N={g.N}")


def test_noalloc_refuses_requests_beyond_the_scratch():
    lib = _lib.load()
    cap = lib.gee_scratch_bytes()
    E, N, K = 10_000_000, 600_000, 50
    need = lib.gee_embed_workspace_bytes(E, N, K, 15, 1, None)
    assert need > cap
    one = torch.zeros(16, dtype=torch.int32, device=DEV)
    Z = torch.zeros(16, dtype=torch.float32, device=DEV)
    # refused on the host before anything is enqueued (the arrays are never touched)
    rc = lib.gee_embed_noalloc(_p(one), _p(one), _p(Z), E, N, _p(one), K, 15, _p(Z), _stream())
    assert rc == GEE_ERR_SCRATCH
    torch.cuda.synchronize()
