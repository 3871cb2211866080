"""The GEE_DEBUG build (internal index checks compiled into the kernels) on the GPU: on
the workloads below it must raise no GEE_DATA_INTERNAL bit and give bitwise the same CSR
and Z as the release build (the checks change no arithmetic). Both libraries are loaded
in this one process, each with its own device state, through the same C ABI."""

import ctypes
import os

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from paper_2406_03726_amd import _lib
from paper_2406_03726_amd.build import LIB_DEBUG
from gee_workloads import powerlaw_10m, random_small_graph

from gpu_util import flags, graph_tensors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dbg():
    if not os.path.exists(LIB_DEBUG):
        pytest.fail(f"{LIB_DEBUG} is missing: build() makes it beside libgee.so")
    lib = ctypes.CDLL(LIB_DEBUG)
    for name, (res, args) in _lib.SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def _p(t):
    return None if t is None else t.data_ptr()


def _bits(lib):
    b = ctypes.c_uint32(0)
    assert lib.gee_get_data_errors(None, ctypes.byref(b)) == 0
    return b.value


def _embed(lib, g, sched=None):
    s, d, w, lab = graph_tensors(g)
    f = flags(g)
    sp = None if sched is None else ctypes.byref(gee.schedule(**sched))
    nb = lib.gee_embed_workspace_bytes(g.E, g.N, g.K, f, int(w is not None), sp)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    Z = torch.full((g.N, g.K), float("nan"), dtype=torch.float32, device="cuda")
    rc = lib.gee_embed_ws(_p(s), _p(d), _p(w), g.E, g.N, _p(lab), g.K, f, _p(Z), sp, _p(ws), nb, None)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return Z


@pytest.mark.parametrize("case", ["powerlaw_10m", "k128", "split_buckets", "small_directed"])
def test_debug_embed_matches_release_without_internal_errors(dbg, case):
    if case == "powerlaw_10m":
        g = powerlaw_10m()
    elif case == "k128":
        g = powerlaw_10m(N=200_000, E=2_000_000, K=128)
    elif case == "split_buckets":  # hub rows: buckets cut into several parts
        g = powerlaw_10m(N=50_000, E=1_000_000, K=33, dmax=20_000.0)
    else:
        g = random_small_graph(77, N=3000, E=30_000, K=7, sym=False).with_options(True, True, True)
    print(f"[gpu-test] debug build {case} N={g.N} E={g.E} K={g.K}", flush=True)
    _bits(dbg)
    Zd = _embed(dbg, g)
    assert _bits(dbg) == 0, "the debug build reported an internal or data error"
    Zr = _embed(_lib.load(), g)
    assert torch.equal(Zd, Zr)


def test_debug_csr_paths_without_internal_errors(dbg):
    """gee_build_csr through both partition passes and pass C (hub rows) and gee_embed_csr."""
    g = powerlaw_10m(N=300_000, E=1_500_000, K=4, dmax=20_000.0)
    print(f"[gpu-test] debug build CSR N={g.N} E={g.E}", flush=True)
    s, d, w, lab = graph_tensors(g)
    f = flags(g)
    for sb in (3, 9):
        sc = gee.schedule(bucket_rows_log2=sb)
        nb = dbg.gee_build_csr_workspace_bytes(g.E, g.N, f, ctypes.byref(sc))
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        cap = 2 * g.E
        rp = torch.empty(g.N + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(cap, dtype=torch.int32, device="cuda")
        val = torch.empty(cap, dtype=torch.float32, device="cuda")
        _bits(dbg)
        assert dbg.gee_build_csr_ws(_p(s), _p(d), _p(w), g.E, g.N, f, _p(rp), _p(col), _p(val), ctypes.byref(sc),
                                    _p(ws), nb, None) == 0
        torch.cuda.synchronize()
        assert _bits(dbg) == 0
        rr, cr, vr = gee.gee_build_csr(s, d, w, g.N, f, sched=dict(bucket_rows_log2=sb))
        torch.cuda.synchronize()
        M = int(rr[-1].item())
        assert torch.equal(rp, rr) and torch.equal(col[:M], cr[:M]) and torch.equal(val[:M], vr[:M])
    M = int(rp[-1].item())
    Z = torch.empty((g.N, g.K), dtype=torch.float32, device="cuda")
    nb = dbg.gee_embed_csr_workspace_bytes(M, g.N, g.K, f, None)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    assert dbg.gee_embed_csr_ws(_p(rp), _p(col), _p(val), M, g.N, _p(lab), g.K, f, _p(Z), None, _p(ws), nb,
                                None) == 0
    torch.cuda.synchronize()
    assert _bits(dbg) == 0
    Zr = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f)
    torch.cuda.synchronize()
    assert torch.equal(Z, Zr)
