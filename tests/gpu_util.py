"""Helpers for the GPU tests: move a workload to the device, run the C ABI, and compare
with the FP64 oracle at the stated tolerance."""

from __future__ import annotations

import numpy as np
import torch

import paper_2406_03726_amd as gee

# Z tolerance: max relative error over entries whose oracle value is non-zero, with FP32
# accumulation against the FP64 oracle; entries the oracle gives as exactly 0 must be 0.
RTOL = 1e-5

DEV = torch.device("cuda:0")


def to_dev(a, dtype):
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def graph_tensors(g):
    return (to_dev(g.src, torch.int32), to_dev(g.dst, torch.int32), to_dev(g.w, torch.float32),
            to_dev(g.labels, torch.int32))


def flags(g):
    return gee.flags_of(g.diag, g.lap, g.cor, g.sym, getattr(g, "deg_io", False))


def embed_graph(g, sched=None):
    s, d, w, lab = graph_tensors(g)
    Z = gee.gee_embed(s, d, w, lab, g.K, flags(g), sched=sched)
    torch.cuda.synchronize()
    return Z


def max_rel_error(Z, R):
    """Largest elementwise relative error over the entries where the oracle is non-zero
    (the 1e-5 bar is relative to each entry); also whether the entries where the oracle is
    exactly zero are exactly zero."""
    Zg = Z.detach().cpu().double().numpy().reshape(R.shape)
    nz = R != 0
    zero_ok = np.all(Zg[~nz] == 0)
    rel = float(np.max(np.abs(Zg[nz] - R[nz]) / np.abs(R[nz]))) if nz.any() else 0.0
    return rel, zero_ok


def rownorm_error(Z, R):
    """Row-normwise error max_i |dZ_i|_inf / |R_i|_inf for signed weights (cancellation)."""
    Zg = Z.detach().cpu().double().numpy().reshape(R.shape)
    rmax = np.max(np.abs(R), axis=1)
    d = np.max(np.abs(Zg - R), axis=1)
    ok = rmax > 0
    err = float(np.max(d[ok] / rmax[ok])) if ok.any() else 0.0
    zero_rows_ok = np.all(d[~ok] <= 1e-30)
    return err, zero_rows_ok


def assert_close(Z, R, what="", rtol=RTOL):
    rel, zero_ok = max_rel_error(Z, R)
    assert zero_ok, f"{what}: non-zero where the oracle is exactly zero"
    assert rel <= rtol, f"{what}: max relative error {rel:.3e} > {rtol:.1e}"
    return rel
