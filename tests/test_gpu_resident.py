"""gee_embed_csr on the bucket kernels (the default for a resident CSR of at most 2^22 rows):
the rows of each bucket's entries come from row_ptr alone. Checked against the FP64 oracle at
the 1e-5 bar on graphs with split buckets (hub rows), 32-row buckets (K > 64), empty rows,
a ragged last bucket, every option combination and unweighted CSRs; two calls are bitwise
equal, and the CSR path's own kernels (a CSR-path schedule) meet the same bar on the same
graphs. A malformed CSR (row pointers out of order, a wrong last pointer, columns outside
[0, N)) raises GEE_DATA_CSR on the call's stream and no other bit; with GEE_NO_VALIDATE it
raises nothing. Needs an MI355X."""

import numpy as np
import pytest
import torch

import paper_2406_03726_amd as gee
from gee_workloads import powerlaw_10m, random_small_graph
from oracle import embed_graph as or_embed_graph

from gpu_util import assert_close, flags, graph_tensors

pytestmark = pytest.mark.gpu

CSR_PATH = dict(wave_entries=1024, waves_per_block=1)  # a schedule that keeps the CSR path's kernels


def _label(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _resident(g):
    s, d, w, lab = graph_tensors(g)
    f = flags(g)
    rp, col, val = gee.gee_build_csr(s, d, w, g.N, f)
    torch.cuda.synchronize()
    return rp, col, val, int(rp[-1].item()), lab, f


CASES = {
    "small_all_options": lambda: random_small_graph(21, N=3000, E=40_000, K=8, weighted=True).with_options(
        True, True, True),
    "hubs_split_buckets": lambda: powerlaw_10m(N=50_000, E=1_000_000, K=33, dmax=20_000.0),
    "k128_ragged": lambda: powerlaw_10m(N=100_003, E=800_000, K=128),
    "k1_unweighted_no_options": lambda: random_small_graph(22, N=4097, E=30_000, K=1, weighted=False),
    "isolated_rows": lambda: random_small_graph(23, N=20_000, E=3_000, K=5, weighted=True).with_options(
        True, True, False),
    "directed_rows": lambda: random_small_graph(24, N=6000, E=50_000, K=12, sym=False).with_options(
        False, True, True),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_resident_bucket_kernels_match_oracle(case):
    g = CASES[case]()
    _label(f"resident CSR, bucket kernels: {case} N={g.N} E={g.E} K={g.K}")
    rp, col, val, M, lab, f = _resident(g)
    gee.gee_get_data_errors()
    Z1 = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f)
    Z2 = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f)
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() == 0
    assert torch.equal(Z1, Z2), "two calls differ"
    R = or_embed_graph(g)
    assert_close(Z1, R, f"{case} (bucket kernels)")
    Zc = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f, sched=CSR_PATH)
    torch.cuda.synchronize()
    assert_close(Zc, R, f"{case} (CSR path's kernels)")


def test_resident_bucket_sizes_from_schedule():
    """bucket_rows_log2 5 and 6 choose 32- or 64-row buckets; both meet the bar."""
    g = powerlaw_10m(N=40_000, E=500_000, K=20, dmax=9000.0)
    rp, col, val, M, lab, f = _resident(g)
    R = or_embed_graph(g)
    for sb in (5, 6):
        for we in (2048, 8192):
            _label(f"resident CSR, bucket_rows_log2={sb} wave_entries={we}")
            Z = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f, sched=dict(bucket_rows_log2=sb, wave_entries=we))
            torch.cuda.synchronize()
            assert_close(Z, R, f"sb={sb} we={we}")


def _bits_after(rp, col, val, M, lab, K, f):
    gee.gee_get_data_errors()
    gee.gee_embed_csr(rp, col, val, M, lab, K, f)
    torch.cuda.synchronize()
    return gee.gee_get_data_errors()


@pytest.mark.parametrize("fault", ["decreasing_row_ptr", "last_pointer", "first_pointer", "column_past_n",
                                   "negative_column"])
def test_resident_bucket_malformed_csr_is_reported(fault):
    g = random_small_graph(25, N=5000, E=60_000, K=6, weighted=True).with_options(True, True, True)
    rp, col, val, M, lab, f = _resident(g)
    rp2, col2 = rp.clone(), col.clone()
    if fault == "decreasing_row_ptr":
        rp2[2500] = rp2[2600] + 5  # row 2499 ends after row 2500 starts
    elif fault == "last_pointer":
        rp2[-1] = M - 1
    elif fault == "first_pointer":
        rp2[0] = 3
    elif fault == "column_past_n":
        col2[M // 2] = g.N + 7
    else:
        col2[M // 3] = -4
    _label(f"malformed resident CSR: {fault}")
    bits = _bits_after(rp2, col2, val, M, lab, g.K, f)
    assert bits == gee.GEE_DATA_CSR, bits
    bits = _bits_after(rp2, col2, val, M, lab, g.K, f | gee.GEE_NO_VALIDATE)
    assert bits == 0, bits
    # the well-formed CSR afterwards: no bits, the oracle's Z
    gee.gee_get_data_errors()
    Z = gee.gee_embed_csr(rp, col, val, M, lab, g.K, f)
    torch.cuda.synchronize()
    assert gee.gee_get_data_errors() == 0
    assert_close(Z, or_embed_graph(g), "well-formed CSR after a malformed one")
