"""CPU checks of the C ABI: the library loads and exports every declared entry point,
and host-side argument checks answer without touching a device."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gee.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gee_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_03726_amd import _lib

    if not os.path.exists(_lib.LIB):
        import __graft_entry__

        __graft_entry__.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gee_embed", "gee_embed_ws", "gee_build_csr", "gee_embed_csr", "gee_class_counts",
                     "gee_get_data_errors", "gee_status_string"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in gee.h but not exported"


def test_binding_covers_every_symbol():
    from paper_2406_03726_amd import _lib

    assert set(declared_functions()) == set(_lib.SYMBOLS)


def test_header_compiles_as_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "gee.h"\nint main(void){ return GEE_ABI_VERSION == 1 ? 0 : 1; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}", "-c", str(src),
                    "-o", str(tmp_path / "t.o")], check=True)


def test_host_only_queries(lib):
    assert lib.gee_abi_version() == 1
    assert lib.gee_status_string(0) == b"ok"
    assert lib.gee_csr_capacity(10, 8) == 20
    assert lib.gee_csr_capacity(10, 0) == 10
    # workspace sizing is pure host arithmetic
    assert lib.gee_embed_workspace_bytes(1000, 100, 3, 15, 1, None) > 0
    assert lib.gee_embed_workspace_bytes(-1, 100, 3, 15, 1, None) == 0
    assert lib.gee_embed_workspace_bytes(1000, 100, 0, 15, 1, None) == 0       # K < 1
    assert lib.gee_embed_workspace_bytes(1000, 100, 129, 15, 1, None) == 0     # K beyond the build
    assert lib.gee_embed_workspace_bytes(1000, 100, 3, 1 << 9, 1, None) == 0    # unknown flag bit
    big = lib.gee_embed_workspace_bytes(2 ** 30, 100, 3, 8, 1, None)
    assert big == 0  # 2^31 entries exceed the int32 CSR
    # original GEE form: counts, per-node table and (Laplacian) degrees, each 256-byte aligned
    assert lib.gee_embed_atomic_workspace_bytes(1000, 3, 8) == 256 + 8192
    assert lib.gee_embed_atomic_workspace_bytes(1000, 3, 15) == 256 + 8192 + 4096
    assert lib.gee_embed_atomic_workspace_bytes(1000, 0, 15) == 0
    assert lib.gee_embed_atomic_workspace_bytes(1000, 129, 15) == 0
    assert lib.gee_embed_atomic_workspace_bytes(-1, 3, 15) == 0
    assert lib.gee_embed_atomic_workspace_bytes(1000, 3, 1 << 9) == 0
    assert lib.gee_embed_atomic_workspace_bytes(2 ** 24 + 1, 3, 15) == 0  # beyond the node limit
    # sparse Z: the embed workspace, room for N K staged (class, value) pairs (twice a dense Z),
    # one int per 256-row tile and one per row
    e = lib.gee_embed_sparse_workspace_bytes(1000, 3000, 5, 15, 1, None)
    assert e >= lib.gee_embed_workspace_bytes(1000, 3000, 5, 15, 1, None) + 2 * 3000 * 5 * 4 + 12 * 4 + 3000 * 4
    assert lib.gee_embed_sparse_workspace_bytes(-1, 3000, 5, 15, 1, None) == 0
    assert lib.gee_embed_sparse_workspace_bytes(1000, 3000, 0, 15, 1, None) == 0
    assert lib.gee_embed_sparse_workspace_bytes(1000, 2 ** 24, 128, 15, 1, None) == 0  # N * K = 2^31


def test_schedule_validation(lib):
    from paper_2406_03726_amd._lib import GeeSchedule

    s = GeeSchedule(0, 0, 0, 0)
    assert lib.gee_default_schedule(10_000_000, 600_000, 50, 15, ctypes.byref(s)) == 0
    assert s.wave_entries >= 256 and 1 <= s.waves_per_block <= 4 and s.tile_entries == 4096
    bad = GeeSchedule(300, 0, 0, 0)  # not a power of two
    assert lib.gee_embed_workspace_bytes(1000, 100, 3, 15, 1, ctypes.byref(bad)) == 0


def test_default_bucket_part_size_follows_the_entries(lib):
    # the bucket path's default part: the largest power of two in [2048, 8192] that leaves at
    # least 2048 parts of the graph's CSR entries (2E under symmetrization; flags 15 = all
    # options with GEE_SYMMETRIZE)
    from paper_2406_03726_amd._lib import GeeSchedule

    def part(E, N, K):
        s = GeeSchedule(0, 0, 0, 0)
        assert lib.gee_default_schedule(E, N, K, 15, ctypes.byref(s)) == 0
        return s.wave_entries

    assert part(223_228, 2000, 3) == 2048            # 446k entries: 218 parts of 2048
    assert part(5_572_753, 10_000, 3) == 4096        # 11.1M entries: 2721 parts of 4096
    assert part(10_000_000, 600_000, 50) == 8192     # 20M entries: 2441 parts of 8192
    assert part(1000, 100, 3) == 2048                # tiny graphs: the smallest part
    assert part(400_000_000, 4_000_000, 50) == 8192  # large graphs: the largest default
    # the boundaries: 2048 parts of 4096 (8,388,608 entries) and of 8192 (16,777,216 entries)
    for e, at, below in ((8_388_608, 4096, 2048), (16_777_216, 8192, 4096)):
        assert part(e // 2, 100_000, 8) == at
        assert part(e // 2 - 1, 100_000, 8) == below
