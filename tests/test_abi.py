"""The C-ABI library loads on any host and exports every symbol kc.h declares.

No compute call is made here: these tests run without a GPU.
"""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1712_03254_amd as kc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = kc.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(kc.EXPORTED) == names


def test_abi_version_and_status_strings():
    text = open(HEADER).read() if os.path.exists(HEADER) else ""
    want = int(re.search(r"#define KC_ABI_VERSION (\d+)u", text).group(1))
    assert kc.kc_abi_version() == want
    lib = kc.load()
    assert lib.kc_status_str(0) == b"KC_OK"
    assert lib.kc_status_str(-5) == b"KC_ERR_OVER_BUDGET"


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "lay.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "kc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(kc_config),
         offsetof(kc_config, seed), offsetof(kc_config, group_bases_log2),
         offsetof(kc_config, hbm_table_budget_bytes), sizeof(kc_stats),
         offsetof(kc_stats, kernel_ms), offsetof(kc_stats, kernel_launches), sizeof(kc_chunk),
         offsetof(kc_chunk, total_bases), sizeof(kc_tune_trial), offsetof(kc_tune_trial, ms));
  printf("%zu %zu %zu %zu %zu\n", sizeof(kc_request), offsetof(kc_request, n_parts),
         sizeof(kc_response), offsetof(kc_response, ctx), offsetof(kc_response, footprint_bytes));
  printf("%zu %zu %zu %zu %zu\n", offsetof(kc_config, shuffle_tile_log2),
         offsetof(kc_tune_trial, shuffle_tile_log2), offsetof(kc_request, ready_event),
         sizeof(kc_server_stats), offsetof(kc_server_stats, device_frees));
  return 0;
}
''')
    exe = tmp_path / "lay"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(kc.KcConfig), kc.KcConfig.seed.offset,
            kc.KcConfig.group_bases_log2.offset, kc.KcConfig.hbm_table_budget_bytes.offset,
            ctypes.sizeof(kc.KcStats), kc.KcStats.kernel_ms.offset,
            kc.KcStats.kernel_launches.offset, ctypes.sizeof(kc.KcChunk),
            kc.KcChunk.total_bases.offset, ctypes.sizeof(kc.KcTuneTrial), kc.KcTuneTrial.ms.offset,
            ctypes.sizeof(kc.KcRequest), kc.KcRequest.n_parts.offset, ctypes.sizeof(kc.KcResponse),
            kc.KcResponse.ctx.offset, kc.KcResponse.footprint_bytes.offset,
            kc.KcConfig.shuffle_tile_log2.offset, kc.KcTuneTrial.shuffle_tile_log2.offset,
            kc.KcRequest.ready_event.offset, ctypes.sizeof(kc.KcServerStats),
            kc.KcServerStats.device_frees.offset]
    assert got == want


@pytest.mark.parametrize("field,value", [("k", 0), ("k", 32), ("n_counters", 3),
                                         ("min_count", 1), ("bloom_hashes", 9),
                                         ("bloom_block_log2", 20), ("bloom_bits_log2", 41),
                                         ("shuffle_tile_log2", 9), ("shuffle_tile_log2", 14),
                                         ("group_bases_log2", 9), ("group_bases_log2", 33)])
def test_config_validation_without_device(field, value):
    cfg = kc.Config(k=21, bloom_bits_log2=20, bloom_hashes=3, bloom_block_log2=12)
    setattr(cfg, field, value)
    with pytest.raises(kc.KcError) as e:
        kc.kc_create(cfg.c(), 0)
    assert e.value.status == kc.KC_ERR_INVALID_ARG


def test_null_context_calls_are_rejected():
    lib = kc.load()
    assert lib.kc_finalize(None, None, None) == kc.KC_ERR_INVALID_ARG
    assert lib.kc_reset(None) == kc.KC_ERR_INVALID_ARG
    lib.kc_destroy(None)
    assert lib.kc_server_set_overlap(None, 1) == kc.KC_ERR_INVALID_ARG
    assert lib.kc_server_release(None, 1) == kc.KC_ERR_INVALID_ARG


def test_probe_library_exports_and_checks_arguments():
    from paper_1712_03254_amd import probe
    text = open(os.path.join(ROOT, "include", "kc_probe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(kcp_[a-z_0-9]+)\s*\(", text)))
    assert names == sorted(probe.EXPORTED)
    lib = probe.load()
    for n in names:
        assert hasattr(lib, n), n
    ms, chk = ctypes.c_float(), ctypes.c_uint64()
    # argument checks run before any device call
    assert lib.kcp_lds_atomics(7, 13, 1, 1, ctypes.byref(ms), ctypes.byref(chk)) == -1
    assert lib.kcp_lds_atomics(0, 16, 1, 1, ctypes.byref(ms), ctypes.byref(chk)) == -1
    assert lib.kcp_lds_atomics(0, 13, 0, 1, ctypes.byref(ms), ctypes.byref(chk)) == -1
    assert lib.kcp_lds_atomics(0, 13, 1, 0, ctypes.byref(ms), ctypes.byref(chk)) == -1


def test_restore_rejects_bad_files_without_a_device(tmp_path):
    lib = kc.load()
    h = ctypes.c_void_p()
    missing = str(tmp_path / "none.kcckpt").encode()
    assert lib.kc_restore(missing, 0, ctypes.byref(h)) == kc.KC_ERR_INVALID_ARG
    junk = tmp_path / "junk.kcckpt"
    junk.write_bytes(bytes(range(256)) * 64)
    assert lib.kc_restore(str(junk).encode(), 0, ctypes.byref(h)) == kc.KC_ERR_INVALID_ARG
    assert b"magic" in lib.kc_last_error(None)
    # right magic, another ABI version
    other = tmp_path / "other.kcckpt"
    other.write_bytes(b"KCCKPT\x00\x01" + (999).to_bytes(4, "little") + bytes(4096))
    assert lib.kc_restore(str(other).encode(), 0, ctypes.byref(h)) == kc.KC_ERR_INVALID_ARG
    assert b"ABI" in lib.kc_last_error(None)
    # right magic and version, truncated
    short = tmp_path / "short.kcckpt"
    short.write_bytes(b"KCCKPT\x00\x01" + kc.kc_abi_version().to_bytes(4, "little") + bytes(16))
    assert lib.kc_restore(str(short).encode(), 0, ctypes.byref(h)) == kc.KC_ERR_INVALID_ARG
    assert not h.value


class _CkptHeader(ctypes.Structure):
    """The checkpoint header as the writer lays it out (a test-side copy)."""
    _fields_ = [("magic", ctypes.c_uint8 * 8), ("abi_version", ctypes.c_uint32),
                ("reserved_", ctypes.c_uint32), ("header_bytes", ctypes.c_uint64),
                ("cfg", kc.KcConfig), ("p_log2", ctypes.c_uint32), ("cap", ctypes.c_uint32),
                ("n_counters", ctypes.c_uint32), ("ovf_log2", ctypes.c_uint32),
                ("n_parts", ctypes.c_uint64), ("bloom_words64", ctypes.c_uint64),
                ("records_offset", ctypes.c_uint64), ("b1_offset", ctypes.c_uint64),
                ("b2_offset", ctypes.c_uint64), ("ovf_keys_offset", ctypes.c_uint64),
                ("ovf_counts_offset", ctypes.c_uint64), ("file_bytes", ctypes.c_uint64),
                ("stats", kc.KcStats)]


def test_restore_checks_the_file_size_before_allocating(tmp_path):
    """A header whose sections are consistent but declare a 2^34-entry overflow
    table and 2^36-bit Bloom levels (about 160 GiB), on a file of a few KiB:
    refused from the file size, before any buffer is sized from the header."""
    lib = kc.load()
    hd = _CkptHeader()
    hd.magic = (ctypes.c_uint8 * 8)(*b"KCCKPT\x00\x01")
    hd.abi_version = kc.kc_abi_version()
    hd.p_log2, hd.cap, hd.n_counters, hd.ovf_log2 = 4, 4096, 2, 34
    hd.n_parts, hd.bloom_words64 = 16, 1 << 30
    hd.records_offset = ctypes.sizeof(_CkptHeader)
    hd.header_bytes = (hd.records_offset + 16 * 24 + 4095) // 4096 * 4096
    table = hd.cap * 8 + hd.cap * 4 * hd.n_counters
    hd.b1_offset = hd.header_bytes + hd.n_parts * table
    hd.b2_offset = hd.b1_offset + hd.bloom_words64 * 8
    hd.ovf_keys_offset = hd.b2_offset + hd.bloom_words64 * 8
    hd.ovf_counts_offset = hd.ovf_keys_offset + (8 << 34)
    hd.file_bytes = hd.ovf_counts_offset + (8 << 34)
    recs = b"".join(u.to_bytes(4, "little") + bytes(4) +
                    (hd.header_bytes + u * table).to_bytes(8, "little") + bytes(8)
                    for u in range(16))
    path = tmp_path / "huge.kcckpt"
    path.write_bytes(bytes(hd) + recs + bytes(4096))
    h = ctypes.c_void_p()
    assert lib.kc_restore(str(path).encode(), 0, ctypes.byref(h)) == kc.KC_ERR_INVALID_ARG
    assert b"file size" in lib.kc_last_error(None)
    assert not h.value
