"""The C ABI library loads and exports every entry point include/rambo.h
declares; host-side argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1910_02611_amd import build as hipbuild
from paper_1910_02611_amd import rambo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = ""
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            with open(os.path.join(ROOT, "include", name)) as f:
                text += f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rambo_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if hipbuild.is_stale():
        hipbuild.build()
    return rambo.lib()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding knows every one of them
    assert set(syms) == set(rambo.EXPORTS)


def test_bad_config_is_rejected_on_the_host(lib):
    bad = [dict(K=0), dict(B=0), dict(B=11), dict(B=5000, K=6000), dict(R=0), dict(R=17), dict(eta=0),
           dict(R=8, eta=5), dict(k=0), dict(k=33), dict(m=63), dict(flags=2)]
    for b in bad:
        c = dict(K=10, B=5, R=2, eta=2, k=31, m=1024, seed=1, flags=0)
        c.update(b)
        cfg = rambo.Config(c["K"], c["B"], c["R"], c["eta"], c["k"], c["flags"], c["m"], c["seed"])
        h = ctypes.c_void_p()
        assert lib.rambo_create(ctypes.byref(cfg), ctypes.byref(h)) == rambo.EINVAL, b
        assert not h.value
        assert b"out of range" in lib.rambo_last_error(None)


def test_null_handle_calls(lib):
    assert lib.rambo_create(None, None) == rambo.EINVAL
    assert lib.rambo_query_kmers(None, None, 0, None, None) == rambo.EINVAL
    assert lib.rambo_insert_seqs(None, None, None, 0, None, 0, None) == rambo.EINVAL
    assert lib.rambo_insert_kmers(None, None, None, 0, None, 0, None) == rambo.EINVAL
    assert lib.rambo_query_termsets(None, None, 0, None, 0, None, None) == rambo.EINVAL
    assert lib.rambo_sync_status(None, None) == rambo.EINVAL
    assert lib.rambo_query_seqs_ids_noalloc(None, None, 0, None, 0, None, None, 0, None, None) == rambo.EINVAL
    assert lib.rambo_query_seqs_ids_noalloc_max_reads(None) == 0
    lib.rambo_destroy(None)


def test_probe_arguments_are_checked_on_the_host(lib):
    # rejected before any launch: a round of streams * run words past 32 bits,
    # a null output, a buffer whose chunks cannot hold one run
    written = ctypes.c_uint64(0)
    dummy = ctypes.c_void_p(4096)
    assert lib.rambo_roofline_append(dummy, 1 << 40, 1 << 20, 1 << 13, 0, 1, ctypes.byref(written), None) \
        == rambo.EINVAL
    assert lib.rambo_roofline_append(dummy, 1 << 20, 16, 16, 0, 1, None, None) == rambo.EINVAL
    assert lib.rambo_roofline_append(dummy, 64, 4, 16, 1, 2, ctypes.byref(written), None) == rambo.EINVAL
