"""The C-ABI library loads and exports every function include/cae.h declares; host-only calls
(sizes, validation, error text) behave as documented.  No GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cae_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def cae():
    from paper_2606_21784_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcae.so not built: run __graft_entry__.build()")
    return _lib


def test_exports_every_declared_symbol(cae):
    L = cae.lib()
    names = _declared("cae.h")
    assert "cae_step" in names and "cae_create" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(cae.EXPORTS) <= set(names)


def test_struct_layouts(cae):
    assert C.sizeof(cae.Market) == 32
    assert C.sizeof(cae.State) == 80
    assert C.sizeof(cae.Sizes) == 32
    assert C.sizeof(cae.Tuning) == 16 + 8 * cae.NUM_CLASSES


def test_header_struct_sizes_match_binding(cae, tmp_path):
    """The header's structs, compiled by the host C compiler, have the binding's sizes."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "sizes.c"
    checks = [("cae_market", C.sizeof(cae.Market)), ("cae_state", C.sizeof(cae.State)),
              ("cae_sizes_t", C.sizeof(cae.Sizes)), ("cae_tuning", C.sizeof(cae.Tuning))]
    src.write_text('#include "cae.h"\n' + "".join(
        "_Static_assert(sizeof(%s) == %d, \"%s\");\n" % (n, z, n) for n, z in checks))
    r = subprocess.run([cc, "-std=c11", "-fsyntax-only", "-I", os.path.join(ROOT, "include"), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_strerror(cae):
    L = cae.lib()
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(L.cae_strerror(code), bytes)


def _sizes(descs):
    from paper_2606_21784_amd import engine
    return engine.sizes(descs)


def test_sizes(cae):
    from paper_2606_21784_amd import engine
    d = engine.markets(256, 1024, 16, 100, M=1024)
    s = _sizes(d)
    assert s.book_words == 1024 * 2 * 256
    assert s.book_bytes == 4 * s.book_words
    assert s.state_bytes == 80 * 1024
    assert s.workspace_bytes > 0 and s.workspace_bytes % 256 == 0
    mixed = np.concatenate([engine.markets(64, 10, 1, 1), engine.markets(1000, 10, 1, 1)])
    assert _sizes(mixed).book_words == 2 * 64 + 2 * 1000


@pytest.mark.parametrize("field,value", [("L", 0), ("L", 1025), ("A", 0), ("Q", 0),
                                         ("K", 2**30 + 1), ("n_noise", 11), ("h", 64),
                                         ("flags", 2), ("flags", 0x200), ("flags", 5 << 16),
                                         ("flags", 1 | (2 << 8))])
def test_invalid_descriptors(cae, field, value):
    from paper_2606_21784_amd import engine
    d = engine.markets(64, 10, 4, 5, M=3)
    d[field][1] = value
    with pytest.raises(cae.CaeError) as ei:
        _sizes(d)
    assert ei.value.code == cae.CAE_EINVAL
    assert "market 1" in str(ei.value)


def test_mid_model_descriptors(cae):
    """The mid-price model takes P_mkt in the flags' upper half; its K must stay below 2^20."""
    from paper_2606_21784_amd import engine
    ok = engine.markets(64, 10, 4, 5, M=2, flags=engine.model_flags(cae.MODEL_MID, 0.25))
    assert int(ok["flags"][0]) == (16384 << 16) | 1
    _sizes(ok)
    bad = engine.markets(64, 10, 2**20, 5, flags=engine.model_flags(cae.MODEL_MID))
    with pytest.raises(cae.CaeError):
        _sizes(bad)
    with pytest.raises(ValueError):
        engine.model_flags(cae.MODEL_LAST, 0.1)
    sm = engine.markets(64, 10, 4, 5, M=2, flags=engine.model_flags(gen=cae.GEN_SPLITMIX))
    assert int(sm["flags"][0]) == 1 << 8
    _sizes(sm)


def test_agents_times_quantity_guard(cae):
    from paper_2606_21784_amd import engine
    d = engine.markets(64, 2**16, 4, 2**16)
    with pytest.raises(cae.CaeError) as ei:
        _sizes(d)
    assert ei.value.code == cae.CAE_EINVAL


def test_null_arguments(cae):
    L = cae.lib()
    assert L.cae_sizes(None, 1, None) == cae.CAE_EINVAL
    assert L.cae_step(None, 1) == cae.CAE_EINVAL
    assert L.cae_read_books(None, None, 0) == cae.CAE_EINVAL
    assert L.cae_clear(0, 1, None, None, None, None) == cae.CAE_EINVAL
    assert L.cae_clear(64, 1, None, None, None, None) == cae.CAE_EINVAL
    assert L.cae_destroy(None) == cae.CAE_OK
    assert b"NULL" in L.cae_last_error() or b"L=" in L.cae_last_error()


def test_size_class(cae):
    from paper_2606_21784_amd import engine
    assert engine.size_class(64, 64) == 0
    assert engine.size_class(65, 64) == 8
    assert engine.size_class(1024, 16384) == 4 * 8 + 7
    assert engine.size_class(256, 1024) == 2 * 8 + 4
    assert engine.size_class(1, 1) == 0
