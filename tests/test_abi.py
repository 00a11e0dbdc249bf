"""C ABI contract on the CPU: the library loads, exports every declared
symbol, sizes workspaces, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hj.h")


@pytest.fixture(scope="module")
def hj():
    import paper_1307_1955_amd.hj as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1307_1955_amd import build
        build.build_all()
    m.load()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hj_[a-z_]+)\s*\(", text)))


def test_header_declares_expected(hj):
    assert declared_functions() == sorted(hj.EXPORTED)


def test_library_exports_every_declared_symbol(hj):
    lib = hj.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_generator_library_exports():
    from paper_1307_1955_amd.gen import device
    lib = device.load()
    for name in ("hjgen_perm_keys", "hjgen_uniform", "hjgen_zipf", "hjgen_iota"):
        assert hasattr(lib, name)


def test_version_and_status_strings(hj):
    assert hj.hj_version() == 100
    lib = hj.load()
    assert lib.hj_status_str(0) == b"ok"
    assert lib.hj_status_str(2) == b"output capacity exceeded"


def test_default_params(hj):
    p = hj.hj_default_params()
    assert p.algo == hj.HJ_PHJ and p.passes == 2 and tuple(p.bits) == (6, 6) and p.flags == 0
    assert p.tile == 0 and p.lds_cap == 0  # chosen from the sizes


def test_resolve_params(hj):
    p = hj.hj_default_params()
    small = hj.hj_resolve_params(p, 1 << 22, 1 << 22)
    big = hj.hj_resolve_params(p, 1 << 23, 1 << 23)
    assert (small.tile, big.tile) == (4096, 8192)
    for q in (small, big):
        assert q.lds_cap % 64 == 0 and 256 <= q.lds_cap <= 8192
        assert (q.algo, q.passes, tuple(q.bits), q.flags) == (p.algo, p.passes, tuple(p.bits), p.flags)
        # the resolved parameters describe the same join: same workspace
        assert hj.hj_workspace_bytes(q, 1 << 22, 1 << 22) > 0
    assert hj.hj_workspace_bytes(big, 1 << 23, 1 << 23) == hj.hj_workspace_bytes(p, 1 << 23, 1 << 23)
    assert hj.hj_workspace_bytes(small, 1 << 22, 1 << 22) == hj.hj_workspace_bytes(p, 1 << 22, 1 << 22)
    # an explicit tile is kept
    e = hj.hj_resolve_params(hj.params("phj", 2, (6, 6), tile=2048), 1 << 23, 1 << 23)
    assert e.tile == 2048
    d = hj.hj_resolve_params(hj.params("phj", 0, (0, 0)), 1000, 5000)
    assert d.passes == 0 and d.lds_cap == 1024 and d.flags & hj.HJ_FLAG_ONE_PASS
    with pytest.raises(hj.HJError):
        hj.hj_resolve_params(hj.params("phj", 2, (6, 6), tile=3000), 10, 10)


@pytest.mark.parametrize("kw", [
    dict(algo="phj", passes=3, bits=(6, 6)),
    dict(algo="phj", passes=1, bits=(0,)),
    dict(algo="phj", passes=1, bits=(14,)),
    dict(algo="phj", passes=2, bits=(9, 8)),
    dict(algo="phj", passes=2, bits=(6, 0)),
    dict(algo="phj", passes=2, bits=(6, 6), tile=3000),
    dict(algo="phj", passes=2, bits=(6, 6), lds_cap=100),
    dict(algo="phj", passes=2, bits=(6, 6), lds_cap=8256),
])
def test_invalid_params_rejected(hj, kw):
    p = hj.params(**kw)
    with pytest.raises(hj.HJError) as e:
        hj.hj_workspace_bytes(p, 1000, 1000)
    assert e.value.status == hj.HJ_ERR_INVALID


def test_flags_and_hash_rejected(hj):
    p = hj.params("shj")
    p.flags = 2
    with pytest.raises(hj.HJError):
        hj.hj_workspace_bytes(p, 10, 10)
    p = hj.params("shj")
    p.hash = 7
    with pytest.raises(hj.HJError):
        hj.hj_workspace_bytes(p, 10, 10)


def test_too_many_rows_rejected(hj):
    with pytest.raises(hj.HJError):
        hj.hj_workspace_bytes(hj.params("shj"), 1 << 31, 10)


def test_workspace_sizes(hj):
    for p in (hj.params("shj"), hj.params("phj", 1, (8,)), hj.params("phj", 2, (6, 6))):
        a = hj.hj_workspace_bytes(p, 1000, 1000)
        b = hj.hj_workspace_bytes(p, 1 << 20, 1 << 20)
        assert 0 < a < b
        assert hj.hj_workspace_bytes(p, 0, 0) > 0
    # PHJ, 2 passes: two partitioned copies (16 B/tuple) plus the HBM-table area
    # (two 8-byte slots and one 4-byte chain link per R tuple)
    n = 1 << 24
    ws = hj.hj_workspace_bytes(hj.params("phj", 2, (6, 6)), n, n)
    assert 16 * 2 * n + 20 * n <= ws < 16 * 2 * n + 20 * n + (64 << 20)
    # SHJ: 2^ceil(log2 2|R|) 8-byte slots plus a 4-byte chain link per R row
    ws = hj.hj_workspace_bytes(hj.params("shj"), n, n)
    assert 8 * 2 * n + 4 * n <= ws < 8 * 2 * n + 4 * n + (8 << 20)


def _raw(hj, p, rn=10, sn=10, rkey=1, skey=1, cap=10, ws=1 << 20, ws_bytes=None, d_count=8):
    R = hj.HjRel(rkey, rkey, rn)
    S = hj.HjRel(skey, skey, sn)
    O = hj.HjOut(8, 8, cap)
    if ws_bytes is None:
        ws_bytes = hj.hj_workspace_bytes(p, rn, sn)
    return hj.load().hj_join(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O),
                             ws, ws_bytes, d_count, None)


def test_validation_before_launch(hj):
    """Every rejected call returns before touching the device (runs without a GPU)."""
    p = hj.params("phj", 2, (6, 6))
    lib = hj.load()
    assert _raw(hj, p, rkey=None) == hj.HJ_ERR_INVALID
    assert b"NULL" in lib.hj_last_error()
    assert _raw(hj, p, skey=None) == hj.HJ_ERR_INVALID
    assert _raw(hj, p, d_count=None) == hj.HJ_ERR_INVALID
    assert _raw(hj, p, ws=None) == hj.HJ_ERR_WORKSPACE
    need = hj.hj_workspace_bytes(p, 10, 10)
    assert _raw(hj, p, ws_bytes=need - 1) == hj.HJ_ERR_WORKSPACE
    assert _raw(hj, p, ws=(1 << 20) + 8) == hj.HJ_ERR_INVALID  # misaligned workspace
    assert _raw(hj, p, rn=1 << 31, ws_bytes=1 << 40) == hj.HJ_ERR_INVALID
    O = hj.HjOut(None, None, 5)
    R = hj.HjRel(1, 1, 10)
    assert lib.hj_join(ctypes.byref(p), ctypes.byref(R), ctypes.byref(R), ctypes.byref(O), 1 << 20, need, 8,
                       None) == hj.HJ_ERR_INVALID
    assert lib.hj_join(ctypes.byref(p), None, ctypes.byref(R), ctypes.byref(O), 1 << 20, need, 8,
                       None) == hj.HJ_ERR_INVALID
