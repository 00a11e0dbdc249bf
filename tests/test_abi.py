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
    small = hj.hj_resolve_params(p, 1 << 23, 1 << 23)
    big = hj.hj_resolve_params(p, 1 << 24, 1 << 24)
    assert (small.tile, big.tile) == (4096, 8192)
    # one pass of 8+ bits takes 8192-tuple tiles from 2^24 tuples on
    one = hj.params("phj", 1, (8,))
    assert hj.hj_resolve_params(one, 1 << 20, (1 << 24) - (1 << 20)).tile == 8192
    assert hj.hj_resolve_params(one, 1 << 20, (1 << 23)).tile == 4096
    assert hj.hj_resolve_params(hj.params("phj", 1, (7,)), 1 << 20, 1 << 24).tile == 4096
    for q in (small, big):
        assert q.lds_cap % 64 == 0 and 256 <= q.lds_cap <= 8192
        assert (q.algo, q.passes, tuple(q.bits), q.flags) == (p.algo, p.passes, tuple(p.bits), p.flags)
        # the resolved parameters describe the same join: same workspace
        assert hj.hj_workspace_bytes(q, 1 << 22, 1 << 22) > 0
    assert hj.hj_workspace_bytes(big, 1 << 24, 1 << 24) == hj.hj_workspace_bytes(p, 1 << 24, 1 << 24)
    assert hj.hj_workspace_bytes(small, 1 << 23, 1 << 23) == hj.hj_workspace_bytes(p, 1 << 23, 1 << 23)
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
    dict(algo="phj", passes=2, bits=(13, 8)),
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


def auto_candidates(hj, n_r, flags, tile=0):
    """The plans HJ_AUTO weighs (csrc/costmodel.cpp), built independently here."""
    c = [hj.params("shj", one_pass=bool(flags))]
    if n_r <= 8192:
        c.append(hj.params("phj", 0, (0, 0), one_pass=bool(flags)))
    B = 0
    while B < 20 and (n_r >> B) > 4096:
        B += 1
    for b in range(max(1, B - 2), min(B + 2, 20) + 1):
        for t in (tile,):  # 0: the library's size rule
            if b <= 13:
                c.append(hj.params("phj", 1, (b,), tile=t, one_pass=bool(flags)))
            if b >= 2:
                for b1 in range(max(1, b // 2 - 1), min(13, b // 2 + 2) + 1):
                    if 1 <= b - b1 <= 13:
                        c.append(hj.params("phj", 2, (b1, b - b1), tile=t, one_pass=bool(flags)))
    return c


@pytest.mark.parametrize("n_r,n_s", [(0, 1000), (1000, 1000), (4416, 50000), (9000, 9000), (100000, 400000),
                                     (1 << 20, 1 << 20), (1 << 22, 1 << 24), (1 << 24, 1 << 24), (3 << 24, 3 << 24),
                                     (1 << 30, 1 << 30), ((1 << 31) - 1, 1 << 20)])
def test_auto_params_are_the_models_choice(hj, n_r, n_s):
    """HJ_AUTO runs the candidate with the least modelled time (hj_model_seconds)."""
    for flags in (0, hj.HJ_FLAG_ONE_PASS):
        for tile in (0, 8192):
            p = hj.params("auto", tile=tile, one_pass=bool(flags))
            q = hj.hj_resolve_params(p, n_r, n_s)
            t_auto = hj.hj_model_seconds(q, n_r, n_s, n_s)
            ts = []
            for c in auto_candidates(hj, n_r, flags, tile):
                try:
                    ts.append(hj.hj_model_seconds(c, n_r, n_s, n_s))
                except hj.HJError:
                    pass
            assert t_auto == pytest.approx(min(ts), rel=1e-12)
            assert hj.hj_workspace_bytes(p, n_r, n_s) == hj.hj_workspace_bytes(q, n_r, n_s)
            if q.algo == hj.HJ_PHJ and q.passes == 0:
                assert q.flags == hj.HJ_FLAG_ONE_PASS  # the direct join always writes in one pass
            else:
                assert q.flags == flags


def test_model_twins_agree(hj):
    """The library's compiled cost model and its Python twin (used to fit the
    constants and to validate them) give the same predictions."""
    from paper_1307_1955_amd import costmodel
    c = costmodel.load()
    for n_r, n_s in [(1000, 1000), (5000, 80000), (100000, 400000), (1 << 20, 1 << 22), (1 << 24, 1 << 24),
                     (3 << 24, 1 << 26), (1 << 28, 1 << 28)]:
        for p in auto_candidates(hj, n_r, 0) + auto_candidates(hj, n_r, 1):
            try:
                want = hj.hj_model_seconds(p, n_r, n_s, n_s // 2)
            except hj.HJError:
                continue
            q = hj.hj_resolve_params(p, n_r, n_s)
            got = costmodel.join_seconds(costmodel.plan_of(q), n_r, n_s, n_s // 2, c)
            assert got == pytest.approx(want, rel=1e-9), (repr(q), n_r, n_s)


def test_model_constants_match_the_calibration():
    """csrc/calib_mi355x.inc is generated from tuning/mi355x_calib.json."""
    import re

    from paper_1307_1955_amd import costmodel
    c = costmodel.load()
    inc = open(costmodel.CALIB_INC).read()
    got = {m.group(1): float(m.group(2)) for m in re.finditer(r"k_(\w+) = ([-+0-9.eE]+);", inc)}
    assert set(got) == set(costmodel.PARAMS)
    for k in costmodel.PARAMS:
        assert got[k] == pytest.approx(c[k], rel=1e-15)


def test_model_geometry_matches_the_kernels():
    """The Python twin's launch geometry (chunk, tile and grid sizes) is the
    one the kernels are compiled with (csrc/hj_internal.h)."""
    import re

    from paper_1307_1955_amd import costmodel
    hdr = open(os.path.join(os.path.dirname(costmodel.__file__), "csrc", "hj_internal.h")).read()

    def const(name):
        m = re.search(r"constexpr \w+ %s = ([^;]+);" % name, hdr)
        assert m, name
        return m.group(1)

    assert int(const("kOvfChunk")) == costmodel.OVF_CHUNK
    assert int(const("kOvfChunkBig")) == costmodel.OVF_CHUNK_BIG
    assert const("kOvfBigPart") == "1u << 16" and costmodel.OVF_BIG_PART == 1 << 16
    assert int(const("kOvfGrid")) == costmodel.OVF_GRID
    assert int(const("kShjTile")) == costmodel.SHJ_TILE
    assert float(const("kShjSlotsPerRow")) == costmodel.SHJ_SLOTS_PER_ROW
    sub = re.search(r"constexpr uint32_t kJoinSub = (\d+)", hdr)
    assert sub and 2 * int(sub.group(1)) == costmodel.JOIN_CHUNK
    # which two-pass plans have a counted pass 2 (no pass-2 histogram and scan)
    assert int(const("kCountedMaxBits")) == costmodel.COUNTED_MAX_BITS
    rule = re.search(r"return passes == 2 && b1 \+ b2 >= (\d+) && b1 \+ b2 <= kCountedMaxBits;", hdr)
    assert rule and int(rule.group(1)) == 4
    assert [b for b in range(2, 16) if costmodel.counted_pass2(2, 1, b - 1)] == list(range(4, 14))
    assert not costmodel.counted_pass2(1, 6, 0)
    assert re.search(r"inline bool counted_clears_tables\(uint32_t b2\) \{ return b2 <= 6; \}", hdr)


def test_table_and_probe_sizes(hj):
    n = 1 << 20
    for p in (hj.params("shj"), hj.params("phj", 1, (8,)), hj.params("phj", 2, (5, 5)),
              hj.params("phj", 0, (0, 0)), hj.params("auto")):
        n_r = 4000 if p.passes == 0 and p.algo == hj.HJ_PHJ else n
        tb = hj.hj_table_bytes(p, n_r)
        assert tb > 0
        t = hj.HjTable()
        t.params = hj.hj_resolve_params(p, n_r, n_r)
        t.n_r, t.r_key, t.r_rid, t.ws, t.ws_bytes = n_r, 256, 256, 1 << 20, tb
        pb = hj.hj_probe_workspace_bytes(t, n)
        assert pb > 0
        if t.params.algo == hj.HJ_PHJ and t.params.passes > 0:
            # build (R) + probe (S) hold what one join holds, minus nothing it needs twice
            assert tb + pb >= hj.hj_workspace_bytes(t.params, n_r, n)
    # SHJ table: 2^ceil(log2 2|R|) 8-byte slots plus a 4-byte link per R row
    tb = hj.hj_table_bytes(hj.params("shj"), 1 << 24)
    assert 8 * 2 * (1 << 24) + 4 * (1 << 24) <= tb < 8 * 2 * (1 << 24) + 4 * (1 << 24) + (1 << 20)
    with pytest.raises(hj.HJError):
        hj.hj_table_bytes(hj.params("phj", 0, (0, 0)), 9000)  # passes 0 needs |R| <= 8192
    with pytest.raises(hj.HJError):
        hj.hj_table_bytes(hj.params("phj", 2, (6, 6)), 1 << 31)


def test_build_probe_validation_before_launch(hj):
    """Rejected build/probe calls return before touching the device (runs without a GPU)."""
    lib = hj.load()
    p = hj.params("phj", 2, (6, 6))
    R = hj.HjRel(256, 256, 1000)
    t = hj.HjTable()
    tb = hj.hj_table_bytes(p, 1000)
    # build: NULL table, NULL or small or misaligned workspace, NULL R arrays
    assert lib.hj_build(ctypes.byref(p), ctypes.byref(R), 1 << 20, tb, None, None) == hj.HJ_ERR_INVALID
    assert lib.hj_build(ctypes.byref(p), ctypes.byref(R), None, tb, None, ctypes.byref(t)) == hj.HJ_ERR_WORKSPACE
    assert lib.hj_build(ctypes.byref(p), ctypes.byref(R), 1 << 20, tb - 1, None, ctypes.byref(t)) == \
        hj.HJ_ERR_WORKSPACE
    assert lib.hj_build(ctypes.byref(p), ctypes.byref(R), (1 << 20) + 8, tb, None, ctypes.byref(t)) == \
        hj.HJ_ERR_INVALID
    Rn = hj.HjRel(None, 256, 1000)
    assert lib.hj_build(ctypes.byref(p), ctypes.byref(Rn), 1 << 20, tb, None, ctypes.byref(t)) == \
        hj.HJ_ERR_INVALID
    # probe: a table whose parameters were not resolved, or without its workspace
    t.params = hj.hj_resolve_params(p, 1000, 1000)
    t.n_r, t.r_key, t.r_rid, t.ws, t.ws_bytes = 1000, 256, 256, 1 << 20, tb
    S = hj.HjRel(256, 256, 500)
    O = hj.HjOut(256, 256, 500)
    pb = hj.hj_probe_workspace_bytes(t, 500)
    probe = lambda tt, ws=1 << 22, wb=pb, d=8, o=O: lib.hj_probe(  # noqa: E731
        ctypes.byref(tt), ctypes.byref(S), ctypes.byref(o), ws, wb, d, None)
    assert probe(t, d=None) == hj.HJ_ERR_INVALID
    assert probe(t, wb=pb - 1) == hj.HJ_ERR_WORKSPACE
    assert probe(t, o=hj.HjOut(None, 256, 5)) == hj.HJ_ERR_INVALID
    bad = hj.HjTable.from_buffer_copy(t)
    bad.params.tile = 0
    assert probe(bad) == hj.HJ_ERR_INVALID
    bad = hj.HjTable.from_buffer_copy(t)
    bad.params.algo = hj.HJ_AUTO
    assert probe(bad) == hj.HJ_ERR_INVALID
    bad = hj.HjTable.from_buffer_copy(t)
    bad.ws = None
    assert probe(bad) == hj.HJ_ERR_INVALID
    bad = hj.HjTable.from_buffer_copy(t)
    bad.ws_bytes = tb - 1
    assert probe(bad) == hj.HJ_ERR_INVALID
    # SHJ probes read R's rids (matches) and R's keys (heavy-key scans) through the table
    ps = hj.params("shj")
    ts = hj.HjTable()
    ts.params = hj.hj_resolve_params(ps, 1000, 1000)
    ts.n_r, ts.r_key, ts.r_rid, ts.ws, ts.ws_bytes = 1000, 256, None, 1 << 20, hj.hj_table_bytes(ps, 1000)
    assert lib.hj_probe_workspace_bytes(ctypes.byref(ts), 500) == 0
    ts.r_key, ts.r_rid = None, 256
    assert lib.hj_probe_workspace_bytes(ctypes.byref(ts), 500) == 0
    # a NULL r_key is rejected before any launch (fake device pointers: a launch would fault)
    assert probe(ts, wb=1 << 22) == hj.HJ_ERR_INVALID
    assert b"key and rid" in lib.hj_last_error()
    ts.r_key = 256
    assert lib.hj_probe_workspace_bytes(ctypes.byref(ts), 500) > 0


def test_batch_bytes_on_host(hj):
    """hj_batch_bytes plans on the host only (no device calls): fake device pointers suffice."""
    lib = hj.load()
    jobs = (hj.HjJob * 3)()
    sizes = [(1000, 5000), (200000, 400000), (3 << 20, 1 << 20)]
    for j, (nr, ns) in enumerate(sizes):
        jobs[j].R = hj.HjRel(256, 256, nr)
        jobs[j].S = hj.HjRel(256, 256, ns)
        jobs[j].out = hj.HjOut(256, 256, ns)
        jobs[j].d_count = 256 + 8 * j
    a = lib.hj_batch_bytes(3, jobs, None)
    assert a > 0
    # at least the largest pipelined job's own workspace (its lane slice)
    q = hj.HjParams()
    lib.hj_default_params(ctypes.byref(q))
    q.algo = hj.HJ_AUTO
    q.flags = hj.HJ_FLAG_ONE_PASS
    assert a >= hj.hj_workspace_bytes(q, 3 << 20, 1 << 20)
    jobs[1].d_count = None
    assert lib.hj_batch_bytes(3, jobs, None) == 0


def test_noalloc_rejects_sizes_beyond_its_array(hj):
    """hj_join_noalloc checks its fixed 64 MiB workspace against the sizes on the
    host, before any device call (runs without a GPU; fake device pointers)."""
    lib = hj.load()
    p = hj.params("phj", 2, (6, 6))
    R = hj.HjRel(256, 256, 1 << 24)
    S = hj.HjRel(256, 256, 1 << 24)
    O = hj.HjOut(256, 256, 1 << 24)
    assert lib.hj_join_noalloc(ctypes.byref(p), ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), 256,
                               None) == hj.HJ_ERR_WORKSPACE
    assert b"fixed" in lib.hj_last_error()
    assert lib.hj_join_noalloc(None, ctypes.byref(R), ctypes.byref(S), ctypes.byref(O), 256,
                               None) == hj.HJ_ERR_INVALID
    assert hj.hj_workspace_bytes(p, 1 << 24, 1 << 24) > 64 << 20


def test_external_validation_before_device(hj):
    """hj_join_external rejects bad arguments before any device call (no GPU here;
    fake pointers)."""
    lib = hj.load()
    p = hj.params("auto", one_pass=True)
    R = hj.HjRel(256, 256, 1000)
    S = hj.HjRel(256, 256, 1000)
    O = hj.HjOut(256, 256, 1000)
    h = ctypes.c_uint64(0)
    info = hj.HjExternalInfo()
    call = lambda ws, wb, r=R, o=O, cnt=ctypes.byref(h): lib.hj_join_external(  # noqa: E731
        ctypes.byref(p), ctypes.byref(r), ctypes.byref(S), ctypes.byref(o), ws, wb, cnt, ctypes.byref(info))
    assert call(1 << 20, (64 << 20) - 1) == hj.HJ_ERR_WORKSPACE
    assert call(None, 64 << 20) == hj.HJ_ERR_WORKSPACE
    assert call((1 << 20) + 8, 64 << 20) == hj.HJ_ERR_INVALID
    assert call(1 << 20, 64 << 20, r=hj.HjRel(None, 256, 5)) == hj.HJ_ERR_INVALID
    assert call(1 << 20, 64 << 20, o=hj.HjOut(None, 256, 5)) == hj.HJ_ERR_INVALID
    assert call(1 << 20, 64 << 20, cnt=None) == hj.HJ_ERR_INVALID
