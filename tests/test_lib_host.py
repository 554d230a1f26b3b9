"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side setup (built without touching a GPU) reproduces the
oracle's operators."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1512_01756_amd as P
from oracle import schur, smpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            names |= set(re.findall(r"\b(smpm_[a-z_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("library not built: run python -m paper_1512_01756_amd.build")
    return P.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared_symbols()
    assert {"smpm_setup", "smpm_solve", "smpm_apply", "smpm_destroy"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(P.EXPORTED)


CASES = [
    (np.linspace(0, 8, 9), np.linspace(0, 1, 3), 11, 0.0),
    (np.array([0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8]), np.array([0, 0.15, 0.45, 1.0]), 5, 0.0),
    (np.array([0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8]), np.array([0, 0.15, 0.45, 1.0]), 5, 1.7),
    (np.linspace(0, 3, 8), np.linspace(0, 1, 2), 4, 0.0),
]


@pytest.mark.parametrize("zlabel", [0, 1])
@pytest.mark.parametrize("xb,zb,n,k", CASES)
def test_host_setup_matches_oracle(lib, xb, zb, n, k, zlabel):
    s = P.Solver(xb, zb, n - 1, kwaves=[k], host_only=True, zlabel=zlabel)
    grid = smpm.Grid(xb, zb, n)
    o = schur.build(grid, kwave=k, zlabel=zlabel)
    kS, d = grid.k, (grid.mx - 1) * (grid.mz if zlabel else 1)
    assert s.info[0]["kS"] == kS and s.info[0]["r"] == grid.r and s.info[0]["d"] == d
    assert s.info[0]["tau"] == pytest.approx(o.tau, rel=1e-15)
    S = s.export(P.TABLE_SCHUR_DENSE).reshape(kS, kS)
    So = o.S.toarray()
    assert np.abs(S - So).max() <= 1e-11 * np.abs(So).max()
    Mi = s.export(P.TABLE_BJINV_DENSE).reshape(kS, kS)
    Mo = np.zeros((kS, kS))
    for idx, Mb in zip(o.bj_index, o.bj_inv):
        Mo[np.ix_(idx, idx)] = Mb
    assert np.abs(Mi - Mo).max() <= 1e-11 * np.abs(Mo).max()
    C = s.export(P.TABLE_COARSE_C).reshape(d, d)
    assert np.abs(C - o.C).max() <= 1e-11 * np.abs(o.C).max()
    SZ = s.export(P.TABLE_SZ).reshape(kS, d)
    assert np.abs(SZ - o.SZ).max() <= 1e-10 * np.abs(o.SZ).max()
    if k == 0.0:
        for table, ref in ((P.TABLE_U_S, o.uS), (P.TABLE_U_L, o.uL), (P.TABLE_U_C, o.uC)):
            v = s.export(table)
            assert np.abs(v - ref).max() < 1e-10
    s.close()


@pytest.mark.parametrize("k", [0.0, 1.7])
def test_fused_schur_times_bj_inverse_matches_oracle(lib, k):
    # uniform strips share blocks, so the setup also stores S M^-1 per half
    xb, zb, n = np.linspace(0, 6, 13), np.linspace(0, 1, 3), 5
    s = P.Solver(xb, zb, n - 1, kwaves=[k], host_only=True)
    o = schur.build(smpm.Grid(xb, zb, n), kwave=k)
    kS = o.grid.k
    Mo = np.zeros((kS, kS))
    for idx, Mb in zip(o.bj_index, o.bj_inv):
        Mo[np.ix_(idx, idx)] = Mb
    ref = o.S.toarray() @ Mo
    F = s.export(P.TABLE_SMINV_DENSE).reshape(kS, kS)
    assert np.abs(F - ref).max() <= 1e-11 * np.abs(ref).max()
    s.close()
    # distinct strips: no fused blocks
    s2 = P.Solver(np.array([0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8]), zb, n - 1, host_only=True)
    with pytest.raises(P.SmpmError):
        s2.export(P.TABLE_SMINV_DENSE)
    s2.close()


@pytest.mark.parametrize("zlabel,k", [(0, 0.0), (1, 1.7)])
def test_saved_tables_load_back_identically(lib, tmp_path, zlabel, k):
    xb = np.array([0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8])
    zb = np.array([0, 0.15, 0.45, 1.0])
    s = P.Solver(xb, zb, 4, kwaves=[k, 2 * k + 0.5], host_only=True, zlabel=zlabel)
    path = str(tmp_path / "tables.bin")
    s.save(path)
    t = P.Solver(load_path=path, host_only=True, zlabel=zlabel)
    assert t.nsys == 2 and t.info == s.info
    for sys in range(2):
        tables = [P.TABLE_SCHUR_DENSE, P.TABLE_BJINV_DENSE, P.TABLE_COARSE_C, P.TABLE_SZ]
        if s.info[sys]["kwave"] == 0.0:
            tables += [P.TABLE_U_S, P.TABLE_U_L, P.TABLE_U_C]
        for table in tables:
            assert np.array_equal(s.export(table, sys), t.export(table, sys)), table
    # a different deflation space, a foreign file and a truncated file are rejected
    with pytest.raises(P.SmpmError):
        P.Solver(load_path=path, host_only=True, zlabel=1 - zlabel)
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a table file")
    with pytest.raises(P.SmpmError):
        P.Solver(load_path=str(bad), host_only=True)
    data = open(path, "rb").read()
    (tmp_path / "short.bin").write_bytes(data[: len(data) // 2])
    with pytest.raises(P.SmpmError):
        P.Solver(load_path=str(tmp_path / "short.bin"), host_only=True, zlabel=zlabel)


def test_uniform_strips_are_deduplicated(lib):
    s = P.Solver(np.linspace(0, 32, 65), np.linspace(0, 1, 5), 6, host_only=True)
    # first strip, interior strips, last strip -> at most 4 distinct half blocks
    assert s.info[0]["unique_W"] <= 4
    s.close()


def test_errors(lib):
    with pytest.raises(P.SmpmError) as e:
        P.Solver(np.linspace(0, 3, 4), np.linspace(0, 1, 2), 4, host_only=True)   # m_x = 3, k = 0
    assert e.value.status == P.ESINGULAR
    # m_x = 3 is fine for k > 0 (nonsingular)
    P.Solver(np.linspace(0, 3, 4), np.linspace(0, 1, 2), 4, kwaves=[2.0], host_only=True).close()
    with pytest.raises(P.SmpmError) as e:
        P.Solver(np.array([0, 1.0, 0.5, 2.0, 3.0]), np.linspace(0, 1, 2), 4, host_only=True)
    assert e.value.status == P.EINVAL
    with pytest.raises(P.SmpmError) as e:
        P.Solver(np.linspace(0, 4, 5), np.linspace(0, 1, 2), 4, kwaves=[-1.0], host_only=True)
    assert e.value.status == P.EINVAL
    with pytest.raises(P.SmpmError) as e:
        P.Solver(np.linspace(0, 4, 5), np.linspace(0, 1, 2), 0, host_only=True)
    assert e.value.status == P.EINVAL
    s = P.Solver(np.linspace(0, 4, 5), np.linspace(0, 1, 2), 4, host_only=True)
    lib_ = P.load()
    st = lib_.smpm_solve(s.h, None, None, None, None, None)
    assert st == P.EUNSUPPORTED
    s.close()


def _system_offsets(data):
    """Byte offsets of the first system's n and of its Schur block id table
    (w_id) in a saved table file: magic, layout version, header, then the
    fields in declaration order (vectors as a u64 length and the values)."""
    import struct
    pos = 8 + 4 + 24
    off_n = pos
    pos += 8 * 4 + 2 * 8 + 2 * 8 + 1          # n .. zm, r, kS, kwave, tau, singular

    def vec(pos, size):
        (cnt,) = struct.unpack_from("<Q", data, pos)
        return pos + 8 + cnt * size, pos + 8

    for size in (8, 8, 8, 8, 4):                # xb, zb, lo, up, strip_class
        pos, _ = vec(pos, size)
    (ncl,) = struct.unpack_from("<Q", data, pos)
    pos += 8
    for _ in range(ncl):
        pos += 8 + 1 + 1                        # hx, west_if, east_if
        for _ in range(5 + 4):                  # G, Dinv, Kinv, betaW, betaE, Wq[2][2]
            pos, _ = vec(pos, 8)
    _, off_wid = vec(pos, 4)
    return off_n, off_wid


def test_corrupt_table_fields_are_rejected(lib, tmp_path):
    # A file with the right magic whose grid size or block ids were changed
    # must be refused (EINVAL) before anything is uploaded.
    import struct
    xb = np.array([0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8])
    zb = np.array([0, 0.15, 0.45, 1.0])
    s = P.Solver(xb, zb, 4, host_only=True)
    path = tmp_path / "tables.bin"
    s.save(str(path))
    s.close()
    data = path.read_bytes()
    off_n, off_wid = _system_offsets(data)
    assert struct.unpack_from("<i", data, off_n)[0] == 5
    assert 0 <= struct.unpack_from("<i", data, off_wid)[0] < 12
    t = P.Solver(load_path=str(path), host_only=True)   # the untouched file loads
    t.close()
    for off, value in ((off_n, 6), (off_n, 40), (off_wid, 4096), (off_wid, -1), (8, 1)):
        bad = bytearray(data)
        struct.pack_into("<i", bad, off, value)
        p2 = tmp_path / "bad.bin"
        p2.write_bytes(bytes(bad))
        with pytest.raises(P.SmpmError) as e:
            P.Solver(load_path=str(p2), host_only=True)
        assert e.value.status == P.EINVAL, (off, value)
