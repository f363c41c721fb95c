"""The row-packed layout planner on the host (csrc/layout_plan.h, built here
with g++ into a small test library; no GPU): the packing units, the per-slot
source blocks and columns, and the per-lane metadata that k_pack_spmv reads.

Checked against the layout's definition on seeded random patterns: every
stored block lands in exactly one slot and every slot of a lane belongs to
that lane's row; a lane serves K consecutive blocks of its row; the first
lane of a row carries the row's lane count and every lane its row's offset in
the unit; a unit's rows fit its lanes, and a unit is closed only when the
next row does not fit (or would widen its columns beyond 16-bit offsets);
rows needing more lanes than a unit or the 8-bit count holds are refused."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1902_01715_amd", "csrc")


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("plan") / "libplan.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-fopenmp", f"-I{CSRC}",
                    os.path.join(HERE, "layout_plan_driver.cpp"), "-o", out], check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.plan_packed.argtypes = [P, P, ctypes.c_int32, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int64,
                                P, P, ctypes.c_int64, P, ctypes.c_int64]
    lib.plan_packed.restype = ctypes.c_int

    def plan(rp, ci, K, unit, span16):
        n = len(rp) - 1
        lanes = np.maximum(1, -(-np.diff(rp) // K))
        cap_units = int(lanes.sum()) + n + 1          # at least one lane per row: units <= rows
        w0 = np.zeros(cap_units + 1, np.int32)
        col = np.zeros(cap_units * unit * K, np.int32)
        mp = np.zeros(cap_units * unit * K, np.int32)
        meta = np.zeros(cap_units * unit, np.uint16)
        rp = np.ascontiguousarray(rp, np.int64)
        ci = np.ascontiguousarray(ci, np.int32)
        nu = lib.plan_packed(rp.ctypes.data, ci.ctypes.data, n, K, unit, int(span16), w0.ctypes.data, len(w0),
                             col.ctypes.data, mp.ctypes.data, len(col), meta.ctypes.data, len(meta))
        assert nu != -2
        if nu < 0:
            return None
        return w0[:nu + 1], col[:nu * unit * K], mp[:nu * unit * K], meta[:nu * unit]
    return plan


def _pattern(rng, n, lmin, lmax, ncols, band):
    lens = rng.integers(lmin, lmax + 1, n)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ci = []
    for r, ln in enumerate(lens):
        lo = max(0, min(ncols - band, r * ncols // n - band // 2))
        ci.append(np.sort(rng.choice(np.arange(lo, lo + band), size=ln, replace=False)))
    return rp, np.concatenate(ci).astype(np.int32) if len(ci) else np.zeros(0, np.int32)


def _check(rp, ci, K, unit, span16, res):
    w0, col, mp, meta = res
    n = len(rp) - 1
    lens = np.diff(rp)
    lr = np.maximum(1, -(-lens // K))
    nunits = len(w0) - 1
    waves = unit // 64
    assert w0[0] == 0 and w0[-1] == n and np.all(np.diff(w0) > 0)
    seen = np.zeros(len(ci), np.int64)
    for u in range(nunits):
        rows = np.arange(w0[u], w0[u + 1])
        used = int(lr[rows].sum())
        assert used <= unit
        cols = np.concatenate([ci[rp[r]:rp[r + 1]] for r in rows])
        if span16 and len(cols):
            assert cols.max() - cols.min() <= 65535
        if u + 1 < nunits:                             # closed only when the next row does not fit
            nxt = w0[u + 1]
            ncols = ci[rp[nxt]:rp[nxt + 1]]
            widened = span16 and len(cols) and len(ncols) and \
                max(cols.max(), ncols.max()) - min(cols.min(), ncols.min()) > 65535
            assert used + lr[nxt] > unit or widened
        m = meta[u * unit:(u + 1) * unit].astype(np.int64)
        lane = 0
        for r in rows:
            for j in range(lr[r]):
                assert m[lane] & 0xFF == r - w0[u]
                assert m[lane] >> 8 == (lr[r] if j == 0 else 0)
                for k in range(K):
                    wv, f = divmod(lane, 64)
                    slot = ((u * waves + wv) * K + k) * 64 + f
                    src = mp[slot]
                    if j * K + k < lens[r]:
                        assert src == rp[r] + j * K + k       # K consecutive blocks of the row
                        assert col[slot] == ci[src]
                        seen[src] += 1
                    else:
                        assert src == -1 and col[slot] == -1
                lane += 1
        assert lane + 0 <= unit
        assert np.all(m[lane:] == 0)                   # unused lanes: no row, offset 0
        for ln in range(lane, unit):
            wv, f = divmod(ln, 64)
            for k in range(K):
                assert mp[((u * waves + wv) * K + k) * 64 + f] == -1
    assert np.all(seen == 1)                           # every block in exactly one slot


@pytest.mark.parametrize("unit", [64, 256])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
@pytest.mark.parametrize("shape", ["short", "medium", "long"])
def test_packed_plan_matches_its_definition(planner, unit, K, shape):
    rng = np.random.default_rng({"short": 1, "medium": 2, "long": 3}[shape] * 100 + K * 10 + unit)
    lmin, lmax, n = {"short": (0, 6, 700), "medium": (8, 40, 300), "long": (80, 300, 60)}[shape]
    rp, ci = _pattern(rng, n, lmin, lmax, 5000, 400)
    res = planner(rp, ci, K, unit, True)
    lr = np.maximum(1, -(-np.diff(rp) // K))
    if lr.max() > min(unit, 255):
        assert res is None                             # a row needs more lanes than a unit holds
        return
    assert res is not None
    _check(rp, ci, K, unit, True, res)


def test_rows_cross_wavefronts_only_in_workgroup_units(planner):
    rng = np.random.default_rng(7)
    rp, ci = _pattern(rng, 200, 20, 60, 3000, 300)
    for unit, crossing in ((64, False), (256, True)):
        w0, _, _, meta = planner(rp, ci, 2, unit, True)
        found = False
        for u in range(len(w0) - 1):
            m = meta[u * unit:(u + 1) * unit].astype(np.int64)
            starts = np.flatnonzero(m >> 8)
            for s in starts:
                found |= s // 64 != (s + (m[s] >> 8) - 1) // 64
        assert found == crossing


def test_seam_in_column_numbering_starts_a_unit(planner):
    # a row-stacked operator: rows of the first block use columns near 70,000,
    # those of the second columns near 0; no unit may span both
    rng = np.random.default_rng(8)
    rp1, ci1 = _pattern(rng, 40, 3, 6, 1000, 100)
    rp2, ci2 = _pattern(rng, 40, 3, 6, 1000, 100)
    rp = np.concatenate([rp1, rp2[1:] + rp1[-1]])
    ci = np.concatenate([ci1 + 70000, ci2])
    for unit in (64, 256):
        res = planner(rp, ci, 1, unit, True)
        _check(rp, ci, 1, unit, True, res)
        assert 40 in set(res[0].tolist())              # the seam row opens a unit
        # without the 16-bit rule the two blocks may share a unit
        res = planner(rp, ci, 1, unit, False)
        _check(rp, ci, 1, unit, False, res)


def test_lane_count_limit(planner):
    # 256 blocks at K = 1 need 256 lanes: more than the 8-bit count holds
    rp = np.array([0, 3, 259, 262], np.int64)
    ci = np.concatenate([np.arange(3), np.arange(256), np.arange(3)]).astype(np.int32)
    assert planner(rp, ci, 1, 256, True) is None
    assert planner(rp, ci, 2, 256, True) is not None   # 128 lanes
    assert planner(rp, ci, 2, 64, True) is None        # 128 lanes > one wavefront
    _check(rp, ci, 4, 64, True, planner(rp, ci, 4, 64, True))


def test_empty_rows_take_one_lane(planner):
    rp = np.array([0, 0, 0, 2, 2], np.int64)
    ci = np.array([5, 9], np.int32)
    w0, col, mp, meta = planner(rp, ci, 2, 64, True)
    assert list(w0) == [0, 4]
    assert list(meta[:5] >> 8) == [1, 1, 1, 1, 0]
    _check(rp, ci, 2, 64, True, (w0, col, mp, meta))
