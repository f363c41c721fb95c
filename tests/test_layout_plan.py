"""The layout planners on the host (csrc/layout_plan.h, built here with g++
into a small test library; no GPU): for the row-packed layout the packing
units, the per-slot source blocks and columns, and the per-lane metadata that
k_pack_spmv reads; for the sliced layout the slot groups per slice, the slots
and the settled padding columns with their 16-bit bases.

Checked against the layout's definition on seeded random patterns: every
stored block lands in exactly one slot and every slot of a lane belongs to
that lane's row; a lane serves K consecutive blocks of its row; the first
lane of a row carries the row's lane count and every lane its row's offset in
the unit; a unit's rows fit its lanes, and a unit is closed only when the
next row does not fit (or would widen its columns beyond 16-bit offsets);
rows needing more lanes than a unit or the 8-bit count holds are refused.  A
slice holds as many slot groups as its longest row needs, lane j of a row its
blocks j, j + L, ...; padding takes its slice's smallest real column, and the
bases are given only when every slice spans at most 65,536 columns."""
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
    lib.plan_sliced.argtypes = [P, P, ctypes.c_int32, ctypes.c_int, P, ctypes.c_int64, P, P, ctypes.c_int64, P, P]
    lib.plan_sliced.restype = ctypes.c_int

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

    def sliced(rp, ci, L):
        n = len(rp) - 1
        ns_cap = n // (64 // L) + 2
        lens = np.diff(rp)
        slots = int(-(-lens // L).sum() * 64 + 64 * ns_cap) * (64 // L)
        sptr = np.zeros(ns_cap + 1, np.int32)
        col = np.zeros(slots, np.int32)
        mp = np.zeros(slots, np.int32)
        base = np.zeros(ns_cap, np.int32)
        nb = ctypes.c_int32(0)
        rp = np.ascontiguousarray(rp, np.int64)
        ci = np.ascontiguousarray(ci, np.int32)
        ns = lib.plan_sliced(rp.ctypes.data, ci.ctypes.data, n, L, sptr.ctypes.data, len(sptr), col.ctypes.data,
                             mp.ctypes.data, len(col), base.ctypes.data, ctypes.byref(nb))
        assert ns >= 0
        g = sptr[ns]
        return sptr[:ns + 1], col[:g * 64], mp[:g * 64], base[:nb.value]
    plan.sliced = sliced
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


@pytest.mark.parametrize("L", [1, 2, 4, 8, 16, 32, 64])
def test_sliced_plan_matches_its_definition(planner, L):
    rng = np.random.default_rng(50 + L)
    rp, ci = _pattern(rng, 333, 0, 90, 20000, 900)
    sptr, col, mp, base = planner.sliced(rp, ci, L)
    n, rps = len(rp) - 1, 64 // L
    lens = np.diff(rp)
    assert len(sptr) - 1 == -(-n // rps) and sptr[0] == 0
    seen = np.zeros(len(ci), np.int64)
    spans = []
    for s in range(len(sptr) - 1):
        rows = np.arange(s * rps, min(n, (s + 1) * rps))
        assert sptr[s + 1] - sptr[s] == (-(-lens[rows] // L)).max()    # the longest row's groups
        real = []
        for g in range(sptr[s], sptr[s + 1]):
            for e in range(64):
                r, k = s * rps + e // L, (g - sptr[s]) * L + e % L
                src, c = mp[g * 64 + e], col[g * 64 + e]
                if r < n and k < lens[r]:
                    assert src == rp[r] + k and c == ci[src]                # lane e % L of row r: blocks j, j + L, ...
                    seen[src] += 1
                    real.append(c)
                else:
                    assert src == -1
        pad = [col[g * 64 + e] for g in range(sptr[s], sptr[s + 1]) for e in range(64)
               if mp[g * 64 + e] < 0]
        lo = min(real) if real else 0
        assert all(c == lo for c in pad)                                # padding: the slice's smallest column
        spans.append((lo, max(real) - lo if real else 0))
    assert np.all(seen == 1)
    if all(sp <= 65535 for _, sp in spans):
        assert list(base) == [lo for lo, _ in spans]
    else:
        assert len(base) == 0


def test_sliced_plan_wide_spans_drop_the_bases(planner):
    # one slice's rows reach columns 0 and 70,000: no 16-bit offsets anywhere
    rp = np.array([0, 2, 3, 4], np.int64)
    ci = np.array([0, 70000, 5, 6], np.int32)
    sptr, col, mp, base = planner.sliced(rp, ci, 1)
    assert len(base) == 0 and list(sptr) == [0, 2]
    ci = np.array([100, 65635, 100, 101], np.int32)                     # span exactly 65,535: fits
    sptr, col, mp, base = planner.sliced(rp, ci, 1)
    assert list(base) == [100]
    # padding slots of rows 1 and 2 (one block each) and of the absent rows
    # take the slice's smallest column
    assert col[64 + 1] == 100 and col[64 + 2] == 100 and col[3] == 100 and col[64 + 63] == 100
