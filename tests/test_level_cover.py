"""Host logic of the batched search (CPU only): the column ranges that the
BFS level launches cover (paper_2601_17026_amd/csrc/level_cover.h, built
here with g++ through tests/level_cover_harness.cpp).

Whole searches are simulated: volumes take part at random, the covered set
starts as every volume between the first and the last taking part, and
live volumes leave a few at a time.  After every choice:
  - every live volume is covered and the covered set has only shrunk;
  - at most max_ranges ranges, sorted and apart, whose columns are exactly
    those of the covered volumes, with consistent thread offsets;
  - the covered columns of volumes that are not live are as few as any
    valid choice allows (brute force over the joinable gaps);
  - with few enough runs of live volumes, exactly the live ones are covered.
"""
import ctypes
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
MAX_RANGES = 16   # the ranges a level launch takes (kMaxRanges)


@pytest.fixture(scope="module")
def cover_fn(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    lib = str(tmp_path_factory.mktemp("level_cover") / "liblevel_cover.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-shared", "-fPIC", "-o", lib,
                    os.path.join(HERE, "level_cover_harness.cpp")], check=True)
    f = ctypes.CDLL(lib).level_cover
    f.restype = ctypes.c_int
    P = ctypes.c_void_p
    f.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, P]

    def call(col_base, cols, live, cover, max_ranges):
        n = len(cols)
        cb = np.ascontiguousarray(col_base, np.int32)
        cl = np.ascontiguousarray(cols, np.int32)
        lv = np.ascontiguousarray(live, np.int8)
        cv = np.ascontiguousarray(cover, np.int8).copy()
        lo = np.full(max_ranges, -7, np.int32)
        pre = np.full(max_ranges + 1, -7, np.int32)
        nr = f(n, cb.ctypes.data, cl.ctypes.data, lv.ctypes.data, cv.ctypes.data, max_ranges,
               lo.ctypes.data, pre.ctypes.data)
        return nr, cv.astype(bool), lo, pre
    return call


def _runs(flags):
    out, i, n = [], 0, len(flags)
    while i < n:
        if flags[i]:
            j = i
            while j + 1 < n and flags[j + 1]:
                j += 1
            out.append((i, j))
            i = j + 1
        else:
            i += 1
    return out


def _min_extra_columns(cols, live, cover_old, max_ranges):
    """Fewest covered columns outside the live volumes over every choice of
    joinable gaps (all volumes of the gap still covered) that leaves at
    most max_ranges runs."""
    runs = _runs(live)
    gaps = []
    for (a0, a1), (b0, _) in zip(runs, runs[1:]):
        if all(cover_old[a1 + 1:b0]):
            gaps.append(int(sum(cols[a1 + 1:b0])))
    need = max(0, len(runs) - max_ranges)
    best = None
    for k in range(need, len(gaps) + 1):
        for sub in itertools.combinations(gaps, k):
            best = sum(sub) if best is None else min(best, sum(sub))
    return best


def _check(cols, col_base, live, cover_old, max_ranges, nr, cover, lo, pre):
    n = len(cols)
    assert nr >= 0, "a choice within the rules must exist"
    assert nr <= max_ranges
    assert (cover <= cover_old).all(), "the covered set may only shrink"
    assert (cover >= live).all(), "every live volume must be covered"
    if not live.any():
        assert nr == 0 and not cover.any()
        return
    # ranges: sorted, apart, exactly the covered volumes' columns
    assert pre[0] == 0
    spans = [(int(lo[r]), int(lo[r] + pre[r + 1] - pre[r])) for r in range(nr)]
    assert all(a < b for a, b in spans)
    assert all(spans[r][1] < spans[r + 1][0] for r in range(nr - 1))
    covered_cols = set()
    for i in range(n):
        if cover[i]:
            covered_cols.update(range(col_base[i], col_base[i] + cols[i]))
    span_cols = set()
    for a, b in spans:
        span_cols.update(range(a, b))
    assert span_cols == covered_cols
    assert nr == len(_runs(cover))
    extra = int(sum(cols[i] for i in range(n) if cover[i] and not live[i]))
    assert extra == _min_extra_columns(cols, live, cover_old, max_ranges)
    if len(_runs(live)) <= max_ranges:
        assert (cover == live).all()


@pytest.mark.parametrize("max_ranges", [1, 2, 3, MAX_RANGES])
def test_simulated_searches(cover_fn, max_ranges):
    rng = np.random.default_rng(100 + max_ranges)
    for trial in range(300):
        n = int(rng.integers(1, 13 if max_ranges < MAX_RANGES else 40))
        cols = rng.integers(1, 7, size=n)
        col_base = np.concatenate([[0], np.cumsum(cols)[:-1]]).astype(np.int64)
        live = rng.random(n) < rng.uniform(0.2, 0.9)
        if not live.any():
            live[rng.integers(n)] = True
        idx = np.flatnonzero(live)
        cover = np.zeros(n, bool)
        cover[idx[0]:idx[-1] + 1] = True   # the volumes between the first and last taking part
        while True:
            nr, new_cover, lo, pre = cover_fn(col_base, cols, live, cover, max_ranges)
            if max_ranges < MAX_RANGES or n <= 14:
                _check(cols, col_base, live, cover, max_ranges, nr, new_cover, lo, pre)
            else:   # too many gaps for the brute force: the other checks
                assert 0 <= nr <= max_ranges
                assert (new_cover <= cover).all() and (new_cover >= live).all()
                assert nr == len(_runs(new_cover))
            cover = new_cover
            if not live.any():
                break
            # a few volumes' searches end at this poll
            leave = np.flatnonzero(live)
            k = int(rng.integers(1, len(leave) + 1))
            live[rng.choice(leave, size=min(k, int(rng.integers(1, 4))), replace=False)] = False


def test_choice_outside_the_rules_is_refused(cover_fn):
    # live volumes 0, 2 and 4 with the volumes between them no longer
    # covered cannot fit one range: -1, and nothing is written
    cols = np.array([2, 1, 3, 1, 2])
    col_base = np.array([0, 2, 3, 6, 7])
    live = np.array([1, 0, 1, 0, 1], bool)
    cover = live.copy()
    nr, new_cover, lo, pre = cover_fn(col_base, cols, live, cover, 1)
    assert nr == -1
    assert (new_cover == cover).all()
    assert (lo == -7).all() and (pre == -7).all()
    # with three ranges allowed the same state is fine
    nr, new_cover, lo, pre = cover_fn(col_base, cols, live, cover, 3)
    assert nr == 3 and list(lo[:3]) == [0, 3, 7] and list(pre[:4]) == [0, 2, 5, 7]
