"""Host logic of the multifrontal symbolic analysis, without a GPU.

The product's nested dissection and front construction (paper_1411_0660_amd/
csrc/symbolic.cpp, host C++) are compiled with g++ together with
tests/symbolic_dump.cpp, run on the sector pattern of the periodic chain
(Eq. (1): the diagonal plus one entry per antiparallel neighbour pair), and
checked against what a multifrontal LU of that pattern needs: a permutation;
pivot blocks that tile the new order in post-order; contribution rows that lie
after their front's pivots and inside the parent front; every original entry
and every entry of the exact symbolic fill of the reordered pattern inside the
front of its column; and the fill and flop counts equal to their formulas over
the fronts.  The GPU tests check the same tree through the library."""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1411_0660_amd", "csrc")

# (L, leaf size); the product's leaf size is 96.  L = 17 at 96 and L = 12 at 8
# hold a front without pivots: a subgraph that the separators above it had
# already disconnected splits with an empty separator, and that front only
# passes its children's updates on to its parent.
CASES = [(L, leaf) for L in (2, 4, 6, 8, 10, 12) for leaf in (8, 96)] + \
        [(L, 8) for L in (5, 7, 9, 11)] + [(17, 96)]
EXACT_FILL_MAX_N = 1000          # the set-based exact fill is checked up to this order


@pytest.fixture(scope="module")
def dump_exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("symbolic") / "symbolic_dump")
    cmd = [gxx, "-O2", "-std=c++17", "-pthread", "-I", CSRC,
           os.path.join(ROOT, "tests", "symbolic_dump.cpp"), os.path.join(CSRC, "symbolic.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def run_dump(exe, L, leaf):
    r = subprocess.run([exe, str(L), str(leaf)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout)


def symbolic_fill(n, rowptr, col, iperm):
    """Exact structure of the factor of the reordered symmetric pattern:
    struct(i) = rows j > i of column i, by elimination with the elimination
    tree (column i inherits the structure of its children minus i)."""
    below = [set() for _ in range(n)]
    for u in range(n):
        for e in range(rowptr[u], rowptr[u + 1]):
            v = col[e]
            i, j = iperm[u], iperm[v]
            if i < j:
                below[i].add(j)
            elif j < i:
                below[j].add(i)
    parent = [-1] * n
    kids = [[] for _ in range(n)]
    out = []
    for i in range(n):
        s = set(below[i])
        for k in kids[i]:
            s |= out[k]
        s.discard(i)
        out.append(s)
        if s:
            parent[i] = min(s)
            kids[parent[i]].append(i)
    return out


@pytest.mark.parametrize("L,leaf", CASES, ids=[f"L{L}-leaf{lf}" for L, lf in CASES])
def test_front_tree_invariants(dump_exe, L, leaf):
    t = run_dump(dump_exe, L, leaf)
    if (L, leaf) in ((12, 8), (17, 96)):
        assert any(f["p"] == 0 for f in t["fronts"])             # the pass-through case is covered
    n = t["n"]
    assert n == math.comb(L, (L + 1) // 2)
    perm = np.array(t["perm"])
    assert sorted(perm.tolist()) == list(range(n))                   # a permutation
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    fronts = t["fronts"]
    # pivot blocks tile [0, n) in front order (post-order: children first)
    pos = 0
    owner = np.empty(n, dtype=np.int64)
    for k, f in enumerate(fronts):
        assert f["first"] == pos and (f["p"] >= 1 or len(f["children"]) >= 2)
        owner[pos:pos + f["p"]] = k
        pos += f["p"]
        for ch in f["children"]:
            assert ch < k and fronts[ch]["parent"] == k
        lvl = 1 + max((fronts[ch]["level"] for ch in f["children"]), default=-1)
        assert f["level"] == lvl
    assert pos == n
    assert t["n_levels"] == 1 + max(f["level"] for f in fronts)
    # contribution rows: sorted, after the front's pivots, inside the parent
    for k, f in enumerate(fronts):
        cr = f["contrib"]
        assert len(cr) == f["c"]
        assert all(a < b for a, b in zip(cr, cr[1:]))
        assert all(x >= f["first"] + f["p"] for x in cr)
        if f["parent"] < 0:
            assert f["c"] == 0                                        # a root front updates nothing
        else:
            P = fronts[f["parent"]]
            prows = set(range(P["first"], P["first"] + P["p"])) | set(P["contrib"])
            assert set(cr) <= prows
    rows_of = [set(range(f["first"], f["first"] + f["p"])) | set(f["contrib"]) for f in fronts]
    # every original entry, and every entry of the exact fill, lies in the
    # front holding the pivot of its column
    rowptr, col = t["rowptr"], t["col"]
    for u in range(n):
        for e in range(rowptr[u], rowptr[u + 1]):
            i, j = sorted((int(iperm[u]), int(iperm[col[e]])))
            assert j in rows_of[owner[i]], (u, col[e])
    exact = 0
    if n <= EXACT_FILL_MAX_N:
        fill = symbolic_fill(n, rowptr, col, iperm)
        for i in range(n):
            assert fill[i] <= rows_of[owner[i]], i
            exact += len(fill[i])
    # counts over the fronts: nnz(L+U) = sum p^2 + 2 p c, entries sum m^2,
    # flops sum 2/3 p^3 + 2 p^2 c + 2 p c^2, and the predicted factor holds at
    # least the exact fill (n diagonal + 2 x the strict lower fill)
    p = np.array([f["p"] for f in fronts], dtype=np.int64)
    c = np.array([f["c"] for f in fronts], dtype=np.int64)
    assert t["nnz_factor"] == int(np.sum(p * p + 2 * p * c))
    assert t["front_entries"] == int(np.sum((p + c) ** 2))
    fl = float(np.sum(2.0 / 3.0 * p ** 3 + 2.0 * p ** 2 * c + 2.0 * p * c ** 2))
    assert abs(t["flops"] - fl) <= 1e-12 * fl
    assert t["nnz_factor"] >= n + 2 * exact


def test_front_tree_is_deterministic(dump_exe):
    a = run_dump(dump_exe, 12, 8)
    b = run_dump(dump_exe, 12, 8)
    assert a == b
