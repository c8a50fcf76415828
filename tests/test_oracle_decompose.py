"""Pins for the oracle's decomposition and grid numbering (Sec. 3.1, 3.3)."""
import os

import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_grid_examples.txt")


def _alg_decompose(N, M, p):
    # Alg. Decompose (Sec. 3.1), branch form: the remainder goes to the first parts.
    q, r = N // M, N % M
    if r > p:
        n = q + 1
        s = n * p
    else:
        n = q
        s = n * p + r
    return n, s


def test_decompose_matches_algorithm_exhaustive():
    for N in range(0, 301):
        for M in range(1, 41):
            parts = [oracle.decompose(N, M, p) for p in range(M)]
            assert parts == [_alg_decompose(N, M, p) for p in range(M)]
            # the parts tile 0..N-1: s_0 = 0 and s_k = s_{k-1} + n_{k-1}
            assert parts[0][1] == 0
            for k in range(1, M):
                assert parts[k][1] == parts[k - 1][1] + parts[k - 1][0]
            assert sum(n for n, _ in parts) == N
            ns = [n for n, _ in parts]
            assert max(ns) - min(ns) <= 1
            assert ns == sorted(ns, reverse=True)  # the larger parts come first


def test_decompose_known_values():
    # 257 half-spectrum bins over 8 parts: the first part gets one extra bin
    assert [oracle.decompose(257, 8, p)[0] for p in range(8)] == [33] + [32] * 7
    # fewer elements than parts leaves trailing parts empty
    assert [oracle.decompose(3, 5, p) for p in range(5)] == [(1, 0), (1, 1), (1, 2), (0, 3), (0, 3)]


def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([tok.strip() for tok in line.split("|")])
    return rows


def test_paper_grid_numbering():
    rows = _golden()
    assert rows
    for row in rows:
        dims = tuple(int(x) for x in row[0].split()[1].split(","))
        if row[1].startswith("coords"):
            coords = tuple(int(x) for x in row[1].split()[1].split(","))
            rank = int(row[2].split()[1])
            # in a layout where grid dir i splits axis i, rank r's block starts
            # at the decompose() start of its coordinates
            lay = oracle.Layout((dims[0] * 2, dims[1] * 2, 5), dims, (0, 1, -1))
            ls, st = lay.block(rank)
            assert st[:2] == (coords[0] * 2, coords[1] * 2)
        else:
            d = int(row[1].split()[1])
            members = [int(x) for x in row[2].split()[1].split(",")]
            lay = oracle.Layout((dims[0] * 2, dims[1] * 2, 5), dims, (0, 1, -1))
            # a subgroup along dir d: ranks that share every other coordinate
            starts = [lay.block(r)[1] for r in members]
            other = [s[1 - d] for s in starts]
            assert len(set(other)) == 1
            assert sorted(s[d] for s in starts) == [2 * c for c in range(dims[d])]


@pytest.mark.parametrize("ndim,ngrid,expect", [
    (3, 1, [(0, -1, -1), (-1, 0, -1)]),
    (3, 2, [(0, 1, -1), (0, -1, 1), (-1, 0, 1)]),
    (4, 3, [(0, 1, 2, -1), (0, 1, -1, 2), (0, -1, 1, 2), (-1, 0, 1, 2)]),
])
def test_paper_layout_chains(ndim, ngrid, expect):
    # Eqs. slab0-slab1 (1 -> 0), pencil0-pencil2 (2 -> 1 in P1, 1 -> 0 in P0),
    # 4d_fft0-4d_fft3 (3 -> 2, 2 -> 1, 1 -> 0).
    assert oracle.paper_layouts(ndim, ngrid) == expect


def test_transform_schedule_is_last_axis_first():
    assert oracle.transform_schedule(oracle.paper_layouts(3, 1)) == [(0, 2), (0, 1), (1, 0)]
    assert oracle.transform_schedule(oracle.paper_layouts(3, 2)) == [(0, 2), (1, 1), (2, 0)]
    assert oracle.transform_schedule(oracle.paper_layouts(4, 3)) == [(0, 3), (1, 2), (2, 1), (3, 0)]
    # slab with the distribution moved from axis 0 to axis 2
    dirs = oracle.layouts_from_steps(3, 1, [(0, 2)])
    assert dirs == [(0, -1, -1), (-1, -1, 0)]
    assert oracle.transform_schedule(dirs) == [(0, 2), (0, 1), (1, 0)]
