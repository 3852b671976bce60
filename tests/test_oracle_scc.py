"""Pins of the literal reading of Definition 6 (Sec. 2.3): the largest
strongly connected component of the input-union symbolic image, plus every
vertex with a path into it.

* Hand-built graphs whose answer is read off the drawing: two cycles with
  tails, an acyclic graph, a self-loop, a tie, a chain between components.
* Brute force on random small graphs: components and paths from the
  transitive closure of the adjacency matrix (no graph library).
* The set lies inside the non-leaving set (cells with an infinite path),
  and equals it when that set holds a single component with a cycle.
"""
import numpy as np
import pytest

import oracle


def _graph(n_cells, K, edges):
    """edges: {(cell, input): [targets]} -> CSR over rows cell * K + input."""
    row_ptr = [0]
    col = []
    for r in range(n_cells * K):
        col += sorted(edges.get(divmod(r, K), []))
        row_ptr.append(len(col))
    return np.array(row_ptr, np.int64), np.array(col, np.int32)


def _set(kept):
    return sorted(int(c) for c in np.nonzero(kept)[0])


CASES = {
    # cycle 0-1-2 (3 cells), cycle 3..7 (5 cells); 8 -> 0, 9 -> 3, 10 -> 9
    "two_cycles": (11, {(0, 0): [1], (1, 1): [2], (2, 0): [0], (3, 0): [4], (4, 0): [5],
                        (5, 1): [6], (6, 0): [7], (7, 0): [3], (8, 0): [0], (9, 1): [3],
                        (10, 1): [9]}, [3, 4, 5, 6, 7, 9, 10]),
    "acyclic": (3, {(0, 0): [1], (1, 0): [2]}, []),
    # 0 -> 0; 1 -> 0; 2 -> 1; 3 has no edge
    "self_loop": (4, {(0, 1): [0], (1, 0): [0], (2, 0): [1]}, [0, 1, 2]),
    # {0, 1} and {2, 3} of equal size: the smaller ids win; 4 -> 2 is not kept
    "tie": (5, {(0, 0): [1], (1, 0): [0], (2, 0): [3], (3, 1): [2], (4, 0): [2]}, [0, 1]),
    # cycle {0, 1, 2} -> chain 3 -> 4 -> cycle {5, 6, 7, 8}: everything has a path into the latter
    "chain": (9, {(0, 0): [1], (1, 0): [2], (2, 0): [0, 3], (3, 0): [4], (4, 0): [5],
                  (5, 0): [6], (6, 0): [7], (7, 0): [8], (8, 0): [5]}, list(range(9))),
}


@pytest.mark.parametrize("name", list(CASES))
def test_hand_built(oracle_lib, name):
    n, edges, want = CASES[name]
    K = 2
    row_ptr, col = _graph(n, K, edges)
    kept, mask = oracle.largest_scc(row_ptr, col, n, K)
    assert _set(kept) == want
    for c in range(n):
        bits = 0
        if kept[c]:
            for u in range(K):
                if any(kept[t] for t in edges.get((c, u), [])):
                    bits |= 1 << u
        assert int(mask[c, 0]) == bits, (name, c)


def _brute(n, K, row_ptr, col):
    A = np.zeros((n, n), dtype=bool)
    for r in range(n * K):
        for t in col[row_ptr[r]:row_ptr[r + 1]]:
            A[r // K, t] = True
    plus = A.copy()  # paths of length >= 1
    for _ in range(n):
        plus = plus | ((plus.astype(np.int64) @ A.astype(np.int64)) > 0)
    star = plus | np.eye(n, dtype=bool)
    best = None
    for v in range(n):
        comp = [w for w in range(n) if star[v, w] and star[w, v]]
        if not plus[v, v]:
            continue  # no cycle through v
        key = (-len(comp), comp[0])
        if best is None or key < best[0]:
            best = (key, comp)
    if best is None:
        return np.zeros(n, np.uint8)
    return np.array([any(star[v, w] for w in best[1]) for v in range(n)], np.uint8)


@pytest.mark.parametrize("seed", range(40))
def test_brute_force(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n, K = int(rng.integers(1, 10)), int(rng.integers(1, 4))
    p = rng.uniform(0.05, 0.35)
    edges = {}
    for c in range(n):
        for u in range(K):
            edges[(c, u)] = [t for t in range(n) if rng.random() < p]
    row_ptr, col = _graph(n, K, edges)
    kept, mask = oracle.largest_scc(row_ptr, col, n, K)
    np.testing.assert_array_equal(kept, _brute(n, K, row_ptr, col))
    nl_kept, _, _ = oracle.prune(row_ptr, col, np.zeros(n * K, np.uint8), n, K, "nonleaving")
    assert not (kept & (1 - nl_kept)).any(), "inside the non-leaving set"


def test_single_component_equals_nonleaving(oracle_lib):
    # a ring of 12 cells with chords, and tails into it: one component with a cycle
    n, K = 20, 3
    edges = {(c, 0): [(c + 1) % 12] for c in range(12)}
    edges.update({(c, 1): [(c + 5) % 12] for c in range(0, 12, 3)})
    edges.update({(c, 2): [c - 12] for c in range(12, 20)})
    row_ptr, col = _graph(n, K, edges)
    kept, mask = oracle.largest_scc(row_ptr, col, n, K)
    nl_kept, nl_mask, _ = oracle.prune(row_ptr, col, np.zeros(n * K, np.uint8), n, K, "nonleaving")
    np.testing.assert_array_equal(kept, nl_kept)
    np.testing.assert_array_equal(mask, nl_mask)
