"""Pins of the oracle's pairwise rescoring stand-in (oracle_contacts).

The paper's Rescore Pose evaluates every ligand atom against every pocket atom
and accumulates the pair terms per pose (Rescore Pose subsections of the
latency and batched implementations); the stand-in pair term is an integer
weight per (ligand type, pocket atom type) for pairs closer than a contact
distance.  The pins below fix it independently of its own code: a hand-computed
case (with a weight table that is not symmetric, and pairs on both sides of the
cutoff), the strict cutoff at a distance that is exact in floating point, a
KD-tree pair search from scipy on random inputs, invariance under a common rigid
motion, and the boundary count.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

from oracle import oracle as O


def _pa(xyz, types, ntypes, weight, dc):
    return O.PocketAtoms(np.asarray(xyz, np.float32), np.asarray(types, np.uint8), ntypes,
                         np.asarray(weight, np.int32), dc)


# Weight table, ligand type (rows) x pocket atom type (columns); not symmetric.
W = [[1, 2, 3],
     [4, 5, 6]]


def test_hand_computed_case():
    # ligand atom 0 (type 0) at the origin, atom 1 (type 1) at (10, 0, 0)
    lig_t = [0, 1]
    lig = [[0, 0, 0], [10, 0, 0]]
    pocket = [[1, 0, 0],      # type 0: 1.0 from atom 0 -> W[0][0] = 1
              [0, 3.5, 0],    # type 1: 3.5 from atom 0 -> W[0][1] = 2
              [0, 0, 4.5],    # type 0: 4.5 from atom 0 -> beyond 4
              [10, 0, 3.9],   # type 2: 3.9 from atom 1 -> W[1][2] = 6
              [13, 0, 0]]     # type 1: 3.0 from atom 1 -> W[1][1] = 5
    ptypes = [0, 1, 0, 2, 1]
    v, b = O.contacts(_pa(pocket, ptypes, 3, W, 4.0), lig_t, lig, tol=0.05)
    assert v == 1 + 2 + 6 + 5
    assert b == 0
    # with the ligand types swapped the rows of W swap: 4 + 5 + 3 + 2
    v2, _ = O.contacts(_pa(pocket, ptypes, 3, W, 4.0), [1, 0], lig)
    assert v2 == 4 + 5 + 3 + 2


def test_cutoff_is_strict_and_boundary_counted():
    # (4, 0, 0) is exactly 4.0 from the origin in floating point: not a contact
    pa = _pa([[4, 0, 0], [0, -3.75, 0]], [2, 0], 3, W, 4.0)
    v, b = O.contacts(pa, [1], [[0, 0, 0]], tol=1e-4)
    assert v == W[1][0]          # only the 3.75 pair
    assert b == abs(W[1][2])     # the pair at the cutoff is a boundary pair
    v, b = O.contacts(pa, [1], [[1e-3, 0, 0]], tol=1e-4)
    assert v == W[1][0] + W[1][2] and b == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_kdtree_pair_search(seed):
    rng = np.random.default_rng(seed)
    n, m, tl, tp = 60, 1500, 4, 5
    lig = rng.uniform(-8, 8, (n, 3))
    lt = rng.integers(0, tl, n)
    pxyz = rng.uniform(-14, 14, (m, 3)).astype(np.float32)
    pt = rng.integers(0, tp, m)
    w = rng.integers(-3, 4, (tl, tp))
    dc = 4.0
    v, b = O.contacts(_pa(pxyz, pt, tp, w, dc), lt, lig, tol=1e-9)
    tree = cKDTree(pxyz.astype(np.float64))
    expect = 0
    for i, js in enumerate(tree.query_ball_point(lig, dc)):
        for j in js:
            expect += int(w[lt[i], pt[j]])
    assert b == 0  # random inputs: no pair within 1e-9 of the cutoff
    assert v == expect
    assert expect != 0


def test_invariant_under_a_common_rigid_motion():
    rng = np.random.default_rng(7)
    lig = rng.uniform(-6, 6, (40, 3))
    lt = rng.integers(0, 2, 40)
    pxyz = rng.uniform(-12, 12, (800, 3))
    pt = rng.integers(0, 3, 800)
    Rm = Rotation.from_rotvec([0.3, -1.1, 0.7]).as_matrix()
    t = np.array([2.5, -1.0, 0.75])
    v0, b0 = O.contacts(_pa(pxyz, pt, 3, W, 3.5), lt, lig, tol=1e-3)
    p1 = (pxyz.astype(np.float32).astype(np.float64) @ Rm.T + t)
    v1, b1 = O.contacts(_pa(p1, pt, 3, W, 3.5), lt, lig @ Rm.T + t, tol=1e-3)
    assert abs(v1 - v0) <= b0 + b1
    assert v0 != 0


def test_empty_pocket_and_empty_ligand():
    pa = _pa(np.zeros((0, 3)), [], 3, W, 4.0)
    assert O.contacts(pa, [0, 1], [[0, 0, 0], [1, 1, 1]]) == (0, 0)
    pa = _pa([[0, 0, 0]], [0], 3, W, 4.0)
    assert O.contacts(pa, [], np.zeros((0, 3))) == (0, 0)
