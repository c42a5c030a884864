"""Pins of the FP64 oracle to things other than itself.

Each test checks one step of Alg. 1 (arXiv:2209.05069, Application Description)
against a closed form, a hand-built case, an independent library routine
(scipy's RegularGridInterpolator, Rotation, shortest_path), or exhaustive search,
so that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import shortest_path
from scipy.spatial.transform import Rotation

import synth
from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# independent helpers (scipy / numpy), written for the tests only
def scipy_interp(values, h, origin):
    T, nz, ny, nx = values.shape
    axes = [origin[0] + h * np.arange(nx), origin[1] + h * np.arange(ny),
            origin[2] + h * np.arange(nz)]
    fns = [RegularGridInterpolator(axes, values[t].transpose(2, 1, 0).astype(np.float64),
                                   method="linear") for t in range(T)]
    lo = np.array([a[0] for a in axes])
    hi = np.array([a[-1] for a in axes])

    def f(types, P):
        P = np.clip(np.asarray(P, np.float64).reshape(-1, 3), lo, hi)
        types = np.asarray(types).reshape(-1)
        out = np.empty(len(P))
        for t in np.unique(types):
            m = types == t
            out[m] = fns[int(t)](P[m])
        return out
    return f


def scipy_score(f, types, P):
    return float(np.sum(f(types, P)))


def topo_scipy(n, bonds):
    A = coo_matrix((np.ones(len(bonds)), (bonds[:, 0], bonds[:, 1])), shape=(n, n))
    return shortest_path(A, directed=False, unweighted=True)


def start_pose(X, q, gc):
    X = X.astype(np.float64)
    c0 = X.mean(0)
    w, x, y, z = (float(v) for v in q)
    return Rotation.from_quat([x, y, z, w]).apply(X - c0) + gc


def align_rot(A, o):
    i, j = divmod(o, A)
    return Rotation.from_euler("xy", [2 * np.pi * i / A, 2 * np.pi * j / A])


def grid_centre(pk):
    nx, ny, nz = pk.shape_xyz
    return np.array(pk.origin) + pk.spacing * (np.array([nx, ny, nz]) - 1) / 2.0


def mask_of(m, n):
    return np.array([(int(m[i >> 6]) >> (i & 63)) & 1 for i in range(n)], bool)


class FakePocket:
    def __init__(self, values, h, origin):
        self.values = np.ascontiguousarray(values, np.float32)
        self.spacing = h
        self.origin = tuple(origin)

    @property
    def shape_xyz(self):
        t, nz, ny, nx = self.values.shape
        return nx, ny, nz


def affine_pocket(coefs, n=16, h=0.5):
    """Per type t, f_t(x,y,z) = c0 + c1 x + c2 y + c3 z + c4 xyz sampled at the grid points;
    dyadic coefficients and spacing keep every stored value exact in float32."""
    o = -h * (n - 1) / 2.0
    ax = o + h * np.arange(n)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    vals = np.stack([c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * Y * Z for c in coefs])
    assert np.array_equal(vals.astype(np.float32).astype(np.float64), vals)
    return FakePocket(vals, h, (o, o, o))


def affine_value(c, p):
    x, y, z = p
    return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y * z


# ---------------------------------------------------------------------------
# Score: trilinear grid interpolation
def test_interp_golden_hand_computed():
    g = json.load(open(os.path.join(HERE, "golden", "trilinear_2x2x2.json")))
    vals = np.array(g["values_zyx"], np.float32)[None]
    pk = FakePocket(vals, g["spacing"], g["origin"])
    for case in g["cases"]:
        assert O.interp(pk, 0, case["p"]) == pytest.approx(case["value"], abs=1e-14)


def test_interp_constant_grid_everywhere():
    pk = FakePocket(np.full((2, 5, 6, 7), 0.625, np.float32), 0.5, (-1.0, 2.0, 0.0))
    rng = np.random.default_rng(1)
    for p in rng.uniform(-10, 10, (50, 3)):
        assert O.interp(pk, 1, p) == 0.625


def test_interp_reproduces_trilinear_polynomials():
    coefs = [(0.25, 0.5, -0.125, 0.75, 0.0625), (-1.0, 0.0, 0.25, -0.5, -0.03125)]
    pk = affine_pocket(coefs)
    rng = np.random.default_rng(2)
    lo = pk.origin[0]
    for p in rng.uniform(lo, -lo, (200, 3)):
        for t in (0, 1):
            assert O.interp(pk, t, p) == pytest.approx(affine_value(coefs[t], p), abs=1e-12)


def test_interp_at_grid_points_returns_stored_value():
    pk = synth.pocket_gaussians(7, 2, 12, 0.5, 10, 2.0)
    rng = np.random.default_rng(3)
    for _ in range(100):
        t = int(rng.integers(0, 2))
        i, j, k = rng.integers(0, 12, 3)
        p = np.array(pk.origin) + pk.spacing * np.array([i, j, k])
        assert O.interp(pk, t, p) == pytest.approx(float(pk.values[t, k, j, i]), abs=1e-12)


def test_interp_clamps_outside_to_edge():
    coefs = [(0.25, 0.5, -0.125, 0.75, 0.0625)]
    pk = affine_pocket(coefs)
    hi = -pk.origin[0]
    rng = np.random.default_rng(4)
    for p in rng.uniform(-3 * hi, 3 * hi, (200, 3)):
        pc = np.clip(p, -hi, hi)
        assert O.interp(pk, 0, p) == pytest.approx(affine_value(coefs[0], pc), abs=1e-12)


def test_interp_upper_faces_stay_inside_the_type_block():
    # type 1 is all NaN: an upper-face sample of type 0 that read one cell past the
    # edge (even with weight 0) would come out NaN.
    coefs = [(0.25, 0.5, -0.125, 0.75, 0.0625)]
    base = affine_pocket(coefs, n=8)
    vals = np.concatenate([base.values, np.full_like(base.values, np.nan)])
    pk = FakePocket(vals, base.spacing, base.origin)
    hi = -pk.origin[0]
    for p in ([hi, hi, hi], [hi, 0.1, -0.3], [0.2, hi, 0.4], [-0.1, 0.3, hi],
              [hi + 5, hi + 1, hi + 2]):
        pc = np.clip(p, -hi, hi)
        assert O.interp(pk, 0, p) == pytest.approx(affine_value(coefs[0], pc), abs=1e-12)


def test_interp_matches_scipy_on_gaussian_grid():
    pk = synth.pocket_gaussians(11, 4, 32, 0.5, 40, 4.0)
    f = scipy_interp(pk.values, pk.spacing, pk.origin)
    rng = np.random.default_rng(5)
    P = rng.uniform(-9, 9, (400, 3))
    T = rng.integers(0, 4, 400)
    ref = f(T, P)
    got = np.array([O.interp(pk, int(t), p) for t, p in zip(T, P)])
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_score_is_sum_over_atoms_by_type():
    coefs = [(0.25, 0.5, -0.125, 0.75, 0.0), (-1.0, 0.0, 0.25, -0.5, 0.0),
             (0.5, -0.25, 0.0, 0.125, 0.0625)]
    pk = affine_pocket(coefs)
    rng = np.random.default_rng(6)
    P = rng.uniform(-3, 3, (17, 3))
    T = rng.integers(0, 3, 17).astype(np.uint8)
    expect = sum(affine_value(coefs[t], p) for t, p in zip(T, P))
    assert O.score(pk, T, P) == pytest.approx(expect, abs=1e-12)


# ---------------------------------------------------------------------------
# Topology, validation, rotations
def test_topo_matches_scipy_shortest_path():
    lib = synth.library_uniform(21, 6, (5, 60), (0, 6))
    for l in range(lib.n_ligands):
        x, t, b, r, m = lib.ligand(l)
        n = len(x)
        np.testing.assert_array_equal(O.topo(n, b), topo_scipy(n, b))
    # a ring (not a tree): 6-cycle with a tail
    bonds = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 5], [5, 0], [3, 6]], np.int32)
    np.testing.assert_array_equal(O.topo(7, bonds), topo_scipy(7, bonds))


def test_check_ligand_accepts_synth_and_rejects_bad_masks():
    pk = synth.pocket_gaussians(1, 4, 16, 0.5, 5, 2.0)
    lib = synth.library_uniform(22, 5, (10, 40), (1, 5))
    for l in range(lib.n_ligands):
        assert O.check_ligand(pk, O.ligand_from_library(lib, l)) == 0
    x, t, b, r, m = lib.ligand(0)
    bad = m.copy()
    bad[0, 0] ^= np.uint64(1) << np.uint64(int(r[0, 0]))         # fixed atom marked moving
    assert O.check_ligand(pk, O.LigandArrays(x, t, b, r, bad)) != 0
    bad = m.copy()
    bad[0, 0] ^= np.uint64(1) << np.uint64(int(r[0, 1]))         # moving atom b cleared
    assert O.check_ligand(pk, O.LigandArrays(x, t, b, r, bad)) != 0
    tb = t.copy()
    tb[0] = 4                                                      # type out of range
    assert O.check_ligand(pk, O.LigandArrays(x, tb, b, r, m)) != 0
    # a bond inside a ring is not rotatable
    xr = np.random.default_rng(0).normal(size=(6, 3)).astype(np.float32)
    ring = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 5], [5, 0]], np.int32)
    rm = np.array([[0b000110]], np.uint64)
    assert O.check_ligand(pk, O.LigandArrays(xr, np.zeros(6, np.uint8), ring,
                                             np.array([[0, 1]], np.int32), rm)) != 0


def test_quaternion_matrix_matches_scipy():
    q = synth.start_quats(5, 20)
    for v in q:
        w, x, y, z = (float(a) for a in v)
        ref = Rotation.from_quat([x, y, z, w]).as_matrix()
        np.testing.assert_allclose(O.quat_matrix(v), ref, atol=1e-12)


def test_alignment_matrix_is_Ry_times_Rx():
    for A in (30, 7):
        for o in (0, 1, A, A + 3, A * A - 1, 5 * A + 11 if A == 30 else 8):
            np.testing.assert_allclose(O.align_matrix(A, o), align_rot(A, o).as_matrix(),
                                       atol=1e-12)


def test_start_quats_are_isotropic():
    q = synth.start_quats(99, 100000).astype(np.float64)
    Rm = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(Rm.mean(0), 0.0, atol=0.01)
    ez = Rm[:, :, 2]
    np.testing.assert_allclose(ez.T @ ez / len(ez), np.eye(3) / 3, atol=0.01)


# ---------------------------------------------------------------------------
# Generate_Starting_Pose, alignment
def _params(**kw):
    p = dict(torsion_steps=36, sweep_passes=1, align_steps=30, top_k=4, final_align=0,
             bump_min_bonds=4, bump_dist=2.0, dedup_rmsd=0.0)
    p.update(kw)
    return p


def test_start_pose_matches_scipy_rotation():
    pk = synth.pocket_gaussians(31, 4, 32, 0.5, 40, 4.0)
    lib = synth.library_from_sizes(31, [15], [0])
    lig = O.ligand_from_library(lib, 0)
    q = synth.start_quats(31, 5)
    res = O.dock_ligand(pk, lig, q, **_params(align_steps=1, top_k=5))
    f = scipy_interp(pk.values, pk.spacing, pk.origin)
    for r in range(5):
        Y = start_pose(lig.xyz, q[r], grid_centre(pk))
        np.testing.assert_allclose(res["restart_pose"][r], Y, atol=1e-12)
        assert res["restart_score"][r] == pytest.approx(scipy_score(f, lig.type, Y), abs=1e-10)


def test_alignment_picks_known_orientation_two_atom_ligand():
    # f_0 = g.p, f_1 = -g.p: the score of a 2-atom ligand is g . (p0 - p1), so the best
    # of the 900 orientations is the one turning p0 - p1 closest to g.  (g has y and z
    # parts: with g = e_x the lattice orientations (a, b) and (a + pi, -b) tie exactly.)
    g = np.array([1.0, 0.375, 0.125])
    pk = affine_pocket([(0, *g, 0), (0, *(-g), 0)], n=32)
    X = np.array([[0.3, -0.2, 0.5], [1.1, 0.9, -0.4]], np.float32)
    lig = O.LigandArrays(X, np.array([0, 1], np.uint8), np.array([[0, 1]], np.int32),
                         np.zeros((0, 2), np.int32), np.zeros((0, 1), np.uint64))
    q = synth.start_quats(41, 6)
    res = O.dock_ligand(pk, lig, q, **_params(top_k=6))
    for r in range(6):
        Y = start_pose(X, q[r], grid_centre(pk))
        v = Y[0] - Y[1]
        table = np.array([align_rot(30, o).apply(v) @ g for o in range(900)])
        best = int(np.argmax(table))
        srt = np.sort(table)
        assert srt[-1] - srt[-2] > 1e-9
        assert int(res["trace"][r, 0]) == best
        assert res["restart_score"][r] == pytest.approx(table[best], abs=1e-12)


def test_rigid_only_poses_are_rigid_and_best_of_900():
    pk = synth.pocket_gaussians(51, 4, 32, 0.5, 40, 4.0)
    lib = synth.library_from_sizes(51, [14], [0])
    lig = O.ligand_from_library(lib, 0)
    q = synth.start_quats(51, 4)
    res = O.dock_ligand(pk, lig, q, **_params(top_k=4))
    f = scipy_interp(pk.values, pk.spacing, pk.origin)
    X = lig.xyz.astype(np.float64)
    for r in range(4):
        # Kabsch (textbook SVD superposition) of the input onto the pose
        P = res["restart_pose"][r]
        Xc, Pc = X - X.mean(0), P - P.mean(0)
        U, S, Vt = np.linalg.svd(Xc.T @ Pc)
        d = np.sign(np.linalg.det(U @ Vt))
        Rk = U @ np.diag([1, 1, d]) @ Vt
        rmsd = np.sqrt(np.mean(np.sum((Xc @ Rk - Pc) ** 2, 1)))
        assert rmsd < 1e-9
        Y = start_pose(X, q[r], grid_centre(pk))
        c = Y.mean(0)
        table = np.array([scipy_score(f, lig.type, align_rot(30, o).apply(Y - c) + c)
                          for o in range(900)])
        assert res["restart_score"][r] == pytest.approx(table.max(), abs=1e-9)
        srt = np.sort(table)
        if srt[-1] - srt[-2] > 1e-9:
            assert int(res["trace"][r, 0]) == int(np.argmax(table))


# ---------------------------------------------------------------------------
# Optimize Pose: exhaustive search on 1-2 bond ligands
def _aligned_pose(pk, lig, q_r, o, A=30):
    Y = start_pose(lig.xyz, q_r, grid_centre(pk))
    c = Y.mean(0)
    return align_rot(A, o).apply(Y - c) + c


def _turn(Y, a, b, M, theta):
    u = (Y[b] - Y[a]) / np.linalg.norm(Y[b] - Y[a])
    Z = Y.copy()
    Z[M] = Y[a] + Rotation.from_rotvec(u * theta).apply(Y[M] - Y[a])
    return Z


def _clash(Z, far):
    d = np.linalg.norm(Z[:, None] - Z[None], axis=-1)
    return bool(np.any(d[far] < 2.0))


@pytest.mark.parametrize("seed", [61, 62, 63])
def test_single_bond_greedy_equals_exhaustive(seed):
    pk = synth.pocket_gaussians(seed, 4, 32, 0.5, 40, 4.0)
    lib = synth.library_from_sizes(seed, [14], [1])
    assert lib.n_rot(0) == 1
    lig = O.ligand_from_library(lib, 0)
    T = 48
    q = synth.start_quats(seed, 3)
    res = O.dock_ligand(pk, lig, q, **_params(torsion_steps=T, top_k=3))
    f = scipy_interp(pk.values, pk.spacing, pk.origin)
    n = lig.n
    D = topo_scipy(n, lig.bonds)
    a, b = lig.rot_bond[0]
    M = mask_of(lig.rot_mask[0], n)
    far = (D >= 4) & (M[:, None] ^ M[None, :])
    checked = 0
    for r in range(3):
        Y = _aligned_pose(pk, lig, q[r], int(res["trace"][r, 0]))
        S = np.full(T, -np.inf)
        for k in range(T):
            Z = _turn(Y, a, b, M, 2 * np.pi * k / T)
            if not _clash(Z, far):
                S[k] = scipy_score(f, lig.type, Z)
        best = int(np.argmax(S))
        srt = np.sort(S[np.isfinite(S)])
        assert res["restart_score"][r] == pytest.approx(S[best], abs=1e-9)
        if len(srt) > 1 and srt[-1] - srt[-2] < 1e-9:
            continue
        assert int(res["trace"][r, 1]) == best
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("seed", [71, 72])
def test_two_bond_greedy_is_a_path_through_the_exhaustive_table(seed):
    pk = synth.pocket_gaussians(seed, 4, 32, 0.5, 40, 4.0)
    lib = synth.library_from_sizes(seed, [13], [2])
    assert lib.n_rot(0) == 2
    lig = O.ligand_from_library(lib, 0)
    T, P = 24, 2
    q = synth.start_quats(seed, 2)
    res = O.dock_ligand(pk, lig, q, **_params(torsion_steps=T, sweep_passes=P, top_k=2))
    f = scipy_interp(pk.values, pk.spacing, pk.origin)
    n = lig.n
    D = topo_scipy(n, lig.bonds)
    far = D >= 4
    Ms = [mask_of(lig.rot_mask[i], n) for i in range(2)]
    for r in range(2):
        Y = _aligned_pose(pk, lig, q[r], int(res["trace"][r, 0]))
        # table over absolute angles, built from the aligned pose (bond 1, then bond 2)
        S = np.full((T, T), -np.inf)
        for k1 in range(T):
            Z1 = _turn(Y, *lig.rot_bond[0], Ms[0], 2 * np.pi * k1 / T)
            for k2 in range(T):
                Z = _turn(Z1, *lig.rot_bond[1], Ms[1], 2 * np.pi * k2 / T)
                if not _clash(Z, far):
                    S[k1, k2] = scipy_score(f, lig.type, Z)
        state = [0, 0]
        expect = []
        ok = True
        for p in range(P):
            for bi in range(2):
                line = np.array([S[(state[0] + j) % T, state[1]] if bi == 0 else
                                 S[state[0], (state[1] + j) % T] for j in range(T)])
                j = int(np.argmax(line))
                srt = np.sort(line[np.isfinite(line)])
                if len(srt) > 1 and srt[-1] - srt[-2] < 1e-9:
                    ok = False
                expect.append(j)
                state[bi] = (state[bi] + j) % T
        if not ok:
            continue
        np.testing.assert_array_equal(res["trace"][r, 1:], expect)
        assert res["restart_score"][r] == pytest.approx(S[state[0], state[1]], abs=1e-9)
        assert res["restart_score"][r] <= np.max(S) + 1e-12


def test_exact_ties_take_the_first_candidate():
    # A constant grid gives every orientation and every torsion step exactly the same
    # score, so each decision must keep the first candidate: orientation 0, step 0.
    pk = FakePocket(np.full((4, 16, 16, 16), 0.5, np.float32), 0.5, (-3.75,) * 3)
    lib = synth.library_from_sizes(81, [16], [3])
    lig = O.ligand_from_library(lib, 0)
    q = synth.start_quats(81, 3)
    res = O.dock_ligand(pk, lig, q, **_params(torsion_steps=36, sweep_passes=2, top_k=3))
    assert np.all(res["trace"] == 0)
    np.testing.assert_array_equal(res["sel_restart"], [0, 1, 2])


# ---------------------------------------------------------------------------
# Bump Check: hand-built chains (distances in closed form)
def _chain(coords, types, rot, moving):
    X = np.array(coords, np.float32)
    n = len(X)
    bonds = np.array([[i, i + 1] for i in range(n - 1)], np.int32)
    m = np.zeros((1, 1), np.uint64)
    for i in moving:
        m[0, 0] |= np.uint64(1) << np.uint64(i)
    return O.LigandArrays(X, np.array(types, np.uint8), bonds, np.array([rot], np.int32), m)


def _hand_dock(lig, T):
    # f_0 = 0, f_1 = x + y/2; identity start, identity-only alignment, so the pose is
    # the input shifted by a constant and only the torsion step matters.
    pk = affine_pocket([(0, 0, 0, 0, 0), (0, 1, 0.5, 0, 0)], n=16)
    q = np.array([[1, 0, 0, 0]], np.float32)
    return O.dock_ligand(pk, lig, q, **_params(torsion_steps=T, align_steps=1, top_k=1))


def test_bump_rejects_one_five_pair_by_hand():
    # Chain 0-1-2-3-4 turned about 1->2 (z axis); atom 4 at radius 1.2, height 0.3;
    # atom 0 at (1.2, 0, -0.9).  d(0,4)^2 = 1.44 (3 - 2 cos phi) < 4 for |phi| < 83.62
    # deg, so with 10-degree steps phi = 90 (k=9, score 0.6) beats the bumped
    # phi = 80 (k=8, score 0.799) and the unconstrained optimum near 26.6 deg.
    lig = _chain([[1.2, 0, -0.9], [0, 0, 0], [0, 0, 1.5], [1.2, 0, 2.4], [1.2, 0, 0.3]],
                 [0, 0, 0, 0, 1], (1, 2), (2, 3, 4))
    res = _hand_dock(lig, 36)
    assert int(res["trace"][0, 1]) == 9


def test_bump_ignores_one_four_pairs_by_hand():
    # Same geometry without atom 4: the close pair (0,3) is only 3 bonds apart, so it
    # is never checked; the best step is phi = 30 deg (k=3): 1.2cos30 + 0.6 sin30.
    lig = _chain([[1.2, 0, -0.9], [0, 0, 0], [0, 0, 1.5], [1.2, 0, 0.3]],
                 [0, 0, 0, 1], (1, 2), (2, 3))
    res = _hand_dock(lig, 36)
    assert int(res["trace"][0, 1]) == 3


def test_all_candidates_bumped_keeps_conformation():
    # Atom 4 sits on the rotation axis, 1.265 A from atom 0 (4 bonds away), for every
    # step: all candidates bump and the pose is kept.
    lig = _chain([[1.2, 0, -0.9], [0, 0, 0], [0, 0, 1.5], [0, 0, 2.9], [0, 0, -0.5]],
                 [0, 0, 0, 0, 1], (1, 2), (2, 3, 4))
    res = _hand_dock(lig, 36)
    assert int(res["trace"][0, 1]) == O.NONE_ACCEPTED
    X = lig.xyz.astype(np.float64)
    np.testing.assert_allclose(res["restart_pose"][0], X - X.mean(0), atol=1e-12)


# ---------------------------------------------------------------------------
# Select Poses: hand-made pose sets
def test_select_hand_made_translations():
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64)
    shifts = [0.0, 1.0, 2.5, 3.0, 6.0]   # plain RMSD between two shifted copies = |shift difference|
    poses = np.stack([base + [s, 0, 0] for s in shifts])
    scores = np.array([5, 4, 3, 2, 1], np.float64)
    np.testing.assert_array_equal(O.select(scores, poses, 10, 2.0), [0, 2, 4])
    np.testing.assert_array_equal(O.select(scores, poses, 2, 2.0), [0, 2])
    np.testing.assert_array_equal(O.select(scores, poses, 10, 0.0), [0, 1, 2, 3, 4])
    # ties in score keep restart order
    np.testing.assert_array_equal(
        O.select(np.array([1, 3, 3, 2.0]), poses[:4], 10, 0.0), [1, 2, 3, 0])


# ---------------------------------------------------------------------------
# whole-ligand invariants, determinism, follow mode
@pytest.fixture(scope="module")
def c1_runs():
    pk, lib, q, s = synth.config(1)
    out = []
    for l in range(3):
        lig = O.ligand_from_library(lib, l)
        res = O.dock_ligand(pk, lig, q, decisions=True, torsion_steps=s["torsion_steps"],
                            sweep_passes=s["sweep_passes"], top_k=s["top_k"],
                            dedup_rmsd=s["dedup_rmsd"])
        out.append((lig, res))
    return pk, q, s, out


def test_geometry_invariants_hold_on_every_restart(c1_runs):
    pk, q, s, runs = c1_runs
    for lig, res in runs:
        n = lig.n
        X = lig.xyz.astype(np.float64)
        D = topo_scipy(n, lig.bonds)
        # atoms in the same rigid piece: not separated by any rotatable bond
        piece = np.zeros((n, n), bool)
        Ms = [mask_of(lig.rot_mask[i], n) for i in range(lig.nrot)]
        same = np.ones((n, n), bool)
        for M in Ms:
            same &= ~(M[:, None] ^ M[None, :])
        piece = same
        dX = np.linalg.norm(X[:, None] - X[None], axis=-1)
        for r in range(len(res["restart_pose"])):
            Y = res["restart_pose"][r]
            dY = np.linalg.norm(Y[:, None] - Y[None], axis=-1)
            np.testing.assert_allclose(dY[D == 1], dX[D == 1], atol=1e-6)  # bond lengths
            np.testing.assert_allclose(dY[D == 2], dX[D == 2], atol=1e-6)  # bond angles
            np.testing.assert_allclose(dY[piece], dX[piece], atol=1e-6)   # rigid pieces
            # float32 input: compare to the exact double values of those inputs
            assert np.max(np.abs(dY[piece] - dX[piece])) < 1e-10
            # no accepted conformation has a clash
            assert not np.any(dY[D >= 4] < 2.0)


def test_each_decision_never_lowers_the_score(c1_runs):
    pk, q, s, runs = c1_runs
    for lig, res in runs:
        ds = res["decision_score"]
        assert np.all(np.diff(ds, axis=1) >= -1e-12)
        np.testing.assert_allclose(ds[:, -1], res["restart_score"], atol=1e-12)


def test_outputs_sorted_and_deduplicated(c1_runs):
    pk, q, s, runs = c1_runs
    for lig, res in runs:
        assert np.all(np.diff(res["pose_score"]) <= 0)
        P = res["pose_xyz"]
        for i in range(len(P)):
            for j in range(i):
                pass
        # kept restarts are pairwise at least dedup_rmsd apart (before the final step)
        RP = res["restart_pose"][res["sel_restart"]]
        for i in range(len(RP)):
            for j in range(i):
                assert np.sqrt(np.mean(np.sum((RP[i] - RP[j]) ** 2, 1))) >= s["dedup_rmsd"]
        # final alignment never lowers a kept pose's score
        assert np.all(res["pose_score"] >= res["restart_score"][res["sel_restart"]] - 1e-12)


def test_deterministic(c1_runs):
    pk, q, s, runs = c1_runs
    lig, res = runs[0]
    res2 = O.dock_ligand(pk, lig, q, decisions=True, torsion_steps=s["torsion_steps"],
                         sweep_passes=s["sweep_passes"], top_k=s["top_k"],
                         dedup_rmsd=s["dedup_rmsd"])
    for k in ("restart_score", "restart_pose", "trace", "pose_score", "pose_xyz", "sel_restart"):
        np.testing.assert_array_equal(res[k], res2[k])


def test_follow_own_decisions_is_exact(c1_runs):
    pk, q, s, runs = c1_runs
    lig, res = runs[1]
    fol = O.dock_ligand(pk, lig, q, torsion_steps=s["torsion_steps"],
                        sweep_passes=s["sweep_passes"], top_k=s["top_k"],
                        dedup_rmsd=s["dedup_rmsd"],
                        follow=dict(trace=res["trace"], sel_restart=res["sel_restart"],
                                    final_trace=res["final_trace"]))
    st = fol["stats"]
    assert st["mismatches"] == 0 and st["exact"] == st["decisions"]
    np.testing.assert_array_equal(fol["pose_score"], res["pose_score"])


def test_follow_flags_a_wrong_decision(c1_runs):
    pk, q, s, runs = c1_runs
    lig, res = runs[2]
    tr = res["trace"].copy()
    # plant a clearly worse alignment choice for restart 0
    table = []
    fol0 = O.dock_ligand(pk, lig, q, torsion_steps=s["torsion_steps"],
                         sweep_passes=s["sweep_passes"], top_k=s["top_k"],
                         follow=dict(trace=tr))
    assert fol0["stats"]["mismatches"] == 0
    tr[0, 0] = (int(tr[0, 0]) + 450) % 900
    fol = O.dock_ligand(pk, lig, q, torsion_steps=s["torsion_steps"],
                        sweep_passes=s["sweep_passes"], top_k=s["top_k"], follow=dict(trace=tr))
    assert fol["stats"]["mismatches"] >= 1
