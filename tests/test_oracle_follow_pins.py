"""Pins of the oracle's follow mode, torsion branch (Optimize Pose of Alg. 1,
arXiv:2209.05069, Application Description: a candidate that fails the Bump
Check is rejected, the best-scoring remaining one is kept).

Follow mode replays another implementation's decisions and classifies each one
as exact, score near-tie, bump near-tie or mismatch; every GPU parity verdict
rests on that classifier.  Each test here plants one choice at one torsion
decision and checks the class the oracle gives it against a ground truth that
does not come from the oracle: closed-form distances and scores on hand-built
chains, or an independent numpy/scipy replay (scipy Rotation for the turns,
scipy RegularGridInterpolator for the scores, scipy shortest_path for the bond
distances) of a config-1 ligand's decision.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import oracle as O
from tests.test_oracle_pins import (_chain, _params, affine_pocket, align_rot, grid_centre,
                                    mask_of, scipy_interp, scipy_score, start_pose, topo_scipy)

TIE_REL = 1e-5
BUMP_TOL = 1e-4


def _follow(pk, lig, q, trace, **kw):
    p = _params(**kw)
    return O.dock_ligand(pk, lig, q, follow=dict(trace=trace, tie_rel=TIE_REL,
                                                  bump_tol=BUMP_TOL), **p)


# ---------------------------------------------------------------------------
# Hand-built chain 0-1-2-3-4 turned about 1->2 (the z axis): atom 4 (type 1) at
# radius 1.2 from the axis, height 0.3, angle phi; atom 0 at (1.2, 0, -0.9).
# d(0,4)^2 = 1.44 (3 - 2 cos phi) (closed form), 4 bonds apart: with 36 steps of
# 10 degrees, k in 0..8 and 28..35 put the pair closer than 2.0 A.
CHAIN = ([[1.2, 0, -0.9], [0, 0, 0], [0, 0, 1.5], [1.2, 0, 2.4], [1.2, 0, 0.3]],
         [0, 0, 0, 0, 1], (1, 2), (2, 3, 4))
T36 = 36


def chain_dist(k):
    phi = 2 * np.pi * k / T36
    return float(np.sqrt(1.44 * (3 - 2 * np.cos(phi))))


def chain_run(trace_k, gx=1.0, gy=0.5, **kw):
    """Follow [alignment 0, torsion step trace_k] on the chain with f_1 = gx x + gy y
    (the pose is the input shifted by its centroid, so atom 4 scores
    gx (1.2 cos phi - cx) + gy (1.2 sin phi - cy) + const)."""
    pk = affine_pocket([(0, 0, 0, 0, 0), (0, gx, gy, 0, 0)], n=16)
    lig = _chain(*CHAIN)
    q = np.array([[1, 0, 0, 0]], np.float32)
    tr = np.array([[0, trace_k]], np.uint16)
    p = dict(torsion_steps=T36, align_steps=1, top_k=1)
    p.update(kw)
    return _follow(pk, lig, q, tr, **p)


def test_chain_closed_form_ground_truth():
    # the oracle's own (free) choice on the chain: phi = 90 deg, as the closed form says
    pk = affine_pocket([(0, 0, 0, 0, 0), (0, 1.0, 0.5, 0, 0)], n=16)
    res = O.dock_ligand(pk, _chain(*CHAIN), np.array([[1, 0, 0, 0]], np.float32),
                        **_params(torsion_steps=T36, align_steps=1, top_k=1))
    assert int(res["trace"][0, 1]) == 9
    assert chain_dist(8) < 2.0 < chain_dist(9)


def test_follow_own_choice_is_exact():
    r = chain_run(9)
    assert list(r["decision_class"][0]) == [O.EXACT, O.EXACT]
    assert r["stats"]["mismatches"] == 0


def test_clearly_worse_free_step_is_a_mismatch():
    # phi = 180 deg: d = 2.68 A (free), score 1.8 below the best free step
    assert chain_dist(18) > 2.5
    r = chain_run(18)
    assert r["decision_class"][0, 1] == O.MISMATCH
    assert r["stats"]["mismatches"] == 1


def test_clearly_bumped_better_scoring_step_is_a_mismatch():
    # phi = 70 deg scores 0.974 (above the free optimum 0.6) but its 1-5 pair is
    # 1.826 A apart, 0.17 A inside the bump distance: the bump rejects it
    assert chain_dist(7) < 2.0 - 0.1
    assert 1.2 * np.cos(np.radians(70)) + 0.6 * np.sin(np.radians(70)) > 0.6 + 0.3
    r = chain_run(7)
    assert r["decision_class"][0, 1] == O.MISMATCH


def test_none_with_a_free_candidate_is_a_mismatch():
    r = chain_run(O.NONE_ACCEPTED)
    assert r["decision_class"][0, 1] == O.MISMATCH


def test_step_beyond_range_is_a_mismatch():
    r = chain_run(T36)
    assert r["decision_class"][0, 1] == O.MISMATCH


def test_all_bumped_decision_none_is_exact_and_any_step_is_a_mismatch():
    # atom 4 on the axis, 1.265 A from atom 0 for every step: all candidates bump
    pk = affine_pocket([(0, 0, 0, 0, 0), (0, 1.0, 0.5, 0, 0)], n=16)
    lig = _chain([[1.2, 0, -0.9], [0, 0, 0], [0, 0, 1.5], [0, 0, 2.9], [0, 0, -0.5]],
                 [0, 0, 0, 0, 1], (1, 2), (2, 3, 4))
    q = np.array([[1, 0, 0, 0]], np.float32)
    kw = dict(torsion_steps=T36, align_steps=1, top_k=1)
    r = _follow(pk, lig, q, np.array([[0, O.NONE_ACCEPTED]], np.uint16), **kw)
    assert r["decision_class"][0, 1] == O.EXACT
    r = _follow(pk, lig, q, np.array([[0, 3]], np.uint16), **kw)
    assert r["decision_class"][0, 1] == O.MISMATCH


def test_exact_symmetric_tie_is_a_score_tie():
    # f_1 = x: the score of atom 4 is 1.2 cos phi + const, so phi = 90 and phi = 270
    # deg (both free, d = 2.08 A) score the same up to FP64 rounding of cos; the
    # oracle keeps the first (k = 9); the other (k = 27) is a score tie, and
    # phi = 100 deg (0.21 lower) is a mismatch
    own = chain_run(9, gx=1.0, gy=0.0)
    assert own["decision_class"][0, 1] == O.EXACT
    r = chain_run(27, gx=1.0, gy=0.0)
    assert r["decision_class"][0, 1] == O.SCORE_TIE
    assert r["stats"]["max_tie_gap"] < 1e-12
    assert r["stats"]["score_ties_beyond_abs"] == 0
    r = chain_run(10, gx=1.0, gy=0.0)
    assert r["decision_class"][0, 1] == O.MISMATCH


def test_near_tie_inside_and_outside_the_tolerance():
    # f_1 = eps * x: candidate k scores 1.2 eps cos(phi_k) + const.  The best
    # free step is phi = 90 deg; phi = 100 deg is lower by 1.2 eps sin(10 deg).
    # With eps = 2^-16 the gap (3.2e-6) is inside the tie tolerance 1e-5 (score
    # below 1): a score tie.  With eps = 2^-12 (gap 5.1e-5) it is a mismatch.
    gap = lambda eps: 1.2 * eps * (np.cos(np.radians(90)) - np.cos(np.radians(100)))
    eps_in, eps_out = 2.0 ** -16, 2.0 ** -12
    assert gap(eps_in) < 0.5 * TIE_REL and gap(eps_out) > 2 * TIE_REL
    r = chain_run(10, gx=eps_in, gy=0.0)
    assert r["decision_class"][0, 1] == O.SCORE_TIE
    assert r["stats"]["max_tie_gap"] == pytest.approx(gap(eps_in), rel=1e-6)
    r = chain_run(10, gx=eps_out, gy=0.0)
    assert r["decision_class"][0, 1] == O.MISMATCH


def test_bump_near_ties_at_the_boundary():
    # bump_dist set within the bump tolerance of the phi = 80 deg pair distance:
    d8 = chain_dist(8)
    # (i) just above it: the oracle calls phi = 80 bumped, but the given choice
    # of phi = 80 (scoring above the best surely-free step) is a bump near-tie
    r = chain_run(8, bump_dist=d8 + 0.5 * BUMP_TOL)
    assert r["decision_class"][0, 1] == O.BUMP_TIE
    # (ii) just below it: the oracle keeps phi = 80 (free, best); a given phi = 90
    # (the best surely-free step) means the other side judged phi = 80 bumped
    r = chain_run(9, bump_dist=d8 - 0.5 * BUMP_TOL)
    assert r["decision_class"][0, 1] == O.BUMP_TIE
    # (iii) the same choices with the boundary well away are a mismatch
    r = chain_run(8, bump_dist=d8 + 10 * BUMP_TOL)
    assert r["decision_class"][0, 1] == O.MISMATCH
    r = chain_run(9, bump_dist=d8 - 10 * BUMP_TOL)
    assert r["decision_class"][0, 1] == O.MISMATCH


# ---------------------------------------------------------------------------
# A config-1 ligand: an independent numpy/scipy replay of the oracle's own
# trace up to one torsion decision gives every candidate's pair distance and
# score; planted choices are picked from that table.
@pytest.fixture(scope="module")
def c1_case():
    pk, lib, q, s = synth.config(1)
    lig = O.ligand_from_library(lib, 0)
    kw = dict(torsion_steps=s["torsion_steps"], sweep_passes=s["sweep_passes"],
              align_steps=s["align_steps"], top_k=s["top_k"], dedup_rmsd=s["dedup_rmsd"])
    own = O.dock_ligand(pk, lig, q, **kw)
    return pk, lig, q, s, kw, own


def candidate_table(pk, lig, q, s, trace_r, r, d):
    """(distance, score) of every candidate at decision d of restart r, replaying
    trace_r[:d] independently of the oracle."""
    A, T, B = s["align_steps"], s["torsion_steps"], lig.nrot
    f = scipy_interp(pk.values, pk.spacing, pk.origin)
    Y = start_pose(lig.xyz, q[r], grid_centre(pk))
    c = Y.mean(0)
    Y = align_rot(A, int(trace_r[0])).apply(Y - c) + c
    masks = [mask_of(lig.rot_mask[b], lig.n) for b in range(B)]

    def turn(Y, b, k):
        a_, b_ = (int(v) for v in lig.rot_bond[b])
        u = (Y[b_] - Y[a_]) / np.linalg.norm(Y[b_] - Y[a_])
        Z = Y.copy()
        Z[masks[b]] = Y[a_] + Rotation.from_rotvec(u * 2 * np.pi * k / T).apply(Y[masks[b]] - Y[a_])
        return Z

    for e in range(1, d):
        k = int(trace_r[e])
        if k != O.NONE_ACCEPTED:
            Y = turn(Y, (e - 1) % B, k)
    b = (d - 1) % B
    topo = topo_scipy(lig.n, lig.bonds)
    M = masks[b]
    elig = (M[:, None] & ~M[None, :]) & (topo >= 4)
    dist, score = np.empty(T), np.empty(T)
    for k in range(T):
        Z = turn(Y, b, k)
        dd = np.linalg.norm(Z[:, None] - Z[None], axis=-1)
        dist[k] = dd[elig].min() if elig.any() else np.inf
        score[k] = scipy_score(f, lig.type, Z)
    return dist, score


def plant_and_check(c1_case, r, d, k_planted):
    pk, lig, q, s, kw, own = c1_case
    tr = own["trace"].copy()
    tr[r, d] = k_planted
    res = O.dock_ligand(pk, lig, q, follow=dict(trace=tr, tie_rel=TIE_REL, bump_tol=BUMP_TOL),
                        **kw)
    cls = res["decision_class"]
    assert cls[r, d] == O.MISMATCH, (r, d, k_planted, cls[r])
    # everything before the planted decision, and every other restart, is exact
    assert np.all(cls[r, :d] == O.EXACT)
    others = np.delete(cls, r, axis=0)
    assert np.all(others == O.EXACT)
    assert res["stats"]["mismatches"] >= 1


def _find(c1_case, want):
    """First (r, d, k, dist, score) over the ligand's torsion decisions where
    want(dist, score, chosen) picks a candidate k."""
    pk, lig, q, s, kw, own = c1_case
    D = own["trace"].shape[1]
    for r in range(3):
        for d in range(1, D):
            dist, score = candidate_table(pk, lig, q, s, own["trace"][r], r, d)
            chosen = int(own["trace"][r, d])
            free = dist >= 2.0
            # the oracle's own step is the best free candidate (independent check)
            assert chosen == int(np.flatnonzero(free)[np.argmax(score[free])])
            k = want(dist, score, chosen)
            if k is not None:
                return r, d, k
    pytest.fail("no decision of the kind wanted")


def test_c1_clearly_worse_free_step_is_a_mismatch(c1_case):
    def want(dist, score, chosen):
        best = score[chosen]
        tol = TIE_REL * max(1.0, abs(best))
        ok = np.flatnonzero((dist >= 2.0 + 0.1) & (score < best - 100 * tol))
        return int(ok[0]) if len(ok) else None
    plant_and_check(c1_case, *_find(c1_case, want))


def test_c1_clearly_bumped_better_scoring_step_is_a_mismatch(c1_case):
    def want(dist, score, chosen):
        best = score[chosen]
        tol = TIE_REL * max(1.0, abs(best))
        ok = np.flatnonzero((dist <= 2.0 - 0.1) & (score > best + 100 * tol))
        return int(ok[0]) if len(ok) else None
    plant_and_check(c1_case, *_find(c1_case, want))


def test_c1_none_with_free_candidates_is_a_mismatch(c1_case):
    def want(dist, score, chosen):
        return O.NONE_ACCEPTED if np.any(dist >= 2.0 + 0.1) else None
    plant_and_check(c1_case, *_find(c1_case, want))
