"""GPU-vs-oracle parity checks (follow mode).

The GPU library returns, per ligand, its decision trace (alignment index and
torsion step of every decision), the kept restarts and the final alignment
indices.  The FP64 oracle replays those decisions; at each one it checks that
the GPU's choice is the oracle's own argmax or a near-tie:
  * score near-tie: |S_gpu_choice - S_best| <= TIE_REL * max(1, |S_best|);
  * bump near-tie: the choice is decided by a pair distance within BUMP_TOL of
    the bump distance.
It then continues with the GPU's choice, so later decisions stay comparable.
Pass/fail bar (FP32 GPU vs FP64 oracle):
  * no mismatching decision;
  * kept restarts form a valid greedy selection under the oracle's scores
    (up to score near-ties and RMSD within RMSD_SEL_TOL of the threshold);
  * final scores within SCORE_REL * max(1, |S|); restart scores likewise;
  * final poses within POSE_RMSD Angstrom RMSD.
"""
import json
import os

import numpy as np

from oracle import oracle as O
from paper_2209_05069_amd import dock as D

TIE_REL = 1e-5
BUMP_TOL = 1e-4
SCORE_REL = 1e-4
POSE_RMSD = 1e-3
RMSD_SEL_TOL = 1e-3


def rmsd(a, b):
    return float(np.sqrt(np.mean(np.sum((np.asarray(a, np.float64) - b) ** 2, axis=-1))))


def check_selection(sel, S, P, K, delta):
    """sel: kept restarts (any order). S/P: oracle restart scores/poses."""
    G = [int(r) for r in sel]
    Gs = set(G)
    assert len(Gs) == len(G), "duplicate kept restart"
    assert len(G) <= K
    tol = TIE_REL * max(1.0, float(np.max(np.abs(S))))
    for i in range(len(G)):
        for j in range(i):
            assert rmsd(P[G[i]], P[G[j]]) >= delta - RMSD_SEL_TOL, "kept poses too similar"
    smin = min(S[g] for g in G) if G else np.inf
    for r in range(len(S)):
        if r in Gs:
            continue
        suppressed = any(rmsd(P[r], P[g]) < delta + RMSD_SEL_TOL and S[g] >= S[r] - tol for g in G)
        below = len(G) == K and S[r] <= smin + tol
        assert suppressed or below, f"restart {r} should have been kept"


def follow_ligand(grid, lig, quats, params, g):
    """Run the oracle in follow mode on GPU outputs g (from dock.ligand_outputs)."""
    assert g["status"] == 0
    return O.dock_ligand(
        grid, lig, quats,
        torsion_steps=params.torsion_steps, sweep_passes=params.sweep_passes,
        align_steps=params.align_steps, top_k=params.top_k, final_align=params.final_align,
        bump_min_bonds=params.bump_min_bonds, bump_dist=params.bump_dist,
        dedup_rmsd=params.dedup_rmsd,
        follow=dict(trace=g["trace"], sel_restart=g["pose_restart"],
                    final_trace=g["final_trace"], tie_rel=TIE_REL, bump_tol=BUMP_TOL))


def check_ligand(grid, lig, quats, params, g, stats=None):
    """Full parity check of one ligand.  Returns the oracle follow result."""
    o = follow_ligand(grid, lig, quats, params, g)
    st = o["stats"]
    assert st["mismatches"] == 0, f"decision mismatches: {st}"
    assert st["decisions"] == params.restarts * (1 + params.sweep_passes * lig.nrot) + (
        g["n_poses"] if params.final_align else 0)
    # restart scores
    S = o["restart_score"]
    rerr = 0.0
    if "restart_score" in g:
        err = np.abs(g["restart_score"] - S) / np.maximum(1.0, np.abs(S))
        assert err.max() <= SCORE_REL, f"restart score rel err {err.max()}"
        rerr = float(err.max())
    check_selection(g["pose_restart"], S, o["restart_pose"], params.top_k, params.dedup_rmsd)
    # final poses and scores (oracle keeps the GPU's output order in follow mode)
    fs = o["pose_score"]
    assert len(fs) == g["n_poses"]
    err = np.abs(g["pose_score"] - fs) / np.maximum(1.0, np.abs(fs))
    assert err.max(initial=0) <= SCORE_REL, f"final score rel err {err.max()}"
    for s in range(len(fs)):
        assert rmsd(g["pose_xyz"][s], o["pose_xyz"][s]) <= POSE_RMSD
    tol = TIE_REL * max(1.0, float(np.max(np.abs(fs), initial=1.0)))
    assert np.all(np.diff(fs) <= tol), "outputs not in final-score order"
    if g["n_poses"]:
        assert g["best_score"] == g["pose_score"][0]
    if stats is not None:
        for k in ("decisions", "exact", "score_ties", "score_ties_beyond_abs", "bump_ties"):
            stats[k] = stats.get(k, 0) + st[k]
        stats["ligands"] = stats.get("ligands", 0) + 1
        stats["max_restart_rel_err"] = max(stats.get("max_restart_rel_err", 0.0), rerr)
        stats["max_tie_gap"] = max(stats.get("max_tie_gap", 0.0), float(st["max_tie_gap"]))
        stats["max_final_rel_err"] = max(stats.get("max_final_rel_err", 0.0), float(err.max(initial=0)))
        stats["max_pose_rmsd"] = max(stats.get("max_pose_rmsd", 0.0),
                                     max((rmsd(g["pose_xyz"][s], o["pose_xyz"][s])
                                          for s in range(len(fs))), default=0.0))
    return o


def report(label, stats):
    """Append one JSON line of parity statistics to the file named by the
    DOCK_PARITY_REPORT environment variable (nothing when it is unset)."""
    path = os.environ.get("DOCK_PARITY_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(dict(label=label, **stats)) + "\n")
