"""FP32-on-GPU against the FP64 oracle, per workload recipe.

For every workload recipe (configs 1-5: small plain, paper-scale plain, large
batched, size grid, serving mix) a sample of ligands stratified by (heavy atoms,
rotatable bonds) is docked by the batched form with the recipe's pocket and
search and checked in follow mode (tests/parity.py).  Config 1 runs in full;
the others use the first 32 of the recipe's start orientations (restarts are
independent, so each of them is computed exactly as in the full run) to keep
the oracle's time bounded.  The statistics (decisions, exact, score ties
relative and beyond 1e-5 absolute, bump ties, largest tie gap, largest final
and restart score error, largest pose RMSD) are printed and, with
DOCK_PARITY_REPORT set, appended to that file as JSON lines.
"""
import numpy as np
import pytest

import synth
from tests.test_gpu_parity import D, check_all, ctx, run_batch  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu

R_SAMPLE = 32


def stratified(lib, per, seed):
    """Ligand indices: `per` drawn (seeded) from each (atom-count quartile,
    bond-count half) cell, plus the largest ligand (the widest kernel slot of
    the recipe)."""
    n, B = lib.n_atoms(), lib.n_rot()
    rng = np.random.default_rng(seed)
    qa = np.quantile(n, [0.25, 0.5, 0.75])
    cell = np.searchsorted(qa, n, side="right") * 2 + (B > np.median(B))
    picks = []
    for c in range(8):
        idx = np.flatnonzero(cell == c)
        if len(idx):
            picks += [int(v) for v in rng.choice(idx, min(per, len(idx)), replace=False)]
    picks.append(int(np.argmax(n * 1000 + B)))
    return sorted(set(picks))


def _run(D, ctx, pk, lib, q, s, ligs, label):
    sub = lib.subset(ligs)
    print(f"[case] {label}: atoms {list(sub.n_atoms())}, bonds {list(sub.n_rot())}", flush=True)
    h, params = run_batch(D, ctx, pk, sub, q, **s)
    st = check_all(D, pk, sub, q, h, params, label=label)
    assert st["ligands"] == sub.n_ligands


def test_config1_in_full(D, ctx):
    pk, lib, q, s = synth.config(1)
    _run(D, ctx, pk, lib, q, s, list(range(lib.n_ligands)), "config 1 (full)")


@pytest.mark.parametrize("cfg", [2, 3])
def test_config_sample(D, ctx, cfg):
    pk, lib, q, s = synth.config(cfg, n_ligands=2000)
    s = dict(s, restarts=R_SAMPLE)
    _run(D, ctx, pk, lib, q[:R_SAMPLE], s, stratified(lib, 2, 2209 + cfg),
         f"config {cfg} (stratified sample, restarts 0-31)")


def test_config4_cells(D, ctx):
    seed = synth.MASTER_SEED + 4
    c2 = synth.CONFIGS[2]
    pk = synth.pocket_gaussians(seed, **c2["pocket"])
    q = synth.start_quats(seed, 128)[:R_SAMPLE]
    s = dict(c2["search"], restarts=R_SAMPLE)
    libs = [synth.library_from_sizes(seed + 1000 * n + B, [n], [B])
            for n, B in ((16, 4), (32, 8), (64, 16), (64, 24), (128, 0), (128, 24))]
    lib = libs[0]
    for other in libs[1:]:
        lib = _concat(lib, other)
    _run(D, ctx, pk, lib, q, s, list(range(lib.n_ligands)),
         "config 4 (one ligand of six size cells, restarts 0-31)")


def test_config5_serving_mix(D, ctx):
    seed = synth.MASTER_SEED + 5
    pk = synth.pocket_gaussians(seed + 100 * 5, 4, 96, 0.375, 160, 9.0)
    lib = synth.library_lognormal(seed + 7, 2000)
    q = synth.start_quats(seed, 256)[:R_SAMPLE]
    s = dict(synth.CONFIGS[2]["search"], restarts=R_SAMPLE)
    _run(D, ctx, pk, lib, q, s, stratified(lib, 2, 2214),
         "config 5 (serving mix, pocket 5, stratified sample, restarts 0-31)")


def _concat(a, b):
    W = max(a.mask_words, b.mask_words)

    def widen(m, w):
        out = np.zeros((len(m), W), np.uint64)
        out[:, :w] = m
        return out
    return synth.Library(
        atom_off=np.concatenate([a.atom_off, a.atom_off[-1] + b.atom_off[1:]]).astype(np.int32),
        xyz=np.concatenate([a.xyz, b.xyz]), type=np.concatenate([a.type, b.type]),
        bond_off=np.concatenate([a.bond_off, a.bond_off[-1] + b.bond_off[1:]]).astype(np.int32),
        bonds=np.concatenate([a.bonds, b.bonds]),
        rot_off=np.concatenate([a.rot_off, a.rot_off[-1] + b.rot_off[1:]]).astype(np.int32),
        rot_bond=np.concatenate([a.rot_bond, b.rot_bond]),
        rot_mask=np.concatenate([widen(a.rot_mask, a.mask_words), widen(b.rot_mask, b.mask_words)]),
        mask_words=W)
