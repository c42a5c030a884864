"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Every comparison uses the follow-mode checks of tests/parity.py on seeded
synthetic inputs.  Marked `gpu`: needs an MI355X and the built libdock.so.
"""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2209_05069_amd import dock
    return dock


@pytest.fixture(scope="module")
def ctx(D):
    c = D.dock_create(0)
    yield c
    D.dock_destroy(c)


def run_batch(D, ctx, pk, lib, quats, **kw):
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    params = D.SearchParams(quats, **kw)
    dl = D.DeviceLibrary(lib)
    res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params,
                          restart_scores=True, trace=True, final_trace=True)
    D.dock_ligands_batch(ctx, pid, dl, params, res)
    torch.cuda.synchronize()
    h = res.to_host()
    D.dock_pocket_unload(ctx, pid)
    return h, params


def check_all(D, pk, lib, quats, h, params, ligands=None, label=""):
    grid = O.Grid.of(pk)
    stats = {}
    ligs = range(lib.n_ligands) if ligands is None else ligands
    for l in ligs:
        g = D.ligand_outputs(h, l, lib.atom_off, lib.rot_off, params)
        assert g["status"] == 0, (l, g["status"])
        parity.check_ligand(grid, O.ligand_from_library(lib, l), quats, params, g, stats)
    print(f"[parity {label}] {stats}", flush=True)
    parity.report(label, stats)
    return stats


def test_config1_full_parity(D, ctx):
    pk, lib, q, s = synth.config(1)
    print("[case] config 1, 8 ligands", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, **s)
    check_all(D, pk, lib, q, h, params, label="c1")


def test_ragged_sizes_and_slots(D, ctx):
    # sizes spanning every LDS bin and slot count, with ragged wave tails
    n = [1, 2, 5, 20, 33, 64, 65, 100, 128, 129, 150, 193, 256]
    b = [0, 0, 1, 3, 5, 8, 4, 12, 16, 10, 20, 24, 30]
    lib = synth.library_from_sizes(301, n, b)
    pk = synth.pocket_gaussians(301, 4, 48, 0.5, 60, 6.0)
    q = synth.start_quats(301, 5)
    print("[case] ragged sizes", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=100, sweep_passes=2, align_steps=7,
                          top_k=8, dedup_rmsd=1.0)
    check_all(D, pk, lib, q, h, params, label="ragged")


def test_alignment_chunks_and_restart_groups(D, ctx):
    # A = 40 splits the 40 y rotations of a lane strip into two parts (32 + 8),
    # each padded to whole waves: 11 restarts per alignment group, so 34
    # restarts leave a one-restart tail group
    lib = synth.library_uniform(305, 4, (10, 60), (1, 5))
    pk = synth.pocket_gaussians(305, 4, 48, 0.5, 60, 6.0)
    q = synth.start_quats(305, 34)
    print("[case] A=40, R=34", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=32, sweep_passes=1, align_steps=40,
                          top_k=4, dedup_rmsd=1.0)
    check_all(D, pk, lib, q, h, params, label="A40")


def test_alignment_three_parts_and_lane_chunks(D, ctx):
    # A = 70: three parts of the y range (32 + 32 + 6), 4 restarts per group
    # (9 restarts: groups of 4, 4, 1); A = 100: four parts and one restart per
    # group, 512 strips
    lib = synth.library_uniform(307, 3, (12, 70), (1, 4))
    pk = synth.pocket_gaussians(307, 4, 48, 0.5, 60, 6.0)
    for A, R in ((70, 9), (100, 3)):
        q = synth.start_quats(307, R)
        print(f"[case] A={A}, R={R}", flush=True)
        h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=16, sweep_passes=1,
                              align_steps=A, top_k=3, dedup_rmsd=1.0)
        check_all(D, pk, lib, q, h, params, label=f"A{A}")


def test_selection_without_lds_room(D, ctx):
    # top-64 of 70 restarts on 240-256-atom ligands: the candidate and kept poses
    # do not fit the final workgroup's LDS, so selection takes the single-wave
    # path over global memory
    n = [240, 256]
    lib = synth.library_from_sizes(306, n, [6, 10])
    pk = synth.pocket_gaussians(306, 4, 48, 0.5, 60, 6.0)
    q = synth.start_quats(306, 70)
    print("[case] K=64 on 256-atom ligands", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=16, sweep_passes=1, align_steps=5,
                          top_k=64, dedup_rmsd=0.5)
    check_all(D, pk, lib, q, h, params, label="K64")


@pytest.mark.parametrize("T", [1, 10, 64, 65, 1024])
def test_torsion_step_counts(D, ctx, T):
    lib = synth.library_uniform(310 + T, 6, (12, 40), (1, 6))
    pk = synth.pocket_gaussians(310, 4, 32, 0.5, 40, 4.0)
    q = synth.start_quats(310, 4)
    print(f"[case] T={T}", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=T, sweep_passes=2, align_steps=12,
                          top_k=4, dedup_rmsd=0.5)
    check_all(D, pk, lib, q, h, params, label=f"T{T}")


@pytest.mark.parametrize("variant", [
    dict(bump_min_bonds=3), dict(bump_min_bonds=5, bump_dist=2.4), dict(dedup_rmsd=0.0),
    dict(final_align=0), dict(top_k=12, dedup_rmsd=3.0), dict(sweep_passes=0)])
def test_search_variants(D, ctx, variant):
    lib = synth.library_uniform(320, 5, (15, 45), (2, 7))
    pk = synth.pocket_gaussians(320, 4, 32, 0.5, 40, 4.0)
    q = synth.start_quats(320, 10)
    kw = dict(torsion_steps=64, sweep_passes=2, align_steps=10, top_k=6, dedup_rmsd=1.5)
    kw.update(variant)
    print(f"[case] variant {variant}", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, **kw)
    check_all(D, pk, lib, q, h, params, label=str(variant))


def _corrupt(lib):
    """Copy of lib with ligand 1 given a bad type, 2 a bad mask, 3 a bad bond index."""
    L = synth.Library(**{k: (getattr(lib, k).copy() if isinstance(getattr(lib, k), np.ndarray)
                             else getattr(lib, k)) for k in (
        "atom_off", "xyz", "type", "bond_off", "bonds", "rot_off", "rot_bond", "rot_mask",
        "mask_words")})
    L.type[L.atom_off[1]] = 9
    r2 = L.rot_off[2]
    L.rot_mask[r2, 0] ^= np.uint64(1) << np.uint64(int(L.rot_bond[r2, 0]))
    L.bonds[L.bond_off[3], 1] = 500
    return L


def test_invalid_ligands_are_flagged_and_others_unaffected(D, ctx):
    lib = synth.library_uniform(330, 6, (15, 30), (2, 4))
    pk = synth.pocket_gaussians(330, 4, 32, 0.5, 40, 4.0)
    q = synth.start_quats(330, 4)
    bad = _corrupt(lib)
    print("[case] invalid ligands", flush=True)
    h, params = run_batch(D, ctx, pk, bad, q, torsion_steps=32, sweep_passes=1, align_steps=6,
                          top_k=4)
    assert list(h["status"]) == [0, 2, 4, 3, 0, 0]
    for l in (1, 2, 3):
        assert h["n_poses"][l] == 0 and h["best_score"][l] == -np.inf
    check_all(D, pk, bad, q, h, params, ligands=[0, 4, 5], label="valid-in-bad-batch")
    # the oracle rejects the same three ligands
    for l in (1, 2, 3):
        assert O.check_ligand(O.Grid.of(pk), O.ligand_from_library(bad, l)) != 0


def test_empty_library(D, ctx):
    lib = synth.library_from_sizes(340, np.zeros(0, np.int32), np.zeros(0, np.int32),
                                   mask_words=1)
    pk = synth.pocket_gaussians(340, 4, 16, 0.5, 5, 2.0)
    q = synth.start_quats(340, 3)
    h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=16, top_k=2)
    assert h["best_score"].size == 0


def test_restarts_fewer_than_top_k_and_rigid_only(D, ctx):
    lib = synth.library_from_sizes(350, [9, 30, 17], [0, 0, 0])
    pk = synth.pocket_gaussians(350, 4, 32, 0.5, 40, 4.0)
    q = synth.start_quats(350, 3)
    h, params = run_batch(D, ctx, pk, lib, q, torsion_steps=16, top_k=8, dedup_rmsd=0.0)
    assert list(h["n_poses"]) == [3, 3, 3]
    check_all(D, pk, lib, q, h, params, label="rigid")


def test_submit_poll_matches_device_batch_and_is_deterministic(D, ctx):
    pk, lib, q, s = synth.config(1)
    h1, params = run_batch(D, ctx, pk, lib, q, **s)
    h2, _ = run_batch(D, ctx, pk, lib, q, **s)
    for k in h1:
        if h1[k] is not None:
            np.testing.assert_array_equal(h1[k], h2[k], err_msg=k)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    hr = D.HostResults(lib.n_ligands, int(lib.atom_off[-1]), int(lib.rot_off[-1]), params,
                       restart_scores=True, trace=True, final_trace=True)
    t = D.dock_submit(ctx, pid, lib, params, hr)
    D.dock_wait(ctx, t)
    with pytest.raises(D.DockError):
        D.dock_poll(ctx, t)
    h3 = hr.to_host()
    for k in h1:
        if h1[k] is not None:
            np.testing.assert_array_equal(h1[k], h3[k], err_msg=k)
    D.dock_pocket_unload(ctx, pid)


def test_config2_full_size_sampled(D, ctx):
    """Full paper-scale workload (10,000 ligands, 96^3 x 4 pocket, R=T=256, P=3,
    K=30) in the benchmark's launch configuration; sampled ligands checked
    against the oracle, properties checked on every ligand."""
    pk, lib, q, s = synth.config(2)
    print("[case] config 2 full size", flush=True)
    h, params = run_batch(D, ctx, pk, lib, q, **s)
    L = lib.n_ligands
    assert np.all(h["status"] == 0)
    assert np.all(h["n_poses"] >= 1)
    K = params.top_k
    ps = h["pose_score"].reshape(L, K)
    assert np.all(h["best_score"] == ps[:, 0])
    for l in range(L):
        npz = h["n_poses"][l]
        assert np.all(np.diff(ps[l, :npz]) <= 0)
    # every output pose keeps the input bond lengths (rigid moves + torsions only)
    worst = 0.0
    for l in range(0, L, 7):
        x, t, b, r, m = lib.ligand(l)
        g = D.ligand_outputs(h, l, lib.atom_off, lib.rot_off, params)
        d0 = np.linalg.norm(x[b[:, 0]] - x[b[:, 1]], axis=1)
        d1 = np.linalg.norm(g["pose_xyz"][:, b[:, 0]] - g["pose_xyz"][:, b[:, 1]], axis=-1)
        worst = max(worst, float(np.abs(d1 - d0).max(initial=0)))
    assert worst < 1e-3, worst
    rng = np.random.default_rng(2209)
    sample = sorted(int(v) for v in rng.choice(L, 3, replace=False))
    check_all(D, pk, lib, q, h, params, ligands=sample, label="c2-sample")


def test_config3_full_size_sampled(D, ctx):
    """The large batched workload at full size (200,000 ligands, 20-100 heavy
    atoms, 0-20 rotatable bonds, 96^3 x 4 pocket, R=T=256, P=3, K=30) in the
    benchmark's launch configuration (batched form, tiles from the autotuner on
    the benchmark's size-stratified 4,096-ligand sample): properties on every
    ligand, sampled ligands against the oracle in follow mode.  The oracle's
    follow mode scores every candidate on every atom and tests every pair, so
    the sample is drawn among the ligands of at most 40 atoms and 6 bonds (large
    ligands meet the oracle in the stratified config-3 case at 32 restarts)."""
    import bench
    pk, lib, q, s = synth.config(3)
    print("[case] config 3 full size", flush=True)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    params = D.SearchParams(q, **s)
    order = bench.stratified_order(lib, 2209)
    tsub = lib.subset(sorted(order[:4096]))
    D.dock_autotune(ctx, pid, D.DeviceLibrary(tsub), params, torch.cuda.current_stream())
    dl = D.DeviceLibrary(lib)
    res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params,
                          restart_scores=True, trace=True, final_trace=True)
    D.dock_ligands_batch(ctx, pid, dl, params, res)
    torch.cuda.synchronize()
    h = res.to_host()
    D.dock_pocket_unload(ctx, pid)
    del res, dl
    L, K = lib.n_ligands, params.top_k
    assert np.all(h["status"] == 0)
    npz = h["n_poses"]
    assert np.all((npz >= 1) & (npz <= K))
    ps = h["pose_score"].reshape(L, K)
    assert np.all(h["best_score"] == ps[:, 0])
    # scores of the kept poses in descending order, every ligand at once
    valid = np.arange(1, K)[None, :] < npz[:, None]
    with np.errstate(invalid="ignore"):  # unused slots hold no score
        assert np.all(np.where(valid, np.diff(ps, axis=1) <= 0, True))
    # bond lengths kept (rigid moves and torsions only) on a seeded sample
    rng = np.random.default_rng(2209)
    worst = 0.0
    for l in sorted(int(v) for v in rng.choice(L, 2000, replace=False)):
        x, t, b, r, m = lib.ligand(l)
        g = D.ligand_outputs(h, l, lib.atom_off, lib.rot_off, params)
        d0 = np.linalg.norm(x[b[:, 0]] - x[b[:, 1]], axis=1)
        d1 = np.linalg.norm(g["pose_xyz"][:, b[:, 0]] - g["pose_xyz"][:, b[:, 1]], axis=-1)
        worst = max(worst, float(np.abs(d1 - d0).max(initial=0)))
    assert worst < 1e-3, worst
    small = np.flatnonzero((lib.n_atoms() <= 40) & (lib.n_rot() <= 6))
    sample = sorted(int(v) for v in rng.choice(small, 3, replace=False))
    check_all(D, pk, lib, q, h, params, ligands=sample, label="c3-full-sample")


def test_plain_form_matches_batched_form_bitwise(D, ctx):
    """The plain (latency) form makes the same decisions with the same arithmetic
    as the batched form; its outputs must be identical, and pass parity."""
    for label, (pk, lib, q, s) in (
            ("c1", synth.config(1)),
            ("ragged", (synth.pocket_gaussians(302, 4, 48, 0.5, 60, 6.0),
                        synth.library_from_sizes(302, [3, 20, 33, 64, 65, 100, 150, 256],
                                                 [0, 3, 5, 8, 4, 12, 20, 24]),
                        synth.start_quats(302, 6),
                        dict(torsion_steps=100, sweep_passes=2, align_steps=7, top_k=8,
                             dedup_rmsd=1.0)))):
        print(f"[case] plain vs batched {label}", flush=True)
        hb, params = run_batch(D, ctx, pk, lib, q, **s)
        hp, pparams = run_batch(D, ctx, pk, lib, q, mode=D.DOCK_MODE_PLAIN, **s)
        for k in hb:
            if hb[k] is not None:
                np.testing.assert_array_equal(hb[k], hp[k], err_msg=f"{label}:{k}")
        check_all(D, pk, lib, q, hp, pparams, label=f"plain-{label}")


def test_scored_sample_count(D, ctx):
    """The torsion samples the kernels report as scored (bump-free candidates x
    moving atoms) agree between the batched and plain forms (same decisions) and
    lie between zero and the all-candidates count."""
    pk, lib, q, s = synth.config(1)
    counts = {}
    for label, mode in (("batched", D.DOCK_MODE_BATCHED), ("plain", D.DOCK_MODE_PLAIN)):
        D.dock_set_timing(ctx, True)
        D.dock_get_timing(ctx)
        run_batch(D, ctx, pk, lib, q, mode=mode, **s)
        tm = D.dock_get_timing(ctx)
        D.dock_set_timing(ctx, False)
        counts[label] = tm["scored_samples"]
    m = [bin(int(w)).count("1") for w in lib.rot_mask.reshape(-1)]
    all_cand = s["restarts"] * s["sweep_passes"] * s["torsion_steps"] * sum(m)
    print(f"[scored] {counts} of {all_cand}", flush=True)
    assert counts["batched"] == counts["plain"]
    assert 0 < counts["batched"] < all_cand


def test_plain_form_matches_batched_form_bitwise_paper_scale(D, ctx):
    """On the paper-scale pocket (where the batched alignment reads most samples
    from the LDS shell bands of the pocket's atlas and the plain form reads every
    sample from global memory), both forms return identical outputs."""
    pk, lib, q, s = synth.config(2, n_ligands=150)
    print("[case] plain vs batched, config 2 pocket, 150 ligands", flush=True)
    hb, params = run_batch(D, ctx, pk, lib, q, **s)
    hp, _ = run_batch(D, ctx, pk, lib, q, mode=D.DOCK_MODE_PLAIN, **s)
    for k in hb:
        if hb[k] is not None:
            np.testing.assert_array_equal(hb[k], hp[k], err_msg=f"c2:{k}")


def test_plain_form_flags_invalid_ligands(D, ctx):
    lib = synth.library_uniform(331, 6, (15, 30), (2, 4))
    pk = synth.pocket_gaussians(331, 4, 32, 0.5, 40, 4.0)
    q = synth.start_quats(331, 4)
    bad = _corrupt(lib)
    h, params = run_batch(D, ctx, pk, bad, q, torsion_steps=32, sweep_passes=1, align_steps=6,
                          top_k=4, mode=D.DOCK_MODE_PLAIN)
    assert list(h["status"]) == [0, 2, 4, 3, 0, 0]
    check_all(D, pk, bad, q, h, params, ligands=[0, 4, 5], label="plain-valid-in-bad-batch")


def test_graph_replays_match_eager(D, ctx):
    """Repeated identical calls are captured as a graph and replayed; every replay,
    with other eager work and synchronisations between replays, must equal the
    first (eager) result bit for bit."""
    pk, lib, q, s = synth.config(1)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    params = D.SearchParams(q, **s)
    dl = D.DeviceLibrary(lib)
    res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params,
                          restart_scores=True, trace=True, final_trace=True)
    other = synth.library_uniform(360, 5, (15, 40), (1, 5))
    do = D.DeviceLibrary(other)
    ro = D.DeviceResults(other.n_ligands, do.n_atoms_total, do.n_rot_total, params)
    st = torch.cuda.Stream()
    D.dock_ligands_batch(ctx, pid, dl, params, res, st)        # first call: eager
    st.synchronize()
    eager = res.to_host()
    for rep in range(4):                                        # capture, then replays
        with torch.cuda.stream(st):
            for t in (res.best_score, res.pose_score, res.pose_xyz, res.restart_score):
                t.fill_(float("nan"))
        D.dock_ligands_batch(ctx, pid, dl, params, res, st)
        st.synchronize()
        got = res.to_host()
        for k in eager:
            if eager[k] is not None:
                np.testing.assert_array_equal(eager[k], got[k], err_msg=f"replay {rep}: {k}")
        D.dock_ligands_batch(ctx, pid, do, params, ro)          # other eager work between
        torch.cuda.synchronize()
    D.dock_pocket_unload(ctx, pid)


def test_production_parameters_every_slot_count(D, ctx):
    """The paper-scale search (A = 30, T = 256, P = 3, K = 30) on the 96^3 x 4
    pocket, with 32 restarts (one whole alignment group), on ligands that take
    every slot count of the kernels: 30 atoms (one 64-lane slot), 75 and 100
    (two), 140 (three) and 200 (four), with 12 to 30 rotatable bonds; both forms
    against the oracle."""
    c2 = synth.CONFIGS[2]
    pk = synth.pocket_gaussians(synth.MASTER_SEED + 2, **c2["pocket"])
    lib = synth.library_from_sizes(308, [30, 75, 100, 140, 200], [12, 20, 20, 30, 30])
    q = synth.start_quats(synth.MASTER_SEED + 2, 32)
    s = dict(c2["search"], restarts=32)
    for mode, label in ((D.DOCK_MODE_BATCHED, "batched"), (D.DOCK_MODE_PLAIN, "plain")):
        print(f"[case] production parameters, slots 1..4, {label}", flush=True)
        h, params = run_batch(D, ctx, pk, lib, q, mode=mode, **s)
        check_all(D, pk, lib, q, h, params, label=f"production-{label}")


def test_no_pruning_ablation_selects_the_same_steps(D, ctx):
    """bump_prune = 0 tests every eligible pair against every candidate and scores
    every candidate, applying the bump verdict afterwards: the decisions and all
    outputs are bit-identical to the pruned path, in both forms, and pass the
    oracle; the kernels report every candidate as scored."""
    pk = synth.pocket_gaussians(309, 4, 48, 0.5, 60, 6.0)
    lib = synth.library_from_sizes(309, [20, 45, 70, 130], [3, 8, 12, 20])
    q = synth.start_quats(309, 8)
    s = dict(torsion_steps=64, sweep_passes=2, align_steps=10, top_k=4, dedup_rmsd=1.0)
    for mode, label in ((D.DOCK_MODE_BATCHED, "batched"), (D.DOCK_MODE_PLAIN, "plain")):
        print(f"[case] no-pruning ablation, {label}", flush=True)
        counts = {}
        out = {}
        for prune in (1, 0):
            D.dock_set_timing(ctx, True)
            D.dock_get_timing(ctx)
            out[prune], params = run_batch(D, ctx, pk, lib, q, mode=mode, bump_prune=prune, **s)
            counts[prune] = D.dock_get_timing(ctx)["scored_samples"]
            D.dock_set_timing(ctx, False)
        for k in out[1]:
            if out[1][k] is not None:
                np.testing.assert_array_equal(out[1][k], out[0][k], err_msg=f"{label}:{k}")
        m = [bin(int(w)).count("1") for w in lib.rot_mask.reshape(-1)]
        all_cand = q.shape[0] * s["sweep_passes"] * s["torsion_steps"] * sum(m)
        print(f"[scored] {label} pruned {counts[1]}, unpruned {counts[0]} of {all_cand}", flush=True)
        assert counts[0] == all_cand and counts[1] < all_cand
        check_all(D, pk, lib, q, out[0], params, label=f"no-pruning-{label}")


def test_submit_admission_budget(D):
    """A context with a device-memory budget admits a request that fits, refuses a
    second one while the first holds its memory (DOCK_EAGAIN, nothing enqueued),
    and admits it once the first has retired; both results equal the
    device-resident batch."""
    pk, lib, q, s = synth.config(1)
    params = D.SearchParams(q, **s)
    need = D.dock_request_bytes(lib, params, D.HostResults(
        lib.n_ligands, int(lib.atom_off[-1]), int(lib.rot_off[-1]), params))
    print(f"[case] admission budget, request needs {need} B", flush=True)
    ref_ctx = D.dock_create(0)
    try:
        ref, _ = run_batch(D, ref_ctx, pk, lib, q, **s)
    finally:
        D.dock_destroy(ref_ctx)
    c = D.dock_create(0, hbm_budget_bytes=need + need // 2)
    try:
        pid = D.dock_pocket_load(c, pk.values, pk.spacing, pk.origin)
        mk = lambda: D.HostResults(lib.n_ligands, int(lib.atom_off[-1]), int(lib.rot_off[-1]),
                                   params)
        ra, rb = mk(), mk()
        ta = D.dock_submit(c, pid, lib, params, ra)
        with pytest.raises(D.DockError) as ei:
            D.dock_submit(c, pid, lib, params, rb)
        assert ei.value.code == D.DOCK_EAGAIN
        D.dock_wait(c, ta)
        tb = D.dock_submit(c, pid, lib, params, rb)
        D.dock_wait(c, tb)
        for r in (ra, rb):
            h = r.to_host()
            for k in ("best_score", "n_poses", "status", "pose_score", "pose_restart", "pose_xyz"):
                np.testing.assert_array_equal(h[k], ref[k], err_msg=k)
        D.dock_pocket_unload(c, pid)
        tiny = D.dock_create(0, hbm_budget_bytes=1)
        try:
            pid2 = D.dock_pocket_load(tiny, pk.values, pk.spacing, pk.origin)
            with pytest.raises(D.DockError) as ei:
                D.dock_submit(tiny, pid2, lib, params, mk())
            assert ei.value.code == D.DOCK_EAGAIN
        finally:
            D.dock_destroy(tiny)
    finally:
        D.dock_destroy(c)


def test_serving_loop_maps_results_to_requests(D, ctx):
    """The serving loop (per-pocket buckets over dock_submit/dock_poll) returns,
    for every request, the best score the device-resident batch gives for the
    same ligand and pocket."""
    from paper_2209_05069_amd import serve as S
    pockets = [synth.pocket_gaussians(370 + p, 4, 32, 0.5, 40, 4.0) for p in range(3)]
    lib = synth.library_uniform(370, 40, (12, 40), (0, 6))
    q = synth.start_quats(370, 8)
    s = dict(torsion_steps=32, sweep_passes=1, align_steps=10, top_k=4, dedup_rmsd=1.0)
    params = D.SearchParams(q, **s)
    pids = {p: D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
            for p, pk in enumerate(pockets)}
    rng = np.random.default_rng(370)
    reqs = [S.Request(i, int(rng.integers(0, 3)), int(rng.integers(0, lib.n_ligands)), 0.0)
            for i in range(120)]
    servers = []
    for kw in (dict(max_batch=16, flush_ms=2.0),                       # size/age buckets
               dict(max_batch=16, max_inflight=2),                     # work-conserving
               dict(max_batch=16, max_inflight=3, return_poses=True)):
        print(f"[case] serving loop, 120 requests over 3 pockets, {kw}", flush=True)
        for rq in reqs:
            rq.t_arrival = 0.0
        srv = S.Server(ctx, pids, lib, params, **kw)
        r = S.run(srv, reqs, S.poisson_arrivals(2000.0, len(reqs), 370), time_limit_s=60.0)
        assert r["completed"] == len(reqs)
        servers.append(srv)
    for p in range(3):
        D.dock_pocket_unload(ctx, pids[p])
    for p, pk in enumerate(pockets):
        h, _ = run_batch(D, ctx, pk, lib, q, **s)
        for req in reqs:
            if req.pocket == p:
                for srv in servers:
                    assert srv.results[req.rid] == h["best_score"][req.ligand], req


def test_autotune_reports_every_bin_and_keeps_results(D, ctx):
    """The per-bin tile choice changes only launch shapes: results stay bitwise
    equal to the default tiles, for the tuned table and for a forced one."""
    pk, lib, q, s = synth.config(2, n_ligands=400)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    params = D.SearchParams(q, **s)
    dl = D.DeviceLibrary(lib)
    print(f"[case] autotune, {lib.n_ligands} paper-scale ligands", flush=True)

    def run():
        res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params,
                              restart_scores=True, trace=True, final_trace=True)
        D.dock_ligands_batch(ctx, pid, dl, params, res)
        torch.cuda.synchronize()
        return res.to_host()

    D.dock_set_tuning(ctx, params, None)
    h0 = run()
    table = D.dock_autotune(ctx, pid, dl, params)
    print(f"[tuning] {table}", flush=True)
    expect = np.bincount((lib.n_atoms() - 1) // 32, minlength=8)
    assert [t["ligands"] for t in table] == list(expect)
    for t in table:
        if t["ligands"] == 0:
            continue
        assert t["dock_waves"] in (2, 4, 8) and t["select_waves"] in (4, 8, 16)
        assert t["falign_waves"] in (2, 4, 8) and t["falign_per_cu"] in (0, 1, 2, 4)
        assert t["falign_xcd"] in (0, 1)
        for k in ("dock", "select", "falign"):
            assert 0 < t[f"{k}_ms"] <= t[f"{k}_ms_default"]
    h1 = run()
    forced = [dict(t, dock_waves=8, select_waves=16, falign_waves=2, falign_per_cu=1,
                   falign_xcd=1 - t["falign_xcd"])
              if t["ligands"] else t for t in table]
    D.dock_set_tuning(ctx, params, forced)
    h2 = run()
    D.dock_set_tuning(ctx, params, None)
    for h in (h1, h2):
        for k, a in h0.items():
            assert np.array_equal(a, h[k]), k
    D.dock_pocket_unload(ctx, pid)


def _contacts_case(D, ctx, pk, lib, q, s, seed, label):
    """Dock with contact scores in both forms; every output pose's GPU score must
    equal the FP64 oracle's on the same pose, up to the weight of pairs within
    1e-4 A of the contact distance; the forms and the submit path agree bitwise."""
    pa = synth.pocket_atoms(seed, pk)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    D.dock_pocket_set_atoms(ctx, pid, pa.xyz, pa.type, pa.ntypes, pa.weight, pa.contact_dist)
    dl = D.DeviceLibrary(lib)
    outs = {}
    for mode in (D.DOCK_MODE_BATCHED, D.DOCK_MODE_PLAIN):
        params = D.SearchParams(q, mode=mode, **s)
        res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params,
                              contacts=True)
        D.dock_ligands_batch(ctx, pid, dl, params, res)
        torch.cuda.synchronize()
        outs[mode] = res.to_host()
    params = D.SearchParams(q, **s)
    hr = D.HostResults(lib.n_ligands, int(lib.atom_off[-1]), int(lib.rot_off[-1]), params,
                       contacts=True)
    D.dock_wait(ctx, D.dock_submit(ctx, pid, lib, params, hr))
    h = outs[D.DOCK_MODE_BATCHED]
    for k in ("pose_contacts", "pose_xyz", "n_poses"):
        assert np.array_equal(h[k], outs[D.DOCK_MODE_PLAIN][k]), k
        assert np.array_equal(h[k], hr.to_host()[k]), k
    opa = O.PocketAtoms.of(pa)
    poses = exact = edge = 0
    for l in range(lib.n_ligands):
        g = D.ligand_outputs(h, l, lib.atom_off, lib.rot_off, params)
        types = lib.type[lib.atom_off[l]:lib.atom_off[l + 1]]
        assert (g["pose_contacts"][g["n_poses"]:] == 0).all()
        for sidx in range(g["n_poses"]):
            v, b = O.contacts(opa, types, g["pose_xyz"][sidx].astype(np.float64), tol=1e-4)
            got = int(g["pose_contacts"][sidx])
            assert abs(got - v) <= b, (l, sidx, got, v, b)
            poses += 1
            exact += got == v
            edge += b > 0
    print(f"[contacts {label}] poses {poses}, exact {exact}, with boundary pairs {edge}, "
          f"{len(pa.type)} pocket atoms, nonzero {(h['pose_contacts'] != 0).sum()}", flush=True)
    assert poses > 0 and (h["pose_contacts"] != 0).any()
    D.dock_pocket_unload(ctx, pid)


def test_pose_contacts_config1(D, ctx):
    pk, lib, q, s = synth.config(1)
    print("[case] contact rescoring, config 1", flush=True)
    _contacts_case(D, ctx, pk, lib, q, s, 11, "c1")


def test_pose_contacts_paper_scale_and_ragged(D, ctx):
    pk, lib, q, s = synth.config(2, n_ligands=40)
    print("[case] contact rescoring, paper-scale pocket, 40 ligands, restarts 0-31", flush=True)
    _contacts_case(D, ctx, pk, lib, q[:32], dict(s, restarts=32), 12, "c2")
    n = [1, 2, 20, 64, 65, 129, 200, 256]
    b = [0, 0, 3, 8, 4, 10, 20, 30]
    rl = synth.library_from_sizes(313, n, b)
    rq = synth.start_quats(313, 6)
    print("[case] contact rescoring, ragged sizes", flush=True)
    _contacts_case(D, ctx, pk, rl, rq, dict(torsion_steps=32, sweep_passes=1, align_steps=7,
                                            top_k=5, dedup_rmsd=1.0), 13, "ragged")


def test_paper_buckets_give_the_same_results(D, ctx):
    """Work lists per (size bin, group of 4 rotatable bonds), as the paper's batched
    form buckets ligands, change only the launch order: results are bitwise equal
    to the size-bin lists, including ligands in the last bond group (28+)."""
    pk, lib, q, s = synth.config(3, n_ligands=300)
    s = dict(s, restarts=32)
    print("[case] paper buckets vs size bins, 300 ligands of the large batched mix", flush=True)
    h0, _ = run_batch(D, ctx, pk, lib, q[:32], **s)
    h1, _ = run_batch(D, ctx, pk, lib, q[:32], bin_mode=1, **s)
    for k, a in h0.items():
        assert np.array_equal(a, h1[k]), k
    n = [1, 2, 5, 20, 33, 64, 65, 100, 128, 129, 150, 193, 256]
    b = [0, 0, 1, 3, 5, 8, 4, 12, 16, 10, 20, 24, 30]
    rl = synth.library_from_sizes(301, n, b)
    rq = synth.start_quats(301, 5)
    kw = dict(torsion_steps=100, sweep_passes=2, align_steps=7, top_k=8, dedup_rmsd=1.0)
    print("[case] paper buckets vs size bins, ragged sizes", flush=True)
    h0, _ = run_batch(D, ctx, pk, rl, rq, **kw)
    h1, params = run_batch(D, ctx, pk, rl, rq, bin_mode=1, **kw)
    for k, a in h0.items():
        assert np.array_equal(a, h1[k]), k
    check_all(D, pk, rl, rq, h1, params, label="paper-buckets-ragged")
