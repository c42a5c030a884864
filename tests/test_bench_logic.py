"""Host-side logic of bench.py (no GPU): the roofline's byte counter is reported
only for the kernel source and workload it was measured on, the sample counts
behind the achieved rate, and the one-GPU guard."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def _source_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_2209_05069_amd", "csrc", "dock_device.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def test_traffic_only_for_the_measured_source_and_workload():
    s3 = dict(synth.CONFIGS[3]["search"])
    L3 = synth.CONFIGS[3]["ligands"]["L"]
    saved = dict(bench.TRAFFIC)
    try:
        bench.TRAFFIC.clear()
        bench.TRAFFIC[(3, 256, L3)] = ("k_dock", _source_sha(), 1.0e11)
        assert bench.kernel_traffic(3, L3, s3, "k_dock") == 1.0e11
        # another kernel, search, library size, config or kernel source: no byte figure
        assert bench.kernel_traffic(3, L3, s3, "k_align") is None
        assert bench.kernel_traffic(3, L3, dict(s3, torsion_steps=10), "k_dock") is None
        assert bench.kernel_traffic(3, L3 - 1, s3, "k_dock") is None
        assert bench.kernel_traffic(2, synth.CONFIGS[2]["ligands"]["L"],
                                    dict(synth.CONFIGS[2]["search"]), "k_dock") is None
        bench.TRAFFIC[(3, 256, L3)] = ("k_dock", "0" * 16, 1.0e11)
        assert bench.kernel_traffic(3, L3, s3, "k_dock") is None
    finally:
        bench.TRAFFIC.clear()
        bench.TRAFFIC.update(saved)


def test_stratified_order_is_a_permutation_taking_cells_in_turn():
    lib = synth.library_uniform(11, 400, (20, 100), (0, 20))
    order = bench.stratified_order(lib, 2209)
    assert sorted(order) == list(range(lib.n_ligands))
    assert order == bench.stratified_order(lib, 2209)
    # the first 8 ligands come from 8 different (atom quartile, bond half) cells
    n, B = lib.n_atoms(), lib.n_rot()
    qa = np.quantile(n, [0.25, 0.5, 0.75])
    cell = np.searchsorted(qa, n, side="right") * 2 + (B > np.median(B))
    assert len(set(cell[order[:8]])) == 8


def test_workload_counts_small_library():
    # rigid: R*(A^2 + 1)*n per ligand (alignment plus the pose score); torsion
    # evaluations R*P*T per rotatable bond; the atom samples behind them move
    # between 1 and n-1 atoms per bond
    pk, lib, q, s = synth.config(1)
    rigid, tors_all, evals = bench.workload_counts(lib, s)
    n = (lib.atom_off[1:] - lib.atom_off[:-1]).astype(int)
    B = (lib.rot_off[1:] - lib.rot_off[:-1]).astype(int)
    R, P, T, A = s["restarts"], s["sweep_passes"], s["torsion_steps"], s["align_steps"]
    assert rigid == R * (A * A + 1) * int(n.sum())
    assert evals == R * P * T * int(B.sum())
    assert R * P * T * int(B.sum()) <= tors_all <= R * P * T * int((B * (n - 1)).sum())


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_valu_instructions_only_for_the_measured_source_and_workload():
    s3 = dict(synth.CONFIGS[3]["search"])
    L3 = synth.CONFIGS[3]["ligands"]["L"]
    saved = dict(bench.VALU_INSTR)
    try:
        bench.VALU_INSTR.clear()
        bench.VALU_INSTR[(3, 256, L3)] = (_source_sha(), 2.0e12)
        assert bench.step_valu_instr(3, L3, s3) == 2.0e12
        assert bench.step_valu_instr(3, L3, dict(s3, restarts=128)) is None
        assert bench.step_valu_instr(3, L3 - 1, s3) is None
        bench.VALU_INSTR[(3, 256, L3)] = ("0" * 16, 2.0e12)
        assert bench.step_valu_instr(3, L3, s3) is None
    finally:
        bench.VALU_INSTR.clear()
        bench.VALU_INSTR.update(saved)


def test_counter_figures_match_the_committed_profile():
    """The byte and VALU-instruction counts bench.py reports for the large batched
    workload are the ones of the committed rocprofv3 summary, taken on the kernel
    source that summary names."""
    import re
    text = open(os.path.join(ROOT, "profiles",
                             "k_align_k_dock_c3_trace_counters_bytes.md")).read()
    sha = re.search(r"Kernel source sha256 prefix:\s*`([0-9a-f]{16})`", text).group(1)
    nbytes = float(re.search(r"k_align \(the dominant kernel\): ([0-9.e+]+) bytes per step",
                             text).group(1))
    valu = float(re.search(r"roofline of the whole step: ([0-9.e+]+) VALU wave-instructions",
                           text).group(1))
    L3 = synth.CONFIGS[3]["ligands"]["L"]
    kernel, tsha, tbytes = bench.TRAFFIC[(3, 256, L3)]
    vsha, vcount = bench.VALU_INSTR[(3, 256, L3)]
    assert kernel == "k_align"
    assert tsha == sha and vsha == sha
    assert tbytes == pytest.approx(nbytes, rel=1e-4)
    assert vcount == pytest.approx(valu, rel=1e-4)
