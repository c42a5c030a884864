"""Host-side logic of bench.py (no GPU): the roofline's byte counter is reported
only for the kernel source and workload it was measured on, the sample counts
behind the achieved rate, and the one-GPU guard."""
import os
import subprocess
import sys

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
    s = dict(synth.CONFIGS[2]["search"])
    L = synth.CONFIGS[2]["ligands"]["L"]
    expect = bench.TRAFFIC_BYTES_PER_STEP if _source_sha() == bench.TRAFFIC_SOURCE_SHA else None
    assert bench.kernel_traffic(2, L, s) == expect
    # any other search, library size or config: no byte figure
    assert bench.kernel_traffic(2, L, dict(s, torsion_steps=10)) is None
    assert bench.kernel_traffic(2, L - 1, s) is None
    assert bench.kernel_traffic(3, synth.CONFIGS[3]["ligands"]["L"],
                                dict(synth.CONFIGS[3]["search"])) is None


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
