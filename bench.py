"""Throughput benchmark of the docking hot path on one MI355X.

Workload (default): the paper-scale synthetic library -- 10,000 random-tree
ligands with U{20..80} heavy atoms and U{2..12} rotatable bonds, a 4-type
96^3 pocket at 0.375 A (160 Gaussians per type), 256 restarts, 256 torsion
steps, 3 sweep passes, 30x30 alignment, top-30 poses with 2 A dedup.
A step docks the whole library (every stage of the hot path) with inputs
already resident in device memory.

Prints one JSON line.  `value` is ligands docked per second.  The roofline
object covers the dominant kernel (the per-restart docking kernels), timed live
with HIP events on the stream they run on; `cpu_baseline` times the FP64
oracle, single-threaded, on a bounded sample of the same library.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations per atom sample (one atom placed and scored):
# rigid transform 18 (3x3 matrix-vector + translation), grid coordinates 6,
# cell fractions 3, trilinear blend 21 (7 lerps x 3), accumulate 1.
FLOP_PER_SAMPLE = 49
PEAK_FP32_TFLOPS = 157.3   # MI355X fp32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--ligands", type=int, default=None, help="truncate the library")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="time budget of the oracle CPU baseline (0: skip)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="run one plain device copy of this size first (reference kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def workload_counts(lib, s):
    """Algorithmic work of one step: atom samples of the docking kernels,
    torsion evaluations and rigid (orientation) evaluations."""
    n = lib.n_atoms().astype(np.int64)
    B = lib.n_rot().astype(np.int64)
    R, T, Pp, A = s["restarts"], s["torsion_steps"], s["sweep_passes"], s["align_steps"]
    # moving atoms per rotatable bond
    m = np.array([bin(int(w)).count("1") for w in lib.rot_mask.reshape(-1)], np.int64)
    m = m.reshape(len(lib.rot_bond), -1).sum(1) if len(lib.rot_bond) else np.zeros(0, np.int64)
    lig_of_rot = np.repeat(np.arange(len(n)), B)
    moving_per_lig = np.bincount(lig_of_rot, weights=m, minlength=len(n)).astype(np.int64)
    samples = int(R * (A * A * n.sum() + Pp * T * moving_per_lig.sum() + n.sum()))
    torsion_evals = int(R * Pp * T * B.sum())
    return samples, torsion_evals


def cpu_baseline(pk, lib, q, s, budget_s):
    """The FP64 oracle as it stands, single-threaded, on ligands of the same
    library taken in a seeded random order until the budget is spent."""
    from oracle import oracle as O
    grid = O.Grid.of(pk)
    rng = np.random.default_rng(2209)
    order = rng.permutation(lib.n_ligands)
    kw = {k: v for k, v in s.items() if k != "restarts"}
    done = 0
    t0 = time.perf_counter()
    for l in order:
        O.dock_ligand(grid, O.ligand_from_library(lib, int(l)), q, **kw)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return dict(value=done / el, unit="ligands/s", cores=1, kind="oracle",
                sample=f"{done} ligands of the same library (seeded random order), "
                       f"FP64 single thread, {el:.1f} s")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); docking shards into "
              "independent ligands, so N GPUs would each run this on their own shard.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2209_05069_amd import dock as D

    t0 = time.time()
    pk, lib, q, s = synth.config(a.config, n_ligands=a.ligands)
    print(f"[bench] workload ready in {time.time() - t0:.1f}s: {lib.n_ligands} ligands, "
          f"{int(lib.atom_off[-1])} atoms, {int(lib.rot_off[-1])} rotatable bonds",
          file=sys.stderr, flush=True)
    ctx = D.dock_create(0)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    params = D.SearchParams(q, **s)
    dl = D.DeviceLibrary(lib)
    res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params)
    stream = torch.cuda.current_stream()
    if a.copy_ref_mib > 0:
        nel = a.copy_ref_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(a.warmup):
        D.dock_ligands_batch(ctx, pid, dl, params, res, stream)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    assert bool((res.status == 0).all()), "some ligands were rejected"

    D.dock_set_timing(ctx, True)
    D.dock_get_timing(ctx)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    step_ms = []
    e0.record(stream)
    for k in range(a.steps):
        es = torch.cuda.Event(enable_timing=True)
        ee = torch.cuda.Event(enable_timing=True)
        es.record(stream)
        D.dock_ligands_batch(ctx, pid, dl, params, res, stream)
        ee.record(stream)
        step_ms.append((es, ee))
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    per_step = [x.elapsed_time(y) for x, y in step_ms]
    tm = D.dock_get_timing(ctx)
    D.dock_set_timing(ctx, False)
    print(f"[bench] timed {a.steps} steps: {total_ms:.1f} ms; phases {tm}", file=sys.stderr,
          flush=True)

    L = lib.n_ligands
    ms = total_ms / a.steps
    samples, tors = workload_counts(lib, s)
    dock_ms = tm["dock_ms"] / max(1, tm["calls"])
    achieved = samples * FLOP_PER_SAMPLE / (dock_ms * 1e-3) / 1e12
    rigid = int(s["restarts"] * L * s["align_steps"] ** 2 +
                int(res.n_poses.sum().item()) * s["align_steps"] ** 2)
    out = {
        "metric": "ligands docked/s + torsion evals/s on 1 MI355X; p50/p99 ligand latency",
        "value": L / (ms * 1e-3),
        "unit": "ligands/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"paper-scale plain workload (config {a.config}): {L} random-tree ligands "
                         f"(heavy atoms U{{20..80}}, rotatable bonds U{{2..12}}), 4-type 96^3 "
                         f"pocket at 0.375 A; R={s['restarts']} restarts, T={s['torsion_steps']} "
                         f"torsion steps, P={s['sweep_passes']} passes, 30x30 alignment, "
                         f"top-{s['top_k']} with {s['dedup_rmsd']} A dedup"),
            "form": "batched (persistent wavefront-per-restart kernels, size-binned)",
            "ligands": L,
        },
        "torsion_evals_per_s": tors / (ms * 1e-3),
        "rigid_evals_per_s": rigid / (ms * 1e-3),
        "latency_ms": {"p50": float(np.percentile(per_step, 50)),
                       "p99": float(np.percentile(per_step, 99)),
                       "note": "batched form: every ligand of a step completes with the step"},
        "phases_ms": {k: tm[k] / max(1, tm["calls"]) for k in ("prep_ms", "dock_ms", "final_ms")},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None,
            "kernel": "k_dock (all size bins of one step)",
            "flop_per_step": samples * FLOP_PER_SAMPLE,
            "atom_samples_per_step": samples,
            "dock_ms_per_step": dock_ms,
        },
    }
    D.dock_destroy(ctx)
    if a.cpu_seconds > 0:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pk, lib, q, s, a.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
