"""Throughput benchmark of the docking hot path on one MI355X.

Workload (default): the large batched library -- 200,000 random-tree ligands
with U{20..100} heavy atoms and U{0..20} rotatable bonds (clipped to what the
tree allows), a 4-type 96^3 pocket at 0.375 A (160 Gaussians per type), 256
restarts, 256 torsion steps, 3 sweep passes, 30x30 alignment, top-30 poses
with 2 A dedup.  A step docks the whole library (every stage of the hot path)
with inputs already resident in device memory.

Prints one JSON line.  `value` is ligands docked per second.  The roofline
object covers the dominant kernel (the alignment or the torsion-sweep kernels
of a step, whichever takes longer), timed live with HIP events on the stream
they run on; `cpu_baseline` times the FP64 oracle, single-threaded, on a
bounded sample of the same library stratified by size.  The plain per-ligand
form is timed on a stratified sample of the same library for the
batched/plain factor, and one ligand at a time for its per-ligand latency.
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
PEAK_FP32_TFLOPS = 157.3   # MI355X fp32 vector peak (256 CU x 2.4 GHz x 256 flop/clk, packed)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # one wave64 FMA per CU per clock (packed FP32 not used)

# HBM bytes of the dominant kernel per step, from two rocprofv3 --pmc runs
# (FETCH_SIZE and WRITE_SIZE, scaled by the factors a plain 256 MiB device copy
# read in the same program).  Valid only for the kernel source they were taken
# on (sha256 prefix) and the workload they were taken on: reported as null
# otherwise.  Key: (config, torsion steps, ligands) -> (kernel, source sha, bytes).
TRAFFIC = {
    # large batched workload, T=256: rocprofv3 FETCH_SIZE / WRITE_SIZE of k_align (all bins),
    # one step, scaled by the 256 MiB reference copy (factors 2.0 and 1.0)
    (3, 256, 200000): ("k_align", "a5b39e79a4970aea", 9.2916e+11),
}

# VALU wave-instructions per step of all docking kernels (rocprofv3 SQ_INSTS_VALU, one
# step), for the VALU-instruction roofline: one wave64 VALU instruction per CU per
# clock, 256 CUs at 2.4 GHz.  Same validity rule as TRAFFIC: (source sha, instructions).
VALU_INSTR = {
    (3, 256, 200000): ("a5b39e79a4970aea", 3.2905e+12),
}
VALU_ROOF_PER_S = 256 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--ligands", type=int, default=None, help="truncate the library")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="time budget of the oracle CPU baseline (0: skip)")
    ap.add_argument("--plain-ligands", type=int, default=512,
                    help="ligands of the stratified sample timed in the plain per-ligand form "
                         "(0: skip)")
    ap.add_argument("--latency-ligands", type=int, default=32,
                    help="ligands docked one per call in the plain form for its per-ligand "
                         "latency (0: skip)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tiles (no per-bin autotuning before the timed steps)")
    ap.add_argument("--save-tuning", type=str, default=None,
                    help="write the autotuned table (with device and search settings) to this "
                         "JSON file")
    ap.add_argument("--tuning-file", type=str, default=None,
                    help="use the table in this JSON file (written by --save-tuning on the same "
                         "device and search settings) instead of autotuning")
    ap.add_argument("--tune-ligands", type=int, default=4096,
                    help="ligands of the size-stratified sample the per-bin autotuner times on")
    ap.add_argument("--graph-steps", type=int, default=2,
                    help="steps replayed from the captured hipGraph after the timed region "
                         "(phase timing off, on a stream of its own), reported as graph_replay (0: skip)")
    ap.add_argument("--bin-mode", type=int, default=0, choices=(0, 1),
                    help="work lists of the batched form: 0 = size bins of 32 heavy atoms, "
                         "1 = the paper's buckets (size bin x group of 4 rotatable bonds)")
    ap.add_argument("--no-prune", action="store_true",
                    help="the no-early-exit ablation: no bump-check pruning (bump_prune=0)")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving workload (8 pockets, Poisson requests) instead")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-loads", type=str, default="0.5,0.8,0.9",
                    help="offered load as fractions of the measured batched saturation")
    ap.add_argument("--serve-max-inflight", type=int, default=4,
                    help="serving: batches in flight at most (work-conserving policy); 0 = "
                         "submit a pocket's bucket when full or after --serve-flush-ms")
    ap.add_argument("--serve-max-batch", type=int, default=4096)
    ap.add_argument("--serve-flush-ms", type=float, default=50.0)
    ap.add_argument("--sweep", action="store_true",
                    help="size grid and library-size sweep, plain vs batched (config 4)")
    ap.add_argument("--sweep-ligands", type=int, default=20000,
                    help="ligands per size-grid cell (batched form)")
    ap.add_argument("--sweep-plain-ligands", type=int, default=2000,
                    help="ligands per size-grid cell timed in the plain form")
    ap.add_argument("--sweep-library", type=str, default="100,1000,10000,100000,1000000")
    ap.add_argument("--torsion-steps", type=int, default=None,
                    help="override T (e.g. 10: the paper's 36-degree torsion steps)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="run one plain device copy of this size first (reference kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def source_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_2209_05069_amd", "csrc", "dock_device.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def kernel_traffic(cfg, L, s, kernel):
    """Measured HBM bytes per step of `kernel`, or None unless they were taken on
    this kernel source, this workload recipe, its full library and its search."""
    import synth
    t = TRAFFIC.get((cfg, s["torsion_steps"], L))
    if (t is None or t[0] != kernel or t[1] != source_sha()
            or s != synth.CONFIGS[cfg]["search"] or L != synth.CONFIGS[cfg]["ligands"]["L"]):
        return None
    return t[2]


def step_valu_instr(cfg, L, s):
    """Measured VALU wave-instructions per step, or None unless they were taken on
    this kernel source, this workload recipe, its full library and its search."""
    import synth
    t = VALU_INSTR.get((cfg, s["torsion_steps"], L))
    if (t is None or t[0] != source_sha() or s != synth.CONFIGS[cfg]["search"]
            or L != synth.CONFIGS[cfg]["ligands"]["L"]):
        return None
    return t[1]


def stratified_order(lib, seed):
    """All ligand indices, ordered so that every prefix takes the (heavy-atom
    quartile, rotatable-bond half) cells in turn, each cell in a seeded random
    order: a prefix is a size-stratified sample of the library."""
    n, B = lib.n_atoms(), lib.n_rot()
    rng = np.random.default_rng(seed)
    qa = np.quantile(n, [0.25, 0.5, 0.75])
    cell = np.searchsorted(qa, n, side="right") * 2 + (B > np.median(B))
    lists = [list(rng.permutation(np.flatnonzero(cell == c))) for c in range(8)]
    out = []
    while any(lists):
        for li in lists:
            if li:
                out.append(int(li.pop()))
    return out


def describe(cfg, L, s):
    import synth
    c = synth.CONFIGS[cfg]
    pk, lg = c["pocket"], c["ligands"]
    names = {1: "small plain workload", 2: "paper-scale plain workload",
             3: "large batched workload"}
    return (f"{names.get(cfg, 'workload')} (config {cfg}): {L} random-tree ligands (heavy atoms "
            f"U{{{lg['atoms'][0]}..{lg['atoms'][1]}}}, rotatable bonds U{{{lg['rot'][0]}.."
            f"{lg['rot'][1]}}}), {pk['ntypes']}-type {pk['n']}^3 pocket at {pk['spacing']} A; "
            f"R={s['restarts']} restarts, T={s['torsion_steps']} torsion steps, "
            f"P={s['sweep_passes']} passes, {s['align_steps']}x{s['align_steps']} alignment, "
            f"top-{s['top_k']} with {s['dedup_rmsd']} A dedup")


def workload_counts(lib, s):
    """Work of one step fixed by the library and the search: atom samples of the
    rigid steps of the docking kernels (alignment of every restart plus its
    final pose score), torsion atom samples if every candidate were scored, and
    torsion evaluations (candidates, counted independently of the bump check)."""
    n = lib.n_atoms().astype(np.int64)
    B = lib.n_rot().astype(np.int64)
    R, T, Pp, A = s["restarts"], s["torsion_steps"], s["sweep_passes"], s["align_steps"]
    # moving atoms per rotatable bond
    m = (np.unpackbits(np.ascontiguousarray(lib.rot_mask).view(np.uint8), axis=None)
         .reshape(len(lib.rot_bond), -1).sum(1).astype(np.int64)
         if len(lib.rot_bond) else np.zeros(0, np.int64))
    lig_of_rot = np.repeat(np.arange(len(n)), B)
    moving_per_lig = np.bincount(lig_of_rot, weights=m, minlength=len(n)).astype(np.int64)
    rigid_samples = int(R * (A * A * n.sum() + n.sum()))
    torsion_all = int(R * Pp * T * moving_per_lig.sum())
    torsion_evals = int(R * Pp * T * B.sum())
    return rigid_samples, torsion_all, torsion_evals


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pk, lib, q, s, budget_s):
    """The FP64 oracle as it stands, on ligands of the same library taken in a
    size-stratified seeded order (stratified_order) until the budget is spent:
    single-threaded (the reported value), then one ligand per thread over the
    host cores given to this job (at most 16; the oracle's C calls release the
    GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    grid = O.Grid.of(pk)
    order = stratified_order(lib, 2209)
    kw = {k: v for k, v in s.items() if k != "restarts"}

    def one(l):
        O.dock_ligand(grid, O.ligand_from_library(lib, l), q, **kw)

    done = 0
    t0 = time.perf_counter()
    for l in order:
        one(l)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    out = dict(value=done / el, unit="ligands/s", cores=1, kind="oracle",
               sample=f"{done} ligands of the same library (stratified by heavy-atom quartile "
                      f"and rotatable-bond half, seeded), full search, FP64 single thread, "
                      f"{el:.1f} s",
               cpu_model=_cpu_model())
    nthr = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                      else (os.cpu_count() or 1)))
    if nthr > 1:
        # as many ligands per thread as the single thread finished in the budget
        sub = order[:done * nthr]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(one, sub))
        el2 = time.perf_counter() - t0
        out["all_cores"] = dict(value=len(sub) / el2, unit="ligands/s", cores=nthr,
                                sample=f"{len(sub)} ligands, one per thread at a time, "
                                       f"{el2:.1f} s")
    return out


def serve_main(a):
    """Serving workload: 8 device-resident pockets (4 types x 96^3 each), a
    Poisson stream of single-ligand requests (each naming a pocket uniformly),
    heavy atoms lognormal (median 40, sigma_log 0.5, clipped 12..150), rotatable
    bonds Poisson(6) clipped 0..30, R=T=256, P=3, K=30.  Offered loads are
    fractions of the batched saturation throughput measured first on the same
    ligand mix."""
    import torch
    import synth
    from paper_2209_05069_amd import dock as D
    from paper_2209_05069_amd import serve as S
    seed = synth.MASTER_SEED + 5
    t0 = time.time()
    pockets = [synth.pocket_gaussians(seed + 100 * p, 4, 96, 0.375, 160, 9.0) for p in range(8)]
    s = dict(synth.CONFIGS[2]["search"])
    q = synth.start_quats(seed, s["restarts"])
    ctx = D.dock_create(0)
    pids = {p: D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
            for p, pk in enumerate(pockets)}
    params = D.SearchParams(q, **s)
    # saturation on this mix: one big device-resident batch (tiles tuned on it first)
    sat_lib = synth.library_lognormal(seed, 6000)
    dl = D.DeviceLibrary(sat_lib)
    tuning = D.dock_autotune(ctx, pids[0], dl, params)
    res = D.DeviceResults(sat_lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params)
    D.dock_ligands_batch(ctx, pids[0], dl, params, res)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    D.dock_ligands_batch(ctx, pids[0], dl, params, res)
    e1.record()
    torch.cuda.synchronize()
    sat = sat_lib.n_ligands / (e0.elapsed_time(e1) * 1e-3)
    print(f"[serve] setup {time.time() - t0:.1f}s, batched saturation {sat:.0f} ligands/s",
          file=sys.stderr, flush=True)
    runs = []
    for load in [float(x) for x in a.serve_loads.split(",")]:
        qps = load * sat
        n = min(int(qps * a.serve_seconds), 2_000_000)
        lib = synth.library_lognormal(seed + 7, n)
        rng = np.random.default_rng(seed + int(1000 * load))
        reqs = [S.Request(i, int(rng.integers(0, 8)), i, 0.0) for i in range(n)]
        arr = S.poisson_arrivals(qps, n, seed + int(1000 * load))
        srv = S.Server(ctx, pids, lib, params, max_batch=a.serve_max_batch,
                       flush_ms=a.serve_flush_ms, max_inflight=a.serve_max_inflight)
        r = S.run(srv, reqs, arr)
        r.update(load=load, offered_qps=qps)
        runs.append(r)
        print(f"[serve] load {load}: {r}", file=sys.stderr, flush=True)
    D.dock_destroy(ctx)
    main_run = runs[-1]
    out = {
        "metric": "ligands docked/s + torsion evals/s on 1 MI355X; p50/p99 ligand latency",
        "value": main_run["ligands_per_s"], "unit": "ligands/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: 8 device-resident 4x96^3 pockets, Poisson requests "
                               "(one ligand each, pocket U{0..7}), heavy atoms lognormal(40, 0.5) "
                               "clipped 12..150, rotatable bonds Poisson(6) clipped 0..30, "
                               "R=T=256, P=3, K=30; buckets per pocket; " +
                               (f"work-conserving: at most {a.serve_max_inflight} batches in "
                                f"flight, oldest bucket first, up to {a.serve_max_batch} ligands"
                                if a.serve_max_inflight > 0 else
                                f"flush at {a.serve_max_batch} ligands or {a.serve_flush_ms} ms")},
        "tuning": {f"atoms {32 * b + 1}-{32 * (b + 1)}": t for b, t in enumerate(tuning)
                   if t["ligands"] > 0},
        "latency_ms": {"p50": main_run["p50_ms"], "p99": main_run["p99_ms"]},
        "batched_saturation_ligands_per_s": sat,
        "runs": runs,
    }
    print(json.dumps(out), flush=True)


def _time_call(D, torch, ctx, pid, lib, params, reps=1):
    dl = D.DeviceLibrary(lib)
    res = D.DeviceResults(lib.n_ligands, dl.n_atoms_total, dl.n_rot_total, params)
    D.dock_ligands_batch(ctx, pid, dl, params, res)      # warm (workspace, tables)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        D.dock_ligands_batch(ctx, pid, dl, params, res)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del dl, res
    return lib.n_ligands / (ms * 1e-3)


def sweep_main(a):
    """Size grid (heavy atoms {16,32,64,128} x rotatable bonds {0,4,8,16,24}) and
    library-size sweep (40 atoms / 8 bonds), plain vs batched, R=128 restarts,
    T=256 steps, P=3, K=30, on the paper-scale pocket.  The plain form is timed on
    the first --sweep-plain-ligands ligands of each library (its throughput does
    not depend on library size beyond a few launches per stream)."""
    import torch
    import synth
    from paper_2209_05069_amd import dock as D
    seed = synth.MASTER_SEED + 4
    c2 = synth.CONFIGS[2]
    pk = synth.pocket_gaussians(seed, **c2["pocket"])
    s = dict(c2["search"])
    s["restarts"] = 128
    q = synth.start_quats(seed, 128)
    ctx = D.dock_create(0)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    if a.no_prune:
        s["bump_prune"] = 0
    pb = D.SearchParams(q, **s)
    pp = D.SearchParams(q, mode=D.DOCK_MODE_PLAIN, **s)
    cells = []
    for n in (16, 32, 64, 128):
        for B in (0, 4, 8, 16, 24):
            if B > max(n - 3, 0):
                cells.append(dict(atoms=n, bonds=B, feasible=False))
                print(f"[sweep] {n} atoms x {B} bonds: infeasible (a tree of {n} atoms has at "
                      f"most {n - 3} non-terminal edges)", file=sys.stderr, flush=True)
                continue
            L = a.sweep_ligands
            lib = synth.library_from_sizes(seed + 1000 * n + B, np.full(L, n, np.int32),
                                           np.full(L, B, np.int32))
            clipped = int((lib.n_rot() < B).sum())
            bat = _time_call(D, torch, ctx, pid, lib, pb)
            sub = lib.subset(range(min(L, a.sweep_plain_ligands)))
            pla = _time_call(D, torch, ctx, pid, sub, pp)
            cells.append(dict(atoms=n, bonds=B, feasible=True, ligands=L, clipped=clipped,
                              batched_ligands_per_s=bat, plain_ligands_per_s=pla,
                              batched_over_plain=bat / pla))
            print(f"[sweep] {n} atoms x {B} bonds: batched {bat:.0f}/s, plain {pla:.0f}/s, "
                  f"x{bat / pla:.2f} (clipped {clipped})", file=sys.stderr, flush=True)
    lib_runs = []
    sizes = [int(x) for x in a.sweep_library.split(",")]
    big = synth.library_from_sizes(seed + 7, np.full(max(sizes), 40, np.int32),
                                   np.full(max(sizes), 8, np.int32))
    for L in sizes:
        lib = big.subset(range(L)) if L < big.n_ligands else big
        bat = _time_call(D, torch, ctx, pid, lib, pb)
        pla = _time_call(D, torch, ctx, pid, lib.subset(range(min(L, a.sweep_plain_ligands))), pp)
        lib_runs.append(dict(ligands=L, batched_ligands_per_s=bat, plain_ligands_per_s=pla))
        print(f"[sweep] library {L}: batched {bat:.0f}/s, plain {pla:.0f}/s", file=sys.stderr,
              flush=True)
    D.dock_destroy(ctx)
    print(json.dumps({"sweep": "size grid and library size (config 4)", "search": s,
                      "cells": cells, "library": lib_runs}), flush=True)


def _events(torch, stream):
    e = torch.cuda.Event(enable_timing=True)
    e.record(stream)
    return e


def plain_form(D, torch, ctx, pid, lib, q, s, order, n_sample, n_latency, stream):
    """The plain per-ligand form on a size-stratified sample of the library (the
    first n_sample of `order`): ligands/s over one call, and per-ligand latency
    from n_latency of them docked one per call (each alone on the GPU)."""
    pparams = D.SearchParams(q, mode=D.DOCK_MODE_PLAIN, **s)
    sub = lib.subset(order[:n_sample])
    dsl = D.DeviceLibrary(sub)
    rsl = D.DeviceResults(sub.n_ligands, dsl.n_atoms_total, dsl.n_rot_total, pparams)
    warm = lib.subset(order[:8])
    dw = D.DeviceLibrary(warm)
    rw = D.DeviceResults(warm.n_ligands, dw.n_atoms_total, dw.n_rot_total, pparams)
    D.dock_ligands_batch(ctx, pid, dw, pparams, rw, stream)
    torch.cuda.synchronize()
    p0 = _events(torch, stream)
    D.dock_ligands_batch(ctx, pid, dsl, pparams, rsl, stream)
    p1 = _events(torch, stream)
    torch.cuda.synchronize()
    pms = p0.elapsed_time(p1)
    out = {"ligands_per_s": sub.n_ligands / (pms * 1e-3), "sample_ligands": sub.n_ligands,
           "sample": "size-stratified (heavy-atom quartile x rotatable-bond half), seeded",
           "ms": pms,
           "form": "one ligand per launch sequence (checks, R restart workgroups, selection, "
                   "one workgroup per kept pose for the final alignment, outputs), "
                   "ligands round-robin over 4 streams"}
    if n_latency > 0:
        lat = []
        for l in order[:n_latency]:
            one = lib.subset([l])
            d1 = D.DeviceLibrary(one)
            r1 = D.DeviceResults(1, d1.n_atoms_total, d1.n_rot_total, pparams)
            torch.cuda.synchronize()
            a = _events(torch, stream)
            D.dock_ligands_batch(ctx, pid, d1, pparams, r1, stream)
            b = _events(torch, stream)
            torch.cuda.synchronize()
            lat.append(a.elapsed_time(b))
        out["latency_ms"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "ligands": len(lat),
                             "note": "one ligand per call, alone on the GPU, from its first "
                                     "kernel to its results"}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); docking shards into "
              "independent ligands, so N GPUs would each run this on their own shard.",
              file=sys.stderr)
        sys.exit(2)
    if a.serve:
        return serve_main(a)
    if a.sweep:
        return sweep_main(a)
    import torch
    import synth
    from paper_2209_05069_amd import dock as D

    t0 = time.time()
    pk, lib, q, s = synth.config(a.config, n_ligands=a.ligands)
    if a.torsion_steps is not None:
        s = dict(s, torsion_steps=a.torsion_steps)
    print(f"[bench] workload ready in {time.time() - t0:.1f}s: {lib.n_ligands} ligands, "
          f"{int(lib.atom_off[-1])} atoms, {int(lib.rot_off[-1])} rotatable bonds",
          file=sys.stderr, flush=True)
    ctx = D.dock_create(0)
    pid = D.dock_pocket_load(ctx, pk.values, pk.spacing, pk.origin)
    prune = 0 if a.no_prune else 1
    params = D.SearchParams(q, bump_prune=prune, bin_mode=a.bin_mode, **s)
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
    order = stratified_order(lib, 2209)
    tuning = None
    tune_key = {"device": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
                "search": {k: s[k] for k in ("restarts", "torsion_steps", "align_steps", "top_k",
                                             "sweep_passes")}}
    if a.tuning_file:
        saved = json.load(open(a.tuning_file))
        if {k: saved.get(k) for k in tune_key} != tune_key:
            raise SystemExit(f"{a.tuning_file} was tuned for {saved.get('device')} "
                             f"{saved.get('search')}, not {tune_key}")
        D.dock_set_tuning(ctx, params, saved["table"])
        tuning = {"from_file": a.tuning_file,
                  "bins": {f"atoms {32 * b + 1}-{32 * (b + 1)}": t
                           for b, t in enumerate(saved["table"]) if t["ligands"] > 0}}
    elif not a.no_tune:
        t1 = time.time()
        tsub = lib.subset(sorted(order[:min(a.tune_ligands, lib.n_ligands)]))
        table = D.dock_autotune(ctx, pid, D.DeviceLibrary(tsub), params, stream)
        tuning = {"sample_ligands": tsub.n_ligands, "seconds": time.time() - t1,
                  "sample": "size-stratified (heavy-atom quartile x rotatable-bond half), seeded",
                  "bins": {f"atoms {32 * b + 1}-{32 * (b + 1)}": t
                           for b, t in enumerate(table) if t["ligands"] > 0}}
        print(f"[bench] autotuned in {tuning['seconds']:.1f}s: {tuning['bins']}",
              file=sys.stderr, flush=True)
        if a.save_tuning:
            with open(a.save_tuning, "w") as f:
                json.dump(dict(tune_key, table=table), f)
    for w in range(a.warmup):
        D.dock_ligands_batch(ctx, pid, dl, params, res, stream)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    assert bool((res.status == 0).all()), "some ligands were rejected"

    D.dock_set_timing(ctx, True)
    D.dock_get_timing(ctx)
    torch.cuda.synchronize()
    step_ms = []
    e0 = _events(torch, stream)
    for k in range(a.steps):
        es = _events(torch, stream)
        D.dock_ligands_batch(ctx, pid, dl, params, res, stream)
        step_ms.append((es, _events(torch, stream)))
    e1 = _events(torch, stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    per_step = [x.elapsed_time(y) for x, y in step_ms]
    tm = D.dock_get_timing(ctx)
    D.dock_set_timing(ctx, False)
    print(f"[bench] timed {a.steps} steps: {total_ms:.1f} ms; phases {tm}", file=sys.stderr,
          flush=True)
    graph_ms = None
    if a.graph_steps > 0:
        # without phase timing, a call repeated with the same arguments on the same
        # (non-null) stream is captured once as a hipGraph and replayed: the first of
        # these two calls runs eagerly, the second captures and launches the graph
        gs = torch.cuda.Stream()
        gs.wait_stream(stream)
        for _ in range(2):
            D.dock_ligands_batch(ctx, pid, dl, params, res, gs)
        torch.cuda.synchronize()
        g0 = _events(torch, gs)
        for _ in range(a.graph_steps):
            D.dock_ligands_batch(ctx, pid, dl, params, res, gs)
        g1 = _events(torch, gs)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / a.graph_steps
        print(f"[bench] {a.graph_steps} graph-replayed steps: {graph_ms:.1f} ms per step",
              file=sys.stderr, flush=True)

    L = lib.n_ligands
    ms = total_ms / a.steps
    rigid_samples, torsion_all, tors = workload_counts(lib, s)
    calls = max(1, tm["calls"])
    align_ms = tm["align_ms"] / calls
    torsion_ms = (tm["dock_ms"] - tm["align_ms"]) / calls
    # Algorithmic work per step.  Alignment (k_align): R * A^2 * n atom samples per
    # ligand.  Torsion sweep (k_dock): as in Alg. 1 a candidate that fails the bump
    # check is not scored, so only the scored torsion samples (counted by the
    # kernels) enter, plus the pose score of every restart (R * n).
    n_tot = int(lib.atom_off[-1])
    align_samples = s["restarts"] * s["align_steps"] ** 2 * n_tot
    scored = tm["scored_samples"] // calls
    if a.no_prune:
        scored = torsion_all  # every candidate is scored, as Alg. 1 scores the bump-free ones
    torsion_samples = scored + s["restarts"] * n_tot
    kernels = {
        "k_align": dict(ms_per_step=align_ms, atom_samples_per_step=align_samples,
                        achieved_tflops=align_samples * FLOP_PER_SAMPLE / (align_ms * 1e-3) / 1e12),
        "k_dock": dict(ms_per_step=torsion_ms, atom_samples_per_step=torsion_samples,
                       torsion_samples_scored=scored,
                       torsion_samples_all_candidates=torsion_all,
                       achieved_tflops=torsion_samples * FLOP_PER_SAMPLE / (torsion_ms * 1e-3) / 1e12),
    }
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    achieved = kd["achieved_tflops"]
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
            "workload": describe(a.config, L, s) + ("; no bump-check pruning (ablation)"
                                                    if a.no_prune else ""),
            "form": "batched (persistent wavefront-per-restart kernels, " +
                    ("work lists per size bin x group of 4 rotatable bonds)" if a.bin_mode
                     else "work lists per size bin)"),
            "ligands": L,
        },
        "torsion_evals_per_s": tors / (ms * 1e-3),
        "rigid_evals_per_s": rigid / (ms * 1e-3),
        "latency_ms": {"p50": float(np.percentile(per_step, 50)),
                       "p99": float(np.percentile(per_step, 99)),
                       "note": "batched form: every ligand of a step is submitted at its start "
                               "and completes with it, so a ligand's latency is the step's"},
        "phases_ms": {k: tm[k] / calls for k in ("prep_ms", "align_ms", "dock_ms", "final_ms")},
        "graph_replay": None if graph_ms is None else {
            "ms_per_step": graph_ms, "ligands_per_s": L / (graph_ms * 1e-3),
            "steps": a.graph_steps,
            "note": "the same step replayed from its captured hipGraph (phase timing off); the "
                    "timed steps above run eagerly because they record phase events"},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": kernel_traffic(a.config, L, s, dom),
            "traffic_unit": "bytes per step (dominant kernel, HBM side of L2)",
            "kernel": f"{dom} (all size bins of one step)",
            "flop_per_step": kd["atom_samples_per_step"] * FLOP_PER_SAMPLE,
            "peak_non_packed": PEAK_FP32_NONPACKED_TFLOPS,
            "frac_non_packed": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "kernels": kernels,
        },
    }
    vi = step_valu_instr(a.config, L, s) if not (a.no_prune or a.bin_mode) else None
    out["valu_roofline"] = None if vi is None else {
        "wave_instr_per_step": vi, "achieved_per_s": vi / (ms * 1e-3),
        "peak_per_s": VALU_ROOF_PER_S, "frac": vi / (ms * 1e-3) / VALU_ROOF_PER_S,
        "note": "VALU wave-instructions of every docking kernel per step (rocprofv3 "
                "SQ_INSTS_VALU on this kernel source and workload) over the live step time; "
                "roof = one wave64 VALU instruction per CU per clock (256 CUs, 2.4 GHz)"}
    out["tuning"] = tuning if tuning is not None else "default tiles (--no-tune)"
    if a.plain_ligands > 0:
        pf = plain_form(D, torch, ctx, pid, lib, q, dict(s, bump_prune=prune), order,
                        min(a.plain_ligands, L), min(a.latency_ligands, L), stream)
        pf["batched_over_plain"] = out["value"] / pf["ligands_per_s"]
        out["plain_form"] = pf
        print(f"[bench] plain form {pf['ligands_per_s']:.0f} ligands/s", file=sys.stderr,
              flush=True)
    D.dock_destroy(ctx)
    if a.cpu_seconds > 0:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pk, lib, q, s, a.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
