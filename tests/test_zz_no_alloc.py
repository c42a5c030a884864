"""dock_ligands_batch_noalloc (tables and workspace in the library's fixed
scratch array) against dock_ligands_batch, through the C ABI.

Both entry points run the same kernels on the same tables, so their outputs are
compared element by element for equality (stricter than the oracle tolerances);
the second, smaller call is also checked against the FP64 oracle in follow
mode.  Two calls in a row on one stream, the second with a smaller input,
exercise the scratch array keeping the first call's contents.
"""
import numpy as np
import pytest

import synth
from tests.test_gpu_parity import D, check_all  # noqa: F401 (fixture)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nctx(D):
    c = D.dock_create(0)
    yield c
    D.dock_destroy(c)


def _results(D, dl, params, trace):
    res = D.DeviceResults(dl.n_ligands, dl.n_atoms_total, dl.n_rot_total, params,
                          restart_scores=True, trace=trace, final_trace=True)
    for k in ("best_score", "n_poses", "status", "pose_score", "pose_restart", "pose_xyz",
              "restart_score", "trace", "final_trace"):
        t = getattr(res, k)
        if t is not None:
            t.fill_(0)
    return res


def _both(D, ctx, pid, lib, q, trace, **kw):
    params = D.SearchParams(q, **kw)
    dl = D.DeviceLibrary(lib)
    ref = _results(D, dl, params, trace)
    got = _results(D, dl, params, trace)
    D.dock_ligands_batch(ctx, pid, dl, params, ref)
    D.dock_ligands_batch_noalloc(ctx, pid, dl, params, got)
    torch.cuda.synchronize()
    return ref.to_host(), got.to_host(), params


def _assert_equal(ref, got):
    for k, a in ref.items():
        if a is None:
            assert got[k] is None, k
            continue
        assert a.dtype == got[k].dtype and a.shape == got[k].shape, k
        assert np.array_equal(a, got[k]), (k, np.flatnonzero(a != got[k])[:8])


def test_noalloc_matches_batch_two_calls_second_smaller(D, nctx):
    # call 1: 300 ligands of the paper-scale library at its full search
    pk2, lib2, q2, s2 = synth.config(2, n_ligands=300)
    pid2 = D.dock_pocket_load(nctx, pk2.values, pk2.spacing, pk2.origin)
    print(f"[case] noalloc call 1: {lib2.n_ligands} ligands, R={len(q2)}, "
          f"T={s2['torsion_steps']}", flush=True)
    ref, got, _ = _both(D, nctx, pid2, lib2, q2, trace=True, **s2)
    assert (got["status"] == 0).all()
    _assert_equal(ref, got)
    # call 2, smaller: 3 small ligands on another pocket, internal trace in scratch
    pk1, lib1, q1, s1 = synth.config(1, n_ligands=3)
    pid1 = D.dock_pocket_load(nctx, pk1.values, pk1.spacing, pk1.origin)
    print(f"[case] noalloc call 2: {lib1.n_ligands} ligands, R={len(q1)}", flush=True)
    ref, got, params = _both(D, nctx, pid1, lib1, q1, trace=False, **s1)
    _assert_equal(ref, got)
    # and the same small request with its trace, against the FP64 oracle
    ref, got, params = _both(D, nctx, pid1, lib1, q1, trace=True, **s1)
    _assert_equal(ref, got)
    check_all(D, pk1, lib1, q1, got, params, label="noalloc-c1")
    D.dock_pocket_unload(nctx, pid1)
    D.dock_pocket_unload(nctx, pid2)


def test_noalloc_rejects_oversize_and_plain_requests(D, nctx):
    pk, lib, q, s = synth.config(2, n_ligands=4000)
    pid = D.dock_pocket_load(nctx, pk.values, pk.spacing, pk.origin)
    params = D.SearchParams(q, **s)
    dl = D.DeviceLibrary(lib)
    res = D.DeviceResults(dl.n_ligands, dl.n_atoms_total, dl.n_rot_total, params)
    print(f"[case] noalloc oversize: {lib.n_ligands} ligands, {dl.n_atoms_total} atoms",
          flush=True)
    with pytest.raises(D.DockError) as e:
        D.dock_ligands_batch_noalloc(nctx, pid, dl, params, res)
    assert e.value.code == D.DOCK_EINVAL and "DOCK_NOALLOC_SCRATCH_BYTES" in str(e.value)
    plain = D.SearchParams(q, **dict(s, mode=D.DOCK_MODE_PLAIN))
    with pytest.raises(D.DockError) as e:
        D.dock_ligands_batch_noalloc(nctx, pid, dl, plain, res)
    assert e.value.code == D.DOCK_EINVAL and "batched" in str(e.value)
    # a request that fits still runs after the refusals
    sub = lib.subset(list(range(50)))
    ref, got, _ = _both(D, nctx, pid, sub, q, trace=False, **s)
    _assert_equal(ref, got)
    D.dock_pocket_unload(nctx, pid)
