"""Properties of the seeded input generators (inputs only: no docking here)."""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components, shortest_path

import synth


def test_library_is_valid_clash_free_and_deterministic():
    lib = synth.library_uniform(123, 40, (12, 90), (0, 12))
    lib2 = synth.library_uniform(123, 40, (12, 90), (0, 12))
    for k in ("atom_off", "xyz", "type", "bonds", "rot_bond", "rot_mask"):
        np.testing.assert_array_equal(getattr(lib, k), getattr(lib2, k))
    assert lib.type.max() < 4
    for l in range(lib.n_ligands):
        x, t, b, r, m = lib.ligand(l)
        n = len(x)
        assert len(b) == n - 1                                   # a tree
        A = coo_matrix((np.ones(len(b)), (b[:, 0], b[:, 1])), shape=(n, n))
        assert connected_components(A, directed=False)[0] == 1
        D = shortest_path(A, directed=False, unweighted=True)
        d = np.linalg.norm(x[:, None] - x[None], axis=-1)
        assert np.all(d[D >= 4] >= 2.0)                           # clash-free input
        bl = d[b[:, 0], b[:, 1]]
        assert np.all((bl > 1.449) & (bl < 1.551))
        assert np.all(np.bincount(b.ravel(), minlength=n) <= 4)   # valence <= 4
        for i, (a, bb) in enumerate(r):
            mov = np.array([(int(m[i, j >> 6]) >> (j & 63)) & 1 for j in range(n)], bool)
            assert mov[bb] and not mov[a]
            # moving set = atoms b reaches once a-b is cut
            keep = ~(((b[:, 0] == a) & (b[:, 1] == bb)) | ((b[:, 0] == bb) & (b[:, 1] == a)))
            Ac = coo_matrix((np.ones(keep.sum()), (b[keep, 0], b[keep, 1])), shape=(n, n))
            lab = connected_components(Ac, directed=False)[1]
            np.testing.assert_array_equal(mov, lab == lab[bb])
            assert not mov[0]                                      # away from the root
        assert np.all(np.diff(r[:, 1]) > 0) if len(r) > 1 else True


def test_sizes_follow_the_requested_ranges():
    lib = synth.library_uniform(7, 2000, (20, 80), (2, 12))
    n = lib.n_atoms()
    assert n.min() == 20 and n.max() == 80
    req = lib.n_rot_requested
    assert req.min() == 2 and req.max() == 12
    assert np.all(lib.n_rot() <= req)
    assert np.mean(lib.n_rot() < req) < 0.05


def test_pocket_values_are_gaussian_sums():
    pk = synth.pocket_gaussians(5, 2, 10, 0.5, 6, 2.0)
    g = pk.gaussians
    o = pk.origin[0]
    rng = np.random.default_rng(0)
    for _ in range(30):
        t = int(rng.integers(0, 2))
        i, j, k = rng.integers(0, 10, 3)
        p = np.array([o + 0.5 * i, o + 0.5 * j, o + 0.5 * k])
        v = sum(a * np.exp(-np.sum((p - c) ** 2) / (2 * s * s))
                for c, s, a in zip(g[t, :, :3], g[t, :, 3], g[t, :, 4]))
        assert abs(float(pk.values[t, k, j, i]) - v) <= 1e-6 * max(1, abs(v))
    assert np.all(np.abs(g[:, :, :3]) <= 2.0)


def test_subset_keeps_ligands():
    lib = synth.library_uniform(9, 10, (10, 30), (1, 4))
    sub = lib.subset([3, 7])
    for a, b in ((0, 3), (1, 7)):
        for u, v in zip(sub.ligand(a), lib.ligand(b)):
            np.testing.assert_array_equal(u, v)
