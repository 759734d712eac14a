"""Properties of the seeded input generators (shapes, compositions,
densities, minimum distances, float32 representability)."""
import numpy as np

from paper_2607_06969_amd import workloads as W


def _f32_exact(a):
    return np.array_equal(np.asarray(a, dtype=np.float64), np.asarray(a, dtype=np.float32).astype(np.float64))


def test_rocksalt_counts_and_layout():
    s = W.rocksalt_gst(16)
    assert s.n_atoms == 3686
    n_te = int((s.species == W.TE).sum())
    n_ge = int((s.species == W.GE).sum())
    n_sb = int((s.species == W.SB).sum())
    assert n_te == 2048 and n_ge == 819 and n_sb == 819
    assert abs(s.cells[0, 0, 0] - 48.0) < 1e-12
    assert _f32_exact(s.pos) and _f32_exact(s.cells)
    frac = s.pos / 48.0
    assert frac.min() >= 0.0 and frac.max() < 1.0
    assert s.n_atoms / 48.0 ** 3 > 0.033


def test_amorphous_batch_min_distance_and_composition():
    s = W.amorphous_batch(n_cfg=6, n_min=64, n_max=150, seed=3)
    sizes = np.diff(s.atom_off)
    assert np.all((sizes >= 64) & (sizes <= 150))
    for c in range(s.n_cfg):
        sub = s.config(c)
        L = sub.cells[0, 0, 0]
        d = sub.pos[:, None, :] - sub.pos[None, :, :]
        d -= L * np.round(d / L)
        r = np.sqrt((d ** 2).sum(-1)) + np.eye(sub.n_atoms) * 1e9
        assert r.min() >= 2.2 - 1e-5
        cnt = np.bincount(sub.species, minlength=3) / sub.n_atoms
        assert np.allclose(cnt, np.array([2, 2, 5]) / 9, atol=1.0 / sub.n_atoms + 1e-9)
        assert abs(sub.n_atoms / L ** 3 - 0.033) < 1e-3


def test_mixed_cells_sizes():
    s = W.mixed_size_cells(n_cells=8, seed=2)
    sizes = np.diff(s.atom_off)
    assert s.n_cfg == 8 and sizes.min() >= 800 and sizes.max() <= 250000


def test_maxwell_boltzmann_temperature_and_momentum():
    s = W.rocksalt_gst(20)
    v = W.maxwell_boltzmann(s.species, W.MASSES_GST, 300.0, seed=1)
    m = np.asarray(W.MASSES_GST)[s.species]
    p = (m[:, None] * v).sum(0)
    assert np.max(np.abs(p)) < 1e-3
    ek = 0.5 * (m[:, None] * v ** 2).sum() / W.ACC_UNIT
    T = 2 * ek / (3 * s.n_atoms * W.KB_EV)
    assert abs(T - 300.0) < 10.0


def test_generators_are_seeded():
    a, b = W.rocksalt_gst(8, seed=5), W.rocksalt_gst(8, seed=5)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.species, b.species)
    assert np.array_equal(W.random_params(W.hp_gst(), 1), W.random_params(W.hp_gst(), 1))
