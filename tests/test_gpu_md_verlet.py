"""GPU velocity-Verlet trajectory against the FP64 reference integrator.

The graph-replayed MD step (float32 forces and velocities, float64 positions)
is compared step by step with oracle/md_ref.py, velocity Verlet in float64 on
the FP64 oracle's forces, over 20 steps of 1 fs on a 460-atom Ge-Sb-Te cell,
once with a 1 A skin (no rebuild) and once with a 0.05 A skin (lists rebuilt
inside the graph during the run).

Tolerances, from the float32 arithmetic of the GPU step:
  - positions are returned in float32: half an ulp at 16-32 A is 1.9e-6 A,
    and the force error (relative 1e-5 at most per atom, accelerations about
    1e-4 A/fs^2) moves an atom by 1e-9 A/fs^2 * (20 fs)^2 / 2 = 2e-7 A at
    most, so |dx| <= 1e-5 A;
  - velocities: the same force error gives 1e-9 * 20 = 2e-8 A/fs, and
    float32 rounding of v (~2e-3 A/fs) 20 * 1e-10, so |dv| <= 1e-6 A/fs
    (rms speed about 2e-3 A/fs);
  - potential energy within 1e-6 eV/atom (the bar of the evaluation), kinetic
    energy within 1e-6 relative.
A wrong unit of acceleration or a wrong kick order moves the trajectory by far
more than these bounds within a few steps.
"""
import numpy as np
import pytest

from paper_2607_06969_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("skin", [1.0, 0.05])
def test_md_trajectory_matches_fp64_verlet(oracle_lib, skin):
    from oracle import md_ref
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    s = W.rocksalt_gst(8, seed=W.SEED_POS + 71)
    p = W.random_params(hp, W.SEED_PARAM + 71)
    v0 = W.maxwell_boltzmann(s.species, W.MASSES_GST, 300.0, seed=W.SEED_VEL + 71)
    masses = np.asarray(W.MASSES_GST)[s.species]
    m = nep.NepModel(hp, p)
    b = nep.Batch.from_system(s)
    md = nep.NepMD(m, b, torch.as_tensor(v0, dtype=torch.float32, device="cuda").contiguous(), W.MASSES_GST,
                   dt_fs=1.0, skin=skin)
    n_steps = 20
    ref = md_ref.velocity_verlet(md_ref.nep_force_fn(hp, p, s), s.pos, v0, masses, 1.0, n_steps)
    L = s.cells[0, 0, 0]
    n = s.n_atoms
    worst = {"x": 0.0, "v": 0.0, "epot": 0.0, "ekin": 0.0}
    for k in range(1, n_steps + 1):
        md.step(1)
        st = md.state()
        d = st["pos"].cpu().numpy().astype(np.float64) - ref["x"][k]
        d -= L * np.round(d / L)
        worst["x"] = max(worst["x"], float(np.max(np.abs(d))))
        worst["v"] = max(worst["v"], float(np.max(np.abs(st["vel"].cpu().numpy() - ref["v"][k]))))
        worst["epot"] = max(worst["epot"], abs(float(st["Epot"][0]) - ref["epot"][k]) / n)
        worst["ekin"] = max(worst["ekin"], abs(float(st["Ekin"][0]) - ref["ekin"][k]) / ref["ekin"][k])
    print(f"skin {skin}: rebuilds {md.stats()['rebuilds']}, worst {worst}")
    if skin < 0.1:
        assert md.stats()["rebuilds"] >= 3
    # the atoms moved by much more than the tolerance
    assert np.max(np.abs(ref["x"][-1] - ref["x"][0])) > 1e-2
    assert worst["x"] <= 1e-5, worst
    assert worst["v"] <= 1e-6, worst
    assert worst["epot"] <= 1e-6, worst
    assert worst["ekin"] <= 1e-6, worst
