"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times:
  - the 900,000-atom rocksalt cell stepped as the timed MD graph (autotuned
    kernel variants, timed-step replay, in-graph list rebuild), every output
    against the FP64 oracle on the same positions;
  - the same cell over 600 steps with its list capacities clamped, so that a
    rebuild overflows and the lists are regrown at full size;
  - the same cell with the model of the paper's Table 2, stepped as the
    benchmark steps it;
  - the float64 evaluation of the same cell (bar 1e-10);
  - the full 256-configuration training batch: loss and parameter gradient;
  - sampled cells (smallest, median, largest) of the 64-cell serving batch,
    evaluated inside the batched MD handle.
Tolerances as in the parity tests (float32 arithmetic against float64):
|dE|/N <= 1e-6 eV/atom, forces and virial <= 1e-5 relative RMS, loss parts
1e-5 relative, gradient 1e-4 relative RMS."""
import numpy as np
import pytest

from paper_2607_06969_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_md_900k_after_timed_steps_matches_oracle(oracle_lib):
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    p = W.random_params(hp, W.SEED_PARAM + 3)
    s = W.rocksalt_gst(100, seed=W.SEED_POS + 3)
    vel = W.maxwell_boltzmann(s.species, W.MASSES_GST, 300.0, seed=W.SEED_VEL)
    m = nep.NepModel(hp, p)
    b = nep.Batch.from_system(s)
    v = torch.as_tensor(vel, dtype=torch.float32, device="cuda").contiguous()
    md = nep.NepMD(m, b, v, W.MASSES_GST, dt_fs=1.0, skin=1.0)
    print(f"[fullsize] MD {s.n_atoms} atoms, variants {m.variants()}", flush=True)
    md.step_timed(60)
    stats = md.stats()
    assert stats["steps"] == 60 and stats["rebuilds"] >= 2, stats
    st = md.state()
    pos = st["pos"].cpu().numpy().astype(np.float64)
    ref = oracle_lib.evaluate(hp, p, W.System(pos, s.species, s.cells, s.atom_off), nbr_mode=1)
    n = s.n_atoms
    dE = abs(float(st["Epot"][0]) - ref["E"][0]) / n
    rF, rV = rel(st["F"].cpu().numpy(), ref["F"]), rel(st["V"][0].cpu().numpy(), ref["V"][0])
    print(f"[fullsize] MD dE/N {dE:.2e} F {rF:.2e} V {rV:.2e}", flush=True)
    assert dE < 1e-6 and rF < 1e-5 and rV < 1e-5


def test_md_900k_regrow_in_long_run_matches_oracle(oracle_lib):
    """The 900,000-atom cell with its list capacities clamped to the longest
    lists built so far: the random-parameter model heats the cell, the lists
    grow, and a rebuild inside the step graph overflows.  The chunk is rolled
    back, the lists regrown and the graph re-captured at full size; afterwards
    the state still matches the FP64 oracle and the total energy is kept."""
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    p = W.random_params(hp, W.SEED_PARAM + 3)
    s = W.rocksalt_gst(100, seed=W.SEED_POS + 3)
    vel = W.maxwell_boltzmann(s.species, W.MASSES_GST, 300.0, seed=W.SEED_VEL)
    m = nep.NepModel(hp, p)
    v = torch.as_tensor(vel, dtype=torch.float32, device="cuda").contiguous()
    md = nep.NepMD(m, nep.Batch.from_system(s), v, W.MASSES_GST, dt_fs=1.0, skin=1.0)
    cap0 = md.capacity(1, 1)  # clamped up to the longest lists so far
    st = md.state()
    n = s.n_atoms
    e0 = (float(st["Epot"][0]) + float(st["Ekin"][0])) / n
    print(f"[fullsize] long MD {n} atoms, capacities {cap0}", flush=True)
    md.step(600)
    stats, cap1 = md.stats(), md.capacity()
    print(f"[fullsize] long MD {stats} capacities {cap1}", flush=True)
    assert stats["steps"] == 600 and stats["regrows"] >= 1, stats
    assert cap1["capR"] > cap0["capR"] or cap1["capA"] > cap0["capA"]
    st = md.state()
    e1 = (float(st["Epot"][0]) + float(st["Ekin"][0])) / n
    pos = st["pos"].cpu().numpy().astype(np.float64)
    ref = oracle_lib.evaluate(hp, p, W.System(pos, s.species, s.cells, s.atom_off), nbr_mode=1)
    dE = abs(float(st["Epot"][0]) - ref["E"][0]) / n
    rF, rV = rel(st["F"].cpu().numpy(), ref["F"]), rel(st["V"][0].cpu().numpy(), ref["V"][0])
    print(f"[fullsize] long MD dE/N {dE:.2e} F {rF:.2e} V {rV:.2e} drift {e1 - e0:.2e} eV/atom", flush=True)
    assert dE < 1e-6 and rF < 1e-5 and rV < 1e-5
    assert abs(e1 - e0) < 1e-5  # 1 fs steps: the total energy is kept (measured 3e-7 eV/atom)


def test_table2_md_900k_matches_oracle(oracle_lib):
    """The MD leg of the paper's own model (Table 2: 10/8 functions, 8/8
    basis, 2- and 3-body terms, cutoffs 7 / 5 A) on the 900,000-atom cell,
    stepped as the benchmark steps it (warm-up, then timed graph replays),
    against the FP64 oracle on the final positions."""
    from paper_2607_06969_amd import nep
    hp = W.hp_table2()
    p = W.random_params(hp, W.SEED_PARAM + 4)
    s = W.rocksalt_gst(100, seed=W.SEED_POS + 3)
    vel = W.maxwell_boltzmann(s.species, W.MASSES_GST, 300.0, seed=W.SEED_VEL)
    m = nep.NepModel(hp, p)
    v = torch.as_tensor(vel, dtype=torch.float32, device="cuda").contiguous()
    md = nep.NepMD(m, nep.Batch.from_system(s), v, W.MASSES_GST, dt_fs=1.0, skin=1.0)
    print(f"[fullsize] Table 2 MD {s.n_atoms} atoms, variants {m.variants()}", flush=True)
    md.step(5)
    md.step_timed(40)
    stats = md.stats()
    assert stats["steps"] == 45 and stats["rebuilds"] >= 1, stats
    st = md.state()
    pos = st["pos"].cpu().numpy().astype(np.float64)
    ref = oracle_lib.evaluate(hp, p, W.System(pos, s.species, s.cells, s.atom_off), nbr_mode=1)
    n = s.n_atoms
    dE = abs(float(st["Epot"][0]) - ref["E"][0]) / n
    rF, rV = rel(st["F"].cpu().numpy(), ref["F"]), rel(st["V"][0].cpu().numpy(), ref["V"][0])
    print(f"[fullsize] Table 2 MD dE/N {dE:.2e} F {rF:.2e} V {rV:.2e} rebuilds {stats['rebuilds']}", flush=True)
    assert dE < 1e-6 and rF < 1e-5 and rV < 1e-5


def test_float64_900k_matches_oracle(oracle_lib):
    """The float64 evaluation of the full 900,000-atom cell against the FP64
    oracle on the same positions, at the float64 bar (1e-10)."""
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    p = W.random_params(hp, W.SEED_PARAM + 3)
    s = W.rocksalt_gst(100, seed=W.SEED_POS + 3)
    m = nep.NepModel(hp, p)
    print(f"[fullsize] float64 {s.n_atoms} atoms", flush=True)
    got = m.compute64(nep.Batch.from_system(s), torch.tensor(p, dtype=torch.float64, device="cuda"),
                      pos=torch.tensor(s.pos, dtype=torch.float64, device="cuda"))
    got = {k: v.cpu().numpy() for k, v in got.items()}
    ref = oracle_lib.evaluate(hp, p, s, nbr_mode=1)
    n = s.n_atoms
    dE = abs(got["E"][0] - ref["E"][0]) / n
    rF, rV = rel(got["F"], ref["F"]), rel(got["V"].reshape(-1), ref["V"].reshape(-1))
    print(f"[fullsize] float64 dE/N {dE:.2e} F {rF:.2e} V {rV:.2e}", flush=True)
    assert dE <= 1e-10 and rF <= 1e-10 and rV <= 1e-10


def test_training_batch_256_matches_oracle(oracle_lib):
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    s = W.amorphous_batch()
    teacher, student = W.random_params(hp, W.SEED_TEACHER), W.random_params(hp, W.SEED_STUDENT)
    lab = oracle_lib.evaluate(hp, teacher, s, nbr_mode=1)
    Er, Fr, Vr = lab["E"], lab["F"].astype(np.float32).astype(np.float64), lab["V"].reshape(-1, 9)
    m = nep.NepModel(hp, student)
    b = nep.Batch.from_system(s)
    print(f"[fullsize] training batch {s.n_cfg} cells, {s.n_atoms} atoms", flush=True)
    for form in (0, 1):
        loss, g = m.loss_grad(b, torch.tensor(Er, device="cuda"), torch.tensor(Fr, dtype=torch.float32, device="cuda"),
                              torch.tensor(Vr, device="cuda"), loss_form=form)
        parts, g_ref = oracle_lib.loss_grad(hp, student, s, Er, Fr, Vr, loss_form=form, nbr_mode=1)
        g = g.cpu().numpy()
        print(f"[fullsize] form {form}: loss rel {rel(loss.cpu().numpy(), parts):.2e} gradient {rel(g, g_ref):.2e}",
              flush=True)
        np.testing.assert_allclose(loss.cpu().numpy(), parts, rtol=1e-5, atol=1e-12)
        assert rel(g, g_ref) < 1e-4


def test_serving_batch_sampled_cells_match_oracle(oracle_lib):
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    p = W.random_params(hp, W.SEED_PARAM + 3)
    s = W.mixed_size_cells()
    vel = W.maxwell_boltzmann(s.species, W.MASSES_GST, 300.0, seed=W.SEED_VEL + 5)
    m = nep.NepModel(hp, p)
    b = nep.Batch.from_system(s)
    v = torch.as_tensor(vel, dtype=torch.float32, device="cuda").contiguous()
    md = nep.NepMD(m, b, v, W.MASSES_GST)
    md.step(3)
    st = md.state()
    pos = st["pos"].cpu().numpy().astype(np.float64)
    F, E, V = st["F"].cpu().numpy(), st["Epot"].cpu().numpy(), st["V"].cpu().numpy()
    n = np.diff(s.atom_off)
    for c in (int(np.argmin(n)), int(np.argsort(n)[len(n) // 2]), int(np.argmax(n))):
        a0, a1 = s.atom_off[c], s.atom_off[c + 1]
        sub = W.System(pos[a0:a1], s.species[a0:a1], s.cells[c:c + 1], np.array([0, a1 - a0]))
        ref = oracle_lib.evaluate(hp, p, sub, nbr_mode=1)
        dE = abs(E[c] - ref["E"][0]) / (a1 - a0)
        rF, rV = rel(F[a0:a1], ref["F"]), rel(V[c], ref["V"][0])
        print(f"[fullsize] serving cell {c} ({a1 - a0} atoms): dE/N {dE:.2e} F {rF:.2e} V {rV:.2e}", flush=True)
        assert dE < 1e-6 and rF < 1e-5 and rV < 1e-5
