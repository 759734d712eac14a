"""Float64 variant of the GPU path (every operator exists in float32 and
float64, Sec. 3.2) against the FP64 oracle, and torch.autograd.gradcheck of
its hand-written parameter backward on the GPU.

Tolerances: both sides compute in float64 and differ only in the order of
rounding, so energy per atom, forces, virial and the parameter gradient agree
to 1e-10 relative (1e-9 for the gradient, whose float64 sums over atoms and
pairs are longer).  gradcheck compares the backward with central differences
of the float64 forward (step 1e-6: truncation ~1e-12, rounding ~1e-10)."""
import numpy as np
import pytest

from paper_2607_06969_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = {
    "cubic64_single": (W.hp_small_single, lambda: W.simple_cubic(), 2001),
    "gst_rocksalt_16": (W.hp_gst, lambda: W.rocksalt_gst(16), 2002),
    "table2_rocksalt_8": (W.hp_table2, lambda: W.rocksalt_gst(8, seed=52), 2003),
    "gst_amorphous_batch": (W.hp_gst, lambda: W.amorphous_batch(n_cfg=6, n_min=64, n_max=300, seed=53), 2004),
}


@pytest.mark.parametrize("name", list(CASES))
def test_compute64_matches_oracle(oracle_lib, name):
    from paper_2607_06969_amd import nep
    hpf, sysf, seed = CASES[name]
    hp, s = hpf(), sysf()
    p = W.random_params(hp, seed)
    print(f"[fp64] {name}: N={s.n_atoms} n_cfg={s.n_cfg}", flush=True)
    ref = oracle_lib.evaluate(hp, p, s, nbr_mode=2)
    m = nep.NepModel(hp, p)
    b = nep.Batch.from_system(s)
    got = m.compute64(b, torch.tensor(p, dtype=torch.float64, device="cuda"), atom_energy=True)
    got = {k: v.cpu().numpy() for k, v in got.items()}
    n = np.diff(s.atom_off)
    print(f"[fp64] {name}: dE/N {np.max(np.abs(got['E'] - ref['E']) / n):.2e} F {rel(got['F'], ref['F']):.2e} "
          f"V {rel(got['V'].reshape(-1, 9), ref['V'].reshape(-1, 9)):.2e}", flush=True)
    assert np.max(np.abs(got["E"] - ref["E"]) / n) <= 1e-10
    assert rel(got["F"], ref["F"]) <= 1e-10, rel(got["F"], ref["F"])
    assert rel(got["V"].reshape(-1, 9), ref["V"].reshape(-1, 9)) <= 1e-10
    if "Ei" in ref:
        assert np.max(np.abs(got["Ei"] - ref["Ei"])) <= 1e-10


def _seeds(form, w, E, F, V, Er, Fr, Vr, off):
    """dL/dE, dL/dF, dL/dV of the loss of Eq. 18-21 in the two normalisations
    the library implements (form 0: pooled over the batch; form 1: per
    configuration, averaged)."""
    n = np.diff(off).astype(np.float64)
    B = len(n)
    dE, dV = E - Er, (V - Vr).reshape(B, 9)
    if form == 0:
        eb = 2 * w[0] / (B * n * n) * dE
        lam = 2 * w[1] / (3 * n.sum()) * (F - Fr)
        mu = 2 * w[2] / (9 * B * n * n)[:, None] * dV
    else:
        eb = 2 * w[0] / (B * n) * dE
        lam = 2 * w[1] / (3 * B * np.repeat(n, n.astype(int)))[:, None] * (F - Fr)
        mu = 2 * w[2] / (9 * B * n)[:, None] * dV
    return eb, lam, mu


@pytest.mark.parametrize("form", [0, 1])
def test_backward64_matches_oracle_loss_gradient(oracle_lib, form):
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=4, n_min=64, n_max=200, seed=95)
    teacher, student = W.random_params(hp, W.SEED_TEACHER), W.random_params(hp, W.SEED_STUDENT)
    lab = oracle_lib.evaluate(hp, teacher, s, nbr_mode=0)
    Er, Fr, Vr = lab["E"], lab["F"], lab["V"].reshape(-1, 9)
    w = (1.0, 2.0, 0.1)
    m = nep.NepModel(hp, student)
    b = nep.Batch.from_system(s)
    P = torch.tensor(student, dtype=torch.float64, device="cuda")
    out = m.compute64(b, P)
    E, F, V = (out[k].cpu().numpy() for k in ("E", "F", "V"))
    eb, lam, mu = _seeds(form, w, E, F, V.reshape(-1, 9), Er, Fr, Vr, s.atom_off)
    g = m.backward_params64(b, P, torch.tensor(eb, device="cuda"), torch.tensor(lam, device="cuda"),
                            torch.tensor(mu, device="cuda")).cpu().numpy()
    parts, g_ref = oracle_lib.loss_grad(hp, student, s, Er, Fr, Vr, weights=w, loss_form=form, nbr_mode=0)
    print(f"[fp64] loss form {form}: gradient rel {rel(g, g_ref):.2e}", flush=True)
    assert rel(g, g_ref) <= 1e-9, rel(g, g_ref)


def test_gradcheck_small_model_every_parameter():
    from paper_2607_06969_amd import nep
    hp = W.hp_small_single()
    s = W.simple_cubic()
    m = nep.NepModel(hp, W.random_params(hp, 2001))
    b = nep.Batch.from_system(s)
    p = torch.tensor(W.random_params(hp, 2001), dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: nep.NepFunction64.apply(x, m, b), (p,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6)


def test_gradcheck_gst_model_fast_mode():
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    s = W.rocksalt_gst(8, seed=51)
    m = nep.NepModel(hp, W.random_params(hp, 2002))
    b = nep.Batch.from_system(s)
    p = torch.tensor(W.random_params(hp, 2002), dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: nep.NepFunction64.apply(x, m, b), (p,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6, fast_mode=True)
