"""GPU optimisation protocol (Sec. 3.3): the Adam kernel against the FP64
reference of oracle/train_ref.py (pinned to torch.optim.Adam), one full
training step (loss gradient of Eq. 18-21 at the step's dynamic weights,
then Adam at the scheduled learning rate) against the oracle's gradient and
the reference Adam, and the loop reducing the loss of a teacher-student fit.

Tolerances: the Adam kernel stores parameters and moments in FP32.  Every
step rounds each stored value (half an ulp, 2^-24 relative) and computes the
update in FP32 (a few ulps of a step that Adam bounds by about
lr * (1 - beta1) / sqrt(1 - beta2) ~ 3.2 lr).  After t steps a parameter
therefore agrees with the FP64 reference to t * (2^-22 |p| + 4e-6 lr), and a
moment to t * 2^-21 of the running sum of the magnitudes of its terms (the
first moment can cancel, so its own magnitude is no scale).  After one full
step (Adam at t = 1) each parameter moved by lr * g / (|g| + eps): every
component must do so for the GPU's own gradient, that gradient must match
the oracle's to the relative RMS bar of the gradient tests (1e-4), and where
|g| exceeds 1e-2 of its RMS (100 times that bar, so the sign is certain)
the step must match the one the oracle's gradient gives."""
import numpy as np
import pytest

from paper_2607_06969_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_adam_kernel_matches_reference():
    from oracle import train_ref as R
    from paper_2607_06969_amd import nep
    rng = np.random.default_rng(7)
    n = 10431
    p0 = rng.normal(scale=0.1, size=n).astype(np.float32)
    p, m, v = (torch.tensor(a, device="cuda") for a in (p0, np.zeros(n, np.float32), np.zeros(n, np.float32)))
    q, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    mag_m = np.zeros(n)
    lr_sum = 0.0
    for t in range(1, 6):
        g0 = (rng.normal(size=n) * 10.0 ** rng.uniform(-4, 1, size=n)).astype(np.float32)
        g = torch.tensor(g0, device="cuda")
        lr = 1e-3 * t
        lr_sum += lr
        nep.adam_step(p, g, m, v, t, lr)
        q, mr, vr = R.adam_step(q, g0.astype(np.float64), mr, vr, t, lr)
        mag_m = 0.9 * mag_m + 0.1 * np.abs(g0)
        torch.cuda.synchronize()
        tol = {"p": t * 2.0 ** -22 * np.abs(q) + 4e-6 * lr_sum,
               "m": t * 2.0 ** -21 * mag_m + 1e-30, "v": t * 2.0 ** -21 * vr + 1e-30}
        for name, got, ref in (("p", p, q), ("m", m, mr), ("v", v, vr)):
            err = np.abs(got.cpu().numpy().astype(np.float64) - ref)
            assert np.all(err <= tol[name]), (t, name, np.max(err / tol[name]))


def test_one_training_step_matches_oracle(oracle_lib):
    from oracle import train_ref as R
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=6, n_min=64, n_max=200, seed=91)
    teacher, student = W.random_params(hp, W.SEED_TEACHER), W.random_params(hp, W.SEED_STUDENT)
    lab = oracle_lib.evaluate(hp, teacher, s, nbr_mode=0)
    Er, Fr, Vr = lab["E"], lab["F"].astype(np.float32).astype(np.float64), lab["V"].reshape(-1, 9)
    total, warm, lr0, lr1 = 20, 4, 2e-3, 1e-5
    ws, we = (1.0, 10.0, 0.1), (10.0, 1.0, 1.0)
    m = nep.NepModel(hp, student)
    tr = nep.Trainer(m, total, warm, lr0, lr1, ws, we, normalised=True, loss_form=1)
    b = nep.Batch.from_system(s)
    loss, lr, w = tr.step(b, torch.tensor(Er, device="cuda"), torch.tensor(Fr, dtype=torch.float32, device="cuda"),
                          torch.tensor(Vr, device="cuda"))
    lr_ref = R.lr_at(0, warm, total, lr0, lr1)
    w_ref = R.loss_weights(lr_ref, lr0, ws, we)
    assert lr == pytest.approx(lr_ref, rel=1e-14) and w == pytest.approx(w_ref, rel=1e-14)
    parts, g = oracle_lib.loss_grad(hp, student, s, Er, Fr, Vr, weights=w_ref, loss_form=1, nbr_mode=0)
    np.testing.assert_allclose(loss.cpu().numpy(), parts, rtol=1e-5)
    gg = tr.last_grad.cpu().numpy().astype(np.float64)
    rms = np.sqrt(np.mean(g * g))
    assert np.sqrt(np.mean((gg - g) ** 2)) < 1e-4 * rms
    p0 = student.astype(np.float32).astype(np.float64)
    got = tr.params.cpu().numpy().astype(np.float64)
    fp32 = 2.0 ** -23 * np.abs(p0) + 4e-6 * lr_ref
    assert np.all(np.abs((got - p0) + lr_ref * gg / (np.abs(gg) + 1e-8)) <= fp32)
    q, _, _ = R.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr_ref)
    sure = np.abs(g) > 1e-2 * rms
    assert np.all(np.abs(got - q)[sure] <= fp32[sure] + 1e-3 * lr_ref)


def test_training_loop_reduces_the_loss():
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=16, n_min=64, n_max=160, seed=92)
    b = nep.Batch.from_system(s)
    teacher = nep.NepModel(hp, W.random_params(hp, W.SEED_TEACHER))
    lab = teacher.compute(b)
    Er, Fr, Vr = lab["E"], lab["F"].contiguous(), lab["V"].reshape(-1, 9).contiguous()
    m = nep.NepModel(hp, W.random_params(hp, W.SEED_STUDENT))
    tr = nep.Trainer(m, total_steps=120, warmup_steps=10, lr_start=3e-3, lr_end=1e-5,
                     w_start=(1.0, 1.0, 0.1), w_end=(1.0, 1.0, 0.1))
    losses = []
    for _ in range(120):
        loss, _, _ = tr.step(b, Er, Fr, Vr)
        losses.append(float(loss[0]))
    print(f"[fit] loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.3 * losses[0]
    assert np.mean(losses[-10:]) < np.mean(losses[:10])
