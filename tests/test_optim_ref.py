"""The optimisation protocol of Sec. 3.3: the FP64 reference pinned to the
library routines the paper names (torch.optim.Adam, LinearLR followed by
CosineAnnealingLR), and the library's host-side schedule and loss weights
against the reference (no GPU needed)."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import train_ref as R


def test_adam_reference_matches_torch_adam():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=257)
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0)
    q, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, 8):
        g = rng.normal(size=257) * (10.0 ** rng.uniform(-3, 1))
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        q, m, v = R.adam_step(q, g, m, v, t, 3e-3)
        assert np.allclose(q, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_schedule_matches_torch_warmup_then_cosine():
    lr0, lr1, W, Ttot = 1e-3, 1e-5, 37, 300
    p = torch.zeros(1, requires_grad=True)
    opt = torch.optim.SGD([p], lr=lr0)
    warm = torch.optim.lr_scheduler.LinearLR(opt, start_factor=1e-4, end_factor=1.0, total_iters=W)
    cos = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=Ttot - W, eta_min=lr1)
    sched = torch.optim.lr_scheduler.SequentialLR(opt, [warm, cos], milestones=[W])
    for step in range(Ttot):
        assert abs(opt.param_groups[0]["lr"] - R.lr_at(step, W, Ttot, lr0, lr1)) <= 1e-12 * lr0, step
        opt.step()
        sched.step()


def test_loss_weights_interpolate_between_start_and_end():
    ws, we = [1.0, 100.0, 0.1], [10.0, 1.0, 1.0]
    assert R.loss_weights(1e-3, 1e-3, ws, we) == pytest.approx(ws)            # start of annealing
    assert R.loss_weights(0.0, 1e-3, ws, we) == pytest.approx(we)             # lr -> 0
    assert R.loss_weights(1e-3, 1e-3, ws, we, normalised=False) == pytest.approx(
        [a * 1e-3 + b * (1 - 1e-3) for a, b in zip(ws, we)])


@pytest.fixture(scope="module")
def lib():
    from paper_2607_06969_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.skip("libnepmi.so not built")
    return _lib.load()


def test_library_schedule_and_weights_match_reference(lib):
    out = C.c_double()
    for W, Ttot in ((37, 300), (0, 10), (5, 5)):
        for step in list(range(0, Ttot + 3)):
            assert lib.nepmi_lr_schedule(step, W, Ttot, 1e-3, 1e-5, 1e-4, C.byref(out)) == 0
            assert out.value == pytest.approx(R.lr_at(step, W, Ttot, 1e-3, 1e-5), rel=1e-14, abs=1e-18)
    ws, we, w = (C.c_double * 3)(1.0, 100.0, 0.1), (C.c_double * 3)(10.0, 1.0, 1.0), (C.c_double * 3)()
    for norm in (0, 1):
        assert lib.nepmi_loss_weights(4e-4, 1e-3, ws, we, norm, w) == 0
        assert list(w) == pytest.approx(R.loss_weights(4e-4, 1e-3, list(ws), list(we), bool(norm)), rel=1e-14)
    assert lib.nepmi_lr_schedule(-1, 3, 10, 1e-3, 1e-5, 1e-4, C.byref(out)) != 0
