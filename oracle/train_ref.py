"""FP64 reference of the optimisation protocol of Sec. 3.3.

TEST INFRASTRUCTURE: only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It never imports the
HIP package, and the HIP package never imports it.

- adam_step: Adam (Sec. 3.3.1) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8
  and no weight decay, bias-corrected, eps added after the square root.
- lr_at: the two-stage schedule of Sec. 3.3.2, a linear warmup of the factor
  from 1e-4 to 1 over the first epoch, then cosine annealing from lr_start to
  lr_end over the remaining steps, updated every step.
- loss_weights: the linear interpolation of Sec. 3.3.3 between the initial
  and final weights, with x = lr as printed or x = lr / lr_start (reading
  documented with the schedule: the printed form is ~w_end at every step
  for learning rates below 1e-2, which the paper's own weight curves do not
  show).
"""
from __future__ import annotations

import math

import numpy as np


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Return (p, m, v) after step t (t >= 1), all float64 arrays."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat_sqrt = np.sqrt(v) / math.sqrt(1.0 - beta2 ** t)
    return p - lr * m_hat / (v_hat_sqrt + eps), m, v


def lr_at(step, warmup_steps, total_steps, lr_start, lr_end, start_factor=1e-4):
    """Learning rate at 0-based training step `step`."""
    if step < warmup_steps:
        return lr_start * (start_factor + (1.0 - start_factor) * step / warmup_steps)
    T = total_steps - warmup_steps
    s = min(step - warmup_steps, T) / T if T > 0 else 1.0
    return lr_end + 0.5 * (lr_start - lr_end) * (1.0 + math.cos(math.pi * s))


def loss_weights(lr, lr_start, w_start, w_end, normalised=True):
    x = lr / lr_start if normalised else lr
    return [ws * x + we * (1.0 - x) for ws, we in zip(w_start, w_end)]
