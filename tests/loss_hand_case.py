"""A loss worked out by hand (shared by the oracle pin and the GPU check).

A single-element model whose site energy is its output bias alone gives
E_c = N_c / 2, F = 0 and V = 0 for any positions, so the residuals of the
chosen labels are known exactly and every loss term can be evaluated by hand.
"""
import numpy as np

from paper_2607_06969_amd import workloads as W


def constant_energy_model():
    """Single-element model whose site energy is the output bias alone
    (W0 = 0, w1 = 0, b1 = 1/2), so that E_c = N_c / 2 and F = V = 0 exactly,
    whatever the positions."""
    hp = W.hp_small_single()
    p = np.zeros(hp.n_params())
    p[-1] = 0.5  # b1 of the only species: the last entry of the flat layout
    return hp, p


def two_config_batch():
    """A dimer (N = 2) and a trimer (N = 3), each in a 20 A cubic box."""
    pos = np.array([[1.0, 1.0, 1.0], [3.5, 1.0, 1.0],
                    [2.0, 2.0, 2.0], [4.5, 2.0, 2.0], [2.0, 4.5, 2.0]])
    cells = np.stack([np.eye(3) * 20.0, np.eye(3) * 20.0])
    return W.System(pos, np.zeros(5, dtype=np.int32), cells, np.array([0, 2, 5], dtype=np.int64))


# Labels chosen by hand.  With the constant-energy model the model's values are
# E = (1, 3/2), F = 0, V = 0, so the residuals are dE = (0.4, -0.9),
# dF = -F_ref and dV = -V_ref:
#   sum dF^2: dimer 0.1^2 + 0.2^2 + 0.3^2 + 0.5^2 = 0.39, trimer 1 + 1 + 1 = 3;
#   sum dV^2: dimer 0.6^2 + 0.8^2 = 1.0, trimer 1.5^2 + 1.2^2 + 0.9^2 = 4.5.
E_REF = np.array([0.6, 2.4])
F_REF = np.array([[0.1, -0.2, 0.3], [0.0, 0.0, 0.5],
                       [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, -1.0]])
V_REF = np.array([[0.6, 0.0, 0.0, 0.0, 0.0, -0.8, 0.0, 0.0, 0.0],
                       [1.5, 1.2, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.9]])
# loss_form 0 (mean squared errors: energy per atom averaged over the B = 2
# configurations, force components pooled over all 3 sum N = 15 of them,
# virial per atom averaged over 9 B = 18 components), weights (1, 1, 0.1):
#   L_E = ((0.4/2)^2 + (0.9/3)^2) / 2       = (0.04 + 0.09) / 2    = 0.065
#   L_F = (0.39 + 3) / 15                                           = 0.226
#   L_V = 0.1 (1.0/2^2 + 4.5/3^2) / 18      = 0.1 (0.25 + 0.5) / 18 = 0.075 / 18
# dL/db1 = sum_c (dL/dE_c) N_c with dL/dE_c = 2 w_E dE_c / (B N_c^2):
#   (2 (0.4) / 8) 2 + (2 (-0.9) / 18) 3 = 0.2 - 0.3 = -0.1
FORM0 = {"w": (1.0, 1.0, 0.1), "parts": (0.065, 0.226, 0.075 / 18), "db1": -0.1}
# loss_form 1 (Eq. 19-21 of each configuration, averaged over the batch),
# weights (2, 3, 0.5):
#   dimer   L_E = 2/2 0.4^2 = 0.16,  L_F = 3/(3*2) 0.39 = 0.195,  L_V = 0.5/(9*2) 1.0 = 1/36
#   trimer  L_E = 2/3 0.9^2 = 0.54,  L_F = 3/(3*3) 3    = 1.0,    L_V = 0.5/(9*3) 4.5 = 1/12
#   batch   L_E = 0.35,  L_F = 0.5975,  L_V = (1/36 + 1/12) / 2 = 1/18
# dL/db1 = sum_c (2 w_E dE_c / (B N_c)) N_c = (2 2 0.4 / 4) 2 + (2 2 (-0.9) / 6) 3 = 0.8 - 1.8 = -1.0
FORM1 = {"w": (2.0, 3.0, 0.5), "parts": (0.35, 0.5975, 1.0 / 18), "db1": -1.0}
