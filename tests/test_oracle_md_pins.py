"""Pins of the FP64 velocity-Verlet reference (oracle/md_ref.py).

The reference is checked against things other than itself: the unit of
acceleration against the library's CODATA constants, one step worked out by
hand on a harmonic spring, the closed-form motion under a constant force, the
second-order scaling of the energy error with the time step (harmonic spring
and a NEP cell), and exact time reversal.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc

from paper_2607_06969_amd import workloads as W


@pytest.fixture(scope="module")
def md_ref():
    from oracle import md_ref as M
    return M


def test_acceleration_unit_from_library_constants(md_ref):
    """1 eV/(A u) in A/fs^2 = (e / u) * 1e-10 from scipy's CODATA constants
    (its CODATA release may differ from the 2018 values of the reference in
    the tenth digit)."""
    want = sc.e / sc.atomic_mass * 1e-10
    assert abs(md_ref.ACC_UNIT / want - 1.0) < 1e-8
    assert abs(md_ref.ACC_UNIT - 9.6485332e-3) < 1e-10


def test_one_step_by_hand(md_ref):
    """Spring F = -k x with k = 1 eV/A^2 on a mass of ACC_UNIT u (so that
    a = -x A/fs^2), x0 = 1 A, v0 = 0, dt = 0.1 fs.  By hand:
    v(1/2) = 0 - 0.05 * 1 = -0.05;  x1 = 1 + 0.1 * (-0.05) = 0.995;
    a1 = -0.995;  v1 = -0.05 + 0.05 * (-0.995) = -0.09975;
    E_kin = m v1^2 / (2 ACC_UNIT) = 0.09975^2 / 2 = 0.0049750312...;
    E_pot = k x1^2 / 2 = 0.4950125."""
    m = np.array([md_ref.ACC_UNIT])
    traj = md_ref.velocity_verlet(lambda x: (0.5 * float(np.sum(x * x)), -x), [[1.0, 0.0, 0.0]],
                                  [[0.0, 0.0, 0.0]], m, 0.1, 1)
    assert abs(traj["x"][1, 0, 0] - 0.995) < 1e-15
    assert abs(traj["v"][1, 0, 0] - (-0.09975)) < 1e-15
    assert abs(traj["ekin"][1] - 0.09975 ** 2 / 2) < 1e-16
    assert abs(traj["epot"][1] - 0.4950125) < 1e-15
    assert abs(traj["ekin"][0]) == 0.0 and abs(traj["epot"][0] - 0.5) < 1e-16


def test_constant_force_is_exact(md_ref):
    """Under a constant force the scheme reproduces x(t) = x0 + v0 t + a t^2/2
    and v(t) = v0 + a t at every step."""
    F = np.array([[0.5, -0.25, 0.125], [0.0, 1.0, -2.0]])
    m = np.array([2.0, 7.5])
    x0 = np.array([[0.0, 1.0, 2.0], [3.0, -1.0, 0.5]])
    v0 = np.array([[0.01, 0.0, -0.02], [0.0, 0.005, 0.0]])
    dt, n = 0.7, 25
    traj = md_ref.velocity_verlet(lambda x: (0.0, F), x0, v0, m, dt, n)
    a = F / m[:, None] * md_ref.ACC_UNIT
    for k in range(n + 1):
        t = k * dt
        np.testing.assert_allclose(traj["x"][k], x0 + v0 * t + 0.5 * a * t * t, rtol=0, atol=1e-13)
        np.testing.assert_allclose(traj["v"][k], v0 + a * t, rtol=0, atol=1e-15)


def _spring_energy_error(md_ref, dt, t_end=20.0):
    m = np.array([1.0])
    w2 = md_ref.ACC_UNIT  # k = 1 eV/A^2, m = 1 u: omega^2 = ACC_UNIT fs^-2
    n = int(round(t_end / dt))
    traj = md_ref.velocity_verlet(lambda x: (0.5 * float(np.sum(x * x)), -x), [[1.0, 0.0, 0.0]],
                                  [[0.0, 0.02, 0.0]], m, dt, n)
    e = traj["epot"] + traj["ekin"]
    return np.max(np.abs(e - e[0])), w2


def test_energy_error_second_order_spring(md_ref):
    """The energy error of velocity Verlet falls as dt^2: halving dt divides it
    by four (a harmonic spring, period about 64 fs)."""
    errs = [_spring_energy_error(md_ref, dt)[0] for dt in (2.0, 1.0, 0.5)]
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


def test_energy_error_second_order_nep(md_ref, oracle_lib):
    """The same dt^2 scaling on a NEP cell with the oracle's forces (64 atoms,
    single-element model, 300 K)."""
    hp = W.hp_small_single()
    s = W.simple_cubic(n=4, spacing=3.1, sigma=0.1, seed=W.SEED_POS + 1)
    p = W.random_params(hp, W.SEED_PARAM + 1)
    masses = np.full(s.n_atoms, 72.63)
    v0 = W.maxwell_boltzmann(s.species, (72.63,), 300.0, seed=W.SEED_VEL + 1)
    f = md_ref.nep_force_fn(hp, p, s)
    errs = []
    for dt in (2.0, 1.0, 0.5):
        traj = md_ref.velocity_verlet(f, s.pos, v0, masses, dt, int(round(16.0 / dt)))
        e = traj["epot"] + traj["ekin"]
        errs.append(np.max(np.abs(e - e[0])))
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0, errs


def test_time_reversal(md_ref, oracle_lib):
    """n steps forward, velocities negated, n steps again: the start is
    recovered to rounding (NEP forces of the 64-atom cell)."""
    hp = W.hp_small_single()
    s = W.simple_cubic(n=4, spacing=3.1, sigma=0.1, seed=W.SEED_POS + 1)
    p = W.random_params(hp, W.SEED_PARAM + 1)
    masses = np.full(s.n_atoms, 72.63)
    v0 = W.maxwell_boltzmann(s.species, (72.63,), 600.0, seed=W.SEED_VEL + 2)
    f = md_ref.nep_force_fn(hp, p, s)
    fw = md_ref.velocity_verlet(f, s.pos, v0, masses, 1.0, 30)
    bw = md_ref.velocity_verlet(f, fw["x"][-1], -fw["v"][-1], masses, 1.0, 30)
    assert np.max(np.abs(bw["x"][-1] - s.pos)) < 1e-11
    assert np.max(np.abs(bw["v"][-1] + v0)) < 1e-13
    # the atoms did move: the check is not trivial
    assert np.max(np.abs(fw["x"][-1] - s.pos)) > 1e-2
    assert math.isfinite(fw["epot"][-1])
