"""FP64 velocity-Verlet NVE reference built on the oracle's forces.

TEST INFRASTRUCTURE: only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It never imports the
HIP package, and the HIP package never imports it.

The paper runs its MD through LAMMPS (Sec. 3.5, Sec. 4.3) and does not print
an integrator; the workload it benchmarks is plain NVE dynamics.  This module
is the textbook velocity-Verlet scheme in float64, with forces from the FP64
oracle (Eq. 3 of the paper) or from any callable:

    v(t + dt/2) = v(t) + (dt/2) a(t)
    x(t + dt)   = x(t) + dt v(t + dt/2)
    v(t + dt)   = v(t + dt/2) + (dt/2) a(t + dt),    a = F / m.

Units are Angstrom, fs, eV and atomic mass units, so a force F (eV/A) on a
mass m (u) accelerates by F / m * ACC_UNIT (A/fs^2), with

    ACC_UNIT = (e / u) * 1e-10   [1 eV/(A u) = e J / (1e-10 m * u kg)
                                   = (e / u) * 1e10 m/s^2, and 1 m/s^2 = 1e-20 A/fs^2]

from the CODATA 2018 values of the elementary charge (exact in the SI) and
the atomic mass constant.  Kinetic energy is sum_i m_i |v_i|^2 / (2 ACC_UNIT)
in eV.
"""
from __future__ import annotations

import numpy as np

# CODATA 2018: elementary charge (C, exact) and atomic mass constant (kg).
ELEMENTARY_CHARGE = 1.602176634e-19
ATOMIC_MASS = 1.66053906660e-27
ACC_UNIT = ELEMENTARY_CHARGE / ATOMIC_MASS * 1e-10


def kinetic_energy(vel, masses) -> float:
    """sum_i m_i |v_i|^2 / 2 in eV (vel in A/fs, masses in u, one per atom)."""
    vel = np.asarray(vel, dtype=np.float64)
    return float(0.5 * np.sum(np.asarray(masses, dtype=np.float64)[:, None] * vel * vel) / ACC_UNIT)


def velocity_verlet(force_fn, x0, v0, masses, dt: float, n_steps: int):
    """Integrate n_steps velocity-Verlet steps from (x0, v0).

    force_fn(x) -> (E_pot, F) with F of shape (N, 3) in eV/A; masses: one per
    atom (u).  Returns a dict of float64 arrays: x, v (n_steps + 1, N, 3),
    epot, ekin (n_steps + 1) and F (n_steps + 1, N, 3), index 0 being the
    initial state.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    v = np.array(v0, dtype=np.float64, copy=True)
    inv_m = ACC_UNIT / np.asarray(masses, dtype=np.float64)[:, None]
    e, f = force_fn(x)
    f = np.asarray(f, dtype=np.float64)
    xs, vs, es, ks, fs = [x.copy()], [v.copy()], [float(e)], [kinetic_energy(v, masses)], [f.copy()]
    for _ in range(n_steps):
        v = v + 0.5 * dt * f * inv_m
        x = x + dt * v
        e, f = force_fn(x)
        f = np.asarray(f, dtype=np.float64)
        v = v + 0.5 * dt * f * inv_m
        xs.append(x.copy())
        vs.append(v.copy())
        es.append(float(e))
        ks.append(kinetic_energy(v, masses))
        fs.append(f.copy())
    return {"x": np.array(xs), "v": np.array(vs), "epot": np.array(es), "ekin": np.array(ks), "F": np.array(fs)}


def nep_force_fn(hp, params, system, nbr_mode: int = 0):
    """force_fn of one periodic configuration of the oracle's NEP: positions
    replace system.pos (unwrapped positions are fine: the oracle sums every
    periodic image)."""
    from copy import copy

    from . import oracle as O

    def f(x):
        s = copy(system)
        s.pos = np.asarray(x, dtype=np.float64)
        out = O.evaluate(hp, params, s, nbr_mode=nbr_mode)
        return float(out["E"].sum()), out["F"]

    return f
