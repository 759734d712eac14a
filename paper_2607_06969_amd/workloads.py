"""Seeded synthetic inputs for the NEP evaluation path.

This module generates positions, species, cells, parameters and velocities.
It holds none of the potential's arithmetic (no basis, descriptor, network,
force or loss code): it is shared by the HIP path's tests and benchmarks and
by the FP64 oracle's tests, which is the only thing the two sides share.

Every generator works in float64, wraps positions into the cell, and then
rounds positions and cell entries to float32, so that a float32 consumer and a
float64 consumer see exactly the same numbers.

Workload shapes follow the Ge-Sb-Te systems of the paper (Sec. 3.2 and
Sec. 4: a cubic Ge2Sb2Te5-like supercell with random occupation, crystalline
rocksalt and amorphous densities).  The paper's own dataset is not available,
so seeded synthetic cells of the same composition and density stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, field

import numpy as np

# Species indices used throughout: Ge = 0, Sb = 1, Te = 2.
GE, SB, TE = 0, 1, 2
# Standard atomic weights (u) for Ge, Sb, Te.
MASSES_GST = (72.630, 121.760, 127.60)
# Boltzmann constant in eV/K.
KB_EV = 8.617333262e-5
# 1 eV/(A*u) expressed in A/fs^2.
ACC_UNIT = 9.648533212e-3

SEED_POS = 1000
SEED_PARAM = 2000
SEED_TEACHER = 3000
SEED_STUDENT = 3001
SEED_VEL = 4000


@dataclass
class HParams:
    """NEP hyper-parameters (Sec. 2.3 notation).

    n_radial / n_angular: number of radial / angular functions (n_max^radial,
    n_max^angular read as counts); basis_radial / basis_angular: number of
    Chebyshev basis functions N_basis; l_max: highest degree of the three-body
    term (l = 1..l_max); use_4body / use_5body: extra angular invariants;
    n_hidden: N_neurons; rc_radial / rc_angular: cutoffs r_max in Angstrom.
    """

    n_species: int
    n_radial: int
    n_angular: int
    basis_radial: int
    basis_angular: int
    l_max: int
    use_4body: int
    use_5body: int
    n_hidden: int
    rc_radial: float
    rc_angular: float

    def as_dict(self):
        return asdict(self)

    @property
    def dim(self) -> int:
        """Descriptor length D."""
        d = self.n_radial + self.l_max * self.n_angular
        d += self.n_angular if self.use_4body else 0
        d += self.n_angular if self.use_5body else 0
        return d

    def n_params(self) -> int:
        t = self.n_species
        c = t * t * (self.n_radial * self.basis_radial + self.n_angular * self.basis_angular)
        mlp = self.n_hidden * self.dim + 2 * self.n_hidden + 1
        return c + t * mlp


def hp_small_single() -> HParams:
    """Single-element model of the 64-atom cubic test cell."""
    return HParams(1, 4, 4, 8, 8, 4, 0, 0, 30, 6.0, 4.0)


def hp_gst() -> HParams:
    """Three-species Ge-Sb-Te model with 4- and 5-body terms (D = 56)."""
    return HParams(3, 8, 8, 12, 12, 4, 1, 1, 50, 6.0, 4.0)


def hp_table2() -> HParams:
    """The NEP of the paper's Table 2 (Sec. 4.1.2): 7.9k parameters."""
    return HParams(3, 10, 8, 8, 8, 4, 0, 0, 50, 7.0, 5.0)


def random_params(hp: HParams, seed: int, std: float = 0.1) -> np.ndarray:
    """Parameters drawn from N(0, std^2), rounded to float32, returned as float64."""
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, std, size=hp.n_params())
    return p.astype(np.float32).astype(np.float64)


@dataclass
class System:
    """A batch of periodic configurations in the user's atom order.

    pos: (N, 3) float64 holding float32-representable values, wrapped into
    the cell; species: (N,) int32; cells: (n_cfg, 3, 3) float64 whose rows are
    the lattice vectors (float32-representable); atom_off: (n_cfg + 1,) int64;
    pbc: (n_cfg, 3) int32 periodicity of each lattice direction, or None for
    periodic in all three (along a non-periodic direction the atoms lie inside
    the cell and have no images).
    """

    pos: np.ndarray
    species: np.ndarray
    cells: np.ndarray
    atom_off: np.ndarray
    meta: dict = field(default_factory=dict)
    pbc: np.ndarray | None = None

    def pbc_array(self) -> np.ndarray:
        if self.pbc is None:
            return np.ones((self.n_cfg, 3), dtype=np.int32)
        return np.ascontiguousarray(np.asarray(self.pbc, dtype=np.int32).reshape(self.n_cfg, 3))

    @property
    def n_atoms(self) -> int:
        return int(self.atom_off[-1])

    @property
    def n_cfg(self) -> int:
        return len(self.atom_off) - 1

    def config(self, c: int) -> "System":
        a, b = int(self.atom_off[c]), int(self.atom_off[c + 1])
        return System(self.pos[a:b].copy(), self.species[a:b].copy(), self.cells[c:c + 1].copy(),
                      np.array([0, b - a], dtype=np.int64), dict(self.meta),
                      None if self.pbc is None else self.pbc_array()[c:c + 1].copy())


def _round_cell(cell: np.ndarray) -> np.ndarray:
    return np.asarray(cell, dtype=np.float64).astype(np.float32).astype(np.float64)


def _wrap_round(pos: np.ndarray, cell: np.ndarray) -> np.ndarray:
    """Wrap into [0, 1) fractional coordinates, then round to float32.

    The rounded value is checked again so that no coordinate lands on the
    upper face of the cell after rounding."""
    inv = np.linalg.inv(cell)
    frac = pos @ inv
    frac -= np.floor(frac)
    out = (frac @ cell).astype(np.float32).astype(np.float64)
    frac2 = out @ inv
    bad = (frac2 >= 1.0) | (frac2 < 0.0)
    if np.any(bad):
        frac2 = np.where(frac2 >= 1.0, 0.0, frac2)
        frac2 = np.where(frac2 < 0.0, 0.0, frac2)
        out = (frac2 @ cell).astype(np.float32).astype(np.float64)
    return out


def simple_cubic(n: int = 4, spacing: float = 3.1, sigma: float = 0.1, seed: int = SEED_POS + 1,
                 species_count: int = 1) -> System:
    """n^3 simple-cubic lattice with Gaussian displacements (std sigma per component)."""
    rng = np.random.default_rng(seed)
    g = np.arange(n, dtype=np.float64) * spacing
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    cell = _round_cell(np.eye(3) * n * spacing)
    pos = _wrap_round(pos, cell)
    species = rng.integers(0, species_count, size=len(pos)).astype(np.int32) if species_count > 1 \
        else np.zeros(len(pos), dtype=np.int32)
    return System(pos, species, cell[None], np.array([0, len(pos)], dtype=np.int64),
                  {"kind": "simple_cubic", "n": n, "spacing": spacing, "sigma": sigma, "seed": seed})


def rocksalt_gst(n: int, a: float = 6.0, sigma: float = 0.15, seed: int = SEED_POS + 2,
                 frac=(0.4, 0.4, 0.2)) -> System:
    """Rocksalt-derived Ge-Sb-Te cell of n^3 sites (n even), site spacing a/2.

    Te occupies the sites with (i + j + k) even; the cation sites receive exact
    counts of Ge / Sb / vacancy in the ratio `frac` by a seeded permutation.
    Displacements are Gaussian with std sigma per component."""
    if n % 2:
        raise ValueError("rocksalt cells need an even number of sites per side")
    rng = np.random.default_rng(seed)
    h = a / 2.0
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    anion = ((i + j + k) % 2) == 0
    n_cat = int((~anion).sum())
    n_ge = int(math.floor(frac[0] * n_cat + 0.5))
    n_sb = int(math.floor(frac[1] * n_cat + 0.5))
    lab = np.full(n_cat, -1, dtype=np.int32)
    lab[:n_ge] = GE
    lab[n_ge:n_ge + n_sb] = SB
    lab = lab[rng.permutation(n_cat)]
    species = np.full(n ** 3, TE, dtype=np.int32)
    species[~anion] = lab
    keep = species >= 0
    pos = np.stack([i, j, k], axis=1).astype(np.float64) * h
    pos = pos[keep]
    species = species[keep]
    pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    cell = _round_cell(np.eye(3) * n * h)
    pos = _wrap_round(pos, cell)
    return System(pos, species, cell[None], np.array([0, len(pos)], dtype=np.int64),
                  {"kind": "rocksalt_gst", "sites_per_side": n, "a": a, "sigma": sigma, "seed": seed})


def _rsa_cell(n_atoms: int, box: float, rmin: float, rng) -> np.ndarray:
    """Random sequential addition of n_atoms points in a periodic cube of side
    `box` with minimum image distance rmin (a simple hard-sphere fluid)."""
    nb = max(1, int(box // rmin))
    w = box / nb
    grid: dict = {}
    pts = []
    tries = 0
    while len(pts) < n_atoms:
        tries += 1
        if tries > 200000 * n_atoms:
            raise RuntimeError("random sequential addition did not converge")
        p = rng.random(3) * box
        c = tuple((p // w).astype(int) % nb)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((c[0] + dx) % nb, (c[1] + dy) % nb, (c[2] + dz) % nb)
                    for q in grid.get(key, ()):
                        d = p - q
                        d -= box * np.round(d / box)
                        if d @ d < rmin * rmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts.append(p)
            grid.setdefault(c, []).append(p)
    return np.array(pts)


def amorphous_batch(n_cfg: int = 256, n_min: int = 64, n_max: int = 512, density: float = 0.033,
                    rmin: float = 2.2, composition=(2, 2, 5), seed: int = SEED_POS + 4) -> System:
    """Batch of amorphous-like Ge-Sb-Te cells with uneven atom counts.

    N_c ~ U{n_min..n_max}; cubic side (N_c / density)^(1/3); species counts in
    the ratio `composition`; positions by random sequential addition with
    minimum pair distance rmin."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_min, n_max + 1, size=n_cfg)
    pos_all, spc_all, cells = [], [], []
    comp = np.asarray(composition, dtype=np.float64)
    comp = comp / comp.sum()
    for nc in sizes:
        nc = int(nc)
        box = float(np.float32((nc / density) ** (1.0 / 3.0)))
        p = _rsa_cell(nc, box, rmin, rng)
        cnt = np.floor(comp * nc + 0.5).astype(int)
        cnt[-1] = nc - cnt[:-1].sum()
        s = np.concatenate([np.full(c, t, dtype=np.int32) for t, c in enumerate(cnt)])
        s = s[rng.permutation(nc)]
        cell = _round_cell(np.eye(3) * box)
        pos_all.append(_wrap_round(p, cell))
        spc_all.append(s)
        cells.append(cell)
    off = np.zeros(n_cfg + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return System(np.concatenate(pos_all), np.concatenate(spc_all), np.stack(cells), off,
                  {"kind": "amorphous_batch", "n_cfg": n_cfg, "n_min": n_min, "n_max": n_max,
                   "density": density, "rmin": rmin, "seed": seed})


def mixed_size_cells(n_cells: int = 64, n_min: float = 1e3, n_max: float = 2e5,
                     seed: int = SEED_POS + 5) -> System:
    """Independent rocksalt Ge-Sb-Te cells with log-uniform atom counts.

    Sites per side: the even integer nearest (N / 0.9)^(1/3)."""
    rng = np.random.default_rng(seed)
    target = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_cells))
    parts = []
    for c, nt in enumerate(target):
        ns = max(2, int(2 * round((nt / 0.9) ** (1.0 / 3.0) / 2.0)))
        parts.append(rocksalt_gst(ns, seed=seed * 1000 + c))
    return concat_systems(parts, {"kind": "mixed_size_cells", "n_cells": n_cells, "seed": seed})


def concat_systems(parts, meta=None) -> System:
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([p.n_atoms for p in parts])
    pbc = None if all(p.pbc is None for p in parts) else np.concatenate([p.pbc_array() for p in parts])
    return System(np.concatenate([p.pos for p in parts]), np.concatenate([p.species for p in parts]),
                  np.concatenate([p.cells for p in parts]), off, dict(meta or {}), pbc)


def maxwell_boltzmann(species: np.ndarray, masses, temperature: float, seed: int = SEED_VEL) -> np.ndarray:
    """Velocities (A/fs) drawn at `temperature` K, zero net momentum, float32-rounded."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)[species]
    # k_B T / m in eV/u -> (A/fs)^2 via ACC_UNIT (1 eV/u = ACC_UNIT A^2/fs^2).
    s = np.sqrt(KB_EV * temperature / m * ACC_UNIT)
    v = rng.normal(0.0, 1.0, size=(len(species), 3)) * s[:, None]
    p = (m[:, None] * v).sum(axis=0)
    v -= p / m.sum()
    return v.astype(np.float32).astype(np.float64)


def synthetic_labels(n_cfg_atoms, seed: int, e_scale=1.0, f_scale=1.0, v_scale=1.0):
    """Random label arrays (energy per config, forces, virial) of the right shapes.

    Used where a test needs labels but not a physical teacher."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(n_cfg_atoms)
    n_cfg = len(sizes)
    e = rng.normal(0.0, e_scale, size=n_cfg) * sizes
    f = rng.normal(0.0, f_scale, size=(int(sizes.sum()), 3)).astype(np.float32).astype(np.float64)
    v = rng.normal(0.0, v_scale, size=(n_cfg, 9)) * sizes[:, None]
    return e, f, v
