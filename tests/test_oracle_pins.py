"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a value the
paper prints, a closed form, a textbook or library routine, an invariant of
the physics, brute force on a tiny input, or finite differences.
"""
import copy
import math
from pathlib import Path

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

from paper_2607_06969_amd import workloads as W

import loss_hand_case as H

GOLDEN = Path(__file__).resolve().parent / "golden"


# ---------------------------------------------------------------- parameter count

def test_table2_parameter_count(oracle_lib):
    """Sec. 4.1.2 / Table 2: the NEP has 7.9k trainable parameters.

    The readings (zeta = 0..N_basis-1, n counts, l = 1..l_max, ordered species
    pairs, per-element network with own output bias) give 7899.  Plausible
    alternatives (N_basis+1 basis functions, n as a maximum index, l from 0,
    shared network, symmetric species pairs) do not round to 7.9k."""
    printed = float([ln for ln in (GOLDEN / "table2_param_count.txt").read_text().splitlines()
                     if ln and not ln.startswith("#")][0])
    n = oracle_lib.param_count(W.hp_table2())
    assert round(n / 100.0) / 10.0 == printed
    T, nR, nA, B, L, H = 3, 10, 8, 8, 4, 50
    D = nR + L * nA
    alternatives = {
        "basis+1": T * T * (nR + nA) * (B + 1) + T * (H * D + 2 * H + 1),
        "n as index": T * T * ((nR + 1) + (nA + 1)) * B + T * (H * ((nR + 1) + L * (nA + 1)) + 2 * H + 1),
        "l from 0": T * T * (nR + nA) * B + T * (H * (D + nA) + 2 * H + 1),
        "shared mlp": T * T * (nR + nA) * B + (H * D + 2 * H + 1),
        "symmetric pairs": (T * (T + 1) // 2) * (nR + nA) * B + T * (H * D + 2 * H + 1),
    }
    for name, v in alternatives.items():
        assert round(v / 100.0) / 10.0 != printed, name


# ---------------------------------------------------------- basis (Eq. 12-15)

@pytest.mark.parametrize("rc,B", [(6.0, 12), (4.0, 8), (7.0, 8)])
def test_chebyshev_basis_closed_forms(oracle_lib, rc, B):
    rs = np.linspace(0.05, rc - 1e-6, 37)
    for r in rs:
        Q, dQ = oracle_lib.basis(r, rc, B)
        fc = 0.5 * (1 + math.cos(math.pi * r / rc))
        x = 2 * (r / rc - 1) ** 2 - 1
        Tk = np.cos(np.arange(B) * np.arccos(np.clip(x, -1, 1)))  # T_k(x) = cos(k arccos x)
        np.testing.assert_allclose(Q, 0.5 * (Tk + 1) * fc, rtol=1e-12, atol=1e-14)
        h = 1e-6
        Qp, _ = oracle_lib.basis(r + h, rc, B)
        Qm, _ = oracle_lib.basis(r - h, rc, B)
        np.testing.assert_allclose(dQ, (Qp - Qm) / (2 * h), rtol=1e-6, atol=1e-8)
    Q0, _ = oracle_lib.basis(0.0, rc, B)
    np.testing.assert_allclose(Q0, np.ones(B), atol=1e-15)  # x = 1 and f_c = 1 at r = 0
    Qc, dQc = oracle_lib.basis(rc, rc, B)
    assert np.all(Qc == 0) and np.all(dQc == 0)
    Qn, dQn = oracle_lib.basis(rc * (1 - 1e-9), rc, B)  # continuity at the cutoff
    assert np.max(np.abs(Qn)) < 1e-15 and np.max(np.abs(dQn)) < 1e-7


# --------------------------------------------- real spherical harmonics (Eq. 16)

def _sphere_quadrature(nt=24, nphi=48):
    x, w = np.polynomial.legendre.leggauss(nt)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    pts, wts = [], []
    for ct, wt in zip(x, w):
        st = math.sqrt(1 - ct * ct)
        for p in phi:
            pts.append((st * math.cos(p), st * math.sin(p), ct))
            wts.append(wt * 2 * np.pi / nphi)
    return np.array(pts), np.array(wts)


def test_ylm_orthonormal_by_quadrature(oracle_lib):
    pts, wts = _sphere_quadrature()
    Y = np.array([oracle_lib.ylm(4, p)[0] for p in pts])
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(24), atol=1e-12)


def test_ylm_matches_scipy_up_to_sign(oracle_lib):
    """Each real component is +-sqrt(2) Re/Im of scipy's complex Y_l^m (or Y_l^0)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        v = rng.normal(size=3)
        r = v * rng.uniform(0.5, 3.0) / np.linalg.norm(v)
        Y, _ = oracle_lib.ylm(4, r)
        th = math.acos(r[2] / np.linalg.norm(r))
        ph = math.atan2(r[1], r[0])
        idx = 0
        for l in range(1, 5):
            ref = [sph_harm_y(l, 0, th, ph).real]
            for m in range(1, l + 1):
                z = sph_harm_y(l, m, th, ph)
                ref += [math.sqrt(2) * z.real, math.sqrt(2) * z.imag]
            got = Y[idx: idx + 2 * l + 1]
            np.testing.assert_allclose(np.abs(got), np.abs(ref), rtol=1e-10, atol=1e-12)
            idx += 2 * l + 1


def test_ylm_addition_theorem_and_gradient(oracle_lib):
    rng = np.random.default_rng(12)
    for _ in range(20):
        a, b = rng.normal(size=3), rng.normal(size=3)
        Ya, dYa = oracle_lib.ylm(4, a)
        Yb, _ = oracle_lib.ylm(4, b)
        c = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
        idx = 0
        for l in range(1, 5):
            s = Ya[idx: idx + 2 * l + 1] @ Yb[idx: idx + 2 * l + 1]
            assert abs(s - (2 * l + 1) / (4 * np.pi) * eval_legendre(l, c)) < 1e-12
            idx += 2 * l + 1
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (oracle_lib.ylm(4, a + e)[0] - oracle_lib.ylm(4, a - e)[0]) / (2 * h)
            np.testing.assert_allclose(dYa[:, k], fd, rtol=1e-6, atol=1e-8)


# --------------------------------------------------------- neighbours

def _pairset(ij, r):
    return {(int(i), int(j), tuple(np.round(v, 9))) for (i, j), v in zip(ij, r)}


def test_pairs_bruteforce_tiny_numpy(oracle_lib):
    """The oracle's brute force against an independent numpy loop over images."""
    s = W.simple_cubic(n=3, spacing=3.0, sigma=0.2, seed=5)  # 9 A box < 2 rc: many images
    rc = 6.0
    ij, r = oracle_lib.pairs(s.pos, s.cells[0], rc, mode=0)
    H = s.cells[0]
    ref = []
    for i in range(s.n_atoms):
        for j in range(s.n_atoms):
            for a in range(-1, 2):
                for b in range(-1, 2):
                    for c in range(-1, 2):
                        if i == j and a == b == c == 0:
                            continue
                        v = s.pos[j] - s.pos[i] + a * H[0] + b * H[1] + c * H[2]
                        if v @ v < rc * rc:
                            ref.append((i, j, v))
    assert _pairset(ij, r) == _pairset([(i, j) for i, j, _ in ref], [v for _, _, v in ref])


def test_pairs_celllist_equals_bruteforce(oracle_lib):
    s = W.rocksalt_gst(8, seed=21)  # 24 A box, 3 bins per direction at rc = 7
    for rc in (6.0, 7.0):
        a = oracle_lib.pairs(s.pos, s.cells[0], rc, mode=0)
        b = oracle_lib.pairs(s.pos, s.cells[0], rc, mode=1)
        assert len(a[0]) == len(b[0])
        assert _pairset(*a) == _pairset(*b)


# ------------------------------------------------- descriptors (Eq. 11, 16, 17)

def _g(oracle_lib, params, hp, a, b, r, angular):
    """g_n(r) for the species pair (a, b) from the oracle's (pinned) basis."""
    T = hp.n_species
    if angular:
        off = T * T * hp.n_radial * hp.basis_radial
        N, B, rc = hp.n_angular, hp.basis_angular, hp.rc_angular
    else:
        off, N, B, rc = 0, hp.n_radial, hp.basis_radial, hp.rc_radial
    c = params[off + (a * T + b) * N * B: off + (a * T + b + 1) * N * B].reshape(N, B)
    Q, _ = oracle_lib.basis(r, rc, B)
    return c @ Q


def test_three_body_equals_legendre_triple_sum(oracle_lib):
    """Addition theorem: sum_m S_nlm^2 = (2l+1)/(4 pi) sum_jk g_n(r_ij) g_n(r_ik) P_l(cos theta_jik)."""
    hp = W.hp_gst()
    s = W.rocksalt_gst(4, seed=8)
    p = W.random_params(hp, 2010)
    out = oracle_lib.evaluate(hp, p, s, nbr_mode=0, want_q=True)
    ij, rv = oracle_lib.pairs(s.pos, s.cells[0], hp.rc_angular, mode=0)
    for i in (0, 5, 17, 40):
        sel = ij[:, 0] == i
        js, rs = ij[sel, 1], rv[sel]
        d = np.linalg.norm(rs, axis=1)
        G = np.array([_g(oracle_lib, p, hp, s.species[i], s.species[j], dd, True) for j, dd in zip(js, d)])
        U = rs / d[:, None]
        C = np.clip(U @ U.T, -1, 1)
        for l in range(1, 5):
            ref = (2 * l + 1) / (4 * np.pi) * np.einsum("jn,kn,jk->n", G, G, eval_legendre(l, C))
            got = out["q"][i, hp.n_radial + (l - 1) * hp.n_angular: hp.n_radial + l * hp.n_angular]
            np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13)
        # 4-body: brute triple product of the traceless tensors; 5-body identity.
        M = np.einsum("ja,jb->jab", U, U) - np.eye(3) / 3
        ref4 = np.einsum("jn,kn,ln,jab,kbc,lca->n", G, G, G, M, M, M)
        off4 = hp.n_radial + 4 * hp.n_angular
        np.testing.assert_allclose(out["q"][i, off4: off4 + 8], ref4, rtol=1e-10, atol=1e-13)
        q1 = out["q"][i, hp.n_radial: hp.n_radial + 8]
        np.testing.assert_allclose(out["q"][i, off4 + 8: off4 + 16], q1 * q1, rtol=1e-13)
        # radial: Eq. 11 against the pair list at the radial cutoff
        ijR, rR = oracle_lib.pairs(s.pos, s.cells[0], hp.rc_radial, mode=0)
        sR = ijR[:, 0] == i
        refR = sum(_g(oracle_lib, p, hp, s.species[i], s.species[j], np.linalg.norm(v), False)
                   for j, v in zip(ijR[sR, 1], rR[sR]))
        np.testing.assert_allclose(out["q"][i, :hp.n_radial], refR, rtol=1e-12, atol=1e-14)


def _mlp_numpy(hp, params, s, q):
    T, H, D = hp.n_species, hp.n_hidden, hp.dim
    off = T * T * (hp.n_radial * hp.basis_radial + hp.n_angular * hp.basis_angular)
    blk = H * D + 2 * H + 1
    w = params[off + s * blk: off + (s + 1) * blk]
    W0, b0, w1, b1 = w[:H * D].reshape(H, D), w[H * D:H * D + H], w[H * D + H:H * D + 2 * H], w[-1]
    return w1 @ np.tanh(W0 @ q + b0) + b1


def test_dimer_closed_form(oracle_lib):
    """Two atoms in vacuum (large box): q_n = g_n(r), q_nl = (2l+1)/(4 pi) g_n^2,
    4-body = (2/9) g_n^3, 5-body = (3/(4 pi))^2 g_n^4, so E is computable by hand."""
    hp = W.hp_gst()
    p = W.random_params(hp, 2011)
    box = 20.0
    u = np.array([0.3, -0.5, 0.81])
    u /= np.linalg.norm(u)
    for r in (2.3, 3.1, 3.9):
        pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0] + r * u])
        spc = np.array([0, 2], dtype=np.int32)
        s = W.System(pos, spc, np.eye(3)[None] * box, np.array([0, 2]))
        out = oracle_lib.evaluate(hp, p, s, nbr_mode=0, want_q=True)
        for i, (a, b) in enumerate([(0, 2), (2, 0)]):
            gR = _g(oracle_lib, p, hp, a, b, r, False)
            gA = _g(oracle_lib, p, hp, a, b, r, True)
            q = np.concatenate([gR] + [(2 * l + 1) / (4 * np.pi) * gA ** 2 for l in range(1, 5)] +
                               [2.0 / 9.0 * gA ** 3, (3 / (4 * np.pi)) ** 2 * gA ** 4])
            np.testing.assert_allclose(out["q"][i], q, rtol=1e-12, atol=1e-14)
            assert abs(out["Ei"][i] - _mlp_numpy(hp, p, a, q)) < 1e-12
        # the force is -dE/dr along the bond, equal and opposite
        h = 1e-6

        def E_at(rr):
            pp = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0] + rr * u])
            return oracle_lib.evaluate(hp, p, W.System(pp, spc, np.eye(3)[None] * box, np.array([0, 2])),
                                       nbr_mode=0)["E"][0]
        dEdr = (E_at(r + h) - E_at(r - h)) / (2 * h)
        np.testing.assert_allclose(out["F"][1], -dEdr * u, rtol=1e-7, atol=1e-10)
        np.testing.assert_allclose(out["F"][0], dEdr * u, rtol=1e-7, atol=1e-10)


# ------------------------------------------------- forces, virial (Eq. 3, 4)

@pytest.fixture(scope="module")
def small_gst():
    hp = W.hp_gst()
    s = W.rocksalt_gst(4, seed=7)
    p = W.random_params(hp, 2002)
    return hp, s, p


def test_forces_are_minus_energy_gradient(oracle_lib, small_gst):
    hp, s, p = small_gst
    out = oracle_lib.evaluate(hp, p, s, nbr_mode=0)
    rng = np.random.default_rng(3)
    h = 1e-5
    for _ in range(12):
        i, a = int(rng.integers(s.n_atoms)), int(rng.integers(3))
        sp, sm = copy.deepcopy(s), copy.deepcopy(s)
        sp.pos[i, a] += h
        sm.pos[i, a] -= h
        fd = -(oracle_lib.evaluate(hp, p, sp, 0)["E"][0] - oracle_lib.evaluate(hp, p, sm, 0)["E"][0]) / (2 * h)
        assert abs(out["F"][i, a] - fd) <= 1e-7 * max(1.0, abs(fd))
    np.testing.assert_allclose(out["F"].sum(axis=0), 0.0, atol=1e-12)


def test_virial_is_minus_strain_derivative(oracle_lib, small_gst):
    hp, s, p = small_gst
    V = oracle_lib.evaluate(hp, p, s, nbr_mode=0)["V"][0]
    np.testing.assert_allclose(V, V.T, atol=1e-11)
    h = 1e-5
    for a in range(3):
        for b in range(3):
            def E_eps(e):
                sp = copy.deepcopy(s)
                M = np.eye(3)
                M[a, b] += e
                sp.pos = s.pos @ M.T
                sp.cells = s.cells @ M.T
                return oracle_lib.evaluate(hp, p, sp, 0)["E"][0]
            fd = -(E_eps(h) - E_eps(-h)) / (2 * h)
            assert abs(V[a, b] - fd) < 1e-7 * max(1.0, abs(fd))


def test_invariances(oracle_lib, small_gst):
    hp, s, p = small_gst
    ref = oracle_lib.evaluate(hp, p, s, nbr_mode=0)
    # rigid rotation of positions and cell
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    R = R @ np.array([[1, 0, 0], [0, math.cos(0.4), -math.sin(0.4)], [0, math.sin(0.4), math.cos(0.4)]])
    sr = copy.deepcopy(s)
    sr.pos = s.pos @ R.T
    sr.cells = s.cells @ R.T
    o = oracle_lib.evaluate(hp, p, sr, nbr_mode=0)
    assert abs(o["E"][0] - ref["E"][0]) < 1e-10
    np.testing.assert_allclose(o["F"], ref["F"] @ R.T, atol=1e-10)
    np.testing.assert_allclose(o["V"][0], R @ ref["V"][0] @ R.T, atol=1e-10)
    # translation, and moving atoms by lattice vectors
    st = copy.deepcopy(s)
    st.pos = s.pos + np.array([0.37, -1.1, 2.9])
    st.pos[3] += s.cells[0][1]
    st.pos[9] -= s.cells[0][0] + s.cells[0][2]
    o = oracle_lib.evaluate(hp, p, st, nbr_mode=0)
    assert abs(o["E"][0] - ref["E"][0]) < 1e-10
    np.testing.assert_allclose(o["F"], ref["F"], atol=1e-10)
    np.testing.assert_allclose(o["V"], ref["V"], atol=1e-10)
    # permutation of atoms (species carried along)
    perm = np.random.default_rng(4).permutation(s.n_atoms)
    sp = copy.deepcopy(s)
    sp.pos, sp.species = s.pos[perm], s.species[perm]
    o = oracle_lib.evaluate(hp, p, sp, nbr_mode=0)
    assert abs(o["E"][0] - ref["E"][0]) < 1e-10
    np.testing.assert_allclose(o["F"], ref["F"][perm], atol=1e-10)
    # swapping the species labels of two atoms of the same species changes nothing
    same = np.where(s.species == s.species[0])[0][:2]
    sw = copy.deepcopy(s)
    sw.pos[same[0]], sw.pos[same[1]] = s.pos[same[1]].copy(), s.pos[same[0]].copy()
    o = oracle_lib.evaluate(hp, p, sw, nbr_mode=0)
    assert abs(o["E"][0] - ref["E"][0]) < 1e-10


def test_supercell_extensivity(oracle_lib):
    hp = W.hp_gst()
    s = W.rocksalt_gst(4, seed=9)
    p = W.random_params(hp, 2012)
    ref = oracle_lib.evaluate(hp, p, s, nbr_mode=0)
    H = s.cells[0]
    shifts = [a * H[0] + b * H[1] + c * H[2] for a in range(2) for b in range(2) for c in range(2)]
    big = W.System(np.concatenate([s.pos + v for v in shifts]), np.tile(s.species, 8), (2 * H)[None],
                   np.array([0, 8 * s.n_atoms]))
    o = oracle_lib.evaluate(hp, p, big, nbr_mode=1)
    assert abs(o["E"][0] - 8 * ref["E"][0]) < 1e-9
    np.testing.assert_allclose(o["V"][0], 8 * ref["V"][0], atol=1e-9)
    np.testing.assert_allclose(o["F"], np.tile(ref["F"], (8, 1)), atol=1e-10)


def test_perfect_lattice_symmetry(oracle_lib):
    """A perfect simple-cubic single-element lattice: every force vanishes and
    the virial is isotropic."""
    hp = W.hp_small_single()
    s = W.simple_cubic(n=4, spacing=3.125, sigma=0.0, seed=1)  # binary-exact sites
    p = W.random_params(hp, 2013)
    o = oracle_lib.evaluate(hp, p, s, nbr_mode=0)
    np.testing.assert_allclose(o["F"], 0.0, atol=1e-12)
    V = o["V"][0]
    np.testing.assert_allclose(V - np.diag(np.diag(V)), 0.0, atol=1e-11)
    np.testing.assert_allclose(np.diag(V), V[0, 0], atol=1e-11)


# ------------------------------------------------- loss and parameter gradient

def test_loss_gradient_finite_differences(oracle_lib):
    """Analytic dL/dtheta against central differences on 20 seeded parameters,
    on a batch of two uneven cells, for both loss forms."""
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=2, n_min=64, n_max=90, seed=31)
    p = W.random_params(hp, SEED := 3001)
    Er, Fr, Vr = W.synthetic_labels(np.diff(s.atom_off), 6)
    rng = np.random.default_rng(SEED)
    idx = np.concatenate([rng.choice(hp.n_params(), 14, replace=False), [0, 865, 1729, 1800, 5000, 10430]])
    for form in (0, 1):
        parts, g = oracle_lib.loss_grad(hp, p, s, Er, Fr, Vr, loss_form=form, nbr_mode=0)
        scale = np.sqrt(np.mean(g ** 2))
        for k in idx:
            h = 1e-5
            pp, pm = p.copy(), p.copy()
            pp[k] += h
            pm[k] -= h
            lp, _ = oracle_lib.loss_grad(hp, pp, s, Er, Fr, Vr, loss_form=form, want_grad=False, nbr_mode=0)
            lm, _ = oracle_lib.loss_grad(hp, pm, s, Er, Fr, Vr, loss_form=form, want_grad=False, nbr_mode=0)
            fd = (lp[0] - lm[0]) / (2 * h)
            assert abs(g[k] - fd) <= 1e-7 * max(abs(fd), scale), (form, k, g[k], fd)


def test_loss_gradient_all_parameters_tiny(oracle_lib):
    """Every component of dL/dtheta on a tiny periodic system by brute-force
    central differences (single-element model)."""
    hp = W.hp_small_single()
    hp.use_4body = 1
    hp.use_5body = 1
    s = W.simple_cubic(n=4, spacing=3.1, sigma=0.15, seed=40)
    p = W.random_params(hp, 2014)
    Er, Fr, Vr = W.synthetic_labels([s.n_atoms], 7)
    parts, g = oracle_lib.loss_grad(hp, p, s, Er, Fr, Vr, nbr_mode=0)
    h = 1e-5
    fd = np.zeros_like(p)
    for k in range(len(p)):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd[k] = (oracle_lib.loss_grad(hp, pp, s, Er, Fr, Vr, want_grad=False, nbr_mode=0)[0][0] -
                 oracle_lib.loss_grad(hp, pm, s, Er, Fr, Vr, want_grad=False, nbr_mode=0)[0][0]) / (2 * h)
    scale = np.sqrt(np.mean(fd ** 2))
    assert np.max(np.abs(g - fd)) < 1e-6 * scale


def test_loss_zero_at_own_labels(oracle_lib):
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=2, n_min=64, n_max=80, seed=32)
    p = W.random_params(hp, 2015)
    ref = oracle_lib.evaluate(hp, p, s, nbr_mode=0)
    parts, g = oracle_lib.loss_grad(hp, p, s, ref["E"], ref["F"], ref["V"].reshape(-1, 9), nbr_mode=0)
    assert abs(parts[0]) < 1e-24
    assert np.max(np.abs(g)) < 1e-12


@pytest.mark.parametrize("form", [0, 1])
def test_loss_hand_evaluated(oracle_lib, form):
    """Loss parts of both forms (the mean-squared reading and Eq. 19-21 per
    configuration) against values worked out by hand above, on two
    configurations of different size, so that any wrong normalisation (N_c
    against sum N_c, B against 1, 3 or 9 dropped) changes the numbers; and the
    energy seed through the one gradient entry it alone determines (b1)."""
    hp, p = H.constant_energy_model()
    s = H.two_config_batch()
    case = H.FORM0 if form == 0 else H.FORM1
    parts, g = oracle_lib.loss_grad(hp, p, s, H.E_REF, H.F_REF, H.V_REF, weights=case["w"],
                                    loss_form=form, nbr_mode=0)
    want = case["parts"]
    np.testing.assert_allclose(parts[1:], want, rtol=1e-14, atol=0)
    np.testing.assert_allclose(parts[0], sum(want), rtol=1e-14)
    np.testing.assert_allclose(g[-1], case["db1"], rtol=1e-13)


# ---------------------------------------------------- non-periodic directions

def _cell_with_vacuum(s, axes, factor=3.0):
    """The same atoms in a cell whose lattice vectors along `axes` are
    `factor` times longer: images along those axes are then farther than any
    cutoff, so the system is effectively not periodic there."""
    cells = s.cells.copy()
    for a in axes:
        cells[0, a] *= factor
    return W.System(s.pos.copy(), s.species.copy(), cells, s.atom_off.copy())


@pytest.mark.parametrize("pbc,axes", [((0, 0, 0), (0, 1, 2)), ((1, 1, 0), (2,)), ((0, 1, 1), (0,))])
def test_non_periodic_directions_equal_vacuum(oracle_lib, pbc, axes):
    """A direction marked non-periodic has no images: E, F and V equal those of
    the same atoms in a cell padded with vacuum along that direction (brute
    force over images in both)."""
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=1, n_min=140, n_max=140, seed=41)
    p = W.random_params(hp, 2041)
    s.pbc = np.array([pbc], dtype=np.int32)
    got = oracle_lib.evaluate(hp, p, s, nbr_mode=0)
    ref = oracle_lib.evaluate(hp, p, _cell_with_vacuum(s, axes), nbr_mode=0)
    periodic = oracle_lib.evaluate(hp, p, W.System(s.pos, s.species, s.cells, s.atom_off), nbr_mode=0)
    np.testing.assert_allclose(got["E"], ref["E"], rtol=1e-13)
    np.testing.assert_allclose(got["F"], ref["F"], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(got["V"], ref["V"], rtol=1e-11, atol=1e-12)
    # and it differs from the fully periodic system (atoms near the faces interact across them there)
    assert abs(got["E"][0] - periodic["E"][0]) > 1e-6


def test_cluster_conserves_momentum_and_angular_momentum(oracle_lib):
    """An isolated cluster (no periodic direction): sum_i F_i = 0, sum_i r_i x F_i = 0
    and a symmetric virial (translation and rotation invariance of Eq. 1)."""
    hp = W.hp_gst()
    s = W.amorphous_batch(n_cfg=1, n_min=120, n_max=120, seed=42)
    s.pbc = np.zeros((1, 3), dtype=np.int32)
    out = oracle_lib.evaluate(hp, W.random_params(hp, 2042), s, nbr_mode=0)
    F = out["F"]
    scale = np.abs(F).max()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale * len(F)
    torque = np.cross(s.pos, F).sum(axis=0)
    assert np.abs(torque).max() < 1e-11 * scale * len(F) * np.abs(s.pos).max()
    V = out["V"][0]
    np.testing.assert_allclose(V, V.T, atol=1e-11 * np.abs(V).max())
