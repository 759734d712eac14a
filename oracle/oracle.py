"""ctypes wrapper of the FP64 CPU oracle (oracle/nep_oracle.c).

TEST INFRASTRUCTURE: only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  It never imports the
HIP package, and the HIP package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB_PATH = HERE / "libnep_oracle.so"
SRC = HERE / "nep_oracle.c"


class OrcHParams(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_radial", C.c_int32), ("n_angular", C.c_int32),
                ("basis_radial", C.c_int32), ("basis_angular", C.c_int32), ("l_max", C.c_int32),
                ("use_4body", C.c_int32), ("use_5body", C.c_int32), ("n_hidden", C.c_int32),
                ("reserved", C.c_int32), ("rc_radial", C.c_double), ("rc_angular", C.c_double)]


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (plain -O2, OpenMP)."""
    if not force and LIB_PATH.exists() and LIB_PATH.stat().st_mtime >= SRC.stat().st_mtime:
        return LIB_PATH
    tmp = LIB_PATH.with_suffix(".so.tmp")
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-Wno-unused-function", "-o", str(tmp), str(SRC), "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            build()
        L = C.CDLL(str(LIB_PATH))
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        hp = C.POINTER(OrcHParams)
        L.orc_param_count.argtypes = [hp, lp]
        L.orc_descriptor_dim.argtypes = [hp]
        L.orc_basis_eval.argtypes = [C.c_double, C.c_double, C.c_int, dp, dp]
        L.orc_ylm_eval.argtypes = [C.c_int, dp, dp, dp]
        L.orc_pairs_of.argtypes = [C.c_int32, dp, dp, C.c_double, C.c_int32, C.c_int64, ip, dp]
        L.orc_pairs_of.restype = C.c_int64
        L.orc_evaluate.argtypes = [hp, dp, C.c_int32, lp, dp, ip, dp, ip, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_loss_grad.argtypes = [hp, dp, C.c_int32, lp, dp, ip, dp, ip, C.c_int32, dp, dp, dp, dp, C.c_int32,
                                    dp, dp]
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _hp(h) -> OrcHParams:
    d = h if isinstance(h, dict) else h.as_dict()
    return OrcHParams(d["n_species"], d["n_radial"], d["n_angular"], d["basis_radial"], d["basis_angular"],
                      d["l_max"], d["use_4body"], d["use_5body"], d["n_hidden"], 0, d["rc_radial"],
                      d["rc_angular"])


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


def param_count(hp) -> int:
    out = C.c_int64()
    if lib().orc_param_count(C.byref(_hp(hp)), C.byref(out)):
        raise ValueError("invalid hyper-parameters")
    return out.value


def descriptor_dim(hp) -> int:
    return lib().orc_descriptor_dim(C.byref(_hp(hp)))


def basis(r: float, rc: float, B: int):
    Q, dQ = np.zeros(B), np.zeros(B)
    _, pq = _d(Q)
    _, pdq = _d(dQ)
    if lib().orc_basis_eval(float(r), float(rc), int(B), Q.ctypes.data_as(C.POINTER(C.c_double)),
                            dQ.ctypes.data_as(C.POINTER(C.c_double))):
        raise ValueError
    return Q, dQ


def ylm(l_max: int, r):
    K = l_max * l_max + 2 * l_max
    Y, dY = np.zeros(K), np.zeros((K, 3))
    rv, pr = _d(np.asarray(r, dtype=np.float64))
    if lib().orc_ylm_eval(int(l_max), pr, Y.ctypes.data_as(C.POINTER(C.c_double)),
                          dY.ctypes.data_as(C.POINTER(C.c_double))):
        raise ValueError
    return Y, dY


def pairs(pos, cell, rc: float, mode: int = 0):
    """(ij (P,2) int32, r (P,3)) of one configuration."""
    pos, pp = _d(pos)
    cell, pc = _d(np.asarray(cell).reshape(9))
    n = len(pos)
    cnt = lib().orc_pairs_of(n, pp, pc, float(rc), int(mode), 0, None, None)
    if cnt < 0:
        raise RuntimeError("pair build failed")
    ij = np.zeros((max(cnt, 1), 2), dtype=np.int32)
    rv = np.zeros((max(cnt, 1), 3))
    cnt2 = lib().orc_pairs_of(n, pp, pc, float(rc), int(mode), cnt, ij.ctypes.data_as(C.POINTER(C.c_int32)),
                              rv.ctypes.data_as(C.POINTER(C.c_double)))
    assert cnt2 == cnt
    return ij[:cnt], rv[:cnt]


def _pbc(system):
    """(array, pointer) of the system's periodicity, or (None, None) if periodic in all directions."""
    pbc = getattr(system, "pbc", None)
    if pbc is None:
        return None, None
    return _i32(np.asarray(pbc).reshape(-1))


def evaluate(hp, params, system, nbr_mode: int = 2, want_q: bool = False):
    """Return dict with E (n_cfg), F (N,3), V (n_cfg,3,3), Ei (N) and optionally q (N,D).
    Directions the system marks non-periodic (system.pbc) have no images."""
    h = _hp(hp)
    P, pP = _d(params)
    pos, ppos = _d(system.pos)
    spc, pspc = _i32(system.species)
    cells, pcell = _d(np.asarray(system.cells).reshape(-1, 9))
    pb, ppb = _pbc(system)
    off, poff = _i64(system.atom_off)
    n_cfg = len(off) - 1
    N = int(off[-1])
    D = descriptor_dim(hp)
    E, F, V, Ei = np.zeros(n_cfg), np.zeros((N, 3)), np.zeros((n_cfg, 9)), np.zeros(N)
    q = np.zeros((N, D)) if want_q else None
    rc = lib().orc_evaluate(C.byref(h), pP, n_cfg, poff, ppos, pspc, pcell, ppb, int(nbr_mode),
                            E.ctypes.data_as(C.POINTER(C.c_double)), F.ctypes.data_as(C.POINTER(C.c_double)),
                            V.ctypes.data_as(C.POINTER(C.c_double)), Ei.ctypes.data_as(C.POINTER(C.c_double)),
                            q.ctypes.data_as(C.POINTER(C.c_double)) if want_q else None)
    if rc:
        raise RuntimeError(f"orc_evaluate failed ({rc})")
    out = {"E": E, "F": F, "V": V.reshape(n_cfg, 3, 3), "Ei": Ei}
    if want_q:
        out["q"] = q
    return out


def loss_grad(hp, params, system, E_ref, F_ref, V_ref, weights=(1.0, 1.0, 0.1), loss_form: int = 0,
              want_grad: bool = True, nbr_mode: int = 2):
    """Return (parts[4] = total, E, F, V terms, grad or None)."""
    h = _hp(hp)
    P, pP = _d(params)
    pos, ppos = _d(system.pos)
    spc, pspc = _i32(system.species)
    cells, pcell = _d(np.asarray(system.cells).reshape(-1, 9))
    pb, ppb = _pbc(system)
    off, poff = _i64(system.atom_off)
    Er, pEr = _d(E_ref)
    Fr, pFr = _d(np.asarray(F_ref).reshape(-1))
    Vr, pVr = _d(np.asarray(V_ref).reshape(-1))
    w, pw = _d(np.asarray(weights, dtype=np.float64))
    parts = np.zeros(4)
    grad = np.zeros(len(P)) if want_grad else None
    rc = lib().orc_loss_grad(C.byref(h), pP, len(off) - 1, poff, ppos, pspc, pcell, ppb, int(nbr_mode), pEr, pFr, pVr,
                             pw, int(loss_form), parts.ctypes.data_as(C.POINTER(C.c_double)),
                             grad.ctypes.data_as(C.POINTER(C.c_double)) if want_grad else None)
    if rc:
        raise RuntimeError(f"orc_loss_grad failed ({rc})")
    return parts, grad


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (n < 1: the OpenMP default)."""
    lib().orc_set_num_threads(int(n))
