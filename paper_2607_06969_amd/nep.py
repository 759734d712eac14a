"""Python face of the HIP NEP library: model handle, batch evaluation,
training gradient, molecular dynamics and a torch.autograd.Function.

Tensors live on the GPU (torch is used for device memory and streams only);
per-batch metadata (atom offsets, cells) are host arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import HParams, _host_f64, _host_i64, _ptr, _stream, check, load


def _dev(t, dtype):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    return t


class Batch:
    """A batch of configurations resident on the GPU.

    pos: (N, 3) float32 CUDA tensor; species: (N,) int32 CUDA tensor;
    atom_off: host int64 (n_cfg + 1); cells: host float64 (n_cfg, 3, 3);
    pbc: host int (n_cfg, 3) of 0/1 per lattice vector, or None (periodic
    in every direction)."""

    def __init__(self, pos, species, atom_off, cells, pbc=None):
        self.pos = _dev(pos, torch.float32)
        self.species = _dev(species, torch.int32)
        self.atom_off = np.ascontiguousarray(np.asarray(atom_off, dtype=np.int64))
        self.cells = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 9))
        self.n_cfg = len(self.atom_off) - 1
        self.n_atoms = int(self.atom_off[-1])
        self.pbc = None
        if pbc is not None:
            self.pbc = np.ascontiguousarray(np.asarray(pbc, dtype=np.int32).reshape(-1, 3))
            if self.pbc.shape[0] != self.n_cfg:
                raise ValueError("pbc must have one row of three flags per configuration")

    @classmethod
    def from_system(cls, system, device="cuda"):
        return cls(torch.as_tensor(system.pos, dtype=torch.float32, device=device).contiguous(),
                   torch.as_tensor(system.species, dtype=torch.int32, device=device).contiguous(),
                   system.atom_off, system.cells, getattr(system, "pbc", None))

    def _meta(self):
        """Host arrays to keep alive for the call, and the pointers to pass
        (pbc: NULL when every direction is periodic)."""
        off, poff = _host_i64(self.atom_off)
        cel, pcel = _host_f64(self.cells)
        ppbc = None if self.pbc is None else self.pbc.ctypes.data_as(C.POINTER(C.c_int32))
        return (off, cel, self.pbc), poff, pcel, ppbc


class NepModel:
    """NEP model handle on the current GPU."""

    def __init__(self, hp, params=None):
        self.hp = hp
        self._hp = HParams.from_any(hp)
        h = C.c_void_p()
        check(load().nepmi_model_create(C.byref(self._hp), C.byref(h)))
        self._h = h
        self.n_params = _lib.param_count(hp)
        self.dim = _lib.descriptor_dim(hp)
        if params is not None:
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().nepmi_model_destroy(h)
            except Exception:
                pass
            self._h = None

    def set_params(self, params):
        p = torch.as_tensor(params, dtype=torch.float32, device="cuda").contiguous()
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.numel()}")
        self._params = p
        check(load().nepmi_model_set_params(self._h, _ptr(p), _stream()))

    def reuse_lists(self, enable=True):
        """Keep neighbour lists between calls on an unchanged batch (same tensors, same contents);
        the caller guarantees the positions and species have not changed (fixed training sets)."""
        check(load().nepmi_model_reuse_lists(self._h, 1 if enable else 0))

    def compute(self, batch: Batch, atom_energy=False, atom_virial=False, noalloc=False):
        """Energy (n_cfg,) float64, forces (N, 3) float32, virial (n_cfg, 3, 3) float64.
        noalloc: use the allocation-free entry point (work space in the library's
        static per-GPU array; the result tensors are still allocated here)."""
        dev = batch.pos.device
        E = torch.empty(batch.n_cfg, dtype=torch.float64, device=dev)
        F = torch.empty(batch.n_atoms, 3, dtype=torch.float32, device=dev)
        V = torch.empty(batch.n_cfg, 9, dtype=torch.float64, device=dev)
        Ea = torch.empty(batch.n_atoms, dtype=torch.float32, device=dev) if atom_energy else None
        Wa = torch.empty(batch.n_atoms, 9, dtype=torch.float32, device=dev) if atom_virial else None
        keep, poff, pcel, ppbc = batch._meta()
        fn = load().nepmi_compute_noalloc if noalloc else load().nepmi_compute
        check(fn(self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(batch.species),
                 _ptr(E), _ptr(F), _ptr(V), _ptr(Ea), _ptr(Wa), _stream()))
        out = {"E": E, "F": F, "V": V.view(-1, 3, 3)}
        if atom_energy:
            out["Ei"] = Ea
        if atom_virial:
            out["Wi"] = Wa.view(-1, 3, 3)
        return out

    def descriptors(self, batch: Batch):
        q = torch.empty(batch.n_atoms, self.dim, dtype=torch.float32, device=batch.pos.device)
        keep, poff, pcel, ppbc = batch._meta()
        check(load().nepmi_descriptors(self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(batch.species),
                                       _ptr(q), _stream()))
        return q

    def neighbors(self, batch: Batch, which=0, cap=128):
        """(count (N,), nbr (N, cap) caller indices, rvec (N, cap, 3)) of the radial (0) or angular (1) list,
        the angular part of the evaluation list (2), or its reverse index in place of the indices (3)."""
        dev = batch.pos.device
        cnt = torch.empty(batch.n_atoms, dtype=torch.int32, device=dev)
        nb = torch.full((batch.n_atoms, cap), -1, dtype=torch.int32, device=dev)
        rv = torch.zeros(batch.n_atoms, cap, 3, dtype=torch.float32, device=dev)
        keep, poff, pcel, ppbc = batch._meta()
        check(load().nepmi_neighbors(self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(batch.species),
                                     int(which), int(cap), _ptr(cnt), _ptr(nb), _ptr(rv), _stream()))
        return cnt, nb, rv

    def autotune(self, batch: Batch):
        """Time every kernel variant on this batch and keep the fastest; returns (desc, force)."""
        ch = (C.c_int32 * 2)()
        keep, poff, pcel, ppbc = batch._meta()
        check(load().nepmi_autotune(self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(batch.species), ch,
                                    _stream()))
        return int(ch[0]), int(ch[1])

    def set_variants(self, desc: int, force: int):
        check(load().nepmi_set_variants(self._h, int(desc), int(force)))

    def variants(self):
        d, f = C.c_int32(), C.c_int32()
        check(load().nepmi_get_variants(self._h, C.byref(d), C.byref(f)))
        return d.value, f.value

    def set_gather_variant(self, v: int):
        """Pin the block size of the force gather (0..3: 256, 128, 512, 1024 threads)."""
        check(load().nepmi_set_gather_variant(self._h, int(v)))

    def gather_variant(self):
        g = C.c_int32()
        check(load().nepmi_get_gather_variant(self._h, C.byref(g)))
        return g.value

    def backward_params(self, batch: Batch, ebar, lam, mu):
        """sum_c ebar_c dE_c/dtheta + sum_i lam_i.dF_i/dtheta + sum_c mu_c:dV_c/dtheta (float32, P).
        Needs a preceding compute() on the same batch."""
        g = torch.empty(self.n_params, dtype=torch.float32, device=batch.pos.device)
        keep, poff, pcel, ppbc = batch._meta()
        check(load().nepmi_backward_params(
            self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(batch.species),
            _ptr(_dev(ebar.contiguous(), torch.float64)), _ptr(_dev(lam.contiguous(), torch.float32)),
            _ptr(_dev(mu.reshape(-1, 9).contiguous(), torch.float64)), _ptr(g), _stream()))
        return g

    def _f64_inputs(self, batch: Batch, params, pos):
        P = _dev(torch.as_tensor(params).contiguous(), torch.float64)
        if P.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {P.numel()}")
        X = batch.pos.double().contiguous() if pos is None else _dev(pos.contiguous(), torch.float64)
        return P, X

    def compute64(self, batch: Batch, params, pos=None, atom_energy=False):
        """Float64 variant (every operator has float32 and float64 forms, Sec. 3.2): energy (n_cfg,),
        forces (N, 3) and virial (n_cfg, 3, 3), all float64, at the float64 parameter vector `params`
        (CUDA tensor, P).  Positions default to the batch's, widened to float64."""
        P, X = self._f64_inputs(batch, params, pos)
        dev = batch.pos.device
        E = torch.empty(batch.n_cfg, dtype=torch.float64, device=dev)
        F = torch.empty(batch.n_atoms, 3, dtype=torch.float64, device=dev)
        V = torch.empty(batch.n_cfg, 9, dtype=torch.float64, device=dev)
        Ea = torch.empty(batch.n_atoms, dtype=torch.float64, device=dev) if atom_energy else None
        keep, poff, pcel, ppbc = batch._meta()
        check(load().nepmi_compute_f64(self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(X), _ptr(batch.species), _ptr(P),
                                       _ptr(E), _ptr(F), _ptr(V), _ptr(Ea), _stream()))
        out = {"E": E, "F": F, "V": V.view(-1, 3, 3)}
        if atom_energy:
            out["Ei"] = Ea
        return out

    def backward_params64(self, batch: Batch, params, ebar, lam, mu, pos=None):
        """Float64 twin of backward_params, at the float64 parameter vector `params`."""
        P, X = self._f64_inputs(batch, params, pos)
        g = torch.empty(self.n_params, dtype=torch.float64, device=batch.pos.device)
        keep, poff, pcel, ppbc = batch._meta()
        check(load().nepmi_backward_params_f64(
            self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(X), _ptr(batch.species), _ptr(P),
            _ptr(_dev(ebar.contiguous(), torch.float64)), _ptr(_dev(lam.reshape(-1, 3).contiguous(), torch.float64)),
            _ptr(_dev(mu.reshape(-1, 9).contiguous(), torch.float64)), _ptr(g), _stream()))
        return g

    def loss_grad(self, batch: Batch, E_ref, F_ref, V_ref, weights=(1.0, 1.0, 0.1), loss_form=0, grad=True):
        """Loss parts (4,) float64 on the GPU and the gradient (P,) float32 (or None)."""
        dev = batch.pos.device
        loss = torch.empty(4, dtype=torch.float64, device=dev)
        g = torch.empty(self.n_params, dtype=torch.float32, device=dev) if grad else None
        keep, poff, pcel, ppbc = batch._meta()
        w, pw = _host_f64(weights)
        check(load().nepmi_loss_grad(
            self._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(batch.species),
            _ptr(_dev(E_ref, torch.float64)), _ptr(_dev(F_ref, torch.float32)),
            _ptr(_dev(V_ref.reshape(-1, 9).contiguous(), torch.float64)), pw, int(loss_form), _ptr(loss), _ptr(g),
            _stream()))
        return loss, g


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Sec. 3.3.1) in place on float32 CUDA tensors; t >= 1."""
    for x in (params, grad, m, v):
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous() or x.numel() != params.numel():
            raise ValueError("adam_step needs contiguous float32 CUDA tensors of one size")
    check(load().nepmi_adam_step(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr),
                                 float(beta1), float(beta2), float(eps), _stream()))


def lr_schedule(step, warmup_steps, total_steps, lr_start, lr_end, start_factor=1e-4):
    """Learning rate at 0-based step (Sec. 3.3.2): linear warmup, then cosine annealing."""
    out = C.c_double()
    check(load().nepmi_lr_schedule(int(step), int(warmup_steps), int(total_steps), float(lr_start), float(lr_end),
                                   float(start_factor), C.byref(out)))
    return out.value


def loss_weights(lr, lr_start, w_start, w_end, normalised=True):
    """Energy, force, virial loss weights at learning rate lr (Sec. 3.3.3)."""
    a, b, w = (C.c_double * 3)(*w_start), (C.c_double * 3)(*w_end), (C.c_double * 3)()
    check(load().nepmi_loss_weights(float(lr), float(lr_start), a, b, 1 if normalised else 0, w))
    return tuple(w)


class Trainer:
    """The training loop of Sec. 3.3 on one batch source: each step computes
    the loss of Eq. 18-21 with the step's dynamic weights and its parameter
    gradient, then one Adam step at the scheduled learning rate.  Parameters,
    moments and gradient stay on the GPU."""

    def __init__(self, model: NepModel, total_steps, warmup_steps, lr_start=1e-3, lr_end=1e-5,
                 w_start=(1.0, 1.0, 0.1), w_end=(1.0, 1.0, 0.1), normalised=True, loss_form=1,
                 betas=(0.9, 0.999), eps=1e-8, reuse_lists=False):
        """reuse_lists: the batches passed to step() are fixed configurations whose tensors are never
        modified, so neighbour lists are kept while the same batch comes back."""
        self.model = model
        if reuse_lists:
            model.reuse_lists(True)
        self.params = model._params.clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.total_steps, self.warmup_steps = int(total_steps), int(warmup_steps)
        self.lr_start, self.lr_end = float(lr_start), float(lr_end)
        self.w_start, self.w_end, self.normalised = tuple(w_start), tuple(w_end), bool(normalised)
        self.loss_form, self.betas, self.eps = int(loss_form), tuple(betas), float(eps)
        self.last_grad = None

    def step(self, batch: Batch, E_ref, F_ref, V_ref):
        """One optimisation step; returns (loss parts (4,) float64 on the GPU, lr, weights)."""
        lr = lr_schedule(self.t, self.warmup_steps, self.total_steps, self.lr_start, self.lr_end)
        w = loss_weights(lr, self.lr_start, self.w_start, self.w_end, self.normalised)
        loss, g = self.model.loss_grad(batch, E_ref, F_ref, V_ref, weights=w, loss_form=self.loss_form)
        self.t += 1
        self.last_grad = g
        adam_step(self.params, g, self.m, self.v, self.t, lr, self.betas[0], self.betas[1], self.eps)
        self.model.set_params(self.params)
        return loss, lr, w


class NepFunction(torch.autograd.Function):
    """(params, batch) -> (E, F, V) with a hand-written parameter backward.

    Gradients flow to the parameter vector only; asking for gradients with
    respect to positions raises."""

    @staticmethod
    def forward(ctx, params, model: NepModel, batch: Batch):
        model.set_params(params.detach())
        out = model.compute(batch)
        ctx.model, ctx.batch = model, batch
        ctx.mark_non_differentiable()
        return out["E"], out["F"], out["V"]

    @staticmethod
    def backward(ctx, gE, gF, gV):
        model, batch = ctx.model, ctx.batch
        if batch.pos.requires_grad:
            raise RuntimeError("position gradients of forces are not provided")
        dev = batch.pos.device
        gE = torch.zeros(batch.n_cfg, dtype=torch.float64, device=dev) if gE is None else gE.to(torch.float64)
        gF = torch.zeros(batch.n_atoms, 3, dtype=torch.float32, device=dev) if gF is None else gF.to(torch.float32)
        gV = torch.zeros(batch.n_cfg, 3, 3, dtype=torch.float64, device=dev) if gV is None else gV.to(torch.float64)
        g = model.backward_params(batch, gE.contiguous(), gF.contiguous(), gV.contiguous())
        return g, None, None


class NepFunction64(torch.autograd.Function):
    """(params float64) -> (E, F, V) float64 with the float64 parameter backward,
    so that torch.autograd.gradcheck can verify the hand-written adjoint on the GPU."""

    @staticmethod
    def forward(ctx, params, model: NepModel, batch: Batch):
        out = model.compute64(batch, params.detach())
        ctx.model, ctx.batch = model, batch
        ctx.save_for_backward(params)
        return out["E"], out["F"], out["V"]

    @staticmethod
    def backward(ctx, gE, gF, gV):
        (params,) = ctx.saved_tensors
        b = ctx.batch
        dev = b.pos.device
        gE = torch.zeros(b.n_cfg, dtype=torch.float64, device=dev) if gE is None else gE.to(torch.float64)
        gF = torch.zeros(b.n_atoms, 3, dtype=torch.float64, device=dev) if gF is None else gF.to(torch.float64)
        gV = torch.zeros(b.n_cfg, 3, 3, dtype=torch.float64, device=dev) if gV is None else gV.to(torch.float64)
        g = ctx.model.backward_params64(b, params.detach(), gE.contiguous(), gF.contiguous(), gV.contiguous())
        return g, None, None


class NepMD:
    """Velocity-Verlet NVE of a batch of cells, replayed as a HIP graph."""

    def __init__(self, model: NepModel, batch: Batch, vel, masses, dt_fs=1.0, skin=1.0):
        self.model, self.batch = model, batch
        vel = _dev(vel, torch.float32)
        keep, poff, pcel, ppbc = batch._meta()
        m, pm = _host_f64(masses)
        h = C.c_void_p()
        check(load().nepmi_md_create(model._h, batch.n_cfg, poff, pcel, ppbc, _ptr(batch.pos), _ptr(vel),
                                     _ptr(batch.species), pm, float(dt_fs), float(skin), C.byref(h), _stream()))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().nepmi_md_destroy(h)
            except Exception:
                pass
            self._h = None

    def step(self, n=1):
        check(load().nepmi_md_step(self._h, int(n), _stream()))

    def step_timed(self, n):
        """Advance n steps; returns the average duration (ms) of the descriptor,
        pair-force and gather kernels over steps 0, 4, 8, ... of these (HIP
        events recorded inside a copy of the step graph that those steps
        replay; the others replay the plain graph)."""
        ms = (C.c_double * 3)()
        check(load().nepmi_md_step_timed(self._h, int(n), ms, _stream()))
        return {"desc": ms[0], "force": ms[1], "gather": ms[2]}

    def state(self):
        b = self.batch
        dev = b.pos.device
        x = torch.empty(b.n_atoms, 3, dtype=torch.float32, device=dev)
        v = torch.empty_like(x)
        f = torch.empty_like(x)
        ep = torch.empty(b.n_cfg, dtype=torch.float64, device=dev)
        ek = torch.empty_like(ep)
        vir = torch.empty(b.n_cfg, 9, dtype=torch.float64, device=dev)
        check(load().nepmi_md_get(self._h, _ptr(x), _ptr(v), _ptr(f), _ptr(ep), _ptr(ek), _ptr(vir), _stream()))
        return {"pos": x, "vel": v, "F": f, "Epot": ep, "Ekin": ek, "V": vir.view(-1, 3, 3)}

    def stats(self):
        s, r, g = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().nepmi_md_stats(self._h, C.byref(s), C.byref(r), C.byref(g)))
        return {"steps": s.value, "rebuilds": r.value, "regrows": g.value}

    def capacity(self, capR=0, capA=0):
        """Set the radial / angular list capacity (0 keeps it; never below the
        longest list built so far) and return the capacities in force."""
        r, a = C.c_int32(), C.c_int32()
        check(load().nepmi_md_capacity(self._h, int(capR), int(capA), C.byref(r), C.byref(a)))
        return {"capR": r.value, "capA": a.value}

    def time_kernels(self, reps=10):
        ms = (C.c_double * 4)()
        check(load().nepmi_md_time_kernels(self._h, int(reps), ms, _stream()))
        return {"desc": ms[0], "force": ms[1], "gather": ms[2], "lists": ms[3]}
