// train_api.hip -- extern "C" entry points of the training path.
#include <algorithm>

#include "model.hpp"

using namespace nepmi;

namespace {

int ensure_train(nepmi_model* m) {
  const Ops* o = m->ops;
  TrainBufs& t = m->tr;
  const size_t ns = (size_t)m->nbr.n_slots, N = (size_t)(m->nbr.N > 0 ? m->nbr.N : 1);
  const size_t nc = (size_t)m->nbr.n_cfg, ni = (size_t)m->red.n_items;
  // the parameter-gradient sums each keep their own partial sums
  const size_t sumE = (size_t)o->H * o->D + (size_t)o->NR * o->T * o->BR + (size_t)o->T * o->NA * o->BA +
                      2 * (size_t)o->H + 1;
  int rc;
  if ((rc = t.F.ensure(12 * N)) || (rc = t.E.ensure(8 * nc)) || (rc = t.V.ensure(72 * nc)) ||
      (rc = t.lam.ensure(12 * N)) || (rc = t.ebar.ensure(8 * nc)) || (rc = t.mu.ensure(72 * nc)) ||
      (rc = t.partF.ensure(8 * ni)) || (rc = t.lam4.ensure(16 * ns)) ||
      (rc = t.Sst.ensure(4 * ns * o->NA * o->K)) || (rc = t.Sdt.ensure(4 * ns * o->NA * o->K)) ||
      (rc = t.q.ensure(4 * ns * o->D)) || (rc = t.qd.ensure(4 * ns * o->D)) ||
      (rc = t.Pb.ensure(4 * ns * o->T * o->BR)) || (rc = t.Pdn.ensure(4 * ns * o->T * o->BR)) ||
      (rc = t.abar.ensure(4 * ns * o->H)) || (rc = t.zneg.ensure(4 * ns * o->H)) || (rc = t.gw1.ensure(4 * ns * o->H)) ||
      (rc = t.eat.ensure(4 * ns)) || (rc = t.qbR.ensure(4 * ns * o->NR)) || (rc = t.FpR.ensure(4 * ns * o->NR)) ||
      (rc = t.GA.ensure(4 * ns * o->T * o->NA * o->BA)) || (rc = t.part.ensure(8 * (size_t)o->T * kRBlocks * sumE)) ||
      (rc = t.grad64.ensure(8 * (size_t)o->P)) || (rc = t.gradf.ensure(4 * (size_t)o->P)) ||
      (rc = t.FpA.ensure(4 * ns * o->D)) || (rc = t.qbA.ensure(4 * ns * o->D)))
    return rc;
  return NEPMI_OK;
}

TrainIO train_io(nepmi_model* m, const double* mu, const double* ebar) {
  TrainBufs& t = m->tr;
  TrainIO io;
  io.ns = m->nbr.n_slots;
  io.pos4 = m->nbr.pos4.ptr<float4>();
  io.cfg_of = m->nbr.cfg_of.ptr<int>();
  io.orig = m->nbr.orig.ptr<int>();
  io.cfgs = m->nbr.cfgs.ptr<CfgDev>();
  io.nbrR = m->nbr.cnbrR.ptr<uint32_t>();  // compact lists written by the forward
  io.cntR = m->nbr.ccntR.ptr<int>();
  io.nbrA = m->nbr.cnbrA.ptr<uint32_t>();
  io.cntA = m->nbr.ccntA.ptr<int>();
  io.lam4 = t.lam4.ptr<float4>();
  io.mu = mu;
  io.ebar = ebar;
  io.Sst = t.Sst.ptr<float>();
  io.Sdt = t.Sdt.ptr<float>();
  io.q = t.q.ptr<float>();
  io.qd = t.qd.ptr<float>();
  io.Pb = t.Pb.ptr<float>();
  io.Pdn = t.Pdn.ptr<float>();
  io.abar = t.abar.ptr<float>();
  io.zneg = t.zneg.ptr<float>();
  io.gw1 = t.gw1.ptr<float>();
  io.eat = t.eat.ptr<float>();
  io.qbR = t.qbR.ptr<float>();
  io.FpR = t.FpR.ptr<float>();
  io.GA = t.GA.ptr<float>();
  io.FpA = t.FpA.ptr<float>();
  io.qbA = t.qbA.ptr<float>();
  io.Ei = nullptr;
  return io;
}

int run_backward(nepmi_model* m, hipStream_t st, const double* ebar, const float* lam, const double* mu,
                 float* dev_grad) {
  NepIO nio = m->io(nullptr, nullptr, nullptr);
  TrainIO io = train_io(m, mu, ebar);
  TrainBufs& t = m->tr;
  return m->ops->backward(st, io, nio.cut, m->params.ptr<float>(), lam, m->nbr.base.ptr<int>(), t.part.ptr<double>(),
                          t.grad64.ptr<double>(), dev_grad);
}

// ---- float64 variant

int ensure_f64(nepmi_model* m) {
  const Ops* o = m->ops;
  F64Bufs& f = m->f64;
  const size_t ns = (size_t)m->nbr.n_slots, N = (size_t)(m->nbr.N > 0 ? m->nbr.N : 1);
  const size_t nc = (size_t)(m->nbr.n_cfg > 0 ? m->nbr.n_cfg : 1);
  // the parameter-gradient sums each keep their own partial sums
  const size_t sumE = (size_t)o->H * o->D + (size_t)o->NR * o->T * o->BR + (size_t)o->T * o->NA * o->BA +
                      2 * (size_t)o->H + 1;
  int rc;
  if ((rc = f.pos4.ensure(32 * ns)) || (rc = f.lam4.ensure(32 * ns)) || (rc = f.ebar1.ensure(8 * nc)) ||
      (rc = f.mu0.ensure(72 * nc)) || (rc = f.Ei.ensure(8 * N)) || (rc = f.Wi.ensure(72 * N)) ||
      (rc = f.Sst.ensure(8 * ns * o->NA * o->K)) || (rc = f.Sdt.ensure(8 * ns * o->NA * o->K)) ||
      (rc = f.q.ensure(8 * ns * o->D)) || (rc = f.qd.ensure(8 * ns * o->D)) ||
      (rc = f.Pb.ensure(8 * ns * o->T * o->BR)) || (rc = f.Pdn.ensure(8 * ns * o->T * o->BR)) ||
      (rc = f.abar.ensure(8 * ns * o->H)) || (rc = f.zneg.ensure(8 * ns * o->H)) || (rc = f.gw1.ensure(8 * ns * o->H)) ||
      (rc = f.eat.ensure(8 * ns)) || (rc = f.qbR.ensure(8 * ns * o->NR)) || (rc = f.FpR.ensure(8 * ns * o->NR)) ||
      (rc = f.GA.ensure(8 * ns * o->T * o->NA * o->BA)) || (rc = f.part.ensure(8 * (size_t)o->T * kRBlocks * sumE)) ||
      (rc = f.FpA.ensure(8 * ns * o->D)) || (rc = f.qbA.ensure(8 * ns * o->D)) ||
      (rc = f.fA.ensure(32 * ns * (size_t)(m->nbr.capA > 0 ? m->nbr.capA : 1))) ||
      (rc = f.aR.ensure(8 * ns * o->T * o->BR)))
    return rc;
  return NEPMI_OK;
}

TrainIOT<double> f64_io(nepmi_model* m, const double* mu, const double* ebar, double* Ei) {
  F64Bufs& f = m->f64;
  TrainIOT<double> io;
  io.ns = m->nbr.n_slots;
  io.pos4 = f.pos4.ptr<double4>();
  io.cfg_of = m->nbr.cfg_of.ptr<int>();
  io.orig = m->nbr.orig.ptr<int>();
  io.cfgs = m->nbr.cfgs.ptr<CfgDev>();
  // the full lists (cutoff, no skin); every kernel tests each pair in float64
  io.nbrR = m->nbr.nbrR.ptr<uint32_t>();
  io.cntR = m->nbr.cntR.ptr<int>();
  io.nbrA = m->nbr.nbrR.ptr<uint32_t>();
  io.cntA = m->nbr.cntR.ptr<int>();
  io.lam4 = f.lam4.ptr<double4>();
  io.mu = mu;
  io.ebar = ebar;
  io.Sst = f.Sst.ptr<double>();
  io.Sdt = f.Sdt.ptr<double>();
  io.q = f.q.ptr<double>();
  io.qd = f.qd.ptr<double>();
  io.Pb = f.Pb.ptr<double>();
  io.Pdn = f.Pdn.ptr<double>();
  io.abar = f.abar.ptr<double>();
  io.zneg = f.zneg.ptr<double>();
  io.gw1 = f.gw1.ptr<double>();
  io.eat = f.eat.ptr<double>();
  io.qbR = f.qbR.ptr<double>();
  io.FpR = f.FpR.ptr<double>();
  io.GA = f.GA.ptr<double>();
  io.FpA = f.FpA.ptr<double>();
  io.qbA = f.qbA.ptr<double>();
  io.Ei = Ei;
  return io;
}

CutoffsT<double> f64_cut(const nepmi_model* m) {
  CutoffsT<double> c;
  c.rcR = m->hp.rc_radial;
  c.rcA = m->hp.rc_angular;
  c.rcR2 = c.rcR * c.rcR;
  c.rcA2 = c.rcA * c.rcA;
  c.rclR2 = c.rcR2;
  c.rclA2 = c.rcA2;
  return c;
}

// Lists from the float32 rounding of the positions with a skin far above its
// rounding error (~1e-5 A at 100 A), so that every pair within a cutoff in
// float64 is listed; the kernels then test each pair in float64.
constexpr double kSkin64 = 0.01;

// lists from the float32 rounding of the positions, then the float64 staging
int prepare64(nepmi_model* m, int n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, const double* dev_pos,
              const int32_t* dev_species, const double* dev_params, hipStream_t st, F64Args& a) {
  if (n_cfg < 1 || !atom_off || atom_off[0] != 0 || atom_off[n_cfg] < 0) {
    set_error("invalid batch");
    return NEPMI_INVALID_ARG;
  }
  const int64_t N = atom_off[n_cfg];
  int rc;
  if ((rc = m->f64.posf.ensure(12 * (size_t)(N > 0 ? N : 1))) ||
      (rc = launch_round_pos(st, 3 * N, dev_pos, m->f64.posf.ptr<float>())) ||
      (rc = m->prepare(n_cfg, atom_off, cells, pbc, m->f64.posf.ptr<float>(), dev_species, st, kSkin64, false)) ||
      (rc = ensure_f64(m)))
    return rc;
  a.atom_off = m->nbr.atom_off_dev.ptr<int64_t>();
  a.n_cfg = n_cfg;
  a.pos = dev_pos;
  a.params = dev_params;
  a.pos4 = m->f64.pos4.ptr<double4>();
  a.Wi = m->f64.Wi.ptr<double>();
  a.vrev = m->nbr.vrev.ptr<uint32_t>();
  a.nbrTA = m->nbr.nbrTA.ptr<uint32_t>();
  a.rowTA = m->nbr.rowTA;
  a.cntAV = m->nbr.cntAV.ptr<int>();
  a.fA = m->f64.fA.ptr<double4>();
  a.aR = m->f64.aR.ptr<double>();
  return launch_stage64(st, f64_io(m, nullptr, nullptr, nullptr), a, m->nbr.pos4.ptr<float4>());
}

}  // namespace

extern "C" {

int nepmi_compute_f64(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                      const double* dev_pos, const int32_t* dev_species, const double* dev_params, double* dev_energy,
                      double* dev_forces, double* dev_virial, double* dev_atom_energy, void* stream) {
  if (!m || !cells || !dev_pos || !dev_species || !dev_params || !dev_energy || !dev_forces || !dev_virial) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  F64Args a;
  int rc;
  if ((rc = prepare64(m, n_cfg, atom_off, cells, pbc, dev_pos, dev_species, dev_params, st, a))) return rc;
  F64Bufs& f = m->f64;
  if ((rc = launch_fill64(st, n_cfg, 1.0, f.ebar1.ptr<double>())) ||
      (rc = launch_fill64(st, 9 * (int64_t)n_cfg, 0.0, f.mu0.ptr<double>())))
    return rc;
  double* Ei = dev_atom_energy ? dev_atom_energy : f.Ei.ptr<double>();
  TrainIOT<double> io = f64_io(m, f.mu0.ptr<double>(), f.ebar1.ptr<double>(), Ei);
  if ((rc = m->ops->forward64(st, io, f64_cut(m), a, dev_forces))) return rc;
  // per-configuration float64 sums in the fixed chunking of the float32 path
  return m->red.run64(st, Ei, a.Wi, dev_energy, dev_virial);
}

int nepmi_backward_params_f64(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                              const double* dev_pos, const int32_t* dev_species, const double* dev_params,
                              const double* dev_ebar, const double* dev_lambda, const double* dev_mu,
                              double* dev_grad, void* stream) {
  if (!m || !cells || !dev_pos || !dev_species || !dev_params || !dev_ebar || !dev_lambda || !dev_mu || !dev_grad) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  F64Args a;
  int rc;
  if ((rc = prepare64(m, n_cfg, atom_off, cells, pbc, dev_pos, dev_species, dev_params, st, a))) return rc;
  TrainIOT<double> io = f64_io(m, dev_mu, dev_ebar, nullptr);
  return m->ops->backward64(st, io, f64_cut(m), a, dev_lambda, m->nbr.base.ptr<int>(), m->f64.part.ptr<double>(),
                            dev_grad);
}


int nepmi_backward_params(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                          const float* dev_pos, const int32_t* dev_species, const double* dev_ebar,
                          const float* dev_lambda, const double* dev_mu, float* dev_grad, void* stream) {
  if (!m || !dev_pos || !dev_species || !dev_ebar || !dev_lambda || !dev_mu || !dev_grad) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = m->prepare(n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st)) || (rc = ensure_train(m))) return rc;
  // the descriptor kernel writes the per-evaluation compact pair lists
  if ((rc = m->ops->desc(st, m->io(nullptr, nullptr, nullptr), m->params.ptr<float>(), false, m->vdesc))) return rc;
  return run_backward(m, st, dev_ebar, dev_lambda, dev_mu, dev_grad);
}

int nepmi_loss_grad(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                    const float* dev_pos, const int32_t* dev_species, const double* dev_E_ref, const float* dev_F_ref,
                    const double* dev_V_ref, const double* weights, int32_t loss_form, double* dev_loss,
                    float* dev_grad, void* stream) {
  if (!m || !dev_pos || !dev_species || !dev_E_ref || !dev_F_ref || !dev_V_ref || !weights || !dev_loss ||
      (loss_form != 0 && loss_form != 1)) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = m->prepare(n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st)) || (rc = ensure_train(m))) return rc;
  TrainBufs& t = m->tr;
  // forward: E, F, V
  NepIO io = m->io(t.F.ptr<float>(), nullptr, nullptr);
  const float* P = m->params.ptr<float>();
  if ((rc = m->ops->desc(st, io, P, true, m->vdesc)) || (rc = m->ops->force(st, io, P, m->vforce)) || (rc = m->ops->gather(st, io, m->vgather)) ||
      (rc = m->red.run(st, io.Ei, io.Wi, nullptr, t.E.ptr<double>(), t.V.ptr<double>(), nullptr)))
    return rc;
  // loss and seeds
  TrainSeedArgs a;
  a.items = m->red.items_dev.ptr<RedItem>();
  a.n_items = m->red.n_items;
  a.item_start = m->red.start_dev.ptr<int>();
  a.n_cfg = n_cfg;
  a.form = loss_form;
  a.w[0] = weights[0];
  a.w[1] = weights[1];
  a.w[2] = weights[2];
  a.inv_3ntot = m->nbr.N > 0 ? 1.0 / (3.0 * (double)m->nbr.N) : 0.0;
  a.off = m->nbr.atom_off_dev.ptr<int64_t>();
  a.F = t.F.ptr<float>();
  a.Fref = dev_F_ref;
  a.E = t.E.ptr<double>();
  a.Eref = dev_E_ref;
  a.V = t.V.ptr<double>();
  a.Vref = dev_V_ref;
  a.lam = t.lam.ptr<float>();
  a.ebar = t.ebar.ptr<double>();
  a.mu = t.mu.ptr<double>();
  a.partF = t.partF.ptr<double>();
  a.loss = dev_loss;
  if ((rc = m->ops->seeds(st, a))) return rc;
  if (!dev_grad) return NEPMI_OK;
  return run_backward(m, st, t.ebar.ptr<double>(), t.lam.ptr<float>(), t.mu.ptr<double>(), dev_grad);
}

}  // extern "C"
