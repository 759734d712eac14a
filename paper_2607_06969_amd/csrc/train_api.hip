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
  const size_t maxE = std::max({(size_t)o->H * o->D, (size_t)o->NR * o->T * o->BR, (size_t)o->T * o->NA * o->BA,
                                (size_t)o->H});
  int rc;
  if ((rc = t.F.ensure(12 * N)) || (rc = t.E.ensure(8 * nc)) || (rc = t.V.ensure(72 * nc)) ||
      (rc = t.lam.ensure(12 * N)) || (rc = t.ebar.ensure(8 * nc)) || (rc = t.mu.ensure(72 * nc)) ||
      (rc = t.partF.ensure(8 * ni)) || (rc = t.lam4.ensure(16 * ns)) ||
      (rc = t.Sst.ensure(4 * ns * o->NA * o->K)) || (rc = t.Sdt.ensure(4 * ns * o->NA * o->K)) ||
      (rc = t.q.ensure(4 * ns * o->D)) || (rc = t.qd.ensure(4 * ns * o->D)) ||
      (rc = t.Pb.ensure(4 * ns * o->T * o->BR)) || (rc = t.Pdn.ensure(4 * ns * o->T * o->BR)) ||
      (rc = t.abar.ensure(4 * ns * o->H)) || (rc = t.zneg.ensure(4 * ns * o->H)) || (rc = t.gw1.ensure(4 * ns * o->H)) ||
      (rc = t.eat.ensure(4 * ns)) || (rc = t.qbR.ensure(4 * ns * o->NR)) || (rc = t.FpR.ensure(4 * ns * o->NR)) ||
      (rc = t.GA.ensure(4 * ns * o->T * o->NA * o->BA)) || (rc = t.part.ensure(8 * (size_t)o->T * 64 * maxE)) ||
      (rc = t.grad64.ensure(8 * (size_t)o->P)) || (rc = t.gradf.ensure(4 * (size_t)o->P)))
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

}  // namespace

extern "C" {

int nepmi_backward_params(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells,
                          const float* dev_pos, const int32_t* dev_species, const double* dev_ebar,
                          const float* dev_lambda, const double* dev_mu, float* dev_grad, void* stream) {
  if (!m || !dev_pos || !dev_species || !dev_ebar || !dev_lambda || !dev_mu || !dev_grad) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = m->prepare(n_cfg, atom_off, cells, dev_pos, dev_species, st)) || (rc = ensure_train(m))) return rc;
  // the descriptor kernel writes the per-evaluation compact pair lists
  if ((rc = m->ops->desc(st, m->io(nullptr, nullptr, nullptr), m->params.ptr<float>(), false, m->vdesc))) return rc;
  return run_backward(m, st, dev_ebar, dev_lambda, dev_mu, dev_grad);
}

int nepmi_loss_grad(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells,
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
  if ((rc = m->prepare(n_cfg, atom_off, cells, dev_pos, dev_species, st)) || (rc = ensure_train(m))) return rc;
  TrainBufs& t = m->tr;
  // forward: E, F, V
  NepIO io = m->io(t.F.ptr<float>(), nullptr, nullptr);
  const float* P = m->params.ptr<float>();
  if ((rc = m->ops->desc(st, io, P, true, m->vdesc)) || (rc = m->ops->force(st, io, P, m->vforce)) || (rc = m->ops->gather(st, io)) ||
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
