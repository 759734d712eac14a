// api.hip -- extern "C" entry points: model handle, compute, descriptors.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "model.hpp"

namespace nepmi {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string("HIP error '") + hipGetErrorString(e) + "' in " + what);
  return NEPMI_HIP_ERROR;
}

template <class S>
static const Ops* ops_of() {
  static const Ops o = {&Launch<S>::desc, &Launch<S>::force, &Launch<S>::gather, &Launch<S>::derive,
                        &TrainLaunch<S>::seeds, &TrainLaunch<S>::backward,
                        &TrainLaunch<S>::forward64, &TrainLaunch<S>::backward64, S::T, S::NR, S::NA, S::BR, S::BA, S::L,
                        S::D, S::NANG, S::H, S::K, S::P, S::P + S::PCR + S::PCA};
  return &o;
}

template <class S>
static bool matches(const nepmi_hparams& h) {
  return h.n_species == S::T && h.n_radial == S::NR && h.n_angular == S::NA && h.basis_radial == S::BR &&
         h.basis_angular == S::BA && h.l_max == S::L && (h.use_4body != 0) == S::F4 && (h.use_5body != 0) == S::F5 &&
         h.n_hidden == S::H;
}

const Ops* find_ops(const nepmi_hparams& h) {
  if (matches<ShapeSmall>(h)) return ops_of<ShapeSmall>();
  if (matches<ShapeGST>(h)) return ops_of<ShapeGST>();
  if (matches<ShapeTable2>(h)) return ops_of<ShapeTable2>();
  return nullptr;
}

static int check_hp(const nepmi_hparams* hp) {
  if (!hp) {
    set_error("null hyper-parameters");
    return NEPMI_INVALID_ARG;
  }
  const nepmi_hparams& h = *hp;
  if (h.n_species < 1 || h.n_radial < 1 || h.n_angular < 0 || h.basis_radial < 1 || h.basis_angular < 0 ||
      h.l_max < 0 || h.l_max > 4 || h.n_hidden < 1 || !(h.rc_radial > 0) || !(h.rc_angular > 0) ||
      h.rc_angular > h.rc_radial || (h.use_4body && h.l_max < 2) || (h.use_5body && h.l_max < 1)) {
    set_error("invalid hyper-parameters");
    return NEPMI_INVALID_ARG;
  }
  return NEPMI_OK;
}

static int64_t param_count(const nepmi_hparams& h) {
  const int64_t D = h.n_radial + (int64_t)h.l_max * h.n_angular + (h.use_4body ? h.n_angular : 0) +
                    (h.use_5body ? h.n_angular : 0);
  const int64_t T = h.n_species;
  return T * T * ((int64_t)h.n_radial * h.basis_radial + (int64_t)h.n_angular * h.basis_angular) +
         T * (h.n_hidden * D + 2 * h.n_hidden + 1);
}

}  // namespace nepmi

using namespace nepmi;

namespace nepmi {

int prepare_eval(EvalWork& w, const Ops* ops, const nepmi_hparams& hp, int n_cfg, const int64_t* atom_off,
                 const double* cells, const int32_t* pbc, const float* pos, const int32_t* species, hipStream_t st, double skin) {
  int rc;
  // the list build's capacity check synchronises the stream once, which also
  // completes the uploads of both setups
  if ((rc = w.nbr.setup(n_cfg, atom_off, cells, pbc, ops->T, hp.rc_radial, hp.rc_angular, skin, st)) ||
      (rc = w.red.setup(n_cfg, atom_off, st)) || (rc = w.nbr.build(st, pos, species)))
    return rc;
  const NbrPipeline& nb = w.nbr;
  const size_t ns = (size_t)nb.n_slots, N = (size_t)(nb.N > 0 ? nb.N : 1);
  if ((rc = w.fp.ensure(4 * ns * (size_t)ops->NANG)) || (rc = w.aR.ensure(4 * ns * (size_t)(ops->T * ops->BR))) ||
      (rc = w.Ei.ensure(4 * N)) || (rc = w.frad.ensure(16 * ns)) ||
      (rc = w.amask.ensure(8 * ns * (size_t)((nb.capA + 63) / 64))) || (rc = w.fA.ensure(16 * ns * (size_t)nb.capA)) ||
      (rc = w.Wi.ensure(36 * N)) || (rc = w.Eproc.ensure(4 * ns)))
    return rc;
  return NEPMI_OK;
}

NepIO eval_io(EvalWork& w, const nepmi_hparams& hp, float* Fuser, float4* Fproc, float* qout) {
  const NbrPipeline& nbr = w.nbr;
  NepIO o;
  o.n_slots = nbr.n_slots;
  o.capR = nbr.capR;
  o.capA = nbr.capA;
  o.pos4 = nbr.pos4.ptr<float4>();
  o.cfg_of = nbr.cfg_of.ptr<int>();
  o.orig = nbr.orig.ptr<int>();
  o.cfgs = nbr.cfgs.ptr<CfgDev>();
  o.nbrR = nbr.nbrR.ptr<uint32_t>();
  o.cntR = nbr.cntR.ptr<int>();
  o.vrev = nbr.vrev.ptr<uint32_t>();
  o.cnR = nbr.cnbrR.ptr<uint32_t>();
  o.ccR = nbr.ccntR.ptr<int>();
  o.cnA = nbr.cnbrA.ptr<uint32_t>();
  o.cpA = nbr.cposA.ptr<uint32_t>();
  o.ccA = nbr.ccntA.ptr<int>();
  o.flags = nbr.flags.ptr<int>();
  const float rcR = (float)hp.rc_radial, rcA = (float)hp.rc_angular;
  o.cut.rcR = rcR;
  o.cut.rcA = rcA;
  o.cut.rcR2 = rcR * rcR;
  o.cut.rcA2 = rcA * rcA;
  o.cut.rclR2 = nbr.rclR2;
  o.cut.rclA2 = nbr.rclA2;
  o.fp = w.fp.ptr<float>();
  o.aR = w.aR.ptr<float>();
  o.Ei = w.Ei.ptr<float>();
  o.qout = qout;
  o.frad = w.frad.ptr<float4>();
  o.fA = w.fA.ptr<float4>();
  o.amask = w.amask.ptr<uint64_t>();
  o.Wi = w.Wi.ptr<float>();
  o.Fuser = Fuser;
  o.Fproc = Fproc;
  o.Eproc = w.Eproc.ptr<float>();
  return o;
}

// E, F, V of a prepared batch: descriptors + network, pair forces, gather,
// float64 sums, optional per-atom copies.
int run_eval(EvalWork& w, const nepmi_model* m, float* dev_forces, double* dev_energy, double* dev_virial,
             float* dev_atom_energy, float* dev_atom_virial, hipStream_t st) {
  NepIO io = eval_io(w, m->hp, dev_forces, nullptr, nullptr);
  const float* P = m->params.ptr<float>();
  int rc;
  if ((rc = m->ops->desc(st, io, P, true, m->vdesc)) || (rc = m->ops->force(st, io, P, m->vforce)) ||
      (rc = m->ops->gather(st, io, m->vgather)))
    return rc;
  if ((rc = w.red.run(st, io.Ei, io.Wi, nullptr, dev_energy, dev_virial, nullptr))) return rc;
  const size_t N = (size_t)w.nbr.N;
  if (dev_atom_energy && N) NEPMI_HIP(hipMemcpyAsync(dev_atom_energy, io.Ei, 4 * N, hipMemcpyDeviceToDevice, st));
  if (dev_atom_virial && N) NEPMI_HIP(hipMemcpyAsync(dev_atom_virial, io.Wi, 36 * N, hipMemcpyDeviceToDevice, st));
  return NEPMI_OK;
}

}  // namespace nepmi

int nepmi_model::prepare(int n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, const float* pos,
                         const int32_t* species, hipStream_t st, double skin, bool may_reuse) {
  // periodicity flags as given (null: every direction periodic)
  std::vector<int32_t> per(3 * (size_t)(n_cfg > 0 ? n_cfg : 0), 1);
  if (pbc) per.assign(pbc, pbc + per.size());
  if (n_cfg >= 1 && atom_off && cells && reuse_lists && may_reuse && last.valid && last.pos == pos &&
      last.species == species && last.skin == skin && last.off.size() == (size_t)n_cfg + 1 &&
      std::equal(last.off.begin(), last.off.end(), atom_off) &&
      std::equal(last.cells.begin(), last.cells.end(), cells) && last.pbc == per)
    return NEPMI_OK;
  last.valid = false;
  int rc;
  if ((rc = prepare_eval(*this, ops, hp, n_cfg, atom_off, cells, pbc, pos, species, st, skin))) return rc;
  if (may_reuse) {
    last.valid = true;
    last.pos = pos;
    last.species = species;
    last.skin = skin;
    last.off.assign(atom_off, atom_off + n_cfg + 1);
    last.cells.assign(cells, cells + 9 * (size_t)n_cfg);
    last.pbc = per;
  }
  return NEPMI_OK;
}

NepIO nepmi_model::io(float* Fuser, float4* Fproc, float* qout) { return eval_io(*this, hp, Fuser, Fproc, qout); }

extern "C" {

const char* nepmi_last_error(void) { return g_last_error.c_str(); }

int nepmi_param_count(const nepmi_hparams* hp, int64_t* out) {
  int rc = check_hp(hp);
  if (rc) return rc;
  if (!out) return NEPMI_INVALID_ARG;
  *out = param_count(*hp);
  return NEPMI_OK;
}

int nepmi_descriptor_dim(const nepmi_hparams* hp, int32_t* out) {
  int rc = check_hp(hp);
  if (rc) return rc;
  if (!out) return NEPMI_INVALID_ARG;
  *out = hp->n_radial + hp->l_max * hp->n_angular + (hp->use_4body ? hp->n_angular : 0) +
         (hp->use_5body ? hp->n_angular : 0);
  return NEPMI_OK;
}

int nepmi_supported(const nepmi_hparams* hp) { return (hp && check_hp(hp) == 0 && find_ops(*hp)) ? 1 : 0; }

int nepmi_model_create(const nepmi_hparams* hp, nepmi_model** out) {
  int rc = check_hp(hp);
  if (rc) return rc;
  if (!out) {
    set_error("null output handle");
    return NEPMI_INVALID_ARG;
  }
  const Ops* ops = find_ops(*hp);
  if (!ops) {
    set_error("no compiled kernel set for these hyper-parameters");
    return NEPMI_UNSUPPORTED;
  }
  nepmi_model* m = new (std::nothrow) nepmi_model();
  if (!m) return NEPMI_INVALID_ARG;
  m->hp = *hp;
  m->ops = ops;
  if (hipGetDevice(&m->device) != hipSuccess || (rc = m->params.ensure(4 * (size_t)ops->P_alloc))) {
    delete m;
    return rc ? rc : NEPMI_HIP_ERROR;
  }
  *out = m;
  return NEPMI_OK;
}

int nepmi_model_set_params(nepmi_model* m, const float* dev_params, void* stream) {
  if (!m || !dev_params) {
    set_error("null model or parameters");
    return NEPMI_INVALID_ARG;
  }
  NEPMI_HIP(hipMemcpyAsync(m->params.p, dev_params, 4 * (size_t)m->ops->P, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  return m->ops->derive((hipStream_t)stream, m->params.ptr<float>());
}

int nepmi_model_reuse_lists(nepmi_model* m, int32_t enable) {
  if (!m) {
    set_error("null model");
    return NEPMI_INVALID_ARG;
  }
  m->reuse_lists = enable != 0;
  m->last.valid = false;
  return NEPMI_OK;
}

void nepmi_model_destroy(nepmi_model* m) { delete m; }

int nepmi_compute(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, const float* dev_pos,
                  const int32_t* dev_species, double* dev_energy, float* dev_forces, double* dev_virial,
                  float* dev_atom_energy, float* dev_atom_virial, void* stream) {
  if (!m || !dev_pos || !dev_species) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = m->prepare(n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st);
  if (rc) return rc;
  return run_eval(*m, m, dev_forces, dev_energy, dev_virial, dev_atom_energy, dev_atom_virial, st);
}

int nepmi_descriptors(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                      const float* dev_pos, const int32_t* dev_species, float* dev_q, void* stream) {
  if (!m || !dev_pos || !dev_species || !dev_q) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = m->prepare(n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st);
  if (rc) return rc;
  NepIO io = m->io(nullptr, nullptr, dev_q);
  return m->ops->desc(st, io, m->params.ptr<float>(), false, m->vdesc);
}

}  // extern "C"

namespace nepmi {
// Export the neighbour list of every atom in caller order (pairs within the
// potential's cutoff only).
__global__ void k_export_lists(int64_t n_slots, const float4* __restrict__ pos4, const int* __restrict__ cfg_of,
                               const int* __restrict__ orig, const CfgDev* __restrict__ cfgs,
                               const uint32_t* __restrict__ nbr, const int* __restrict__ cnt, float rc2, int cap,
                               int* __restrict__ out_cnt, int* __restrict__ out_nbr, float* __restrict__ out_r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  const int c = cfg_of[p];
  if (c < 0) return;
  const int i = orig[p];
  const float4 xi = pos4[p];
  float H[9];
  for (int x = 0; x < 9; ++x) H[x] = cfgs[c].H[x];
  int n = 0;
  for (int k = 0; k < cnt[p]; ++k) {
    const uint32_t e = nbr[group_index(n_slots, p, k)];
    const int q = (int)(e & kNbrMask);
    const float4 xq = pos4[q];
    float sx, sy, sz;
    image_shift(H, e >> kNbrShift, sx, sy, sz);
    const float rx = (xq.x - xi.x) + sx, ry = (xq.y - xi.y) + sy, rz = (xq.z - xi.z) + sz;
    if (pair_d2(rx, ry, rz) < rc2) {
      if (n < cap) {
        out_nbr[(int64_t)i * cap + n] = orig[q];
        out_r[((int64_t)i * cap + n) * 3 + 0] = rx;
        out_r[((int64_t)i * cap + n) * 3 + 1] = ry;
        out_r[((int64_t)i * cap + n) * 3 + 2] = rz;
      }
      ++n;
    }
  }
  out_cnt[i] = n;
}

// Export the angular part of every atom's list (which = 2: neighbour caller
// index and pair vector of each entry, in the order of that part) or, for the
// same entries found through the mask over the whole list (which = 3), the
// reverse index: the position of the atom in the angular part of its
// neighbour's list, with the pair vector of the entry.
__global__ void k_export_angular(int64_t n_slots, const float4* __restrict__ pos4, const int* __restrict__ cfg_of,
                                 const int* __restrict__ orig, const CfgDev* __restrict__ cfgs,
                                 const uint32_t* __restrict__ nbr, const int* __restrict__ cnt,
                                 const uint32_t* __restrict__ nbrTA, int rowTA, const int* __restrict__ cntAV,
                                 const uint32_t* __restrict__ angm, const uint32_t* __restrict__ vrev, int which,
                                 int cap, int* __restrict__ out_cnt, int* __restrict__ out_nbr,
                                 float* __restrict__ out_r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  const int c = cfg_of[p];
  if (c < 0) return;
  const int i = orig[p];
  const float4 xi = pos4[p];
  float H[9];
  for (int x = 0; x < 9; ++x) H[x] = cfgs[c].H[x];
  auto put = [&](int a, uint32_t e, int v) {
    if (a >= cap) return;
    const float4 xq = pos4[e & kNbrMask];
    float sx, sy, sz;
    image_shift(H, e >> kNbrShift, sx, sy, sz);
    out_nbr[(int64_t)i * cap + a] = v;
    out_r[((int64_t)i * cap + a) * 3 + 0] = (xq.x - xi.x) + sx;
    out_r[((int64_t)i * cap + a) * 3 + 1] = (xq.y - xi.y) + sy;
    out_r[((int64_t)i * cap + a) * 3 + 2] = (xq.z - xi.z) + sz;
  };
  int n = 0;
  if (which == 2) {
    n = cntAV[p];
    for (int a = 0; a < n; ++a) {
      const uint32_t e = nbrTA[p * rowTA + a];
      put(a, e, orig[e & kNbrMask]);
    }
  } else {
    for (int k = 0; k < cnt[p]; ++k) {
      if (!((angm[(int64_t)(k >> 5) * n_slots + p] >> (k & 31)) & 1u)) continue;
      const int64_t gi = group_index(n_slots, p, k);
      put(n++, nbr[gi], (int)vrev[gi]);
    }
  }
  out_cnt[i] = n;
}
}  // namespace nepmi

extern "C" int nepmi_neighbors(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                               const float* dev_pos, const int32_t* dev_species, int32_t which, int32_t cap,
                               int32_t* dev_count, int32_t* dev_nbr, float* dev_rvec, void* stream) {
  if (!m || !dev_pos || !dev_species || !dev_count || !dev_nbr || !dev_rvec || cap < 0 || which < 0 || which > 3) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = m->prepare(n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st);
  if (rc) return rc;
  const int64_t ns = m->nbr.n_slots;
  if (which >= 2) {
    hipLaunchKernelGGL(k_export_angular, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns,
                       m->nbr.pos4.ptr<float4>(), m->nbr.cfg_of.ptr<int>(), m->nbr.orig.ptr<int>(),
                       m->nbr.cfgs.ptr<CfgDev>(), m->nbr.nbrR.ptr<uint32_t>(), m->nbr.cntR.ptr<int>(),
                       m->nbr.nbrTA.ptr<uint32_t>(), m->nbr.rowTA, m->nbr.cntAV.ptr<int>(),
                       m->nbr.angm.ptr<uint32_t>(), m->nbr.vrev.ptr<uint32_t>(), which, cap, dev_count, dev_nbr,
                       dev_rvec);
    NEPMI_HIP(hipGetLastError());
    return NEPMI_OK;
  }
  const float rc1 = (float)(which ? m->hp.rc_angular : m->hp.rc_radial);
  hipLaunchKernelGGL(k_export_lists, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns,
                     m->nbr.pos4.ptr<float4>(), m->nbr.cfg_of.ptr<int>(), m->nbr.orig.ptr<int>(),
                     m->nbr.cfgs.ptr<CfgDev>(), m->nbr.nbrR.ptr<uint32_t>(),
                     m->nbr.cntR.ptr<int>(), rc1 * rc1, cap, dev_count, dev_nbr,
                     dev_rvec);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}
