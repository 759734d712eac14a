// model.hpp -- the model handle and per-shape kernel dispatch.
#pragma once

#include <vector>

#include "nep_kernels.hpp"
#include "reduce.hpp"
#include "train.hpp"

namespace nepmi {

// Kernel set of one compiled shape.
struct Ops {
  int (*desc)(hipStream_t, const NepIO&, const float*, bool, int);
  int (*force)(hipStream_t, const NepIO&, const float*, int);
  int (*gather)(hipStream_t, const NepIO&, int);
  int (*derive)(hipStream_t, float*);
  int (*seeds)(hipStream_t, const TrainSeedArgs&);
  int (*backward)(hipStream_t, TrainIO, const Cutoffs&, const float*, const float*, const int*, double*, double*,
                  float*);
  int (*forward64)(hipStream_t, TrainIOT<double>, const CutoffsT<double>&, const F64Args&, double*);
  int (*backward64)(hipStream_t, TrainIOT<double>, const CutoffsT<double>&, const F64Args&, const double*, const int*,
                    double*, double*);
  int T, NR, NA, BR, BA, L, D, NANG, H, K;
  int64_t P;
  int64_t P_alloc;  // P parameters + the derived coefficient table
};

const Ops* find_ops(const nepmi_hparams& hp);

// Training-only buffers (see train.hip).
struct TrainBufs {
  DevBuf F, E, V, lam, ebar, mu, partF, lam4;
  DevBuf Sst, Sdt, q, qd, Pb, Pdn, abar, zneg, gw1, eat, qbR, FpR, GA, part, grad64, gradf, FpA, qbA;
};

// Buffers of the float64 variant (see train.hip).
struct F64Bufs {
  DevBuf posf, pos4, lam4, ebar1, mu0, Ei, Wi, fA, aR;
  DevBuf Sst, Sdt, q, qd, Pb, Pdn, abar, zneg, gw1, eat, qbR, FpR, GA, part, FpA, qbA;
};

// Work space of one evaluation (E, F, V): neighbour lists and processing
// order, reduction plan and the per-slot arrays the kernels hand to each other.
struct EvalWork {
  NbrPipeline nbr;
  Reducer red;
  DevBuf fp, aR, Ei, frad, fA, amask, Wi, Eproc;
  // Take every buffer from `a` (see Arena); releases what is held.
  void use_arena(Arena* a) {
    nbr.use_arena(a);
    red.use_arena(a);
    for (DevBuf* b : {&fp, &aR, &Ei, &frad, &fA, &amask, &Wi, &Eproc}) {
      b->release();
      b->arena = a;
    }
  }
};

// Neighbour lists (pairs within the cutoffs + skin), work buffers and
// reduction plan of a batch in `w`.
int prepare_eval(EvalWork& w, const Ops* ops, const nepmi_hparams& hp, int n_cfg, const int64_t* atom_off,
                 const double* cells, const int32_t* pbc, const float* pos, const int32_t* species, hipStream_t st, double skin);
// Kernel arguments of an evaluation on `w` (optional caller-order forces,
// slot-order forces and descriptors).
NepIO eval_io(EvalWork& w, const nepmi_hparams& hp, float* Fuser, float4* Fproc, float* qout);

}  // namespace nepmi

struct nepmi_model : nepmi::EvalWork {
  nepmi_hparams hp{};
  const nepmi::Ops* ops = nullptr;
  nepmi::DevBuf params;
  nepmi::TrainBufs tr;
  nepmi::F64Bufs f64;
  int device = 0;
  int vdesc = 0, vforce = 0;  // kernel variants in use (see nepmi_autotune)
  int vgather = 0;            // block size of the gather (see kGatherVariants)
  bool pinned = false;        // variants chosen by nepmi_set_variants: MD creation keeps them
  // Prepare the batch: neighbour lists (pairs within the cutoffs + skin),
  // work buffers and reduction plan.  With reuse_lists set and may_reuse, a
  // batch identical to the previous one (same sizes, cells and device
  // pointers) keeps what the previous call prepared.
  int prepare(int n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, const float* pos, const int32_t* species,
              hipStream_t st, double skin = 0.0, bool may_reuse = true);
  bool reuse_lists = false;
  struct {
    bool valid = false;
    const float* pos = nullptr;
    const int32_t* species = nullptr;
    double skin = 0.0;
    std::vector<int64_t> off;
    std::vector<double> cells;
    std::vector<int32_t> pbc;
  } last;
  nepmi::NepIO io(float* Fuser, float4* Fproc, float* qout);
};

namespace nepmi {
// E, F, V of a batch prepared in `w` with the model's parameters and kernel
// variants (descriptors + network, pair forces, gather, float64 sums, and the
// optional per-atom copies).
int run_eval(EvalWork& w, const nepmi_model* m, float* dev_forces, double* dev_energy, double* dev_virial,
             float* dev_atom_energy, float* dev_atom_virial, hipStream_t st);
// Time every compiled variant of k_desc and k_force on `io` and keep the
// fastest in the model (see tune.hip).
int autotune_io(nepmi_model* m, const NepIO& io, hipStream_t st, int reps);
}  // namespace nepmi
