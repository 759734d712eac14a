// train.hpp -- training kernels: loss seeds and the parameter gradient.
#pragma once

#include "reduce.hpp"

namespace nepmi {

// Blocks per species of the gradient sums over atoms (a fixed number: the
// summation order, hence every bit of the gradient, does not depend on the
// launch).  The partial-sum buffer holds T * kRBlocks * (largest sum) doubles.
// On the 256-cell batch: 64 blocks 2.27 ms per loss and gradient, 128 1.96,
// 256 1.88, 512 2.06.
constexpr int kRBlocks = 256;

// Per-slot training state; every array is column-major [dim][ns].  R is the
// arithmetic precision (float, or double for the float64 variant).
template <class R>
struct TrainIOT {
  int64_t ns;
  const Vec4<R>* pos4;
  const int* cfg_of;
  const int* orig;
  const CfgDev* cfgs;
  const uint32_t* nbrR;
  const int* cntR;
  const uint32_t* nbrA;
  const int* cntA;
  Vec4<R>* lam4;       // [ns] dL/dF in slot order
  const double* mu;    // [n_cfg][9] dL/dV
  const double* ebar;  // [n_cfg] dL/dE
  R* Sst;              // [NA*K] S, then sigma = dE/dS
  R* Sdt;              // [NA*K] Sdot, then Sbar = dj/dS
  R* q;                // [D]
  R* qd;               // [D]
  R* Pb;               // [T*BR] sum_j Q_k per neighbour species
  R* Pdn;              // [T*BR] -sum_j dQ_k (u.t)
  R* abar;             // [H]
  R* zneg;             // [H] -w1 (1 - h^2)
  R* gw1;              // [H] dj/dw1
  R* eat;              // [1] ebar of the atom's configuration
  R* qbR;              // [NR] dj/dq (radial)
  R* FpR;              // [NR] dE/dq (radial)
  R* GA;               // [T*NA*BA] angular coefficient gradient of the atom
  R* FpA;              // [D] dE/dq (rows NR..D-1 used), network pass -> sigma pass
  R* qbA;              // [D] dj/dq (rows NR..D-1 used), network pass -> sigma pass
  R* Ei;               // [N] site energies, caller order (float64 variant only; may be null)
};
using TrainIO = TrainIOT<float>;

struct TrainSeedArgs {
  const RedItem* items;
  int n_items;
  const int* item_start;
  int n_cfg;
  int form;
  double w[3];
  double inv_3ntot;
  const int64_t* off;
  const float* F;
  const float* Fref;
  const double* E;
  const double* Eref;
  const double* V;
  const double* Vref;
  float* lam;
  double* ebar;
  double* mu;
  double* partF;
  double* loss;
};

// Inputs of the float64 variant: positions in caller order, float64 (the
// neighbour lists are built from their float32 rounding; every pair is then
// tested and evaluated in float64).
struct F64Args {
  const int64_t* atom_off;  // device [n_cfg + 1]
  int n_cfg;
  const double* pos;        // device [N][3]
  const double* params;     // device [P], the parameter layout of the model
  double4* pos4;            // work: [ns] positions in slot order
  double* Wi;               // work: [N][9] per-atom virial, caller order
  const uint32_t* vrev;     // reverse index of the Verlet list (grouped as the list)
  const uint32_t* nbrTA;    // angular part (rc_angular + skin) of each list, row-major, rows of rowTA
  int rowTA;
  const int* cntAV;         // [ns] entries in that part
  double4* fA;              // work: [capA][ns] dE_i/dr_ij of the angular part of i's list, by position
  double* aR;               // work: [T][ns][BR] radial adjoint rows
};

template <class S>
struct TrainLaunch {
  static int seeds(hipStream_t st, const TrainSeedArgs& a);
  static int backward(hipStream_t st, TrainIO io, const Cutoffs& cut, const float* params, const float* lam,
                      const int* base, double* part, double* grad64, float* grad);
  // float64 variant: forces, site energies (io.Ei) and per-atom virials
  // (a.Wi), all in caller order; the caller sums them per configuration ...
  static int forward64(hipStream_t st, TrainIOT<double> io, const CutoffsT<double>& cut, const F64Args& a,
                       double* forces);
  // ... and the parameter gradient of ebar.E + lambda.F + mu:V
  static int backward64(hipStream_t st, TrainIOT<double> io, const CutoffsT<double>& cut, const F64Args& a,
                        const double* lam, const int* base, double* part, double* grad);
};

// float64 helpers: stage positions in slot order, round positions to float32
// (for the neighbour lists), fill a float64 array.
int launch_stage64(hipStream_t st, const TrainIOT<double>& io, const F64Args& a, const float4* pos4f);
int launch_round_pos(hipStream_t st, int64_t n, const double* a, float* b);
int launch_fill64(hipStream_t st, int64_t n, double v, double* a);

}  // namespace nepmi
