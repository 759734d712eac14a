// train.hpp -- training kernels: loss seeds and the parameter gradient.
#pragma once

#include "reduce.hpp"

namespace nepmi {

// Per-slot training state; every array is column-major [dim][ns].
struct TrainIO {
  int64_t ns;
  const float4* pos4;
  const int* cfg_of;
  const int* orig;
  const CfgDev* cfgs;
  const uint32_t* nbrR;
  const int* cntR;
  const uint32_t* nbrA;
  const int* cntA;
  float4* lam4;        // [ns] dL/dF in slot order
  const double* mu;    // [n_cfg][9] dL/dV
  const double* ebar;  // [n_cfg] dL/dE
  float* Sst;          // [NA*K] S, then sigma = dE/dS
  float* Sdt;          // [NA*K] Sdot, then Sbar = dj/dS
  float* q;            // [D]
  float* qd;           // [D]
  float* Pb;           // [T*BR] sum_j Q_k per neighbour species
  float* Pdn;          // [T*BR] -sum_j dQ_k (u.t)
  float* abar;         // [H]
  float* zneg;         // [H] -w1 (1 - h^2)
  float* gw1;          // [H] dj/dw1
  float* eat;          // [1] ebar of the atom's configuration
  float* qbR;          // [NR] dj/dq (radial)
  float* FpR;          // [NR] dE/dq (radial)
  float* GA;           // [T*NA*BA] angular coefficient gradient of the atom
};

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

template <class S>
struct TrainLaunch {
  static int seeds(hipStream_t st, const TrainSeedArgs& a);
  static int backward(hipStream_t st, TrainIO io, const Cutoffs& cut, const float* params, const float* lam,
                      const int* base, double* part, double* grad64, float* grad);
};

}  // namespace nepmi
