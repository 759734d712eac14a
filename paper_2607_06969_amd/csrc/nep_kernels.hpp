// nep_kernels.hpp -- NEP evaluation kernels for gfx950, templated on the shape.
//
// One thread evaluates one atom slot; every wavefront holds one species (see
// nbr.hip), so species-pair coefficients c[Z_i][.] and the network weights of
// Z_i are read through the scalar unit.  Coefficients that depend on the
// neighbour's species are read from LDS.
//
//   k_desc   filters the Verlet list into compact lists of the pairs inside
//            the radial and angular cutoffs, then computes the
//            descriptors (Eq. 11, 16, 17 and the 4-/5-body invariants), the
//            network (Sec. 2.3), site energy E_i, and the adjoints the force
//            kernel needs: dE_i/dq for the angular descriptors, and
//            a_i[b][k] = sum_n dE_i/dq_n c^R[Z_i][b][n][k] for the radial ones.
//   k_force  pair forces dE_i/dr_ij and the per-atom virial (Eq. 3, Eq. 4).
//            Radial pairs gather the neighbour's a_j[Z_i] and add both
//            directions at once; angular pairs write dE_i/dr_ij to a pair
//            buffer (no atomics), and S_i is recomputed rather than stored.
//   k_gather F_i = radial part + sum_j (f_ij - f_ji) over the angular pair
//            buffer; f_ji is found in j's compact list (Eq. 3).
#pragma once

#include "common.hpp"

namespace nepmi {

struct NepIO {
  int64_t n_slots;
  const float4* pos4;
  const int* cfg_of;
  const int* orig;
  const CfgDev* cfgs;
  const uint32_t* nbrR;  // Verlet list (rc_radial + skin)
  const int* cntR;
  uint32_t* cnR;         // compact list: pairs within rc_radial (written by k_desc)
  int* ccR;
  uint32_t* cnA;         // compact list: pairs within rc_angular (written by k_desc)
  int* ccA;
  int* flags;
  Cutoffs cut;
  float* fp;     // [NANG][n_slots]  dE_i/dq (angular descriptors)
  float* aR;     // [n_slots][T*BR]  radial adjoint
  float* Ei;     // [N] caller order (site energies)
  float* qout;   // [N][D] caller order, optional
  float4* frad;  // [n_slots] radial force part
  float4* fA;    // [capA][n_slots] angular pair forces dE_i/dr_ij
  float* Wi;     // [N][9] caller order, per-atom virial
  float* Fuser;  // [N][3] caller order, optional
  float4* Fproc; // [n_slots], optional
  float* Eproc;  // [n_slots] site energies in slot order, optional
};

constexpr int kVariants = 4;  // compiled variants of k_desc and of k_force

template <class S>
struct Launch {
  static int desc(hipStream_t st, const NepIO& io, const float* params, bool want_adjoint, int variant);
  static int force(hipStream_t st, const NepIO& io, const float* params, int variant);
  static int gather(hipStream_t st, const NepIO& io);
};

}  // namespace nepmi
