// nep_kernels.hpp -- NEP evaluation kernels for gfx950, templated on the shape.
//
// One thread evaluates one atom slot; every wavefront holds one species (see
// nbr.hip), so species-pair coefficients c[Z_i][.] and the network weights of
// Z_i are read through the scalar unit.  Coefficients that depend on the
// neighbour's species are read from LDS.  The kernels use a derived copy of
// the Chebyshev coefficients stored after the parameters (k_derive), in which
// the "+1" of Q_k = (T_k + 1) f_c / 2 is folded into column 0.
//
//   k_desc   filters the Verlet list into compact lists of the pairs inside
//            the radial and angular cutoffs (accumulating the radial sums on
//            the way), then computes the descriptors (Eq. 11, 16, 17 and the
//            4-/5-body invariants), the network (Sec. 2.3), site energy E_i,
//            and the adjoints the force kernel needs: dE_i/dq for the angular
//            descriptors, and atil_i[b][k] = sum_n dE_i/dq_n ctil[Z_i][b][n][k]
//            for the radial ones.
//   k_force  pair forces dE_i/dr_ij and the per-atom virial (Eq. 3, Eq. 4).
//            Radial pairs gather the neighbour's atil_j[Z_i] and add both
//            directions at once; for angular pairs, dE_i/dr_ij is added to
//            i's own force and kept in i's compact slot (no atomics).  S_i is
//            recomputed rather than stored.
//   k_gather F_i = own part - sum_j dE_j/dr_ji over i's angular pairs (Eq. 3),
//            finding i's slot in j's compact list from the reverse index
//            built with the lists and j's entry mask.
#pragma once

#include "common.hpp"

namespace nepmi {

struct NepIO {
  int64_t n_slots;
  int capR;              // rows of the Verlet list and of the pair buffer
  int capA;              // rows of the compact angular list
  const float4* pos4;
  const int* cfg_of;
  const int* orig;
  const CfgDev* cfgs;
  const uint32_t* nbrR;  // Verlet list (rc_radial + skin), in groups of four entries
  const int* cntR;
  const uint32_t* vrev;  // position of i in the angular part (rc_angular + skin) of j's Verlet list,
                         // 0xFFFFFFFF outside that part; grouped as nbrR
  uint32_t* cnR;         // compact list: pairs within rc_radial (written by k_desc)
  int* ccR;
  uint32_t* cnA;         // compact list: pairs within rc_angular (written by k_desc)
  uint32_t* cpA;         // own angular-part position | reverse position << 16, grouped as cnA
  int* ccA;
  int* flags;
  Cutoffs cut;
  float* fp;     // [NANG][n_slots]  dE_i/dq (angular descriptors)
  float* aR;     // [T][n_slots][BR] radial adjoint, part b = atil_i[b][.]
  float* Ei;     // [N] caller order (site energies)
  float* qout;   // [N][D] caller order, optional
  float4* frad;  // [n_slots] own force part (radial pairs both ways, angular dE_i/dr_ij)
  float4* fA;    // [capA][n_slots] angular pair forces dE_i/dr_ij in i's compact slots
  uint64_t* amask; // [ceil(capA/64)][n_slots] entries of the angular part of i's Verlet list that are
                   // in its compact angular list
  float* Wi;     // [N][9] caller order, per-atom virial
  float* Fuser;  // [N][3] caller order, optional
  float4* Fproc; // [n_slots], optional
  float* Eproc;  // [n_slots] site energies in slot order, optional
};

constexpr int kDescVariants = 10;  // compiled variants of k_desc (4..7: network in its own kernel;
                                   // 8, 9: variant 0 in blocks of 128 and 512 threads)
constexpr int kForceVariants = 6;  // compiled variants of k_force (4, 5: variant 0 in blocks of 128, 512)
constexpr int kGatherVariants = 4; // k_gather in blocks of 256, 128, 512, 1024 threads

template <class S>
struct Launch {
  static int desc(hipStream_t st, const NepIO& io, const float* params, bool want_adjoint, int variant);
  static int force(hipStream_t st, const NepIO& io, const float* params, int variant);
  static int gather(hipStream_t st, const NepIO& io, int variant);
  // Writes the derived coefficient table after the P parameters (the
  // parameter buffer holds P + PCR + PCA floats).
  static int derive(hipStream_t st, float* params);
};

}  // namespace nepmi
