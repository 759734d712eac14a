// train.hip -- loss (Eq. 18-21), adjoint seeds and the parameter gradient.
//
// With seeds ebar_c = dL/dE_c, lambda_i = dL/dF_i and mu_c = dL/dV_c, the
// gradient is d/dtheta of  sum_c ebar_c E_c + sum_i lambda_i.F_i + sum_c mu_c:V_c.
// By Eq. 3 and Eq. 4,  sum_i lambda_i.F_i + mu:V = - sum_ij (dE_i/dr_ij).t_ij
// with t_ij = lambda_j - lambda_i + mu r_ij, i.e. minus the directional
// derivative of E along t: - sum_i dE_i/dq_i . qdot_i, where qdot_i is the
// tangent of the descriptors.  Per atom the objective is therefore
//   j_i = ebar E_i - z . (W0 qdot_i),   z = w1 (1 - h^2),  h = tanh(W0 q_i + b0),
// whose derivatives with respect to the network weights and, through q_i and
// qdot_i (both linear in the coefficients c), with respect to c^R and c^A give
// the gradient.  Descriptors are recomputed; nothing per pair is stored.
//
//   k_train_atom    tangent pass + second-order network adjoint (per atom)
//   k_train_coefA   angular coefficient gradient (per atom, over its pairs)
//   k_outer2 / k_colsum4 per-species sums over atoms (fixed order, float64)
#include <cstdlib>

#include "train.hpp"

namespace nepmi {

constexpr int kTB = 256;

// Symmetric 3x3 as (xx, yy, zz, xy, xz, yz); full-matrix gradient convention
// dE = sum_ab M_ab dA_ab.  A_n from S_n2m (l = 2 content of S).
template <class R>
__device__ __forceinline__ void sym_from_s2(const R* s2, R (&A)[6]) {
  const R azz = s2[0] * (R(1.0) / (R(3.0) * ShC<R>::k20));
  const R dif = s2[3] * (R(1.0) / ShC<R>::k22);
  A[0] = R(0.5) * (dif - azz);
  A[1] = -R(0.5) * (dif + azz);
  A[2] = azz;
  A[3] = s2[4] * (R(1.0) / ShC<R>::k21);
  A[4] = s2[1] * (R(1.0) / ShC<R>::k21);
  A[5] = s2[2] * (R(1.0) / ShC<R>::k21);
}

template <class R>
__device__ __forceinline__ void sym_mul_sym(const R (&A)[6], const R (&B)[6], R (&C)[9]) {
  // C = A B (general 3x3, row-major)
  const R a[9] = {A[0], A[3], A[4], A[3], A[1], A[5], A[4], A[5], A[2]};
  const R b[9] = {B[0], B[3], B[4], B[3], B[1], B[5], B[4], B[5], B[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// sum_ab M_ab N_ab for symmetric M, N
template <class R>
__device__ __forceinline__ R sym_dot(const R (&M)[6], const R (&N)[6]) {
  return M[0] * N[0] + M[1] * N[1] + M[2] * N[2] + R(2.0) * (M[3] * N[3] + M[4] * N[4] + M[5] * N[5]);
}

// Gradient with respect to S_n2m of a function whose gradient w.r.t. A is M.
template <class R>
__device__ __forceinline__ void chain_s2(const R (&M)[6], R (&g)[5]) {
  g[0] = (M[2] - R(0.5) * (M[0] + M[1])) * (R(1.0) / (R(3.0) * ShC<R>::k20));
  g[1] = R(2.0) * M[4] * (R(1.0) / ShC<R>::k21);
  g[2] = R(2.0) * M[5] * (R(1.0) / ShC<R>::k21);
  g[3] = R(0.5) * (M[0] - M[1]) * (R(1.0) / ShC<R>::k22);
  g[4] = R(2.0) * M[3] * (R(1.0) / ShC<R>::k21);
}

template <class R>
__device__ __forceinline__ void sym_sq6(const R (&A)[6], R (&B)[6]) {
  const R xx = A[0], yy = A[1], zz = A[2], xy = A[3], xz = A[4], yz = A[5];
  B[0] = xx * xx + xy * xy + xz * xz;
  B[1] = xy * xy + yy * yy + yz * yz;
  B[2] = xz * xz + yz * yz + zz * zz;
  B[3] = xx * xy + xy * yy + xz * yz;
  B[4] = xx * xz + xy * yz + xz * zz;
  B[5] = xy * xz + yy * yz + yz * zz;
}

template <class R>
__device__ __forceinline__ void load_cell9(const CfgDev* __restrict__ cfgs, int c, R (&H)[9]) {
#pragma unroll
  for (int x = 0; x < 9; ++x) H[x] = c >= 0 ? cell_rows(cfgs[c], R())[x] : R(0);
}

template <class R>
struct PV {
  R rx, ry, rz, d2;
  int q, zj;
};

// Pair vector of list entry e whose neighbour position xq is already loaded.
template <class R>
__device__ __forceinline__ PV<R> pvec_at(uint32_t e, Vec4<R> xq, Vec4<R> xi, const R (&H)[9]) {
  PV<R> v;
  v.q = (int)(e & kNbrMask);
  R sx, sy, sz;
  image_shift(H, e >> kNbrShift, sx, sy, sz);
  v.rx = (xq.x - xi.x) + sx;
  v.ry = (xq.y - xi.y) + sy;
  v.rz = (xq.z - xi.z) + sz;
  v.d2 = pair_d2(v.rx, v.ry, v.rz);
  v.zj = species_of(xq);
  return v;
}

template <class R>
__device__ __forceinline__ PV<R> pvec(const Vec4<R>* __restrict__ pos4, uint32_t e, Vec4<R> xi, const R (&H)[9]) {
  return pvec_at(e, pos4[e & kNbrMask], xi, H);
}

// The pair lists walked here (compact lists of the forward in float32, the
// Verlet list in float64) are stored in groups of four entries (walk_groups).

// ---------------------------------------------------------------- seeds

// Per reduction item (a chunk of one configuration's atoms, caller order):
// lambda_i = 2 cF (F_i - Fref_i) and the partial sum of (F - Fref)^2.
__global__ __launch_bounds__(kTB) void k_loss_forces(const RedItem* __restrict__ items, int form, double wF,
                                                     double inv_3ntot, int n_cfg, const int64_t* __restrict__ off,
                                                     const float* __restrict__ F, const float* __restrict__ Fref,
                                                     float* __restrict__ lam, double* __restrict__ part) {
  __shared__ double sh[kTB];
  const RedItem it = items[blockIdx.x];
  const double Nc = (double)(off[it.cfg + 1] - off[it.cfg]);
  const double cF = form == 0 ? wF * inv_3ntot : wF / (3.0 * n_cfg * Nc);
  double acc = 0.0;
  for (int64_t a = it.a0 + threadIdx.x; a < it.a1; a += kTB)
    for (int x = 0; x < 3; ++x) {
      const double d = (double)F[3 * a + x] - (double)Fref[3 * a + x];
      acc += d * d;
      lam[3 * a + x] = (float)(2.0 * cF * d);
    }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kTB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * cF;
}

// Energy and virial terms, seeds ebar_c and mu_c, and the loss parts.  One
// block: a thread per configuration, then fixed-order sums in float64.
__global__ __launch_bounds__(kTB) void k_loss_final(int n_cfg, int form, double wE, double wV,
                                                    const int64_t* __restrict__ off,
                                                    const int* __restrict__ item_start,
                                                    const double* __restrict__ partF, const double* __restrict__ E,
                                                    const double* __restrict__ Eref, const double* __restrict__ V,
                                                    const double* __restrict__ Vref, double* __restrict__ ebar,
                                                    double* __restrict__ mu, double* __restrict__ loss) {
  __shared__ double sh[3][kTB];
  double LE = 0.0, LF = 0.0, LV = 0.0;
  const double B = (double)n_cfg;
  for (int c = threadIdx.x; c < n_cfg; c += kTB) {
    const double Nc = (double)(off[c + 1] - off[c]);
    const double cE = form == 0 ? wE / (B * Nc * Nc) : wE / (B * Nc);
    const double cV = form == 0 ? wV / (9.0 * B * Nc * Nc) : wV / (9.0 * B * Nc);
    const double dE = E[c] - Eref[c];
    LE += cE * dE * dE;
    ebar[c] = 2.0 * cE * dE;
    for (int x = 0; x < 9; ++x) {
      const double dV = V[9 * c + x] - Vref[9 * c + x];
      LV += cV * dV * dV;
      mu[9 * c + x] = 2.0 * cV * dV;
    }
    for (int w = item_start[c]; w < item_start[c + 1]; ++w) LF += partF[w];
  }
  sh[0][threadIdx.x] = LE;
  sh[1][threadIdx.x] = LF;
  sh[2][threadIdx.x] = LV;
  __syncthreads();
  for (int st = kTB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int x = 0; x < 3; ++x) sh[x][threadIdx.x] += sh[x][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    loss[0] = sh[0][0] + sh[1][0] + sh[2][0];
    loss[1] = sh[0][0];
    loss[2] = sh[1][0];
    loss[3] = sh[2][0];
  }
}

// lambda to slot order (Vec4<R>); zero on padding slots
template <class R>
__global__ void k_lam_slots(int64_t ns, const int* __restrict__ orig, const R* __restrict__ lam,
                            Vec4<R>* __restrict__ lam4) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const int i = orig[p];
  lam4[p] = i >= 0 ? make_v4<R>(lam[3 * (int64_t)i], lam[3 * (int64_t)i + 1], lam[3 * (int64_t)i + 2], R(0))
                   : make_v4<R>(R(0), R(0), R(0), R(0));
}

// ------------------------------------------------- tangent + network adjoint

// PHASE 1: the tangent pass (radial and angular sums, q and qdot, S and Sdot);
// PHASE 2: the network adjoint (abar, z, dj/dw1, dE/dq, dj/dq), from q and qdot;
// PHASE 3: sigma = dE/dS and Sbar = dj/dS, from S, Sdot, dE/dq and dj/dq.
// Apart, the phases need far fewer registers than one kernel doing all three;
// every hand-over goes through the per-slot arrays of io.
// PHASE 1 runs on a grid (slot blocks, 1 + NA / NC): blockIdx.y = 0 takes the
// radial sums, blockIdx.y = 1 + h the angular chunk h.  The parts write
// disjoint outputs, and running them side by side rather than one after
// another keeps a batch of a few ten thousand atoms from leaving SIMDs idle.
// PHASE 3 runs on a grid (slot blocks, NA), one angular function per row.
// FWD: forward quantities only (q, S, E_i, dE/dq, sigma), for the float64
// evaluation: the tangent parts and the second-order adjoint are skipped.
template <class S, int NC, class R, int PHASE, bool FWD = false>
__global__ __launch_bounds__(kTB) void k_train_atom(TrainIOT<R> io, CutoffsT<R> cut, const R* __restrict__ params) {
  constexpr int T = S::T, NR = S::NR, NA = S::NA, BR = S::BR, BA = S::BA, L = S::L, K = S::K, D = S::D, H = S::H;
  static_assert(NA % NC == 0, "chunk must divide n_angular");
  static_assert(PHASE >= 1 && PHASE <= 3, "phases 1-3");
  constexpr bool kTangent = PHASE == 1, kNet = PHASE == 2, kSigma = PHASE == 3;
  __shared__ R cA_s[kTangent ? T * T * NA * BA : 1];
  if constexpr (kTangent) {
    for (int t = threadIdx.x; t < T * T * NA * BA; t += kTB) cA_s[t] = params[S::PCR + t];
    __syncthreads();
  }
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (p >= ns) return;
  const Vec4<R> xi = io.pos4[p];
  const int Zs = __builtin_amdgcn_readfirstlane(species_of(xi));
  const int c = io.cfg_of[p];
  if (c < 0) {
    // padding: zero every per-slot output that is summed over species ranges
    if constexpr (kTangent) {
      if (blockIdx.y != 0) return;
      for (int d = 0; d < D; ++d) io.q[d * ns + p] = io.qd[d * ns + p] = R(0);
      for (int k = 0; k < T * BR; ++k) io.Pb[k * ns + p] = io.Pdn[k * ns + p] = R(0);
    }
    if constexpr (kNet) {
      for (int h = 0; h < H; ++h) io.abar[h * ns + p] = io.zneg[h * ns + p] = io.gw1[h * ns + p] = R(0);
      for (int n = 0; n < NR; ++n) io.qbR[n * ns + p] = io.FpR[n * ns + p] = R(0);
      io.eat[p] = R(0);
    }
    return;
  }
  const R eb = (R)io.ebar[c];
  if constexpr (kTangent) {
  R Hc[9];
  load_cell9(io.cfgs, c, Hc);
  const R rcR_inv = R(1.0) / cut.rcR, rcA_inv = R(1.0) / cut.rcA;
  const Vec4<R> li = io.lam4[p];
  // lambda_j of each pair, loaded by the pair walker ahead of its prefetches
  auto lam_of = [&](int, uint32_t e) { return io.lam4[e & kNbrMask]; };
  R mu[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) mu[x] = (R)io.mu[9 * c + x];

  // ---- radial: P_b[k] = sum_{j in b} Q_k, Pd_b[k] = sum_{j in b} dQ_k (u.t)
  if (blockIdx.y == 0) {
    R P[T][BR], Pd[T][BR];
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int k = 0; k < BR; ++k) P[b][k] = Pd[b][k] = R(0);
    (void)Pd;
    const int n = io.cntR[p];
    walk_groups(reinterpret_cast<const uint4*>(io.nbrR), ns, p, n, io.pos4, lam_of,
                                          [&](int, uint32_t e, Vec4<R> xq, uint32_t, Vec4<R> lj) {
      const PV<R> v = pvec_at(e, xq, xi, Hc);
      if (v.d2 < cut.rcR2) {
        const R d = sqrt_(v.d2), inv = R(1.0) / d;
        R Q[BR], dQ[BR];
        cheb_basis_d<BR>(d, rcR_inv, Q, dQ);
        if constexpr (FWD) {
#pragma unroll
          for (int b = 0; b < T; ++b) {
            const R m = (T == 1 || v.zj == b) ? R(1.0) : R(0.0);
#pragma unroll
            for (int kk = 0; kk < BR; ++kk) P[b][kk] = fma_(m, Q[kk], P[b][kk]);
          }
        } else {
          const R tx = lj.x - li.x + mu[0] * v.rx + mu[1] * v.ry + mu[2] * v.rz;
          const R ty = lj.y - li.y + mu[3] * v.rx + mu[4] * v.ry + mu[5] * v.rz;
          const R tz = lj.z - li.z + mu[6] * v.rx + mu[7] * v.ry + mu[8] * v.rz;
          const R ut = (v.rx * tx + v.ry * ty + v.rz * tz) * inv;
#pragma unroll
          for (int b = 0; b < T; ++b) {
            const R m = (T == 1 || v.zj == b) ? R(1.0) : R(0.0);
            const R mut = m * ut;
#pragma unroll
            for (int kk = 0; kk < BR; ++kk) {
              P[b][kk] = fma_(m, Q[kk], P[b][kk]);
              Pd[b][kk] = fma_(mut, dQ[kk], Pd[b][kk]);
            }
          }
        }
      }
    });
    const R* cR = params + (int64_t)Zs * (T * NR * BR);
#pragma unroll
    for (int nn = 0; nn < NR; ++nn) {
      R a = R(0), ad = R(0);
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) {
          a = fma_(cR[(b * NR + nn) * BR + kk], P[b][kk], a);
          ad = fma_(cR[(b * NR + nn) * BR + kk], Pd[b][kk], ad);
        }
      io.q[(int64_t)nn * ns + p] = a;
      if constexpr (!FWD) io.qd[(int64_t)nn * ns + p] = ad;
    }
    if constexpr (!FWD) {
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) {
          io.Pb[(b * BR + kk) * ns + p] = P[b][kk];
          io.Pdn[(b * BR + kk) * ns + p] = -Pd[b][kk];
        }
    }
  }
  // ---- angular: S and Sdot in chunks of NC functions (stored for the adjoint)
  if (blockIdx.y > 0) {
    const int h = (int)blockIdx.y - 1;
    const int nA = io.cntA[p];
    R Sg[NC][K], Sd[NC][K];
#pragma unroll
    for (int nn = 0; nn < NC; ++nn)
#pragma unroll
      for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = Sd[nn][lm] = R(0);
    walk_groups(reinterpret_cast<const uint4*>(io.nbrA), ns, p, nA, io.pos4, lam_of,
                                          [&](int, uint32_t e, Vec4<R> xq, uint32_t, Vec4<R> lj) {
      const PV<R> v = pvec_at(e, xq, xi, Hc);
      if (v.d2 < cut.rcA2) {
        const R d = sqrt_(v.d2), inv = R(1.0) / d;
        const R ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
        R Q[BA], dQ[BA];
        cheb_basis_d<BA>(d, rcA_inv, Q, dQ);
        R Y[K], Dl[K];
        real_sph<L>(ux, uy, uz, Y);
        const R* cl = cA_s + ((Zs * T + v.zj) * NA + h * NC) * BA;
        if constexpr (FWD) {
#pragma unroll
          for (int nn = 0; nn < NC; ++nn) {
            R g = R(0);
#pragma unroll
            for (int kk = 0; kk < BA; ++kk) g = fma_(cl[nn * BA + kk], Q[kk], g);
#pragma unroll
            for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = fma_(g, Y[lm], Sg[nn][lm]);
          }
          (void)Dl;
          (void)dQ;
          return;
        }
        const R tx = lj.x - li.x + mu[0] * v.rx + mu[1] * v.ry + mu[2] * v.rz;
        const R ty = lj.y - li.y + mu[3] * v.rx + mu[4] * v.ry + mu[5] * v.rz;
        const R tz = lj.z - li.z + mu[6] * v.rx + mu[7] * v.ry + mu[8] * v.rz;
        const R ut = ux * tx + uy * ty + uz * tz;
        // grad_r Y_lm . t = grad P_lm . (t - (u.t) u) / d
        real_sph_dir<L>(ux, uy, uz, (tx - ut * ux) * inv, (ty - ut * uy) * inv, (tz - ut * uz) * inv, Dl);
#pragma unroll
        for (int nn = 0; nn < NC; ++nn) {
          R g = R(0), gp = R(0);
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) {
            g = fma_(cl[nn * BA + kk], Q[kk], g);
            gp = fma_(cl[nn * BA + kk], dQ[kk], gp);
          }
          const R gput = gp * ut;
#pragma unroll
          for (int lm = 0; lm < K; ++lm) {
            Sg[nn][lm] = fma_(g, Y[lm], Sg[nn][lm]);
            Sd[nn][lm] = fma_(gput, Y[lm], fma_(g, Dl[lm], Sd[nn][lm]));
          }
        }
      }
    });
#pragma unroll
    for (int nn = 0; nn < NC; ++nn) {
      const int n = h * NC + nn;
#pragma unroll
      for (int lm = 0; lm < K; ++lm) {
        io.Sst[(int64_t)(n * K + lm) * ns + p] = Sg[nn][lm];
        if constexpr (!FWD) io.Sdt[(int64_t)(n * K + lm) * ns + p] = Sd[nn][lm];
      }
      R q1 = R(0), qd1 = R(0);
#pragma unroll
      for (int l = 1; l <= L; ++l) {
        R s = R(0), sd = R(0);
#pragma unroll
        for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) {
          s = fma_(Sg[nn][lm], Sg[nn][lm], s);
          sd = fma_(Sg[nn][lm], Sd[nn][lm], sd);
        }
        io.q[(int64_t)(NR + (l - 1) * NA + n) * ns + p] = s;
        if constexpr (!FWD) io.qd[(int64_t)(NR + (l - 1) * NA + n) * ns + p] = R(2.0) * sd;
        if (l == 1) {
          q1 = s;
          qd1 = R(2.0) * sd;
        }
      }
      if constexpr (S::F4) {
        R A[6], Ad[6], A2[6];
        sym_from_s2(&Sg[nn][3], A);
        sym_from_s2(&Sd[nn][3], Ad);
        sym_sq6(A, A2);
        io.q[(int64_t)(S::OFF4 + n) * ns + p] = sym_dot(A2, A);
        if constexpr (!FWD) io.qd[(int64_t)(S::OFF4 + n) * ns + p] = R(3.0) * sym_dot(A2, Ad);
      }
      if constexpr (S::F5) {
        io.q[(int64_t)(S::OFF5 + n) * ns + p] = q1 * q1;
        if constexpr (!FWD) io.qd[(int64_t)(S::OFF5 + n) * ns + p] = R(2.0) * q1 * qd1;
      }
    }
  }
  }  // tangent pass
  if constexpr (kNet) {
  // ---- network, second-order adjoint; pass 1: abar, z, dj/dw1
  const R* W0 = params + S::PCR + S::PCA + (int64_t)Zs * S::PMLP;
  const R* b0 = W0 + H * D;
  const R* w1 = b0 + H;
  {
    R q[D], qd[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      q[d] = io.q[(int64_t)d * ns + p];
      qd[d] = FWD ? R(0) : io.qd[(int64_t)d * ns + p];
    }
    R Esite = w1[H];  // E_i = b1 + sum_h w1_h h_h (written by the float64 variant)
    for (int hh = 0; hh < H; ++hh) {
      R a = b0[hh], ad = R(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        a = fma_(W0[hh * D + d], q[d], a);
        if constexpr (!FWD) ad = fma_(W0[hh * D + d], qd[d], ad);
      }
      const R t = tanh_(a);
      Esite = fma_(w1[hh], t, Esite);
      const R s2 = R(1.0) - t * t;
      const R z = w1[hh] * s2;
      if constexpr (!FWD) {
        io.abar[(int64_t)hh * ns + p] = z * (eb + R(2.0) * t * ad);
        io.gw1[(int64_t)hh * ns + p] = eb * t - s2 * ad;
      }
      io.zneg[(int64_t)hh * ns + p] = -z;
    }
    if constexpr (sizeof(R) == 8) {
      if (io.Ei) io.Ei[io.orig[p]] = Esite;
    }
  }
  if constexpr (!FWD) io.eat[p] = eb;
  // pass 2: qbar = W0^T abar, Fp = W0^T z
  R qb[D], Fp[D];
#pragma unroll
  for (int d = 0; d < D; ++d) qb[d] = Fp[d] = R(0);
  for (int hh = 0; hh < H; ++hh) {
    const R z = -io.zneg[(int64_t)hh * ns + p];
    const R ab = FWD ? R(0) : io.abar[(int64_t)hh * ns + p];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if constexpr (!FWD) qb[d] = fma_(ab, W0[hh * D + d], qb[d]);
      Fp[d] = fma_(z, W0[hh * D + d], Fp[d]);
    }
  }
#pragma unroll
  for (int nn = 0; nn < NR; ++nn) {
    if constexpr (!FWD) io.qbR[(int64_t)nn * ns + p] = qb[nn];
    io.FpR[(int64_t)nn * ns + p] = Fp[nn];
  }
#pragma unroll
  for (int d = NR; d < D; ++d) {
    if constexpr (!FWD) io.qbA[(int64_t)d * ns + p] = qb[d];
    io.FpA[(int64_t)d * ns + p] = Fp[d];
  }
  }  // network
  if constexpr (!kSigma) return;
  // dE/dq_d and dj/dq_d of descriptor d, as the network pass stored them
  auto Fp_at = [&](int d) { return io.FpA[(int64_t)d * ns + p]; };
  auto qb_at = [&](int d) { return io.qbA[(int64_t)d * ns + p]; };
  // ---- sigma = dE/dS and Sbar = dj/dS from the stored S and Sdot
  {
    const int n = blockIdx.y;
    R Sg[K], Sd[K];
#pragma unroll
    for (int lm = 0; lm < K; ++lm) {
      Sg[lm] = io.Sst[(int64_t)(n * K + lm) * ns + p];
      Sd[lm] = FWD ? R(0) : io.Sdt[(int64_t)(n * K + lm) * ns + p];
    }
    R g4s[5] = {0, 0, 0, 0, 0}, g4b[5] = {0, 0, 0, 0, 0};
    if constexpr (S::F4) {
      R A[6], Ad[6], A2[6], Msig[6], Mbar[6];
      sym_from_s2(&Sg[3], A);
      sym_from_s2(&Sd[3], Ad);
      sym_sq6(A, A2);
      R AAd[9], AdA[9];
      sym_mul_sym(A, Ad, AAd);
      sym_mul_sym(Ad, A, AdA);
      const R fp4 = Fp_at(S::OFF4 + n), qb4 = FWD ? R(0) : qb_at(S::OFF4 + n);
      const int ix[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
#pragma unroll
      for (int x = 0; x < 6; ++x) {
        const R sym = AAd[3 * ix[x][0] + ix[x][1]] + AdA[3 * ix[x][0] + ix[x][1]];
        Msig[x] = R(3.0) * fp4 * A2[x];
        Mbar[x] = R(3.0) * qb4 * A2[x] - R(3.0) * fp4 * sym;
      }
      chain_s2(Msig, g4s);
      chain_s2(Mbar, g4b);
    }
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      const R fp3 = Fp_at(NR + (l - 1) * NA + n), qb3 = FWD ? R(0) : qb_at(NR + (l - 1) * NA + n);
      R fp5 = R(0), qb5 = R(0);
      if constexpr (S::F5) {
        fp5 = Fp_at(S::OFF5 + n);
        qb5 = FWD ? R(0) : qb_at(S::OFF5 + n);
      }
      R cs = R(2.0) * fp3;   // sigma = cs S
      R cbS = R(2.0) * qb3;  // Sbar = cbS S + cbD Sdot
      R cbD = -R(2.0) * fp3;
      if (S::F5 && l == 1) {
        const R q1 = io.q[(int64_t)(NR + n) * ns + p], qd1 = FWD ? R(0) : io.qd[(int64_t)(NR + n) * ns + p];
        cs += R(4.0) * fp5 * q1;
        cbS += R(4.0) * qb5 * q1 - R(4.0) * fp5 * qd1;
        cbD += -R(4.0) * fp5 * q1;
      }
#pragma unroll
      for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) {
        R sg = cs * Sg[lm];
        R sb = cbS * Sg[lm] + cbD * Sd[lm];
        if (S::F4 && l == 2) {
          sg += g4s[lm - 3];
          sb += g4b[lm - 3];
        }
        io.Sst[(int64_t)(n * K + lm) * ns + p] = sg;
        if constexpr (!FWD) io.Sdt[(int64_t)(n * K + lm) * ns + p] = sb;
      }
    }
  }
}

// ------------------------------------------------ angular coefficient pass

// GA[(b NA + n) BA + k] = sum over angular pairs j of species b of
//   (alpha_n + gamma_n) Q_k + beta_n dQ_k,
// alpha_n = sum_lm Sbar Y, beta_n = -(u.t) sum_lm sigma Y, gamma_n = -sum_lm sigma grad Y.t
// One thread per (atom, n): grid (slot blocks, NA).  The NA walks of an atom's
// pairs run side by side instead of one after another, so a batch of a few
// ten thousand atoms still puts several waves on every SIMD.
template <class S, class R>
__global__ __launch_bounds__(kTB) void k_train_coefA(TrainIOT<R> io, CutoffsT<R> cut, const R* __restrict__ params) {
  constexpr int T = S::T, NA = S::NA, BA = S::BA, L = S::L, K = S::K;
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  const int n = blockIdx.y;
  if (p >= ns) return;
  const int c = io.cfg_of[p];
  if (c < 0) {
    for (int b = 0; b < T; ++b)
      for (int kk = 0; kk < BA; ++kk) io.GA[(int64_t)((b * NA + n) * BA + kk) * ns + p] = R(0);
    return;
  }
  const Vec4<R> xi = io.pos4[p];
  R Hc[9];
  load_cell9(io.cfgs, c, Hc);
  const R rcA_inv = R(1.0) / cut.rcA;
  const Vec4<R> li = io.lam4[p];
  // lambda_j of each pair, loaded by the pair walker ahead of its prefetches
  auto lam_of = [&](int, uint32_t e) { return io.lam4[e & kNbrMask]; };
  R mu[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) mu[x] = (R)io.mu[9 * c + x];
  const int nA = io.cntA[p];
  {
    R sg[K], sb[K];
#pragma unroll
    for (int lm = 0; lm < K; ++lm) {
      sg[lm] = io.Sst[(int64_t)(n * K + lm) * ns + p];
      sb[lm] = io.Sdt[(int64_t)(n * K + lm) * ns + p];
    }
    R G[T][BA];
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int k = 0; k < BA; ++k) G[b][k] = R(0);
    walk_groups(reinterpret_cast<const uint4*>(io.nbrA), ns, p, nA, io.pos4, lam_of,
                                          [&](int, uint32_t e, Vec4<R> xq, uint32_t, Vec4<R> lj) {
      const PV<R> v = pvec_at(e, xq, xi, Hc);
      if (v.d2 < cut.rcA2) {
        const R d = sqrt_(v.d2), inv = R(1.0) / d;
        const R ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
        R Q[BA], dQ[BA];
        cheb_basis_d<BA>(d, rcA_inv, Q, dQ);
        const R tx = lj.x - li.x + mu[0] * v.rx + mu[1] * v.ry + mu[2] * v.rz;
        const R ty = lj.y - li.y + mu[3] * v.rx + mu[4] * v.ry + mu[5] * v.rz;
        const R tz = lj.z - li.z + mu[6] * v.rx + mu[7] * v.ry + mu[8] * v.rz;
        const R ut = ux * tx + uy * ty + uz * tz;
        R Y[K], Dl[K];
        real_sph<L>(ux, uy, uz, Y);
        real_sph_dir<L>(ux, uy, uz, (tx - ut * ux) * inv, (ty - ut * uy) * inv, (tz - ut * uz) * inv, Dl);
        R al = R(0), sy = R(0), ga = R(0);
#pragma unroll
        for (int lm = 0; lm < K; ++lm) {
          al = fma_(sb[lm], Y[lm], al);
          sy = fma_(sg[lm], Y[lm], sy);
          ga = fma_(sg[lm], Dl[lm], ga);
        }
        const R cq = al - ga, cd = -ut * sy;
#pragma unroll
        for (int b = 0; b < T; ++b) {
          const R m = (T == 1 || v.zj == b) ? R(1.0) : R(0.0);
          const R mq = m * cq, md = m * cd;
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) G[b][kk] = fma_(mq, Q[kk], fma_(md, dQ[kk], G[b][kk]));
        }
      }
    });
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int kk = 0; kk < BA; ++kk) io.GA[(int64_t)((b * NA + n) * BA + kk) * ns + p] = G[b][kk];
  }
}

// ---------------------------------------------------- species reductions

constexpr int kRB = 256;       // threads per reduction block
constexpr int kRChunk = 32;    // slots staged per step
constexpr int kRS = kRChunk + 1;  // LDS row stride: odd, so that lanes reading
                                  // one column of different rows hit distinct banks

// part[(s * kRBlocks + blk) * A*B + e] = sum over slots i of species s handled
// by block blk of  X1[a][i] Y1[b][i] + X2[a][i] Y2[b][i]  (e = a*B + b).
// Chunks of kRChunk slots are staged in LDS, every load of a chunk issued
// before the first store (so a chunk costs one memory latency); each thread
// owns a kOB x kOB block of entries, so one set of LDS reads feeds kOB^2
// products: 4 x 4 when that still leaves at least 128 blocks of entries, else
// 2 x 2 (small products would otherwise run on a few threads).  Per chunk an
// entry is summed in float in slot order, then added in float64.
template <int A, int B>
constexpr int outer_block() {
  return ((A + 3) / 4) * ((B + 3) / 4) >= 128 ? 4 : 2;
}
template <class X, int A, int B>
__device__ __forceinline__ void outer_sum_block(int64_t ns, const int* __restrict__ base, const X* __restrict__ X1,
                                                const X* __restrict__ Y1, const X* __restrict__ X2,
                                                const X* __restrict__ Y2, double* __restrict__ part, X* lds) {
  X* sx1 = lds;  // LDS rows of X1, X2, Y1, Y2 (2 (A + B) kRS values)
  X* sx2 = sx1 + A * kRS;
  X* sy1 = sx2 + A * kRS;
  X* sy2 = sy1 + B * kRS;
  constexpr int kOB = outer_block<A, B>();
  constexpr int nbB = (B + kOB - 1) / kOB, nblk = ((A + kOB - 1) / kOB) * nbB;
  static_assert(nblk <= kRB, "one entry block per thread");
  constexpr int TA = (A * kRChunk + kRB - 1) / kRB, TB = (B * kRChunk + kRB - 1) / kRB;
  const int s = blockIdx.y, blk = blockIdx.x;
  const int p0 = base[s], p1 = base[s + 1];
  const bool own = (int)threadIdx.x < nblk;
  const int a0 = own ? ((int)threadIdx.x / nbB) * kOB : 0, b0 = own ? ((int)threadIdx.x % nbB) * kOB : 0;
  int ra[kOB], rb[kOB];  // LDS rows, clamped (entries past A or B are computed and dropped)
#pragma unroll
  for (int r = 0; r < kOB; ++r) {
    ra[r] = min(a0 + r, A - 1) * kRS;
    rb[r] = min(b0 + r, B - 1) * kRS;
  }
  double acc[kOB][kOB];
#pragma unroll
  for (int r = 0; r < kOB; ++r)
#pragma unroll
    for (int c = 0; c < kOB; ++c) acc[r][c] = 0.0;
  for (int c0 = p0 + blk * kRChunk; c0 < p1; c0 += kRBlocks * kRChunk) {
    const int nc = min(kRChunk, p1 - c0);
    X va1[TA], va2[TA], vb1[TB], vb2[TB];
#pragma unroll
    for (int u = 0; u < TA; ++u) {
      const int t = threadIdx.x + u * kRB, r = t / kRChunk, i = t % kRChunk;
      const bool ok = t < A * kRChunk && i < nc;
      va1[u] = ok ? X1[(int64_t)r * ns + c0 + i] : X(0);
      va2[u] = ok ? X2[(int64_t)r * ns + c0 + i] : X(0);
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int t = threadIdx.x + u * kRB, r = t / kRChunk, i = t % kRChunk;
      const bool ok = t < B * kRChunk && i < nc;
      vb1[u] = ok ? Y1[(int64_t)r * ns + c0 + i] : X(0);
      vb2[u] = ok ? Y2[(int64_t)r * ns + c0 + i] : X(0);
    }
    __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
    for (int u = 0; u < TA; ++u) {
      const int t = threadIdx.x + u * kRB;
      if (t < A * kRChunk) {
        sx1[(t / kRChunk) * kRS + t % kRChunk] = va1[u];
        sx2[(t / kRChunk) * kRS + t % kRChunk] = va2[u];
      }
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int t = threadIdx.x + u * kRB;
      if (t < B * kRChunk) {
        sy1[(t / kRChunk) * kRS + t % kRChunk] = vb1[u];
        sy2[(t / kRChunk) * kRS + t % kRChunk] = vb2[u];
      }
    }
    __syncthreads();
    if (own) {
      X s1[kOB][kOB];
#pragma unroll
      for (int r = 0; r < kOB; ++r)
#pragma unroll
        for (int c = 0; c < kOB; ++c) s1[r][c] = X(0);
      for (int i = 0; i < kRChunk; ++i) {
        X x1[kOB], x2[kOB], y1[kOB], y2[kOB];
#pragma unroll
        for (int r = 0; r < kOB; ++r) {
          x1[r] = sx1[ra[r] + i];
          x2[r] = sx2[ra[r] + i];
          y1[r] = sy1[rb[r] + i];
          y2[r] = sy2[rb[r] + i];
        }
#pragma unroll
        for (int r = 0; r < kOB; ++r)
#pragma unroll
          for (int c = 0; c < kOB; ++c) s1[r][c] = fma_(x1[r], y1[c], fma_(x2[r], y2[c], s1[r][c]));
      }
#pragma unroll
      for (int r = 0; r < kOB; ++r)
#pragma unroll
        for (int c = 0; c < kOB; ++c) acc[r][c] += (double)s1[r][c];
    }
  }
  if (!own) return;
#pragma unroll
  for (int r = 0; r < kOB; ++r)
#pragma unroll
    for (int c = 0; c < kOB; ++c)
      if (a0 + r < A && b0 + c < B) part[((int64_t)s * kRBlocks + blk) * (A * B) + (a0 + r) * B + b0 + c] = acc[r][c];
}

// Two outer-product sums in one launch, grid (kRBlocks, T, 2): blockIdx.z
// picks the product (A0 x B0 or A1 x B1); one LDS buffer fits either.
template <class X, int A0, int B0, int A1, int B1>
__global__ __launch_bounds__(kRB) void k_outer2(int64_t ns, const int* __restrict__ base, const X* __restrict__ X1a,
                                                const X* __restrict__ Y1a, const X* __restrict__ X2a,
                                                const X* __restrict__ Y2a, double* __restrict__ Pa,
                                                const X* __restrict__ X1b, const X* __restrict__ Y1b,
                                                const X* __restrict__ X2b, const X* __restrict__ Y2b,
                                                double* __restrict__ Pb) {
  constexpr int L0 = 2 * (A0 + B0) * kRS, L1 = 2 * (A1 + B1) * kRS;
  __shared__ X lds[L0 > L1 ? L0 : L1];
  if (blockIdx.z == 0)
    outer_sum_block<X, A0, B0>(ns, base, X1a, Y1a, X2a, Y2a, Pa, lds);
  else
    outer_sum_block<X, A1, B1>(ns, base, X1b, Y1b, X2b, Y2b, Pb, lds);
}

// part[(s * kRBlocks + blk) * A + a] = sum over the block's slots of X[a][i].
// A block of kCB threads; wavefront w takes rows w, w + kCB/64, ...  Lanes sit
// on consecutive slots (coalesced), and all of a wavefront's rows are loaded
// before any is reduced (one memory latency per 64-slot chunk); each chunk is
// summed across the lanes in a fixed butterfly order (lane 0's sum is used),
// then added in float64.
constexpr int kCB = 1024;
template <class X, int A>
__device__ __forceinline__ void colsum_block(int64_t ns, const int* __restrict__ base, const X* __restrict__ Xa,
                                             double* __restrict__ part) {
  constexpr int NW = kCB / kWave, RPW = (A + NW - 1) / NW;
  const int s = blockIdx.y, blk = blockIdx.x;
  const int p0 = base[s], p1 = base[s + 1];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  double acc[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) acc[r] = 0.0;
  for (int c0 = p0 + blk * kWave; c0 < p1; c0 += kRBlocks * kWave) {
    const int i = c0 + lane;
    X v[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int a = wv + NW * r;
      v[r] = (a < A && i < p1) ? Xa[(int64_t)a * ns + i] : X(0);
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off);
      acc[r] += (double)v[r];
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int a = wv + NW * r;
      if (a < A) part[((int64_t)s * kRBlocks + blk) * A + a] = acc[r];
    }
  }
}

// Four column sums in one launch, grid (kRBlocks, T, 4): blockIdx.z picks
// the sum (X0 has A0 rows, X1 and X2 A1 rows, X3 one row).
template <class X, int A0, int A1>
__global__ __launch_bounds__(kCB) void k_colsum4(int64_t ns, const int* __restrict__ base, const X* __restrict__ X0,
                                                 double* __restrict__ P0, const X* __restrict__ X1,
                                                 double* __restrict__ P1, const X* __restrict__ X2,
                                                 double* __restrict__ P2, const X* __restrict__ X3,
                                                 double* __restrict__ P3) {
  switch (blockIdx.z) {
    case 0: colsum_block<X, A0>(ns, base, X0, P0); break;
    case 1: colsum_block<X, A1>(ns, base, X1, P1); break;
    case 2: colsum_block<X, A1>(ns, base, X2, P2); break;
    default: colsum_block<X, 1>(ns, base, X3, P3); break;
  }
}

// The gradient sums of one backward pass, each with its own region of the
// partial-sum buffer, finished by one launch.  Segment g covers threads
// [first[g], first[g + 1]), one per (species s, entry e):
// grad[dst(s, e)] = sum_blk part[part_off + (s kRBlocks + blk) E + e];  dst = off + s * sstride + map(e)
// map: kind 0 identity; kind 1: e = n*(T*BR) + b*BR + k -> (b*NR + n)*BR + k
constexpr int kPartSegs = 6;
struct PartSeg {
  int E, kind;
  int64_t part_off, off, sstride;
};
struct PartPlan {
  int T, NR, BR, n;
  int64_t first[kPartSegs + 1];
  PartSeg seg[kPartSegs];
  int64_t used;  // doubles of the partial-sum buffer taken so far
  // region of the next segment's partial sums (host side)
  double* add(double* part, int E, int64_t off, int64_t sstride, int kind) {
    if (n >= kPartSegs) std::abort();  // a fixed set of sums per backward pass
    PartSeg& g = seg[n];
    g.E = E;
    g.kind = kind;
    g.part_off = used;
    g.off = off;
    g.sstride = sstride;
    first[n + 1] = first[n] + (int64_t)T * E;
    ++n;
    used += (int64_t)T * kRBlocks * E;
    return part + g.part_off;
  }
};
static PartPlan part_plan(int T, int NR, int BR) {
  PartPlan pl{};
  pl.T = T;
  pl.NR = NR;
  pl.BR = BR;
  return pl;
}
__global__ void k_part_final(PartPlan pl, const double* __restrict__ part, double* __restrict__ grad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= pl.first[pl.n]) return;
  int g = 0;
  while (g + 1 < pl.n && t >= pl.first[g + 1]) ++g;
  const int E = pl.seg[g].E, kind = pl.seg[g].kind, T = pl.T, NR = pl.NR, BR = pl.BR;
  const int64_t off = pl.seg[g].off, sstride = pl.seg[g].sstride;
  const int64_t u = t - pl.first[g];
  const int s = (int)(u / E), e = (int)(u % E);
  // four interleaved partial sums, combined in a fixed order; 64 loads are
  // issued per round trip
  static_assert(kRBlocks % 64 == 0, "partials come in sixty-fours");
  double a4[4] = {0.0, 0.0, 0.0, 0.0};
  const double* src = part + pl.seg[g].part_off + (int64_t)s * kRBlocks * E + e;
  for (int blk = 0; blk < kRBlocks; blk += 64) {
    double v[64];
#pragma unroll
    for (int u = 0; u < 64; ++u) v[u] = src[(int64_t)(blk + u) * E];
#pragma unroll
    for (int u = 0; u < 64; ++u) a4[u & 3] += v[u];
  }
  const double acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  int64_t dst = e;
  if (kind == 1) {
    const int n = e / (T * BR), r = e % (T * BR), b = r / BR, k = r % BR;
    dst = ((int64_t)b * NR + n) * BR + k;
  }
  grad[off + (int64_t)s * sstride + dst] = acc;
}

__global__ void k_to_float(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

static inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------- float64 variant

__global__ void k_fill64(int64_t n, double v, double* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_round_pos(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Positions in slot order, float64, wrapped by the same lattice vector as the
// float32 staging that built the lists: that vector is the integer nearest to
// (x_f - x_f,wrapped) H^-1, where x_f is the float32 rounding of the position.
__global__ void k_stage64(int64_t ns, const int* __restrict__ orig, const int* __restrict__ cfg_of,
                          const CfgDev* __restrict__ cfgs, const float4* __restrict__ pos4f,
                          const double* __restrict__ pos, double4* __restrict__ pos4) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const float4 wf = pos4f[p];
  const int i = orig[p], c = cfg_of[p];
  if (i < 0 || c < 0) {
    pos4[p] = make_double4(0.0, 0.0, 0.0, (double)species_of(wf));
    return;
  }
  const CfgDev& C = cfgs[c];
  const double x[3] = {pos[3 * (int64_t)i], pos[3 * (int64_t)i + 1], pos[3 * (int64_t)i + 2]};
  const double dx[3] = {(double)(float)x[0] - (double)wf.x, (double)(float)x[1] - (double)wf.y,
                        (double)(float)x[2] - (double)wf.z};
  double m[3];
  for (int a = 0; a < 3; ++a) m[a] = rint(dx[0] * C.Hinv[a] + dx[1] * C.Hinv[3 + a] + dx[2] * C.Hinv[6 + a]);
  double w[3];
  for (int a = 0; a < 3; ++a) w[a] = x[a] - m[0] * C.Hd[a] - m[1] * C.Hd[3 + a] - m[2] * C.Hd[6 + a];
  pos4[p] = make_double4(w[0], w[1], w[2], (double)species_of(wf));
}

// Constants of the float64 force kernels.  Float64 instructions take no
// 64-bit literal operands, so every constant of the pair arithmetic that the
// compiler hoists out of a pair loop holds two registers for the whole loop
// (about a hundred of them here, which spills).  The kernels read them instead
// through a pointer made opaque once per pair: they are then loaded with scalar
// loads where they are used.
struct K64 {
  double sc[12];  // sin(pi w) = w sum_k sc[k] w^(2k),  sc[k] = (-1)^k pi^(2k+1) / (2k+1)!
  double cc[12];  // cos(pi w) = sum_k cc[k] w^(2k),    cc[k] = (-1)^k pi^(2k) / (2k)!
  double pi;
  double c1, k20, k21, k22, k30, k31, k32, k32s, k33, k40, k41, k42, k42s, k43, k44, k44s;
  double n3, n5, n6, n7, n10, n14, n15, n21, n30, n35, n60, n140;
};

constexpr K64 make_k64() {
  using C = ShC<double>;
  K64 k{};
  // Taylor series of sin and cos at 0; on |w| <= 1/2 the first omitted terms,
  // (pi/2)^25 / 25! and (pi/2)^24 / 24!, are below 2e-20.
  double s = C::pi, c = 1.0;
  for (int j = 0; j < 12; ++j) {
    k.sc[j] = s;
    k.cc[j] = c;
    s = -s * C::pi * C::pi / ((2.0 * j + 2.0) * (2.0 * j + 3.0));
    c = -c * C::pi * C::pi / ((2.0 * j + 1.0) * (2.0 * j + 2.0));
  }
  k.pi = C::pi;
  k.c1 = C::c1;
  k.k20 = C::k20;
  k.k21 = C::k21;
  k.k22 = C::k22;
  k.k30 = C::k30;
  k.k31 = C::k31;
  k.k32 = C::k32;
  k.k32s = C::k32s;
  k.k33 = C::k33;
  k.k40 = C::k40;
  k.k41 = C::k41;
  k.k42 = C::k42;
  k.k42s = C::k42s;
  k.k43 = C::k43;
  k.k44 = C::k44;
  k.k44s = C::k44s;
  k.n3 = 3.0;
  k.n5 = 5.0;
  k.n6 = 6.0;
  k.n7 = 7.0;
  k.n10 = 10.0;
  k.n14 = 14.0;
  k.n15 = 15.0;
  k.n21 = 21.0;
  k.n30 = 30.0;
  k.n35 = 35.0;
  k.n60 = 60.0;
  k.n140 = 140.0;
  return k;
}
__device__ const K64 kK64 = make_k64();

// The table through an address the compiler cannot see as loop-invariant, in
// the constant address space (scalar loads).
using K64c = const __attribute__((address_space(4))) K64;
__device__ __forceinline__ K64c& k64_opaque() {
  uint64_t a = reinterpret_cast<uint64_t>(&kK64);
  __asm__ volatile("" : "+s"(a));
  return *reinterpret_cast<K64c*>(a);
}

// sin(pi t) and cos(pi t) for t in [0, 1]: with w = t - 1/2,
// sin(pi t) = cos(pi w) and cos(pi t) = -sin(pi w), |w| <= 1/2.
__device__ __forceinline__ void sincospi64(K64c& K, double t, double& sn, double& cs) {
  const double w = t - 0.5, w2 = w * w;
  double s = K.sc[11], c = K.cc[11];
#pragma unroll
  for (int j = 10; j >= 0; --j) {
    s = fma(s, w2, K.sc[j]);
    c = fma(c, w2, K.cc[j]);
  }
  sn = c;
  cs = -(w * s);
}

// The Chebyshev basis of Eq. 12-15 with its radial derivative, as
// cheb_basis_d, for d < rc, on the float64 force kernels' constants.
template <int B>
__device__ __forceinline__ void cheb_basis64(K64c& K, double d, double rc_inv, double (&Q)[B], double (&dQ)[B]) {
  const double t = d * rc_inv;
  const double y = t - 1.0;
  const double x = 2.0 * y * y - 1.0;
  const double dx = 4.0 * y * rc_inv;
  double sn, cs;
  sincospi64(K, t, sn, cs);
  const double fc = 0.5 * (1.0 + cs);
  const double dfc = -0.5 * K.pi * rc_inv * sn;
  double tm = 1.0, tk = x, dtm = 0.0, dtk = 1.0;
  Q[0] = fc;
  dQ[0] = dfc;
  if (B > 1) {
    Q[1] = 0.5 * (x + 1.0) * fc;
    dQ[1] = 0.5 * (dx * fc + (x + 1.0) * dfc);
  }
#pragma unroll
  for (int k = 2; k < B; ++k) {
    const double tn = 2.0 * x * tk - tm;
    const double dtn = 2.0 * tk + 2.0 * x * dtk - dtm;
    tm = tk;
    tk = tn;
    dtm = dtk;
    dtk = dtn;
    Q[k] = 0.5 * (tn + 1.0) * fc;
    dQ[k] = 0.5 * (dtn * dx * fc + (tn + 1.0) * dfc);
  }
}

// Real harmonics and their gradient one degree l at a time (the polynomials
// of real_sph / real_sph_grad_dot, split by l), so that a float64 pair keeps
// at most 2l + 1 harmonics and weights live.  Yl[m] = P_{l,m}(x, y, z) for
// m = 0..2l, in the order of real_sph.
template <int l>
__device__ __forceinline__ void real_sph_l(K64c& K, double x, double y, double z, double (&Yl)[2 * l + 1]) {
  if constexpr (l == 1) {
    Yl[0] = K.c1 * z;
    Yl[1] = K.c1 * x;
    Yl[2] = K.c1 * y;
  } else if constexpr (l == 2) {
    const double z2 = z * z;
    Yl[0] = K.k20 * (K.n3 * z2 - 1.0);
    Yl[1] = K.k21 * x * z;
    Yl[2] = K.k21 * y * z;
    Yl[3] = K.k22 * (x * x - y * y);
    Yl[4] = K.k21 * x * y;
  } else if constexpr (l == 3) {
    const double z2 = z * z;
    const double x2my2 = x * x - y * y;
    const double p = K.n5 * z2 - 1.0;
    Yl[0] = K.k30 * z * (K.n5 * z2 - K.n3);
    Yl[1] = K.k31 * x * p;
    Yl[2] = K.k31 * y * p;
    Yl[3] = K.k32 * z * x2my2;
    Yl[4] = K.k32s * x * y * z;
    Yl[5] = K.k33 * x * (x * x - K.n3 * y * y);
    Yl[6] = K.k33 * y * (K.n3 * x * x - y * y);
  } else {
    static_assert(l == 4, "l_max <= 4");
    const double z2 = z * z;
    const double x2my2 = x * x - y * y;
    const double q = K.n7 * z2 - K.n3;
    const double r = K.n7 * z2 - 1.0;
    Yl[0] = K.k40 * (K.n35 * z2 * z2 - K.n30 * z2 + K.n3);
    Yl[1] = K.k41 * x * z * q;
    Yl[2] = K.k41 * y * z * q;
    Yl[3] = K.k42 * x2my2 * r;
    Yl[4] = K.k42s * x * y * r;
    Yl[5] = K.k43 * x * z * (x * x - K.n3 * y * y);
    Yl[6] = K.k43 * y * z * (K.n3 * x * x - y * y);
    Yl[7] = K.k44 * (x2my2 * x2my2 - 4.0 * x * x * y * y);
    Yl[8] = K.k44s * x * y * x2my2;
  }
}

// (gx, gy, gz) += sum_m Gl[m] grad_u P_{l,m}(u), degree l only.
template <int l>
__device__ __forceinline__ void real_sph_grad_acc_l(K64c& K, double x, double y, double z,
                                                    const double (&G)[2 * l + 1], double& gx, double& gy,
                                                    double& gz) {
  if constexpr (l == 1) {
    gx += K.c1 * G[1];
    gy += K.c1 * G[2];
    gz += K.c1 * G[0];
  } else if constexpr (l == 2) {
    gz += K.n6 * K.k20 * z * G[0];
    gx += K.k21 * z * G[1];
    gz += K.k21 * x * G[1];
    gy += K.k21 * z * G[2];
    gz += K.k21 * y * G[2];
    gx += 2.0 * K.k22 * x * G[3];
    gy -= 2.0 * K.k22 * y * G[3];
    gx += K.k21 * y * G[4];
    gy += K.k21 * x * G[4];
  } else if constexpr (l == 3) {
    const double z2 = z * z, x2 = x * x, y2 = y * y;
    const double p = K.n5 * z2 - 1.0;
    gz += K.k30 * (K.n15 * z2 - K.n3) * G[0];
    gx += K.k31 * p * G[1];
    gz += K.n10 * K.k31 * x * z * G[1];
    gy += K.k31 * p * G[2];
    gz += K.n10 * K.k31 * y * z * G[2];
    gx += 2.0 * K.k32 * x * z * G[3];
    gy -= 2.0 * K.k32 * y * z * G[3];
    gz += K.k32 * (x2 - y2) * G[3];
    gx += K.k32s * y * z * G[4];
    gy += K.k32s * x * z * G[4];
    gz += K.k32s * x * y * G[4];
    gx += K.n3 * K.k33 * (x2 - y2) * G[5];
    gy -= K.n6 * K.k33 * x * y * G[5];
    gx += K.n6 * K.k33 * x * y * G[6];
    gy += K.n3 * K.k33 * (x2 - y2) * G[6];
  } else {
    static_assert(l == 4, "l_max <= 4");
    const double z2 = z * z, x2 = x * x, y2 = y * y;
    const double q = K.n7 * z2 - K.n3;
    const double r = K.n7 * z2 - 1.0;
    gz += K.k40 * (K.n140 * z2 * z - K.n60 * z) * G[0];
    gx += K.k41 * z * q * G[1];
    gz += K.k41 * x * (K.n21 * z2 - K.n3) * G[1];
    gy += K.k41 * z * q * G[2];
    gz += K.k41 * y * (K.n21 * z2 - K.n3) * G[2];
    gx += 2.0 * K.k42 * x * r * G[3];
    gy -= 2.0 * K.k42 * y * r * G[3];
    gz += K.n14 * K.k42 * z * (x2 - y2) * G[3];
    gx += K.k42s * y * r * G[4];
    gy += K.k42s * x * r * G[4];
    gz += K.n14 * K.k42s * x * y * z * G[4];
    gx += K.n3 * K.k43 * z * (x2 - y2) * G[5];
    gy -= K.n6 * K.k43 * x * y * z * G[5];
    gz += K.k43 * x * (x2 - K.n3 * y2) * G[5];
    gx += K.n6 * K.k43 * x * y * z * G[6];
    gy += K.n3 * K.k43 * z * (x2 - y2) * G[6];
    gz += K.k43 * y * (K.n3 * x2 - y2) * G[6];
    gx += 4.0 * K.k44 * x * (x2 - K.n3 * y2) * G[7];
    gy += 4.0 * K.k44 * y * (y2 - K.n3 * x2) * G[7];
    gx += K.k44s * y * (K.n3 * x2 - y2) * G[8];
    gy += K.k44s * x * (x2 - K.n3 * y2) * G[8];
  }
}

// One degree l of an angular pair, for the NP functions n of one pass:
// Z_j += sum_m sigma_{j,lm} Y_lm and grad += sum_m G_lm grad P_lm with
// G_lm = sum_j sigma_{j,lm} g_j.
template <int l, int NP, int K>
__device__ __forceinline__ void ang_degree64(K64c& KC, const double (&sg)[NP][K], double ux, double uy, double uz,
                                             const double (&g)[NP], double (&Z)[NP], double& gx, double& gy,
                                             double& gz) {
  constexpr int base = l * l - 1;  // index of (l, m = 0) in real_sph's order
  double Y[2 * l + 1], G[2 * l + 1];
  real_sph_l<l>(KC, ux, uy, uz, Y);
#pragma unroll
  for (int m = 0; m < 2 * l + 1; ++m) G[m] = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int m = 0; m < 2 * l + 1; ++m) {
      Z[j] = fma(sg[j][base + m], Y[m], Z[j]);
      G[m] = fma(sg[j][base + m], g[j], G[m]);
    }
  real_sph_grad_acc_l<l>(KC, ux, uy, uz, G, gx, gy, gz);
}

// The part of dE_a/dr_ab of the angular descriptors (Eq. 11-17) that the NP
// functions n of one pass contribute, for centre a and neighbour b at
// r_ab = d u:  with g_n = sum_k c[Za][Zb][n][k] Q_k(d),
//   u sum_n g'_n Z_n + (I - u u^T) grad_u(sum_lm G_lm P_lm) / d,
//   Z_n = sum_lm sigma_nlm Y_lm(u),  G_lm = sum_n sigma_nlm g_n,
// sigma = dE_a/dS_a.  cl: the NP x BA rows of c[Za][Zb] of the pass.
template <class S, int NP>
__device__ __forceinline__ void ang_pair_grad64(K64c& KC, const double (&sg)[NP][S::K], const double* cl, double ux,
                                                double uy, double uz, double d, double d_inv, double rcA_inv,
                                                double& fx, double& fy, double& fz) {
  constexpr int BA = S::BA, L = S::L, K = S::K;
  double g[NP], gp[NP];
  {
    double Q[BA], dQ[BA];
    cheb_basis64<BA>(KC, d, rcA_inv, Q, dQ);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int k = 0; k < BA; ++k) {
        a = fma(cl[j * BA + k], Q[k], a);
        b = fma(cl[j * BA + k], dQ[k], b);
      }
      g[j] = a;
      gp[j] = b;
    }
  }
  double Z[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) Z[j] = 0.0;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  ang_degree64<1, NP, K>(KC, sg, ux, uy, uz, g, Z, gx, gy, gz);
  if constexpr (L >= 2) ang_degree64<2, NP, K>(KC, sg, ux, uy, uz, g, Z, gx, gy, gz);
  if constexpr (L >= 3) ang_degree64<3, NP, K>(KC, sg, ux, uy, uz, g, Z, gx, gy, gz);
  if constexpr (L >= 4) ang_degree64<4, NP, K>(KC, sg, ux, uy, uz, g, Z, gx, gy, gz);
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j) s = fma(gp[j], Z[j], s);
  const double ug = ux * gx + uy * gy + uz * gz;
  fx = s * ux + (gx - ug * ux) * d_inv;
  fy = s * uy + (gy - ug * uy) * d_inv;
  fz = s * uz + (gz - ug * uz) * d_inv;
}

// Radial adjoint in float64, atil_i[b][k] = sum_n dE_i/dq_n c[Z_i][b][n][k],
// stored [T][slot][B_R] (the pair kernel reads i's part Z_j and j's part Z_i,
// 12 contiguous values each, instead of two 8 x 12 coefficient blocks per pair).
template <class S>
__global__ __launch_bounds__(kTB) void k_radial_adj64(int64_t ns, const int* __restrict__ cfg_of,
                                                      const double4* __restrict__ pos4,
                                                      const double* __restrict__ FpR,
                                                      const double* __restrict__ params, double* __restrict__ aR) {
  constexpr int T = S::T, NR = S::NR, BR = S::BR;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (p >= ns || cfg_of[p] < 0) return;
  const int Zi = species_of(pos4[p]);
  double fp[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n) fp[n] = FpR[(int64_t)n * ns + p];
#pragma unroll
  for (int b = 0; b < T; ++b) {
    const double* c = params + ((int64_t)(Zi * T + b) * NR) * BR;
#pragma unroll
    for (int k = 0; k < BR; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int n = 0; n < NR; ++n) acc = fma(fp[n], c[n * BR + k], acc);
      aR[((int64_t)b * ns + p) * BR + k] = acc;
    }
  }
}


// Forces and per-atom virials in float64 (Eq. 3, Eq. 4), from the adjoints
// that the atom pass leaves with zero tangent seeds:
// F_i = sum_j (dE_i/dr_ij - dE_j/dr_ji), W_i = - sum_j dE_i/dr_ij (x) r_ij,
// caller order for F and W.
//
// k_ang_force64: for every entry of the angular part of i's list (rc_angular
// + skin), dE_i/dr_ij of the angular descriptors, from i's own sigma, goes to
// fA at the entry's position (zero beyond rc_angular).  The functions n are
// taken NP at a time: their sigma rows (NP K values) are read once into
// registers and every entry of the atom is visited per pass, its partial
// derivative added to fA.  The coefficient blocks c[Z_i][Z_j] sit in LDS.
template <class S, int NP>
__global__ __launch_bounds__(kTB) void k_ang_force64(TrainIOT<double> io, CutoffsT<double> cut,
                                                     const double* __restrict__ params,
                                                     const uint32_t* __restrict__ nbrTA, int rowTA,
                                                     const int* __restrict__ cntAV, double4* __restrict__ fA) {
  constexpr int NA = S::NA, BA = S::BA, K = S::K;
  static_assert(NA % NP == 0, "passes of NP functions");
  constexpr int NCA = S::T * S::T * NA * BA;
  __shared__ double cAs[NCA];
  for (int x = threadIdx.x; x < NCA; x += kTB) cAs[x] = params[S::PCR + x];
  __syncthreads();
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (p >= ns) return;
  const int c = io.cfg_of[p];
  if (c < 0) return;
  const double4 xi = io.pos4[p];
  const int Zi = species_of(xi);
  double Hc[9];
  load_cell9(io.cfgs, c, Hc);
  const double rcA_inv = 1.0 / cut.rcA;
  const uint32_t* row = nbrTA + p * rowTA;
  const int n = cntAV[p];
#pragma unroll 1
  for (int h = 0; h < NA; h += NP) {
    double sg[NP][K];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int lm = 0; lm < K; ++lm) sg[j][lm] = io.Sst[(int64_t)((h + j) * K + lm) * ns + p];
    for (int ka = 0; ka < n; ++ka) {
      const PV<double> v = pvec(io.pos4, row[ka], xi, Hc);
      double ax = 0.0, ay = 0.0, az = 0.0;
      if (v.d2 < cut.rcA2) {
        const double d = sqrt(v.d2);
        const double d_inv = 1.0 / d;
        const double* cl = cAs + ((Zi * S::T + v.zj) * NA + h) * BA;
        ang_pair_grad64<S, NP>(k64_opaque(), sg, cl, v.rx * d_inv, v.ry * d_inv, v.rz * d_inv, d, d_inv, rcA_inv,
                               ax, ay, az);
      }
      double4* o = fA + (int64_t)ka * ns + p;
      if (h > 0) {
        const double4 prev = *o;
        ax += prev.x;
        ay += prev.y;
        az += prev.z;
      }
      *o = make_double4(ax, ay, az, 0.0);
    }
  }
}

// k_force64 walks i's whole list once.  A radial pair takes both directions
// at once through the two adjoint rows of k_radial_adj64:
// dE_i/dd = sum_k atil_i[Z_j][k] dQ_k and dE_j/dd = sum_k atil_j[Z_i][k] dQ_k.
// An entry of the angular part adds i's own angular dE_i/dr_ij (fA at its
// position in i's angular part, also into W_i) and subtracts the partner's
// dE_j/dr_ji, which sits at i's position in the angular part of j's list
// (the reverse index).
template <class S>
__global__ __launch_bounds__(kTB) void k_force64(TrainIOT<double> io, CutoffsT<double> cut,
                                                 const double* __restrict__ aR, const uint32_t* __restrict__ vrev,
                                                 const double4* __restrict__ fA, double* __restrict__ F,
                                                 double* __restrict__ W) {
  constexpr int BR = S::BR;
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (p >= ns) return;
  const int c = io.cfg_of[p];
  if (c < 0) return;
  const int i = io.orig[p];
  const double4 xi = io.pos4[p];
  const int Zi = species_of(xi);
  double Hc[9];
  load_cell9(io.cfgs, c, Hc);
  const double rcR_inv = 1.0 / cut.rcR;
  // i's own adjoint rows atil_i[b][.] for every neighbour species b, held for
  // the whole walk (read once instead of once per pair)
  double Ai[S::T][BR];
#pragma unroll
  for (int b = 0; b < S::T; ++b)
#pragma unroll
    for (int kk = 0; kk < BR; ++kk) Ai[b][kk] = aR[((int64_t)b * ns + p) * BR + kk];
  double Fx = 0.0, Fy = 0.0, Fz = 0.0, Wm[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) Wm[x] = 0.0;
  const int n = io.cntR[p];
  int ka = 0;  // position in the angular part of i's list
  for (int k = 0; k < n; ++k) {
    const int64_t gk = group_index(ns, p, k);
    const uint32_t rv = vrev[gk];
    const PV<double> v = pvec(io.pos4, io.nbrR[gk], xi, Hc);
    double fx = 0.0, fy = 0.0, fz = 0.0;  // dE_i/dr_ij
    if (v.d2 < cut.rcR2) {
      const double d = sqrt(v.d2);
      const double d_inv = 1.0 / d;
      const double ux = v.rx * d_inv, uy = v.ry * d_inv, uz = v.rz * d_inv;
      double Q[BR], dQ[BR];
      cheb_basis64<BR>(k64_opaque(), d, rcR_inv, Q, dQ);
      const double* aj = aR + ((int64_t)Zi * ns + v.q) * BR;
      double own = 0.0, rev = 0.0;
#pragma unroll
      for (int b = 0; b < S::T; ++b) {
        double t = 0.0;
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) t = fma(Ai[b][kk], dQ[kk], t);
        own = v.zj == b ? t : own;
      }
#pragma unroll
      for (int kk = 0; kk < BR; ++kk) rev = fma(aj[kk], dQ[kk], rev);
      fx = own * ux;
      fy = own * uy;
      fz = own * uz;
      // minus dE_j/dr_ji of the radial descriptors (r_ji = -r_ij)
      Fx += rev * ux;
      Fy += rev * uy;
      Fz += rev * uz;
    }
    if (rv != 0xFFFFFFFFu) {
      const double4 a = fA[(int64_t)ka++ * ns + p];
      fx += a.x;
      fy += a.y;
      fz += a.z;
      // a partner that was not found (0xFFFFFFFE) has made the list build fail
      // already; the test only keeps the read in bounds
      if (rv <= 0xFFFFu) {
        const double4 b = fA[(int64_t)rv * ns + v.q];
        Fx -= b.x;
        Fy -= b.y;
        Fz -= b.z;
      }
    }
    Fx += fx;
    Fy += fy;
    Fz += fz;
    const double f[3] = {fx, fy, fz}, r[3] = {v.rx, v.ry, v.rz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Wm[3 * a + b] -= f[a] * r[b];
  }
  F[3 * (int64_t)i] = Fx;
  F[3 * (int64_t)i + 1] = Fy;
  F[3 * (int64_t)i + 2] = Fz;
#pragma unroll
  for (int x = 0; x < 9; ++x) W[9 * (int64_t)i + x] = Wm[x];
}

// ------------------------------------------------------------ launchers

template <class S>
int TrainLaunch<S>::seeds(hipStream_t st, const TrainSeedArgs& a) {
  hipLaunchKernelGGL(k_loss_forces, dim3(a.n_items), dim3(kTB), 0, st, a.items, a.form, a.w[1], a.inv_3ntot, a.n_cfg,
                     a.off, a.F, a.Fref, a.lam, a.partF);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kTB), 0, st, a.n_cfg, a.form, a.w[0], a.w[2], a.off, a.item_start,
                     a.partF, a.E, a.Eref, a.V, a.Vref, a.ebar, a.mu, a.loss);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

// Per-species sums over atoms of every parameter gradient, each into its own
// region of part, then one launch finishes them all into grad (float64):
//   W0: sum abar q^T - z qdot^T;  c^R: sum qbar_R (x) P - dE/dq_R (x) P';
//   c^A: sum of the per-atom bins;  b0: sum abar;  w1: sum dj/dw1;  b1: sum ebar.
template <class S, class R>
static void species_sums(hipStream_t st, const TrainIOT<R>& io, const int* base, double* part, double* grad) {
  constexpr int T = S::T, H = S::H;
  const int64_t ns = io.ns;
  PartPlan pl = part_plan(T, S::NR, S::BR);
  double* pW0 = pl.add(part, S::H * S::D, S::PCR + S::PCA, S::PMLP, 0);
  double* pcR = pl.add(part, S::NR * T * S::BR, 0, (int64_t)T * S::NR * S::BR, 1);
  hipLaunchKernelGGL((k_outer2<R, S::H, S::D, S::NR, S::T * S::BR>), dim3(kRBlocks, T, 2), dim3(kRB), 0, st, ns, base,
                     io.abar, io.q, io.zneg, io.qd, pW0, io.qbR, io.Pb, io.FpR, io.Pdn, pcR);
  double* pA = pl.add(part, T * S::NA * S::BA, S::PCR, (int64_t)T * S::NA * S::BA, 0);
  double* pb0 = pl.add(part, H, S::PCR + S::PCA + (int64_t)H * S::D, S::PMLP, 0);
  double* pw1 = pl.add(part, H, S::PCR + S::PCA + (int64_t)H * S::D + H, S::PMLP, 0);
  double* pb1 = pl.add(part, 1, S::PCR + S::PCA + (int64_t)H * S::D + 2 * H, S::PMLP, 0);
  hipLaunchKernelGGL((k_colsum4<R, S::T * S::NA * S::BA, S::H>), dim3(kRBlocks, T, 4), dim3(kCB), 0, st, ns, base,
                     io.GA, pA, io.abar, pb0, io.gw1, pw1, io.eat, pb1);
  hipLaunchKernelGGL(k_part_final, dim3(blocks(pl.first[pl.n], 256)), dim3(256), 0, st, pl, part, grad);
}

// The network pass of the float training path on the fp32 matrix cores: the
// same quantities as the network phase of k_train_atom (abar, -z and dj/dw1
// per hidden unit; qbar = W0^T abar and dE/dq = W0^T z), from the four
// products a = W0 q + b0, adot = W0 qdot, W0^T abar and W0^T z.  As in the
// evaluation's network, the 16-block 4x4x1 instruction lets every lane supply
// its own atom's vector as B and a weight row selected by lane % 4 as A, so
// each lane accumulates four entries of its own atom; the weights of the
// block's species sit in LDS as [Z][h][d] and [Z][d][h], zero padded.  Every
// lane runs the matrix instructions (slots past the end and padding slots
// with zero inputs); only real atoms store, and padding slots store zeros
// where the species sums read them.
typedef float tnetx4 __attribute__((ext_vector_type(4)));

template <class S>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(2))) void k_train_net(TrainIO io,
                                                                                         const float* __restrict__ params) {
  constexpr int T = S::T, NR = S::NR, D = S::D, H = S::H;
  constexpr int HP = (H + 3) / 4 * 4, DP = (D + 3) / 4 * 4;
  __shared__ float W0s[T * HP * DP];
  __shared__ float W0Ts[T * DP * HP];
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  const bool in = p < ns;
  const int64_t pc = in ? p : ns - 1;
  {
    // the species of this block's wavefronts (each is uniform)
    const int64_t b0 = (int64_t)blockIdx.x * kTB;
    unsigned need = 0;
#pragma unroll
    for (int w = 0; w < kTB / kWave; ++w) {
      const int64_t s0 = b0 + w * kWave;
      need |= 1u << species_of(io.pos4[s0 < ns ? s0 : ns - 1]);
    }
    for (int z = 0; z < T; ++z) {
      if (!(need >> z & 1u)) continue;
      const float* W0g = params + S::PCR + S::PCA + (int64_t)z * S::PMLP;
      for (int t = threadIdx.x; t < HP * DP; t += kTB) {
        const int h = t / DP, d = t % DP;
        const float w = (h < H && d < D) ? W0g[h * D + d] : 0.0f;
        W0s[(z * HP + h) * DP + d] = w;
        W0Ts[(z * DP + d) * HP + h] = w;
      }
    }
    __syncthreads();
  }
  if (__builtin_amdgcn_readfirstlane((int)(p - threadIdx.x % kWave >= ns))) return;  // wavefront past the end
  const int Zs = __builtin_amdgcn_readfirstlane(species_of(io.pos4[pc]));
  const int c = io.cfg_of[pc];
  const bool active = in && c >= 0;
  const float eb = active ? (float)io.ebar[c] : 0.f;
  const int lq = threadIdx.x & 3;
  const float* b0g = params + S::PCR + S::PCA + (int64_t)Zs * S::PMLP + H * D;
  const float* w1g = b0g + H;
  // forward: a_h and adot_h, four hidden units per group
  tnetx4 acc[HP / 4], accd[HP / 4];
#pragma unroll
  for (int hg = 0; hg < HP / 4; ++hg)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[hg][r] = (4 * hg + r < H) ? b0g[4 * hg + r] : 0.f;
      accd[hg][r] = 0.f;
    }
  {
    float q[DP], qd[DP];
#pragma unroll
    for (int d = 0; d < DP; ++d) {
      q[d] = (d < D && active) ? io.q[(int64_t)d * ns + p] : 0.f;
      qd[d] = (d < D && active) ? io.qd[(int64_t)d * ns + p] : 0.f;
    }
    const float* Wz = W0s + (Zs * HP + lq) * DP;
#pragma unroll
    for (int dg = 0; dg < DP / 4; ++dg) {
#pragma unroll
      for (int hg = 0; hg < HP / 4; ++hg) {
        const float4 w = *reinterpret_cast<const float4*>(Wz + 4 * hg * DP + 4 * dg);
        acc[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, q[4 * dg + 0], acc[hg], 0, 0, 0);
        acc[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, q[4 * dg + 1], acc[hg], 0, 0, 0);
        acc[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, q[4 * dg + 2], acc[hg], 0, 0, 0);
        acc[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, q[4 * dg + 3], acc[hg], 0, 0, 0);
        accd[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, qd[4 * dg + 0], accd[hg], 0, 0, 0);
        accd[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, qd[4 * dg + 1], accd[hg], 0, 0, 0);
        accd[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, qd[4 * dg + 2], accd[hg], 0, 0, 0);
        accd[hg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, qd[4 * dg + 3], accd[hg], 0, 0, 0);
      }
    }
  }
  // per hidden unit: abar = z (ebar + 2 h adot), z = w1 (1 - h^2), dj/dw1
  float zt[HP], ab[HP];
#pragma unroll
  for (int hg = 0; hg < HP / 4; ++hg)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int h = 4 * hg + r;
      zt[h] = ab[h] = 0.f;
      if (h < H) {
        const float t = tanh_(acc[hg][r]), ad = accd[hg][r];
        const float s2 = 1.0f - t * t;
        const float z = w1g[h] * s2;
        if (active) {
          zt[h] = z;
          ab[h] = z * (eb + 2.0f * t * ad);
        }
        if (in) {
          io.abar[(int64_t)h * ns + p] = ab[h];
          io.gw1[(int64_t)h * ns + p] = active ? eb * t - s2 * ad : 0.f;
          io.zneg[(int64_t)h * ns + p] = -zt[h];
        }
      }
    }
  if (in) io.eat[p] = eb;
  // backward: qbar_d = sum_h abar_h W0[h][d], dE/dq_d = sum_h z_h W0[h][d]
  tnetx4 qba[DP / 4], fpa[DP / 4];
#pragma unroll
  for (int dg = 0; dg < DP / 4; ++dg) qba[dg] = fpa[dg] = tnetx4{0.f, 0.f, 0.f, 0.f};
  {
    const float* WzT = W0Ts + (Zs * DP + lq) * HP;
#pragma unroll
    for (int hg = 0; hg < HP / 4; ++hg) {
#pragma unroll
      for (int dg = 0; dg < DP / 4; ++dg) {
        const float4 w = *reinterpret_cast<const float4*>(WzT + 4 * dg * HP + 4 * hg);
        qba[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, ab[4 * hg + 0], qba[dg], 0, 0, 0);
        qba[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, ab[4 * hg + 1], qba[dg], 0, 0, 0);
        qba[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, ab[4 * hg + 2], qba[dg], 0, 0, 0);
        qba[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, ab[4 * hg + 3], qba[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, zt[4 * hg + 0], fpa[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, zt[4 * hg + 1], fpa[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, zt[4 * hg + 2], fpa[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, zt[4 * hg + 3], fpa[dg], 0, 0, 0);
      }
    }
  }
  if (!in) return;
#pragma unroll
  for (int dg = 0; dg < DP / 4; ++dg)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = 4 * dg + r;
      if (d < NR) {
        io.qbR[(int64_t)d * ns + p] = qba[dg][r];
        io.FpR[(int64_t)d * ns + p] = fpa[dg][r];
      } else if (d < D && active) {
        io.qbA[(int64_t)d * ns + p] = qba[dg][r];
        io.FpA[(int64_t)d * ns + p] = fpa[dg][r];
      }
    }
}

template <class S>
int TrainLaunch<S>::backward(hipStream_t st, TrainIO io, const Cutoffs& cut, const float* params, const float* lam,
                             const int* base, double* part, double* grad64, float* grad) {
  const int64_t ns = io.ns;
  hipLaunchKernelGGL(k_lam_slots<float>, dim3(blocks(ns, 256)), dim3(256), 0, st, ns, io.orig, lam,
                     const_cast<float4*>(io.lam4));
  constexpr int NC = S::NA >= 4 ? 2 : 1;
  hipLaunchKernelGGL((k_train_atom<S, NC, float, 1>), dim3(blocks(ns, kTB), 1 + S::NA / NC), dim3(kTB), 0, st, io, cut, params);
  hipLaunchKernelGGL(k_train_net<S>, dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, params);
  hipLaunchKernelGGL((k_train_atom<S, NC, float, 3>), dim3(blocks(ns, kTB), S::NA), dim3(kTB), 0, st, io, cut, params);
  hipLaunchKernelGGL((k_train_coefA<S, float>), dim3(blocks(ns, kTB), S::NA), dim3(kTB), 0, st, io, cut, params);
  species_sums<S, float>(st, io, base, part, grad64);
  hipLaunchKernelGGL(k_to_float, dim3(blocks(S::P, 256)), dim3(256), 0, st, (int64_t)S::P, grad64, grad);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

// float64: positions staged, then the atom pass with zero tangent seeds
// (lambda = 0, mu = 0, ebar = 1), which leaves E_i, dE/dq and dE/dS.
static int stage64(hipStream_t st, const TrainIOT<double>& io, const F64Args& a, const float4* pos4f) {
  hipLaunchKernelGGL(k_stage64, dim3(blocks(io.ns, 256)), dim3(256), 0, st, io.ns, io.orig, io.cfg_of, io.cfgs, pos4f,
                     a.pos, a.pos4);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S>
int TrainLaunch<S>::forward64(hipStream_t st, TrainIOT<double> io, const CutoffsT<double>& cut, const F64Args& a,
                              double* forces) {
  const int64_t ns = io.ns;
  hipLaunchKernelGGL(k_fill64, dim3(blocks(4 * ns, 256)), dim3(256), 0, st, 4 * ns, 0.0,
                     reinterpret_cast<double*>(io.lam4));
  constexpr int NC = S::NA >= 4 ? 2 : 1;
  hipLaunchKernelGGL((k_train_atom<S, NC, double, 1, true>), dim3(blocks(ns, kTB), 1 + S::NA / NC), dim3(kTB), 0, st,
                     io, cut, a.params);
  hipLaunchKernelGGL((k_train_atom<S, NC, double, 2, true>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, cut,
                     a.params);
  hipLaunchKernelGGL((k_train_atom<S, NC, double, 3, true>), dim3(blocks(ns, kTB), S::NA), dim3(kTB), 0, st, io, cut,
                     a.params);
  // the radial adjoint rows of every atom
  hipLaunchKernelGGL((k_radial_adj64<S>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, ns, io.cfg_of, io.pos4, io.FpR,
                     a.params, a.aR);
  // the angular part of every list, then each list once
  constexpr int NP = S::NA % 2 == 0 ? 2 : 1;
  hipLaunchKernelGGL((k_ang_force64<S, NP>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, cut, a.params, a.nbrTA,
                     a.rowTA, a.cntAV, a.fA);
  hipLaunchKernelGGL((k_force64<S>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, cut, a.aR, a.vrev, a.fA, forces,
                     a.Wi);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S>
int TrainLaunch<S>::backward64(hipStream_t st, TrainIOT<double> io, const CutoffsT<double>& cut, const F64Args& a,
                               const double* lam, const int* base, double* part, double* grad) {
  const int64_t ns = io.ns;
  hipLaunchKernelGGL(k_lam_slots<double>, dim3(blocks(ns, 256)), dim3(256), 0, st, ns, io.orig, lam, io.lam4);
  constexpr int NC = S::NA >= 4 ? 2 : 1;
  hipLaunchKernelGGL((k_train_atom<S, NC, double, 1>), dim3(blocks(ns, kTB), 1 + S::NA / NC), dim3(kTB), 0, st, io, cut, a.params);
  hipLaunchKernelGGL((k_train_atom<S, NC, double, 2>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, cut, a.params);
  hipLaunchKernelGGL((k_train_atom<S, NC, double, 3>), dim3(blocks(ns, kTB), S::NA), dim3(kTB), 0, st, io, cut, a.params);
  hipLaunchKernelGGL((k_train_coefA<S, double>), dim3(blocks(ns, kTB), S::NA), dim3(kTB), 0, st, io, cut, a.params);
  species_sums<S, double>(st, io, base, part, grad);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int launch_stage64(hipStream_t st, const TrainIOT<double>& io, const F64Args& a, const float4* pos4f) {
  return stage64(st, io, a, pos4f);
}

int launch_round_pos(hipStream_t st, int64_t n, const double* a, float* b) {
  if (n > 0) hipLaunchKernelGGL(k_round_pos, dim3(blocks(n, 256)), dim3(256), 0, st, n, a, b);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int launch_fill64(hipStream_t st, int64_t n, double v, double* a) {
  if (n > 0) hipLaunchKernelGGL(k_fill64, dim3(blocks(n, 256)), dim3(256), 0, st, n, v, a);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template struct TrainLaunch<ShapeSmall>;
template struct TrainLaunch<ShapeGST>;
template struct TrainLaunch<ShapeTable2>;

}  // namespace nepmi
