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
//   k_outer / k_colsum  per-species sums over atoms (fixed order, float64)
#include "train.hpp"

namespace nepmi {

constexpr int kTB = 256;

// Symmetric 3x3 as (xx, yy, zz, xy, xz, yz); full-matrix gradient convention
// dE = sum_ab M_ab dA_ab.  A_n from S_n2m (l = 2 content of S).
__device__ __forceinline__ void sym_from_s2(const float* s2, float (&A)[6]) {
  const float azz = s2[0] * (1.0f / (3.0f * sh::k20));
  const float dif = s2[3] * (1.0f / sh::k22);
  A[0] = 0.5f * (dif - azz);
  A[1] = -0.5f * (dif + azz);
  A[2] = azz;
  A[3] = s2[4] * (1.0f / sh::k21);
  A[4] = s2[1] * (1.0f / sh::k21);
  A[5] = s2[2] * (1.0f / sh::k21);
}

__device__ __forceinline__ void sym_mul_sym(const float (&A)[6], const float (&B)[6], float (&C)[9]) {
  // C = A B (general 3x3, row-major)
  const float a[9] = {A[0], A[3], A[4], A[3], A[1], A[5], A[4], A[5], A[2]};
  const float b[9] = {B[0], B[3], B[4], B[3], B[1], B[5], B[4], B[5], B[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// sum_ab M_ab N_ab for symmetric M, N
__device__ __forceinline__ float sym_dot(const float (&M)[6], const float (&N)[6]) {
  return M[0] * N[0] + M[1] * N[1] + M[2] * N[2] + 2.0f * (M[3] * N[3] + M[4] * N[4] + M[5] * N[5]);
}

// Gradient with respect to S_n2m of a function whose gradient w.r.t. A is M.
__device__ __forceinline__ void chain_s2(const float (&M)[6], float (&g)[5]) {
  g[0] = (M[2] - 0.5f * (M[0] + M[1])) * (1.0f / (3.0f * sh::k20));
  g[1] = 2.0f * M[4] * (1.0f / sh::k21);
  g[2] = 2.0f * M[5] * (1.0f / sh::k21);
  g[3] = 0.5f * (M[0] - M[1]) * (1.0f / sh::k22);
  g[4] = 2.0f * M[3] * (1.0f / sh::k21);
}

__device__ __forceinline__ void sym_sq6(const float (&A)[6], float (&B)[6]) {
  const float xx = A[0], yy = A[1], zz = A[2], xy = A[3], xz = A[4], yz = A[5];
  B[0] = xx * xx + xy * xy + xz * xz;
  B[1] = xy * xy + yy * yy + yz * yz;
  B[2] = xz * xz + yz * yz + zz * zz;
  B[3] = xx * xy + xy * yy + xz * yz;
  B[4] = xx * xz + xy * yz + xz * zz;
  B[5] = xy * xz + yy * yz + yz * zz;
}

__device__ __forceinline__ void load_cell9(const CfgDev* __restrict__ cfgs, int c, float (&H)[9]) {
#pragma unroll
  for (int x = 0; x < 9; ++x) H[x] = c >= 0 ? cfgs[c].H[x] : 0.f;
}

struct PV {
  float rx, ry, rz, d2;
  int q, zj;
};

__device__ __forceinline__ PV pvec(const float4* __restrict__ pos4, uint32_t e, float4 xi, const float (&H)[9]) {
  PV v;
  v.q = (int)(e & kNbrMask);
  const float4 xq = pos4[v.q];
  float sx, sy, sz;
  image_shift(H, e >> kNbrShift, sx, sy, sz);
  v.rx = (xq.x - xi.x) + sx;
  v.ry = (xq.y - xi.y) + sy;
  v.rz = (xq.z - xi.z) + sz;
  v.d2 = pair_d2(v.rx, v.ry, v.rz);
  v.zj = __float_as_int(xq.w);
  return v;
}

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

// Energy and virial terms, seeds ebar_c and mu_c, and the loss parts.
__global__ void k_loss_final(int n_cfg, int form, double wE, double wV, const int64_t* __restrict__ off,
                             const int* __restrict__ item_start, const double* __restrict__ partF,
                             const double* __restrict__ E, const double* __restrict__ Eref,
                             const double* __restrict__ V, const double* __restrict__ Vref, double* __restrict__ ebar,
                             double* __restrict__ mu, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double LE = 0.0, LF = 0.0, LV = 0.0;
  const double B = (double)n_cfg;
  for (int c = 0; c < n_cfg; ++c) {
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
  loss[0] = LE + LF + LV;
  loss[1] = LE;
  loss[2] = LF;
  loss[3] = LV;
}

// lambda to slot order (float4); zero on padding slots
__global__ void k_lam_slots(int64_t ns, const int* __restrict__ orig, const float* __restrict__ lam,
                            float4* __restrict__ lam4) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const int i = orig[p];
  lam4[p] = i >= 0 ? make_float4(lam[3 * (int64_t)i], lam[3 * (int64_t)i + 1], lam[3 * (int64_t)i + 2], 0.f)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
}

// ------------------------------------------------- tangent + network adjoint

template <class S, int NC>
__global__ __launch_bounds__(kTB) void k_train_atom(TrainIO io, Cutoffs cut, const float* __restrict__ params) {
  constexpr int T = S::T, NR = S::NR, NA = S::NA, BR = S::BR, BA = S::BA, L = S::L, K = S::K, D = S::D, H = S::H;
  static_assert(NA % NC == 0, "chunk must divide n_angular");
  __shared__ float cA_s[T * T * NA * BA];
  for (int t = threadIdx.x; t < T * T * NA * BA; t += kTB) cA_s[t] = params[S::PCR + t];
  __syncthreads();
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (p >= ns) return;
  const float4 xi = io.pos4[p];
  const int Zs = __builtin_amdgcn_readfirstlane(__float_as_int(xi.w));
  const int c = io.cfg_of[p];
  if (c < 0) {
    // padding: zero every per-slot output that is summed over species ranges
    for (int d = 0; d < D; ++d) io.q[d * ns + p] = io.qd[d * ns + p] = 0.f;
    for (int h = 0; h < H; ++h) io.abar[h * ns + p] = io.zneg[h * ns + p] = io.gw1[h * ns + p] = 0.f;
    for (int k = 0; k < T * BR; ++k) io.Pb[k * ns + p] = io.Pdn[k * ns + p] = 0.f;
    for (int n = 0; n < NR; ++n) io.qbR[n * ns + p] = io.FpR[n * ns + p] = 0.f;
    io.eat[p] = 0.f;
    return;
  }
  float Hc[9];
  load_cell9(io.cfgs, c, Hc);
  const float rcR_inv = 1.0f / cut.rcR, rcA_inv = 1.0f / cut.rcA;
  const float4 li = io.lam4[p];
  float mu[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) mu[x] = (float)io.mu[9 * c + x];
  const float eb = (float)io.ebar[c];

  // ---- radial: P_b[k] = sum_{j in b} Q_k, Pd_b[k] = sum_{j in b} dQ_k (u.t)
  {
    float P[T][BR], Pd[T][BR];
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int k = 0; k < BR; ++k) P[b][k] = Pd[b][k] = 0.f;
    const int n = io.cntR[p];
    for (int k = 0; k < n; ++k) {
      const PV v = pvec(io.pos4, io.nbrR[(int64_t)k * ns + p], xi, Hc);
      if (v.d2 < cut.rcR2) {
        const float d = sqrtf(v.d2), inv = 1.0f / d;
        float Q[BR], dQ[BR];
        cheb_basis_d<BR>(d, rcR_inv, Q, dQ);
        const float4 lj = io.lam4[v.q];
        const float tx = lj.x - li.x + mu[0] * v.rx + mu[1] * v.ry + mu[2] * v.rz;
        const float ty = lj.y - li.y + mu[3] * v.rx + mu[4] * v.ry + mu[5] * v.rz;
        const float tz = lj.z - li.z + mu[6] * v.rx + mu[7] * v.ry + mu[8] * v.rz;
        const float ut = (v.rx * tx + v.ry * ty + v.rz * tz) * inv;
#pragma unroll
        for (int b = 0; b < T; ++b) {
          const float m = (T == 1 || v.zj == b) ? 1.0f : 0.0f;
          const float mut = m * ut;
#pragma unroll
          for (int kk = 0; kk < BR; ++kk) {
            P[b][kk] = fmaf(m, Q[kk], P[b][kk]);
            Pd[b][kk] = fmaf(mut, dQ[kk], Pd[b][kk]);
          }
        }
      }
    }
    const float* cR = params + (int64_t)Zs * (T * NR * BR);
#pragma unroll
    for (int nn = 0; nn < NR; ++nn) {
      float a = 0.f, ad = 0.f;
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) {
          a = fmaf(cR[(b * NR + nn) * BR + kk], P[b][kk], a);
          ad = fmaf(cR[(b * NR + nn) * BR + kk], Pd[b][kk], ad);
        }
      io.q[(int64_t)nn * ns + p] = a;
      io.qd[(int64_t)nn * ns + p] = ad;
    }
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int kk = 0; kk < BR; ++kk) {
        io.Pb[(b * BR + kk) * ns + p] = P[b][kk];
        io.Pdn[(b * BR + kk) * ns + p] = -Pd[b][kk];
      }
  }
  // ---- angular: S and Sdot in chunks of NC functions (stored for the adjoint)
  const int nA = io.cntA[p];
  for (int h = 0; h < NA / NC; ++h) {
    float Sg[NC][K], Sd[NC][K];
#pragma unroll
    for (int nn = 0; nn < NC; ++nn)
#pragma unroll
      for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = Sd[nn][lm] = 0.f;
    for (int k = 0; k < nA; ++k) {
      const PV v = pvec(io.pos4, io.nbrA[(int64_t)k * ns + p], xi, Hc);
      if (v.d2 < cut.rcA2) {
        const float d = sqrtf(v.d2), inv = 1.0f / d;
        const float ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
        float Q[BA], dQ[BA];
        cheb_basis_d<BA>(d, rcA_inv, Q, dQ);
        const float4 lj = io.lam4[v.q];
        const float tx = lj.x - li.x + mu[0] * v.rx + mu[1] * v.ry + mu[2] * v.rz;
        const float ty = lj.y - li.y + mu[3] * v.rx + mu[4] * v.ry + mu[5] * v.rz;
        const float tz = lj.z - li.z + mu[6] * v.rx + mu[7] * v.ry + mu[8] * v.rz;
        const float ut = ux * tx + uy * ty + uz * tz;
        float Y[K], Dl[K];
        real_sph<L>(ux, uy, uz, Y);
        // grad_r Y_lm . t = grad P_lm . (t - (u.t) u) / d
        real_sph_dir<L>(ux, uy, uz, (tx - ut * ux) * inv, (ty - ut * uy) * inv, (tz - ut * uz) * inv, Dl);
        const float* cl = cA_s + ((Zs * T + v.zj) * NA + h * NC) * BA;
#pragma unroll
        for (int nn = 0; nn < NC; ++nn) {
          float g = 0.f, gp = 0.f;
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) {
            g = fmaf(cl[nn * BA + kk], Q[kk], g);
            gp = fmaf(cl[nn * BA + kk], dQ[kk], gp);
          }
          const float gput = gp * ut;
#pragma unroll
          for (int lm = 0; lm < K; ++lm) {
            Sg[nn][lm] = fmaf(g, Y[lm], Sg[nn][lm]);
            Sd[nn][lm] = fmaf(gput, Y[lm], fmaf(g, Dl[lm], Sd[nn][lm]));
          }
        }
      }
    }
#pragma unroll
    for (int nn = 0; nn < NC; ++nn) {
      const int n = h * NC + nn;
#pragma unroll
      for (int lm = 0; lm < K; ++lm) {
        io.Sst[(int64_t)(n * K + lm) * ns + p] = Sg[nn][lm];
        io.Sdt[(int64_t)(n * K + lm) * ns + p] = Sd[nn][lm];
      }
      float q1 = 0.f, qd1 = 0.f;
#pragma unroll
      for (int l = 1; l <= L; ++l) {
        float s = 0.f, sd = 0.f;
#pragma unroll
        for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) {
          s = fmaf(Sg[nn][lm], Sg[nn][lm], s);
          sd = fmaf(Sg[nn][lm], Sd[nn][lm], sd);
        }
        io.q[(int64_t)(NR + (l - 1) * NA + n) * ns + p] = s;
        io.qd[(int64_t)(NR + (l - 1) * NA + n) * ns + p] = 2.0f * sd;
        if (l == 1) {
          q1 = s;
          qd1 = 2.0f * sd;
        }
      }
      if constexpr (S::F4) {
        float A[6], Ad[6], A2[6];
        sym_from_s2(&Sg[nn][3], A);
        sym_from_s2(&Sd[nn][3], Ad);
        sym_sq6(A, A2);
        io.q[(int64_t)(S::OFF4 + n) * ns + p] = sym_dot(A2, A);
        io.qd[(int64_t)(S::OFF4 + n) * ns + p] = 3.0f * sym_dot(A2, Ad);
      }
      if constexpr (S::F5) {
        io.q[(int64_t)(S::OFF5 + n) * ns + p] = q1 * q1;
        io.qd[(int64_t)(S::OFF5 + n) * ns + p] = 2.0f * q1 * qd1;
      }
    }
  }
  // ---- network, second-order adjoint; pass 1: abar, z, dj/dw1
  const float* W0 = params + S::PCR + S::PCA + (int64_t)Zs * S::PMLP;
  const float* b0 = W0 + H * D;
  const float* w1 = b0 + H;
  {
    float q[D], qd[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      q[d] = io.q[(int64_t)d * ns + p];
      qd[d] = io.qd[(int64_t)d * ns + p];
    }
    for (int hh = 0; hh < H; ++hh) {
      float a = b0[hh], ad = 0.f;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        a = fmaf(W0[hh * D + d], q[d], a);
        ad = fmaf(W0[hh * D + d], qd[d], ad);
      }
      const float t = tanhf(a);
      const float s2 = 1.0f - t * t;
      const float z = w1[hh] * s2;
      io.abar[(int64_t)hh * ns + p] = z * (eb + 2.0f * t * ad);
      io.zneg[(int64_t)hh * ns + p] = -z;
      io.gw1[(int64_t)hh * ns + p] = eb * t - s2 * ad;
    }
  }
  io.eat[p] = eb;
  // pass 2: qbar = W0^T abar, Fp = W0^T z
  float qb[D], Fp[D];
#pragma unroll
  for (int d = 0; d < D; ++d) qb[d] = Fp[d] = 0.f;
  for (int hh = 0; hh < H; ++hh) {
    const float ab = io.abar[(int64_t)hh * ns + p], z = -io.zneg[(int64_t)hh * ns + p];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      qb[d] = fmaf(ab, W0[hh * D + d], qb[d]);
      Fp[d] = fmaf(z, W0[hh * D + d], Fp[d]);
    }
  }
#pragma unroll
  for (int nn = 0; nn < NR; ++nn) {
    io.qbR[(int64_t)nn * ns + p] = qb[nn];
    io.FpR[(int64_t)nn * ns + p] = Fp[nn];
  }
  // ---- sigma = dE/dS and Sbar = dj/dS from the stored S and Sdot
  for (int n = 0; n < NA; ++n) {
    float Sg[K], Sd[K];
#pragma unroll
    for (int lm = 0; lm < K; ++lm) {
      Sg[lm] = io.Sst[(int64_t)(n * K + lm) * ns + p];
      Sd[lm] = io.Sdt[(int64_t)(n * K + lm) * ns + p];
    }
    float g4s[5] = {0, 0, 0, 0, 0}, g4b[5] = {0, 0, 0, 0, 0};
    if constexpr (S::F4) {
      float A[6], Ad[6], A2[6], Msig[6], Mbar[6];
      sym_from_s2(&Sg[3], A);
      sym_from_s2(&Sd[3], Ad);
      sym_sq6(A, A2);
      float AAd[9], AdA[9];
      sym_mul_sym(A, Ad, AAd);
      sym_mul_sym(Ad, A, AdA);
      float fp4 = 0.f, qb4 = 0.f;
#pragma unroll
      for (int x = 0; x < NA; ++x)
        if (x == n) {
          fp4 = Fp[S::OFF4 + x];
          qb4 = qb[S::OFF4 + x];
        }
      const int ix[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
#pragma unroll
      for (int x = 0; x < 6; ++x) {
        const float sym = AAd[3 * ix[x][0] + ix[x][1]] + AdA[3 * ix[x][0] + ix[x][1]];
        Msig[x] = 3.0f * fp4 * A2[x];
        Mbar[x] = 3.0f * qb4 * A2[x] - 3.0f * fp4 * sym;
      }
      chain_s2(Msig, g4s);
      chain_s2(Mbar, g4b);
    }
#pragma unroll
    for (int l = 1; l <= L; ++l) {
      float fp3 = 0.f, qb3 = 0.f, fp5 = 0.f, qb5 = 0.f;
#pragma unroll
      for (int x = 0; x < NA; ++x)
        if (x == n) {
          fp3 = Fp[NR + (l - 1) * NA + x];
          qb3 = qb[NR + (l - 1) * NA + x];
          if (S::F5) {
            fp5 = Fp[S::OFF5 + x];
            qb5 = qb[S::OFF5 + x];
          }
        }
      float cs = 2.0f * fp3;   // sigma = cs S
      float cbS = 2.0f * qb3;  // Sbar = cbS S + cbD Sdot
      float cbD = -2.0f * fp3;
      if (S::F5 && l == 1) {
        const float q1 = io.q[(int64_t)(NR + n) * ns + p], qd1 = io.qd[(int64_t)(NR + n) * ns + p];
        cs += 4.0f * fp5 * q1;
        cbS += 4.0f * qb5 * q1 - 4.0f * fp5 * qd1;
        cbD += -4.0f * fp5 * q1;
      }
#pragma unroll
      for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) {
        float sg = cs * Sg[lm];
        float sb = cbS * Sg[lm] + cbD * Sd[lm];
        if (S::F4 && l == 2) {
          sg += g4s[lm - 3];
          sb += g4b[lm - 3];
        }
        io.Sst[(int64_t)(n * K + lm) * ns + p] = sg;
        io.Sdt[(int64_t)(n * K + lm) * ns + p] = sb;
      }
    }
  }
}

// ------------------------------------------------ angular coefficient pass

// GA[(b NA + n) BA + k] = sum over angular pairs j of species b of
//   (alpha_n + gamma_n) Q_k + beta_n dQ_k,
// alpha_n = sum_lm Sbar Y, beta_n = -(u.t) sum_lm sigma Y, gamma_n = -sum_lm sigma grad Y.t
template <class S>
__global__ __launch_bounds__(kTB) void k_train_coefA(TrainIO io, Cutoffs cut, const float* __restrict__ params) {
  constexpr int T = S::T, NA = S::NA, BA = S::BA, L = S::L, K = S::K;
  const int64_t ns = io.ns;
  const int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (p >= ns) return;
  const int c = io.cfg_of[p];
  if (c < 0) {
    for (int x = 0; x < T * NA * BA; ++x) io.GA[(int64_t)x * ns + p] = 0.f;
    return;
  }
  const float4 xi = io.pos4[p];
  float Hc[9];
  load_cell9(io.cfgs, c, Hc);
  const float rcA_inv = 1.0f / cut.rcA;
  const float4 li = io.lam4[p];
  float mu[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) mu[x] = (float)io.mu[9 * c + x];
  const int nA = io.cntA[p];
  for (int n = 0; n < NA; ++n) {
    float sg[K], sb[K];
#pragma unroll
    for (int lm = 0; lm < K; ++lm) {
      sg[lm] = io.Sst[(int64_t)(n * K + lm) * ns + p];
      sb[lm] = io.Sdt[(int64_t)(n * K + lm) * ns + p];
    }
    float G[T][BA];
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int k = 0; k < BA; ++k) G[b][k] = 0.f;
    for (int k = 0; k < nA; ++k) {
      const PV v = pvec(io.pos4, io.nbrA[(int64_t)k * ns + p], xi, Hc);
      if (v.d2 < cut.rcA2) {
        const float d = sqrtf(v.d2), inv = 1.0f / d;
        const float ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
        float Q[BA], dQ[BA];
        cheb_basis_d<BA>(d, rcA_inv, Q, dQ);
        const float4 lj = io.lam4[v.q];
        const float tx = lj.x - li.x + mu[0] * v.rx + mu[1] * v.ry + mu[2] * v.rz;
        const float ty = lj.y - li.y + mu[3] * v.rx + mu[4] * v.ry + mu[5] * v.rz;
        const float tz = lj.z - li.z + mu[6] * v.rx + mu[7] * v.ry + mu[8] * v.rz;
        const float ut = ux * tx + uy * ty + uz * tz;
        float Y[K], Dl[K];
        real_sph<L>(ux, uy, uz, Y);
        real_sph_dir<L>(ux, uy, uz, (tx - ut * ux) * inv, (ty - ut * uy) * inv, (tz - ut * uz) * inv, Dl);
        float al = 0.f, sy = 0.f, ga = 0.f;
#pragma unroll
        for (int lm = 0; lm < K; ++lm) {
          al = fmaf(sb[lm], Y[lm], al);
          sy = fmaf(sg[lm], Y[lm], sy);
          ga = fmaf(sg[lm], Dl[lm], ga);
        }
        const float cq = al - ga, cd = -ut * sy;
#pragma unroll
        for (int b = 0; b < T; ++b) {
          const float m = (T == 1 || v.zj == b) ? 1.0f : 0.0f;
          const float mq = m * cq, md = m * cd;
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) G[b][kk] = fmaf(mq, Q[kk], fmaf(md, dQ[kk], G[b][kk]));
        }
      }
    }
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int kk = 0; kk < BA; ++kk) io.GA[(int64_t)((b * NA + n) * BA + kk) * ns + p] = G[b][kk];
  }
}

// ---------------------------------------------------- species reductions

constexpr int kRB = 256;       // threads per reduction block
constexpr int kRChunk = 32;    // slots staged per step
constexpr int kRBlocks = 64;   // blocks per species (fixed: deterministic order)
constexpr int kMaxE = 16;      // entries per thread (A*B <= 4096)

// part[(s * kRBlocks + blk) * A*B + e] = sum over slots i of species s handled
// by block blk of  X1[a][i] Y1[b][i] + X2[a][i] Y2[b][i]  (e = a*B + b).
__global__ __launch_bounds__(kRB) void k_outer(int64_t ns, const int* __restrict__ base, int A, int B,
                                               const float* __restrict__ X1, const float* __restrict__ Y1,
                                               const float* __restrict__ X2, const float* __restrict__ Y2,
                                               double* __restrict__ part) {
  extern __shared__ float smem[];
  float* sx1 = smem;
  float* sy1 = sx1 + A * kRChunk;
  float* sx2 = sy1 + B * kRChunk;
  float* sy2 = sx2 + A * kRChunk;
  const int s = blockIdx.y, blk = blockIdx.x;
  const int p0 = base[s], p1 = base[s + 1];
  const int AB = A * B;
  double acc[kMaxE];
#pragma unroll
  for (int j = 0; j < kMaxE; ++j) acc[j] = 0.0;
  for (int c0 = p0 + blk * kRChunk; c0 < p1; c0 += kRBlocks * kRChunk) {
    const int nc = min(kRChunk, p1 - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < A * kRChunk; t += kRB) {
      const int a = t / kRChunk, i = t % kRChunk;
      sx1[t] = i < nc ? X1[(int64_t)a * ns + c0 + i] : 0.f;
      sx2[t] = i < nc ? X2[(int64_t)a * ns + c0 + i] : 0.f;
    }
    for (int t = threadIdx.x; t < B * kRChunk; t += kRB) {
      const int b = t / kRChunk, i = t % kRChunk;
      sy1[t] = i < nc ? Y1[(int64_t)b * ns + c0 + i] : 0.f;
      sy2[t] = i < nc ? Y2[(int64_t)b * ns + c0 + i] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMaxE; ++j) {
      const int e = threadIdx.x + j * kRB;
      if (e < AB) {
        const int a = e / B, b = e % B;
        float s1 = 0.f;
        for (int i = 0; i < kRChunk; ++i)
          s1 = fmaf(sx1[a * kRChunk + i], sy1[b * kRChunk + i], fmaf(sx2[a * kRChunk + i], sy2[b * kRChunk + i], s1));
        acc[j] += (double)s1;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxE; ++j) {
    const int e = threadIdx.x + j * kRB;
    if (e < AB) part[((int64_t)s * kRBlocks + blk) * AB + e] = acc[j];
  }
}

// part[(s * kRBlocks + blk) * A + a] = sum over the block's slots of X[a][i]
__global__ __launch_bounds__(kRB) void k_colsum(int64_t ns, const int* __restrict__ base, int A,
                                                const float* __restrict__ X, double* __restrict__ part) {
  const int s = blockIdx.y, blk = blockIdx.x;
  const int p0 = base[s], p1 = base[s + 1];
  for (int a = threadIdx.x; a < A; a += kRB) {
    double acc = 0.0;
    for (int c0 = p0 + blk * kRChunk; c0 < p1; c0 += kRBlocks * kRChunk) {
      const int c1 = min(c0 + kRChunk, p1);
      float s1 = 0.f;
      for (int i = c0; i < c1; ++i) s1 += X[(int64_t)a * ns + i];
      acc += (double)s1;
    }
    part[((int64_t)s * kRBlocks + blk) * A + a] = acc;
  }
}

// grad[dst(s, e)] = sum_blk part[s][blk][e];  dst = off + s * sstride + map(e)
// map: kind 0 identity; kind 1: e = n*(T*BR) + b*BR + k -> (b*NR + n)*BR + k
__global__ void k_part_final(int T, int E, const double* __restrict__ part, int64_t off, int64_t sstride, int kind,
                             int NR, int BR, double* __restrict__ grad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)T * E) return;
  const int s = (int)(t / E), e = (int)(t % E);
  double acc = 0.0;
  for (int blk = 0; blk < kRBlocks; ++blk) acc += part[((int64_t)s * kRBlocks + blk) * E + e];
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

// ------------------------------------------------------------ launchers

template <class S>
int TrainLaunch<S>::seeds(hipStream_t st, const TrainSeedArgs& a) {
  hipLaunchKernelGGL(k_loss_forces, dim3(a.n_items), dim3(kTB), 0, st, a.items, a.form, a.w[1], a.inv_3ntot, a.n_cfg,
                     a.off, a.F, a.Fref, a.lam, a.partF);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, a.n_cfg, a.form, a.w[0], a.w[2], a.off, a.item_start,
                     a.partF, a.E, a.Eref, a.V, a.Vref, a.ebar, a.mu, a.loss);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S>
int TrainLaunch<S>::backward(hipStream_t st, TrainIO io, const Cutoffs& cut, const float* params, const float* lam,
                             const int* base, double* part, double* grad64, float* grad) {
  const int64_t ns = io.ns;
  hipLaunchKernelGGL(k_lam_slots, dim3(blocks(ns, 256)), dim3(256), 0, st, ns, io.orig, lam,
                     const_cast<float4*>(io.lam4));
  constexpr int NC = S::NA >= 4 ? 2 : 1;
  hipLaunchKernelGGL((k_train_atom<S, NC>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, cut, params);
  hipLaunchKernelGGL((k_train_coefA<S>), dim3(blocks(ns, kTB)), dim3(kTB), 0, st, io, cut, params);
  constexpr int T = S::T;
  const dim3 g(kRBlocks, T);
  // W0: sum abar q^T - z qdot^T
  {
    const int A = S::H, B = S::D;
    const size_t sm = sizeof(float) * (size_t)(2 * A + 2 * B) * kRChunk;
    hipLaunchKernelGGL(k_outer, g, dim3(kRB), sm, st, ns, base, A, B, io.abar, io.q, io.zneg, io.qd, part);
    hipLaunchKernelGGL(k_part_final, dim3(blocks((int64_t)T * A * B, 256)), dim3(256), 0, st, T, A * B, part,
                       S::PCR + S::PCA, S::PMLP, 0, 0, 0, grad64);
  }
  // c^R: sum qbar_R (x) P - Fp_R (x) P'
  {
    const int A = S::NR, B = T * S::BR;
    const size_t sm = sizeof(float) * (size_t)(2 * A + 2 * B) * kRChunk;
    hipLaunchKernelGGL(k_outer, g, dim3(kRB), sm, st, ns, base, A, B, io.qbR, io.Pb, io.FpR, io.Pdn, part);
    hipLaunchKernelGGL(k_part_final, dim3(blocks((int64_t)T * A * B, 256)), dim3(256), 0, st, T, A * B, part,
                       (int64_t)0, (int64_t)T * S::NR * S::BR, 1, S::NR, S::BR, grad64);
  }
  // c^A
  {
    const int A = T * S::NA * S::BA;
    hipLaunchKernelGGL(k_colsum, g, dim3(kRB), 0, st, ns, base, A, io.GA, part);
    hipLaunchKernelGGL(k_part_final, dim3(blocks((int64_t)T * A, 256)), dim3(256), 0, st, T, A, part, S::PCR,
                       (int64_t)A, 0, 0, 0, grad64);
  }
  // b0, w1, b1
  {
    const int H = S::H;
    hipLaunchKernelGGL(k_colsum, g, dim3(kRB), 0, st, ns, base, H, io.abar, part);
    hipLaunchKernelGGL(k_part_final, dim3(blocks((int64_t)T * H, 256)), dim3(256), 0, st, T, H, part,
                       S::PCR + S::PCA + (int64_t)H * S::D, S::PMLP, 0, 0, 0, grad64);
    hipLaunchKernelGGL(k_colsum, g, dim3(kRB), 0, st, ns, base, H, io.gw1, part);
    hipLaunchKernelGGL(k_part_final, dim3(blocks((int64_t)T * H, 256)), dim3(256), 0, st, T, H, part,
                       S::PCR + S::PCA + (int64_t)H * S::D + H, S::PMLP, 0, 0, 0, grad64);
    hipLaunchKernelGGL(k_colsum, g, dim3(kRB), 0, st, ns, base, 1, io.eat, part);
    hipLaunchKernelGGL(k_part_final, dim3(1), dim3(64), 0, st, T, 1, part,
                       S::PCR + S::PCA + (int64_t)H * S::D + 2 * H, S::PMLP, 0, 0, 0, grad64);
  }
  hipLaunchKernelGGL(k_to_float, dim3(blocks(S::P, 256)), dim3(256), 0, st, (int64_t)S::P, grad64, grad);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template struct TrainLaunch<ShapeSmall>;
template struct TrainLaunch<ShapeGST>;
template struct TrainLaunch<ShapeTable2>;

}  // namespace nepmi
