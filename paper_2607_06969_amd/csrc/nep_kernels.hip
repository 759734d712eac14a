// nep_kernels.hip -- descriptor/network, pair-force and gather kernels.
#include "nep_kernels.hpp"
#include "nbr.hpp"

namespace nepmi {

constexpr int kBlock = 256;

// Pair vector r_ij = (x_j - x_i) + image shift, computed with the same
// rounding from either side so that r_ji = -r_ij exactly.
struct PairVec {
  float rx, ry, rz, d2;
  int q, zj;
};

__device__ __forceinline__ PairVec pair_vec(const float4* __restrict__ pos4, uint32_t e, float4 xi, const float (&H)[9]) {
  PairVec v;
  v.q = (int)(e & kNbrMask);
  const float4 xq = pos4[v.q];
  float sx, sy, sz;
  image_shift(H, e >> kNbrShift, sx, sy, sz);
  v.rx = (xq.x - xi.x) + sx;
  v.ry = (xq.y - xi.y) + sy;
  v.rz = (xq.z - xi.z) + sz;
  v.d2 = v.rx * v.rx + v.ry * v.ry + v.rz * v.rz;
  v.zj = __float_as_int(xq.w);
  return v;
}

__device__ __forceinline__ void load_cell(const CfgDev* __restrict__ cfgs, int c, float (&H)[9]) {
  if (c >= 0) {
#pragma unroll
    for (int x = 0; x < 9; ++x) H[x] = cfgs[c].H[x];
  } else {
#pragma unroll
    for (int x = 0; x < 9; ++x) H[x] = 0.f;
  }
}

// S_n2m -> symmetric traceless A_n = sum_j g_n (u u^T - I/3) (l = 2 content).
// Returns A as (xx, yy, zz, xy, xz, yz).
__device__ __forceinline__ void a_from_s2(const float* s2, float (&A)[6]) {
  const float azz = s2[0] * (1.0f / (3.0f * sh::k20));
  const float dif = s2[3] * (1.0f / sh::k22);
  A[0] = 0.5f * (dif - azz);
  A[1] = -0.5f * (dif + azz);
  A[2] = azz;
  A[3] = s2[4] * (1.0f / sh::k21);
  A[4] = s2[1] * (1.0f / sh::k21);
  A[5] = s2[2] * (1.0f / sh::k21);
}

// A^2 as (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void sym_sq(const float (&A)[6], float (&B)[6]) {
  const float xx = A[0], yy = A[1], zz = A[2], xy = A[3], xz = A[4], yz = A[5];
  B[0] = xx * xx + xy * xy + xz * xz;
  B[1] = xy * xy + yy * yy + yz * yz;
  B[2] = xz * xz + yz * yz + zz * zz;
  B[3] = xx * xy + xy * yy + xz * yz;
  B[4] = xx * xz + xy * yz + xz * zz;
  B[5] = xy * xz + yy * yz + yz * zz;
}

// tr(A^3) = sum_ab (A^2)_ab A_ab for symmetric A
__device__ __forceinline__ float tr_cube(const float (&A)[6]) {
  float B[6];
  sym_sq(A, B);
  return B[0] * A[0] + B[1] * A[1] + B[2] * A[2] + 2.0f * (B[3] * A[3] + B[4] * A[4] + B[5] * A[5]);
}

// ------------------------------------------------------------------ k_desc

template <class S, int NSPLIT, int WPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_desc(
    int64_t n_slots, const float4* __restrict__ pos4, const int* __restrict__ cfg_of, const int* __restrict__ orig,
    const CfgDev* __restrict__ cfgs, const uint32_t* __restrict__ nbrR, const int* __restrict__ cntR,
    uint32_t* __restrict__ cnR, int* __restrict__ ccR, uint32_t* __restrict__ cnA, int* __restrict__ ccA,
    Cutoffs cut, const float* __restrict__ params, float* __restrict__ fp, float* __restrict__ aR,
    float* __restrict__ Ei, float* __restrict__ qout, float* __restrict__ Eproc, int want_adjoint) {
  constexpr int T = S::T, NR = S::NR, NA = S::NA, BR = S::BR, BA = S::BA, L = S::L, K = S::K, D = S::D, H = S::H;
  constexpr int NH = NA / NSPLIT;
  static_assert(NA % NSPLIT == 0, "NSPLIT must divide n_angular");
  __shared__ float cA_s[T * T * NA * BA];
  for (int t = threadIdx.x; t < T * T * NA * BA; t += kBlock) cA_s[t] = params[S::PCR + t];
  __syncthreads();

  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n_slots) return;
  const float4 xi = pos4[p];
  const int Zs = __builtin_amdgcn_readfirstlane(__float_as_int(xi.w));
  const int c = cfg_of[p];
  const bool active = c >= 0;
  float Hc[9];
  load_cell(cfgs, c, Hc);
  const float rcR_inv = 1.0f / cut.rcR, rcA_inv = 1.0f / cut.rcA;

  // ---- filter the Verlet list into the pairs inside the two cutoffs
  int nR = 0, nA = 0;
  if (active) {
    const int n = cntR[p];
    for (int k = 0; k < n; ++k) {
      const uint32_t e = nbrR[(int64_t)k * n_slots + p];
      const PairVec v = pair_vec(pos4, e, xi, Hc);
      if (v.d2 < cut.rcR2) {
        cnR[(int64_t)nR * n_slots + p] = e;
        ++nR;
        if (v.d2 < cut.rcA2) {
          cnA[(int64_t)nA * n_slots + p] = e;
          ++nA;
        }
      }
    }
  }
  ccR[p] = nR;
  ccA[p] = nA;

  float q[D];
  // ---- radial descriptors, Eq. 11: q_n = sum_b sum_k c^R[Z_i][b][n][k] P_b[k],
  //      P_b[k] = sum over neighbours j of species b of Q_k(r_ij)
  {
    float P[T][BR];
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int k = 0; k < BR; ++k) P[b][k] = 0.f;
    for (int k = 0; k < nR; ++k) {
      const PairVec v = pair_vec(pos4, cnR[(int64_t)k * n_slots + p], xi, Hc);
      float Q[BR];
      cheb_basis<BR>(sqrtf(v.d2), rcR_inv, Q);
#pragma unroll
      for (int b = 0; b < T; ++b) {
        const float m = (T == 1 || v.zj == b) ? 1.0f : 0.0f;
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) P[b][kk] = fmaf(m, Q[kk], P[b][kk]);
      }
    }
    const float* cR = params + (int64_t)Zs * (T * NR * BR);
#pragma unroll
    for (int nn = 0; nn < NR; ++nn) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) acc = fmaf(cR[(b * NR + nn) * BR + kk], P[b][kk], acc);
      q[nn] = acc;
    }
  }

  // ---- angular descriptors, Eq. 16-17, in NSPLIT groups of n
#pragma unroll
  for (int h = 0; h < NSPLIT; ++h) {
    float Sg[NH][K];
#pragma unroll
    for (int nn = 0; nn < NH; ++nn)
#pragma unroll
      for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = 0.f;
    for (int k = 0; k < nA; ++k) {
      const PairVec v = pair_vec(pos4, cnA[(int64_t)k * n_slots + p], xi, Hc);
      {
        const float d = sqrtf(v.d2);
        const float inv = 1.0f / d;
        float Q[BA];
        cheb_basis<BA>(d, rcA_inv, Q);
        const float* cl = cA_s + ((Zs * T + v.zj) * NA + h * NH) * BA;
        float g[NH];
#pragma unroll
        for (int nn = 0; nn < NH; ++nn) {
          float acc = 0.f;
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) acc = fmaf(cl[nn * BA + kk], Q[kk], acc);
          g[nn] = acc;
        }
        float Y[K];
        real_sph<L>(v.rx * inv, v.ry * inv, v.rz * inv, Y);
#pragma unroll
        for (int nn = 0; nn < NH; ++nn)
#pragma unroll
          for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = fmaf(g[nn], Y[lm], Sg[nn][lm]);
      }
    }
    // invariants of this group
#pragma unroll
    for (int nn = 0; nn < NH; ++nn) {
      const int n = h * NH + nn;
#pragma unroll
      for (int l = 1; l <= L; ++l) {
        float s = 0.f;
#pragma unroll
        for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) s = fmaf(Sg[nn][lm], Sg[nn][lm], s);
        q[NR + (l - 1) * NA + n] = s;
      }
      if constexpr (S::F4) {
        float A[6];
        a_from_s2(&Sg[nn][3], A);
        q[S::OFF4 + n] = tr_cube(A);
      }
      if constexpr (S::F5) q[S::OFF5 + n] = q[NR + n] * q[NR + n];
    }
  }

  // ---- network of Sec. 2.3 (weights of species Z_i through the scalar unit)
  const float* W0 = params + S::PCR + S::PCA + (int64_t)Zs * S::PMLP;
  const float* b0 = W0 + H * D;
  const float* w1 = b0 + H;
  float E = w1[H];
  float Fp[D];
#pragma unroll
  for (int d = 0; d < D; ++d) Fp[d] = 0.f;
  for (int hh = 0; hh < H; ++hh) {
    float a = b0[hh];
#pragma unroll
    for (int d = 0; d < D; ++d) a = fmaf(W0[hh * D + d], q[d], a);
    const float t = tanhf(a);
    E = fmaf(w1[hh], t, E);
    const float z = w1[hh] * (1.0f - t * t);
#pragma unroll
    for (int d = 0; d < D; ++d) Fp[d] = fmaf(z, W0[hh * D + d], Fp[d]);
  }
  if (!active) return;
  const int i = orig[p];
  Ei[i] = E;
  if (Eproc) Eproc[p] = E;
  if (qout) {
#pragma unroll
    for (int d = 0; d < D; ++d) qout[(int64_t)i * D + d] = q[d];
  }
  if (!want_adjoint) return;
#pragma unroll
  for (int d = NR; d < D; ++d) fp[(int64_t)(d - NR) * n_slots + p] = Fp[d];
  const float* cR = params + (int64_t)Zs * (T * NR * BR);
#pragma unroll
  for (int b = 0; b < T; ++b)
#pragma unroll
    for (int kk = 0; kk < BR; ++kk) {
      float acc = 0.f;
#pragma unroll
      for (int nn = 0; nn < NR; ++nn) acc = fmaf(Fp[nn], cR[(b * NR + nn) * BR + kk], acc);
      aR[p * (T * BR) + b * BR + kk] = acc;
    }
}

// ----------------------------------------------------------------- k_force

template <class S, int NSPLIT, int WPE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WPE))) void k_force(
    int64_t n_slots, const float4* __restrict__ pos4, const int* __restrict__ cfg_of, const int* __restrict__ orig,
    const CfgDev* __restrict__ cfgs, const uint32_t* __restrict__ cnR, const int* __restrict__ ccR,
    const uint32_t* __restrict__ cnA, const int* __restrict__ ccA, Cutoffs cut, const float* __restrict__ params,
    const float* __restrict__ fp, const float* __restrict__ aR, float4* __restrict__ frad, float4* __restrict__ fA,
    float* __restrict__ Wi) {
  constexpr int T = S::T, NR = S::NR, NA = S::NA, BR = S::BR, BA = S::BA, L = S::L, K = S::K;
  constexpr int NH = NA / NSPLIT;
  __shared__ float cA_s[T * T * NA * BA];
  for (int t = threadIdx.x; t < T * T * NA * BA; t += kBlock) cA_s[t] = params[S::PCR + t];
  __syncthreads();

  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n_slots) return;
  const float4 xi = pos4[p];
  const int Zs = __builtin_amdgcn_readfirstlane(__float_as_int(xi.w));
  const int c = cfg_of[p];
  if (c < 0) return;
  float Hc[9];
  load_cell(cfgs, c, Hc);
  const float rcR_inv = 1.0f / cut.rcR, rcA_inv = 1.0f / cut.rcA;

  float Fx = 0.f, Fy = 0.f, Fz = 0.f;
  float W[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) W[x] = 0.f;

  // ---- radial pairs: f_ij - f_ji = (s_own + s_rev) u_ij
  {
    float a_own[T][BR];
#pragma unroll
    for (int b = 0; b < T; ++b)
#pragma unroll
      for (int kk = 0; kk < BR; ++kk) a_own[b][kk] = aR[p * (T * BR) + b * BR + kk];
    const int n = ccR[p];
    for (int k = 0; k < n; ++k) {
      const PairVec v = pair_vec(pos4, cnR[(int64_t)k * n_slots + p], xi, Hc);
      {
        const float d = sqrtf(v.d2);
        const float inv = 1.0f / d;
        float Q[BR], dQ[BR];
        cheb_basis_d<BR>(d, rcR_inv, Q, dQ);
        float s_own = 0.f;
#pragma unroll
        for (int b = 0; b < T; ++b) {
          float sb = 0.f;
#pragma unroll
          for (int kk = 0; kk < BR; ++kk) sb = fmaf(a_own[b][kk], dQ[kk], sb);
          s_own = (T == 1 || v.zj == b) ? sb : s_own;
        }
        const float* ar = aR + (int64_t)v.q * (T * BR) + Zs * BR;
        float s_rev = 0.f;
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) s_rev = fmaf(ar[kk], dQ[kk], s_rev);
        const float ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
        const float st = s_own + s_rev;
        Fx = fmaf(st, ux, Fx);
        Fy = fmaf(st, uy, Fy);
        Fz = fmaf(st, uz, Fz);
        const float fx = s_own * ux, fy = s_own * uy, fz = s_own * uz;
        W[0] -= fx * v.rx; W[1] -= fx * v.ry; W[2] -= fx * v.rz;
        W[3] -= fy * v.rx; W[4] -= fy * v.ry; W[5] -= fy * v.rz;
        W[6] -= fz * v.rx; W[7] -= fz * v.ry; W[8] -= fz * v.rz;
      }
    }
  }

  // ---- angular pairs, in NSPLIT groups of n
  const int nA = ccA[p];
#pragma unroll
  for (int h = 0; h < NSPLIT; ++h) {
    // recompute S for this group
    float Sg[NH][K];
#pragma unroll
    for (int nn = 0; nn < NH; ++nn)
#pragma unroll
      for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = 0.f;
    for (int k = 0; k < nA; ++k) {
      const PairVec v = pair_vec(pos4, cnA[(int64_t)k * n_slots + p], xi, Hc);
      {
        const float d = sqrtf(v.d2);
        const float inv = 1.0f / d;
        float Q[BA];
        cheb_basis<BA>(d, rcA_inv, Q);
        const float* cl = cA_s + ((Zs * T + v.zj) * NA + h * NH) * BA;
        float g[NH];
#pragma unroll
        for (int nn = 0; nn < NH; ++nn) {
          float acc = 0.f;
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) acc = fmaf(cl[nn * BA + kk], Q[kk], acc);
          g[nn] = acc;
        }
        float Y[K];
        real_sph<L>(v.rx * inv, v.ry * inv, v.rz * inv, Y);
#pragma unroll
        for (int nn = 0; nn < NH; ++nn)
#pragma unroll
          for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = fmaf(g[nn], Y[lm], Sg[nn][lm]);
      }
    }
    // sigma = dE_i/dS for this group (in place)
#pragma unroll
    for (int nn = 0; nn < NH; ++nn) {
      const int n = h * NH + nn;
      float s4[5];
      if constexpr (S::F4) {
        // d tr(A^3)/dS_n2m through A(S): 3 Fp4 A^2 contracted with dA/dS
        float A[6], B[6];
        a_from_s2(&Sg[nn][3], A);
        sym_sq(A, B);
        const float f4 = 3.0f * fp[(int64_t)(S::OFF4 - NR + n) * n_slots + p];
#pragma unroll
        for (int x = 0; x < 6; ++x) B[x] *= f4;
        s4[0] = (B[2] - 0.5f * (B[0] + B[1])) * (1.0f / (3.0f * sh::k20));
        s4[1] = 2.0f * B[4] * (1.0f / sh::k21);
        s4[2] = 2.0f * B[5] * (1.0f / sh::k21);
        s4[3] = 0.5f * (B[0] - B[1]) * (1.0f / sh::k22);
        s4[4] = 2.0f * B[3] * (1.0f / sh::k21);
      }
      float psi1 = 2.0f * fp[(int64_t)(0 * NA + n) * n_slots + p];
      if constexpr (S::F5) {
        const float q1 = Sg[nn][0] * Sg[nn][0] + Sg[nn][1] * Sg[nn][1] + Sg[nn][2] * Sg[nn][2];
        psi1 = fmaf(4.0f * q1, fp[(int64_t)(S::OFF5 - NR + n) * n_slots + p], psi1);
      }
#pragma unroll
      for (int l = 1; l <= L; ++l) {
        const float psi = (l == 1) ? psi1 : 2.0f * fp[(int64_t)((l - 1) * NA + n) * n_slots + p];
#pragma unroll
        for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) Sg[nn][lm] *= psi;
      }
      if constexpr (S::F4) {
#pragma unroll
        for (int m = 0; m < 5; ++m) Sg[nn][3 + m] += s4[m];
      }
    }
    // pair forces of this group: f = u sum_n g'_n Z_n + (I - u u^T) v / d,
    // Z_n = sum_lm sigma_nlm Y_lm, v = sum_lm G_lm grad P_lm, G_lm = sum_n sigma_nlm g_n
    for (int k = 0; k < nA; ++k) {
      const PairVec v = pair_vec(pos4, cnA[(int64_t)k * n_slots + p], xi, Hc);
      float fx = 0.f, fy = 0.f, fz = 0.f;
      {
        const float d = sqrtf(v.d2);
        const float inv = 1.0f / d;
        const float ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
        float Y[K];
        real_sph<L>(ux, uy, uz, Y);
        float Q[BA], dQ[BA];
        cheb_basis_d<BA>(d, rcA_inv, Q, dQ);
        const float* cl = cA_s + ((Zs * T + v.zj) * NA + h * NH) * BA;
        float G[K];
#pragma unroll
        for (int lm = 0; lm < K; ++lm) G[lm] = 0.f;
        float s = 0.f;
#pragma unroll
        for (int nn = 0; nn < NH; ++nn) {
          float g = 0.f, gp = 0.f;
#pragma unroll
          for (int kk = 0; kk < BA; ++kk) {
            const float cc = cl[nn * BA + kk];
            g = fmaf(cc, Q[kk], g);
            gp = fmaf(cc, dQ[kk], gp);
          }
          float zn = 0.f;
#pragma unroll
          for (int lm = 0; lm < K; ++lm) {
            zn = fmaf(Sg[nn][lm], Y[lm], zn);
            G[lm] = fmaf(Sg[nn][lm], g, G[lm]);
          }
          s = fmaf(gp, zn, s);
        }
        float vx, vy, vz;
        real_sph_grad_dot<L>(ux, uy, uz, G, vx, vy, vz);
        const float uv = ux * vx + uy * vy + uz * vz;
        fx = s * ux + (vx - uv * ux) * inv;
        fy = s * uy + (vy - uv * uy) * inv;
        fz = s * uz + (vz - uv * uz) * inv;
        W[0] -= fx * v.rx; W[1] -= fx * v.ry; W[2] -= fx * v.rz;
        W[3] -= fy * v.rx; W[4] -= fy * v.ry; W[5] -= fy * v.rz;
        W[6] -= fz * v.rx; W[7] -= fz * v.ry; W[8] -= fz * v.rz;
      }
      float4* dst = fA + (int64_t)k * n_slots + p;
      if (h == 0) {
        *dst = make_float4(fx, fy, fz, 0.f);
      } else {
        const float4 o = *dst;
        *dst = make_float4(o.x + fx, o.y + fy, o.z + fz, 0.f);
      }
    }
  }
  frad[p] = make_float4(Fx, Fy, Fz, 0.f);
  const int i = orig[p];
#pragma unroll
  for (int x = 0; x < 9; ++x) Wi[(int64_t)i * 9 + x] = W[x];
}

// ---------------------------------------------------------------- k_gather

__global__ __launch_bounds__(kBlock) void k_gather(int64_t n_slots, const int* __restrict__ orig,
                                                   const uint32_t* __restrict__ cnA, const int* __restrict__ ccA,
                                                   const float4* __restrict__ frad, const float4* __restrict__ fA,
                                                   float* __restrict__ Fuser, float4* __restrict__ Fproc,
                                                   int* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n_slots) return;
  const int i = orig[p];
  if (i < 0) {
    if (Fproc) Fproc[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float4 F = frad[p];
  const int n = ccA[p];
  for (int k = 0; k < n; ++k) {
    const uint32_t e = cnA[(int64_t)k * n_slots + p];
    const int q = (int)(e & kNbrMask);
    // the pair seen from q: slot p with the opposite image shift
    const uint32_t want = (uint32_t)p | ((26u - (e >> kNbrShift)) << kNbrShift);
    const int nq = ccA[q];
    int j = 0;
    while (j < nq && cnA[(int64_t)j * n_slots + q] != want) ++j;
    const float4 a = fA[(int64_t)k * n_slots + p];
    if (j < nq) {
      const float4 b = fA[(int64_t)j * n_slots + q];
      F.x += a.x - b.x;
      F.y += a.y - b.y;
      F.z += a.z - b.z;
    } else {
      atomicOr(&flags[kFlagAsym], 1);
    }
  }
  if (Fuser) {
    Fuser[(int64_t)i * 3 + 0] = F.x;
    Fuser[(int64_t)i * 3 + 1] = F.y;
    Fuser[(int64_t)i * 3 + 2] = F.z;
  }
  if (Fproc) Fproc[p] = F;
}

// ------------------------------------------------------------- launchers

// Kernel variants: (groups of angular functions per pass, waves per SIMD the
// register allocation must allow).  Every variant computes the same result;
// descriptor variants are bitwise identical, force variants differ only in
// the order the per-group pair forces are added.
template <class S, int NS>
constexpr int groups() {
  return NS <= S::NA ? NS : S::NA;
}

template <class S, int NS, int W>
static int launch_desc(hipStream_t st, const NepIO& io, const float* params, bool want_adjoint) {
  const unsigned g = (unsigned)((io.n_slots + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_desc<S, groups<S, NS>(), W>), dim3(g), dim3(kBlock), 0, st, io.n_slots, io.pos4, io.cfg_of,
                     io.orig, io.cfgs, io.nbrR, io.cntR, io.cnR, io.ccR, io.cnA, io.ccA, io.cut, params, io.fp, io.aR,
                     io.Ei, io.qout, io.Eproc, want_adjoint ? 1 : 0);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S, int NS, int W>
static int launch_force(hipStream_t st, const NepIO& io, const float* params) {
  const unsigned g = (unsigned)((io.n_slots + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_force<S, groups<S, NS>(), W>), dim3(g), dim3(kBlock), 0, st, io.n_slots, io.pos4, io.cfg_of,
                     io.orig, io.cfgs, io.cnR, io.ccR, io.cnA, io.ccA, io.cut, params, io.fp, io.aR, io.frad, io.fA,
                     io.Wi);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S>
int Launch<S>::desc(hipStream_t st, const NepIO& io, const float* params, bool want_adjoint, int variant) {
  switch (variant) {
    case 1: return launch_desc<S, 4, 3>(st, io, params, want_adjoint);
    case 2: return launch_desc<S, 4, 2>(st, io, params, want_adjoint);
    case 3: return launch_desc<S, 8, 3>(st, io, params, want_adjoint);
    default: return launch_desc<S, 2, 2>(st, io, params, want_adjoint);
  }
}

template <class S>
int Launch<S>::force(hipStream_t st, const NepIO& io, const float* params, int variant) {
  switch (variant) {
    case 1: return launch_force<S, 4, 2>(st, io, params);
    case 2: return launch_force<S, 4, 3>(st, io, params);
    case 3: return launch_force<S, 8, 3>(st, io, params);
    default: return launch_force<S, 2, 2>(st, io, params);
  }
}

template <class S>
int Launch<S>::gather(hipStream_t st, const NepIO& io) {
  const unsigned g = (unsigned)((io.n_slots + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_gather, dim3(g), dim3(kBlock), 0, st, io.n_slots, io.orig, io.cnA, io.ccA, io.frad, io.fA,
                     io.Fuser, io.Fproc, io.flags);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template struct Launch<ShapeSmall>;
template struct Launch<ShapeGST>;
template struct Launch<ShapeTable2>;

}  // namespace nepmi
