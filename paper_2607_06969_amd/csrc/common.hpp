// common.hpp -- shared definitions of the HIP NEP library (gfx950).
//
// Compile-time model shapes, the per-configuration table, device math for the
// Chebyshev radial basis (Eq. 12-15) and the real spherical harmonics (Eq. 16),
// and host-side error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/nepmi.h"

namespace nepmi {

// ---------------------------------------------------------------- model shape

// Compile-time NEP shape.  Kernels keep per-atom accumulators in registers, so
// every array length is a template constant.
template <int T_, int NR_, int NA_, int BR_, int BA_, int L_, int F4_, int F5_, int H_>
struct Shape {
  static constexpr int T = T_;    // species
  static constexpr int NR = NR_;  // radial functions
  static constexpr int NA = NA_;  // angular functions
  static constexpr int BR = BR_;  // Chebyshev basis size, radial
  static constexpr int BA = BA_;  // Chebyshev basis size, angular
  static constexpr int L = L_;    // l_max of the three-body term
  static constexpr bool F4 = F4_ != 0;
  static constexpr bool F5 = F5_ != 0;
  static constexpr int H = H_;    // hidden neurons
  static constexpr int K = L * L + 2 * L;  // real (l, m) components, l = 1..L
  static constexpr int OFF4 = NR + L * NA;
  static constexpr int OFF5 = OFF4 + (F4 ? NA : 0);
  static constexpr int D = OFF5 + (F5 ? NA : 0);
  static constexpr int NANG = D - NR;  // descriptors that depend on S
  static constexpr int64_t PCR = (int64_t)T * T * NR * BR;
  static constexpr int64_t PCA = (int64_t)T * T * NA * BA;
  static constexpr int64_t PMLP = (int64_t)H * D + 2 * H + 1;
  static constexpr int64_t P = PCR + PCA + T * PMLP;
};

// Shapes compiled into the library: the 64-atom single-element test model,
// the three-species Ge-Sb-Te model with 4- and 5-body terms, and the model of
// the paper's Table 2.
using ShapeSmall = Shape<1, 4, 4, 8, 8, 4, 0, 0, 30>;
using ShapeGST = Shape<3, 8, 8, 12, 12, 4, 1, 1, 50>;
using ShapeTable2 = Shape<3, 10, 8, 8, 8, 4, 0, 0, 50>;

constexpr int kWave = 64;
constexpr int kNbrShift = 27;  // neighbour entry: index (27 bits) | image code (5 bits)
constexpr uint32_t kNbrMask = (1u << kNbrShift) - 1u;
constexpr int kMaxAtoms = (1 << kNbrShift) - 1;

// One periodic configuration as the kernels see it.
struct CfgDev {
  float H[9];       // lattice vectors as rows, float32
  double Hd[9];     // same, float64
  double Hinv[9];   // inverse, float64 (fractional = x . Hinv)
  int nb[3];        // bins per direction
  int bin_off;      // first global bin of this configuration
  int64_t atom_off; // first atom (caller's order)
  int n_atoms;
  int pad;
};

// Runtime (non-shape) parameters of a launch.
struct Cutoffs {
  float rcR, rcA;        // cutoffs of the potential
  float rcR2, rcA2;      // squared
  float rclR2, rclA2;    // squared list cutoffs (cutoff + skin)
};

// ------------------------------------------------------------ device helpers

// Image code = 9 (w0 + 1) + 3 (w1 + 1) + (w2 + 1), w in {-1, 0, 1}; the shift is
// w0 a + w1 b + w2 c for lattice rows a, b, c.  Digits by multiply-shift
// (exact for code < 27: floor(57 c / 512) = floor(c / 9), floor(11 r / 32) =
// floor(r / 3) for r < 9).  Every w_a is -1, 0 or 1, so the shift of code
// 26 - code is the exact negative of the shift of code.
__device__ __forceinline__ void image_shift(const float* __restrict__ H, uint32_t code, float& sx, float& sy,
                                            float& sz) {
  // 24-bit products (full-rate multiplies; every operand is below 2^9)
  const uint32_t d0 = __umul24(code, 57u) >> 9;
  const uint32_t r = code - __umul24(9u, d0);
  const uint32_t d1 = __umul24(r, 11u) >> 5;
  const uint32_t d2 = r - __umul24(3u, d1);
  const float w0 = (float)((int)d0 - 1);
  const float w1 = (float)((int)d1 - 1);
  const float w2 = (float)((int)d2 - 1);
  sx = w0 * H[0] + w1 * H[3] + w2 * H[6];
  sy = w0 * H[1] + w1 * H[4] + w2 * H[7];
  sz = w0 * H[2] + w1 * H[5] + w2 * H[8];
}

// Chebyshev radial basis of Eq. 12-15:
//   x = 2 (d/rc - 1)^2 - 1,  f_c = (1 + cos(pi d/rc)) / 2,  Q_k = (T_k(x) + 1)/2 f_c.
// Valid for d < rc (the caller tests the cutoff).
template <int B>
__device__ __forceinline__ void cheb_basis(float d, float rc_inv, float (&Q)[B]) {
  const float t = d * rc_inv;
  const float y = t - 1.0f;
  const float x = 2.0f * y * y - 1.0f;
  const float fc = 0.5f * (1.0f + cospif(t));
  const float hf = 0.5f * fc;
  float tm = 1.0f, tk = x;
  Q[0] = fc;
  if (B > 1) Q[1] = hf * (x + 1.0f);
#pragma unroll
  for (int k = 2; k < B; ++k) {
    const float tn = 2.0f * x * tk - tm;
    tm = tk;
    tk = tn;
    Q[k] = hf * (tn + 1.0f);
  }
}

// Basis and its radial derivative dQ_k/dd.
template <int B>
__device__ __forceinline__ void cheb_basis_d(float d, float rc_inv, float (&Q)[B], float (&dQ)[B]) {
  const float t = d * rc_inv;
  const float y = t - 1.0f;
  const float x = 2.0f * y * y - 1.0f;
  const float dx = 4.0f * y * rc_inv;
  float sn, cs;
  sincospif(t, &sn, &cs);
  const float fc = 0.5f * (1.0f + cs);
  const float dfc = -0.5f * 3.14159265358979323846f * rc_inv * sn;
  float tm = 1.0f, tk = x, dtm = 0.0f, dtk = 1.0f;
  Q[0] = fc;
  dQ[0] = dfc;
  if (B > 1) {
    Q[1] = 0.5f * (x + 1.0f) * fc;
    dQ[1] = 0.5f * (dx * fc + (x + 1.0f) * dfc);
  }
#pragma unroll
  for (int k = 2; k < B; ++k) {
    const float tn = 2.0f * x * tk - tm;
    const float dtn = 2.0f * tk + 2.0f * x * dtk - dtm;
    tm = tk;
    tk = tn;
    dtm = dtk;
    dtk = dtn;
    Q[k] = 0.5f * (tn + 1.0f) * fc;
    dQ[k] = 0.5f * (dtn * dx * fc + (tn + 1.0f) * dfc);
  }
}

// Workgroups of a launch are dispatched round-robin over the XCDs, each with
// its own L2: block b runs on XCD b % kXcds.  Per-atom kernels take their
// tile from this remapping instead of blockIdx.x, so that every XCD walks one
// contiguous range of slots (spatially close atoms, whose neighbours' data
// then stay in that XCD's L2).  It is a bijection on [0, gridDim.x).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile() {
  const unsigned b = blockIdx.x, nb = gridDim.x;
  const unsigned x = b % kXcds, i = b / kXcds, per = nb / kXcds, rem = nb % kXcds;
  return (int64_t)(x * per + (x < rem ? x : rem) + i);
}

// |r|^2 with a fixed operation order (fused), shared by every kernel that
// compares pair distances so that all of them agree on which pairs are in.
__device__ __forceinline__ float pair_d2(float rx, float ry, float rz) {
  return fmaf(rz, rz, fmaf(ry, ry, rx * rx));
}

// 1/sqrt(x) with the hardware reciprocal square root (1 ulp).
__device__ __forceinline__ float rsqrt_hw(float x) { return __builtin_amdgcn_rsqf(x); }

// sin(pi u) and cos(pi u) for |u| <= 1/2 by their Taylor series to degree 13
// and 12: coefficients (-1)^k pi^(2k+1)/(2k+1)! and (-1)^k pi^(2k)/(2k)!; the
// truncation error is below (pi/2)^15/15! < 7e-10 and (pi/2)^14/14! < 7e-9.
namespace taylor {
constexpr double kPi = 3.14159265358979323846;
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
constexpr double ipow(double x, int n) { return n == 0 ? 1.0 : x * ipow(x, n - 1); }
constexpr float sin_c(int k) { return (float)((k % 2 ? -1.0 : 1.0) * ipow(kPi, 2 * k + 1) / fact(2 * k + 1)); }
constexpr float cos_c(int k) { return (float)((k % 2 ? -1.0 : 1.0) * ipow(kPi, 2 * k) / fact(2 * k)); }
}  // namespace taylor

__device__ __forceinline__ float sinpi_small(float u, float w /* u*u */) {
  constexpr float a0 = taylor::sin_c(0), a1 = taylor::sin_c(1), a2 = taylor::sin_c(2), a3 = taylor::sin_c(3);
  constexpr float a4 = taylor::sin_c(4), a5 = taylor::sin_c(5), a6 = taylor::sin_c(6);
  float p = fmaf(a6, w, a5);
  p = fmaf(p, w, a4);
  p = fmaf(p, w, a3);
  p = fmaf(p, w, a2);
  p = fmaf(p, w, a1);
  p = fmaf(p, w, a0);
  return p * u;
}

__device__ __forceinline__ float cospi_small(float w /* u*u */) {
  constexpr float b0 = taylor::cos_c(0), b1 = taylor::cos_c(1), b2 = taylor::cos_c(2), b3 = taylor::cos_c(3);
  constexpr float b4 = taylor::cos_c(4), b5 = taylor::cos_c(5), b6 = taylor::cos_c(6);
  float p = fmaf(b6, w, b5);
  p = fmaf(p, w, b4);
  p = fmaf(p, w, b3);
  p = fmaf(p, w, b2);
  p = fmaf(p, w, b1);
  return fmaf(p, w, b0);
}

// Radial factors of Eq. 12-15 for t = d / rc in [0, 1):
//   x = 2 (t - 1)^2 - 1,  hf = f_c / 2 = (1 + cos(pi t)) / 4.
// With cos(pi t) = -sin(pi (t - 1/2)) the argument stays in [-1/2, 1/2].
struct RadialF {
  float x, hf;
};
__device__ __forceinline__ RadialF radial_f(float t) {
  const float y = t - 1.0f;
  const float u = t - 0.5f;
  RadialF r;
  r.x = fmaf(2.0f * y, y, -1.0f);
  r.hf = fmaf(-0.25f, sinpi_small(u, u * u), 0.25f);
  return r;
}

// The same with the derivatives needed by the pair forces:
//   dxhf = (dx/dd) hf = 4 (t - 1) / rc * hf,  dfc2 = (df_c/dd) / 2 = -pi sin(pi t) / (4 rc),
// so that dQ_k/dd = dxhf T'_k(x) + dfc2 (T_k(x) + 1).
struct RadialFD {
  float x, hf, dxhf, dfc2;
};
__device__ __forceinline__ RadialFD radial_fd(float t, float rc_inv) {
  const float y = t - 1.0f;
  const float u = t - 0.5f;
  const float w = u * u;
  RadialFD r;
  r.x = fmaf(2.0f * y, y, -1.0f);
  r.hf = fmaf(-0.25f, sinpi_small(u, w), 0.25f);
  r.dxhf = (4.0f * rc_inv) * y * r.hf;
  r.dfc2 = (-0.25f * 3.14159265358979323846f) * rc_inv * cospi_small(w);
  return r;
}

// Chebyshev polynomials T_0..T_{B-1} at x (three-term recurrence).
template <int B>
__device__ __forceinline__ void cheb_t(float x, float (&Tk)[B]) {
  Tk[0] = 1.0f;
  if (B > 1) Tk[1] = x;
  const float x2 = 2.0f * x;
#pragma unroll
  for (int k = 2; k < B; ++k) Tk[k] = fmaf(x2, Tk[k - 1], -Tk[k - 2]);
}

// T_k and T'_k = dT_k/dx (T'_0 = 0, T'_1 = 1, T'_{k+1} = 2 T_k + 2x T'_k - T'_{k-1}).
template <int B>
__device__ __forceinline__ void cheb_tt(float x, float (&Tk)[B], float (&Dk)[B]) {
  Tk[0] = 1.0f;
  Dk[0] = 0.0f;
  if (B > 1) {
    Tk[1] = x;
    Dk[1] = 1.0f;
  }
  const float x2 = 2.0f * x;
#pragma unroll
  for (int k = 2; k < B; ++k) {
    Tk[k] = fmaf(x2, Tk[k - 1], -Tk[k - 2]);
    Dk[k] = fmaf(2.0f, Tk[k - 1], fmaf(x2, Dk[k - 1], -Dk[k - 2]));
  }
}

// Real orthonormal spherical harmonics Y_lm(u) of a unit vector u for
// l = 1..L, ordered per l as m = 0, then (cos m, sin m) for m = 1..l.
// Written as polynomials in the components of u (normalisation
// sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), times sqrt(2) for m > 0).
namespace sh {
constexpr float c1 = 0.488602511902919921f;     // sqrt(3/(4pi))
constexpr float k20 = 0.315391565252520051f;    // sqrt(5/(16pi))
constexpr float k21 = 1.092548430592079070f;    // sqrt(15/(4pi))
constexpr float k22 = 0.546274215296039535f;    // sqrt(15/(16pi))
constexpr float k30 = 0.373176332590115391f;    // sqrt(7/(16pi))
constexpr float k31 = 0.457045799464465736f;    // sqrt(21/(32pi))
constexpr float k32 = 1.445305721320277027f;    // sqrt(105/(16pi))
constexpr float k32s = 2.890611442640554055f;   // sqrt(105/(4pi))
constexpr float k33 = 0.590043589926643510f;    // sqrt(35/(32pi))
constexpr float k40 = 0.105785546915204322f;    // (3/16) sqrt(1/pi)
constexpr float k41 = 0.669046543557289168f;    // (3/4) sqrt(5/(2pi))
constexpr float k42 = 0.473087347878780009f;    // (3/8) sqrt(5/pi)
constexpr float k42s = 0.946174695757560018f;   // (3/4) sqrt(5/pi)
constexpr float k43 = 1.770130769779930531f;    // (3/4) sqrt(35/(2pi))
constexpr float k44 = 0.625835735449176135f;    // (3/16) sqrt(35/pi)
constexpr float k44s = 2.503342941796704538f;   // (3/4) sqrt(35/pi)
}  // namespace sh

template <int L>
__device__ __forceinline__ void real_sph(float x, float y, float z, float (&Y)[L * L + 2 * L]) {
  using namespace sh;
  Y[0] = c1 * z;
  Y[1] = c1 * x;
  Y[2] = c1 * y;
  if constexpr (L >= 2) {
    const float z2 = z * z;
    Y[3] = k20 * (3.0f * z2 - 1.0f);
    Y[4] = k21 * x * z;
    Y[5] = k21 * y * z;
    Y[6] = k22 * (x * x - y * y);
    Y[7] = k21 * x * y;
    if constexpr (L >= 3) {
      const float x2my2 = x * x - y * y;
      const float p = 5.0f * z2 - 1.0f;
      Y[8] = k30 * z * (5.0f * z2 - 3.0f);
      Y[9] = k31 * x * p;
      Y[10] = k31 * y * p;
      Y[11] = k32 * z * x2my2;
      Y[12] = k32s * x * y * z;
      Y[13] = k33 * x * (x * x - 3.0f * y * y);
      Y[14] = k33 * y * (3.0f * x * x - y * y);
      if constexpr (L >= 4) {
        const float q = 7.0f * z2 - 3.0f;
        const float r = 7.0f * z2 - 1.0f;
        Y[15] = k40 * (35.0f * z2 * z2 - 30.0f * z2 + 3.0f);
        Y[16] = k41 * x * z * q;
        Y[17] = k41 * y * z * q;
        Y[18] = k42 * x2my2 * r;
        Y[19] = k42s * x * y * r;
        Y[20] = k43 * x * z * (x * x - 3.0f * y * y);
        Y[21] = k43 * y * z * (3.0f * x * x - y * y);
        Y[22] = k44 * (x2my2 * x2my2 - 4.0f * x * x * y * y);
        Y[23] = k44s * x * y * x2my2;
      }
    }
  }
}

// g = sum_lm G_lm grad_u P_lm(u), where P_lm is the polynomial of real_sph
// (extended off the unit sphere).  The gradient of Y_lm(r/|r|) with respect to
// r is (I - u u^T) grad_u P_lm / |r|; the caller applies that projection.
template <int L>
__device__ __forceinline__ void real_sph_grad_dot(float x, float y, float z, const float (&G)[L * L + 2 * L],
                                                  float& gx, float& gy, float& gz) {
  using namespace sh;
  gx = c1 * G[1];
  gy = c1 * G[2];
  gz = c1 * G[0];
  if constexpr (L >= 2) {
    gz += 6.0f * k20 * z * G[3];
    gx += k21 * z * G[4];
    gz += k21 * x * G[4];
    gy += k21 * z * G[5];
    gz += k21 * y * G[5];
    gx += 2.0f * k22 * x * G[6];
    gy -= 2.0f * k22 * y * G[6];
    gx += k21 * y * G[7];
    gy += k21 * x * G[7];
    if constexpr (L >= 3) {
      const float z2 = z * z, x2 = x * x, y2 = y * y;
      const float p = 5.0f * z2 - 1.0f;
      gz += k30 * (15.0f * z2 - 3.0f) * G[8];
      gx += k31 * p * G[9];
      gz += 10.0f * k31 * x * z * G[9];
      gy += k31 * p * G[10];
      gz += 10.0f * k31 * y * z * G[10];
      gx += 2.0f * k32 * x * z * G[11];
      gy -= 2.0f * k32 * y * z * G[11];
      gz += k32 * (x2 - y2) * G[11];
      gx += k32s * y * z * G[12];
      gy += k32s * x * z * G[12];
      gz += k32s * x * y * G[12];
      gx += 3.0f * k33 * (x2 - y2) * G[13];
      gy -= 6.0f * k33 * x * y * G[13];
      gx += 6.0f * k33 * x * y * G[14];
      gy += 3.0f * k33 * (x2 - y2) * G[14];
      if constexpr (L >= 4) {
        const float q = 7.0f * z2 - 3.0f;
        const float r = 7.0f * z2 - 1.0f;
        gz += k40 * (140.0f * z2 * z - 60.0f * z) * G[15];
        gx += k41 * z * q * G[16];
        gz += k41 * x * (21.0f * z2 - 3.0f) * G[16];
        gy += k41 * z * q * G[17];
        gz += k41 * y * (21.0f * z2 - 3.0f) * G[17];
        gx += 2.0f * k42 * x * r * G[18];
        gy -= 2.0f * k42 * y * r * G[18];
        gz += 14.0f * k42 * z * (x2 - y2) * G[18];
        gx += k42s * y * r * G[19];
        gy += k42s * x * r * G[19];
        gz += 14.0f * k42s * x * y * z * G[19];
        gx += 3.0f * k43 * z * (x2 - y2) * G[20];
        gy -= 6.0f * k43 * x * y * z * G[20];
        gz += k43 * x * (x2 - 3.0f * y2) * G[20];
        gx += 6.0f * k43 * x * y * z * G[21];
        gy += 3.0f * k43 * z * (x2 - y2) * G[21];
        gz += k43 * y * (3.0f * x2 - y2) * G[21];
        gx += 4.0f * k44 * x * (x2 - 3.0f * y2) * G[22];
        gy += 4.0f * k44 * y * (y2 - 3.0f * x2) * G[22];
        gx += k44s * y * (3.0f * x2 - y2) * G[23];
        gy += k44s * x * (x2 - 3.0f * y2) * G[23];
      }
    }
  }
}

// Dl[lm] = w . grad_u P_lm(u) for every component (P_lm as in real_sph).
template <int L>
__device__ __forceinline__ void real_sph_dir(float x, float y, float z, float wx, float wy, float wz,
                                             float (&Dl)[L * L + 2 * L]) {
  using namespace sh;
  Dl[0] = c1 * wz;
  Dl[1] = c1 * wx;
  Dl[2] = c1 * wy;
  if constexpr (L >= 2) {
    Dl[3] = 6.0f * k20 * z * wz;
    Dl[4] = k21 * (z * wx + x * wz);
    Dl[5] = k21 * (z * wy + y * wz);
    Dl[6] = 2.0f * k22 * (x * wx - y * wy);
    Dl[7] = k21 * (y * wx + x * wy);
    if constexpr (L >= 3) {
      const float z2 = z * z, x2 = x * x, y2 = y * y;
      const float p = 5.0f * z2 - 1.0f;
      Dl[8] = k30 * (15.0f * z2 - 3.0f) * wz;
      Dl[9] = k31 * (p * wx + 10.0f * x * z * wz);
      Dl[10] = k31 * (p * wy + 10.0f * y * z * wz);
      Dl[11] = k32 * (2.0f * x * z * wx - 2.0f * y * z * wy + (x2 - y2) * wz);
      Dl[12] = k32s * (y * z * wx + x * z * wy + x * y * wz);
      Dl[13] = k33 * (3.0f * (x2 - y2) * wx - 6.0f * x * y * wy);
      Dl[14] = k33 * (6.0f * x * y * wx + 3.0f * (x2 - y2) * wy);
      if constexpr (L >= 4) {
        const float q = 7.0f * z2 - 3.0f;
        const float r = 7.0f * z2 - 1.0f;
        Dl[15] = k40 * (140.0f * z2 * z - 60.0f * z) * wz;
        Dl[16] = k41 * (z * q * wx + x * (21.0f * z2 - 3.0f) * wz);
        Dl[17] = k41 * (z * q * wy + y * (21.0f * z2 - 3.0f) * wz);
        Dl[18] = k42 * (2.0f * x * r * wx - 2.0f * y * r * wy + 14.0f * z * (x2 - y2) * wz);
        Dl[19] = k42s * (y * r * wx + x * r * wy + 14.0f * x * y * z * wz);
        Dl[20] = k43 * (3.0f * z * (x2 - y2) * wx - 6.0f * x * y * z * wy + x * (x2 - 3.0f * y2) * wz);
        Dl[21] = k43 * (6.0f * x * y * z * wx + 3.0f * z * (x2 - y2) * wy + y * (3.0f * x2 - y2) * wz);
        Dl[22] = k44 * (4.0f * x * (x2 - 3.0f * y2) * wx + 4.0f * y * (y2 - 3.0f * x2) * wy);
        Dl[23] = k44s * (y * (3.0f * x2 - y2) * wx + x * (x2 - 3.0f * y2) * wy);
      }
    }
  }
}

// Unnormalised harmonics: Y_lm(u) = kappa_lm Praw_lm(u), where Praw_lm is
// the polynomial of real_sph without its constant (same order).  The kernels
// accumulate sums of Praw and apply kappa once per atom.
template <int L>
struct Kappa {
  static constexpr int K = L * L + 2 * L;
  float v[K > 0 ? K : 1];
  constexpr Kappa() : v() {
    using namespace sh;
    const float all[24] = {c1,  c1,  c1,  k20, k21,  k21, k22, k21, k30, k31, k31, k32,
                           k32s, k33, k33, k40, k41, k41, k42, k42s, k43, k43, k44, k44s};
    for (int i = 0; i < K; ++i) v[i] = all[i];
  }
};

template <int L>
__device__ __forceinline__ void raw_sph(float x, float y, float z, float (&P)[L * L + 2 * L]) {
  P[0] = z;
  P[1] = x;
  P[2] = y;
  if constexpr (L >= 2) {
    const float z2 = z * z, xy = x * y;
    const float dxy = (x - y) * (x + y);  // x^2 - y^2
    P[3] = fmaf(3.0f, z2, -1.0f);
    P[4] = x * z;
    P[5] = y * z;
    P[6] = dxy;
    P[7] = xy;
    if constexpr (L >= 3) {
      const float p5 = fmaf(5.0f, z2, -1.0f);
      const float x3 = x * (dxy - 2.0f * y * y);  // x (x^2 - 3 y^2)
      const float y3 = y * (dxy + 2.0f * x * x);  // y (3 x^2 - y^2)
      P[8] = z * (p5 - 2.0f);                     // z (5 z^2 - 3)
      P[9] = x * p5;
      P[10] = y * p5;
      P[11] = z * dxy;
      P[12] = xy * z;
      P[13] = x3;
      P[14] = y3;
      if constexpr (L >= 4) {
        const float q7 = fmaf(7.0f, z2, -3.0f);
        const float r7 = q7 + 2.0f;  // 7 z^2 - 1
        P[15] = fmaf(z2, fmaf(35.0f, z2, -30.0f), 3.0f);
        P[16] = P[4] * q7;
        P[17] = P[5] * q7;
        P[18] = dxy * r7;
        P[19] = xy * r7;
        P[20] = z * x3;
        P[21] = z * y3;
        P[22] = fmaf(dxy, dxy, -4.0f * xy * xy);
        P[23] = xy * dxy;
      }
    }
  }
}

// v = sum_lm G_lm grad_u Praw_lm(u) (Praw extended off the unit sphere as
// polynomials); the caller projects out the radial component.
template <int L>
__device__ __forceinline__ void raw_sph_grad_dot(float x, float y, float z, const float (&G)[L * L + 2 * L], float& gx,
                                                 float& gy, float& gz) {
  gx = G[1];
  gy = G[2];
  gz = G[0];
  if constexpr (L >= 2) {
    // 3z^2-1: (0,0,6z)  xz: (z,0,x)  yz: (0,z,y)  x^2-y^2: (2x,-2y,0)  xy: (y,x,0)
    const float g6 = 2.0f * G[6];
    gx = fmaf(z, G[4], fmaf(x, g6, fmaf(y, G[7], gx)));
    gy = fmaf(z, G[5], fmaf(-y, g6, fmaf(x, G[7], gy)));
    gz = fmaf(6.0f * z, G[3], fmaf(x, G[4], fmaf(y, G[5], gz)));
    if constexpr (L >= 3) {
      const float z2 = z * z, xy = x * y, xz = x * z, yz = y * z;
      const float dxy = (x - y) * (x + y);
      const float p5 = fmaf(5.0f, z2, -1.0f);
      // z(5z^2-3): (0,0,15z^2-3)  x(5z^2-1): (p5,0,10xz)  y(5z^2-1): (0,p5,10yz)
      // z(x^2-y^2): (2xz,-2yz,dxy)  xyz: (yz,xz,xy)
      // x(x^2-3y^2): (3dxy,-6xy,0)  y(3x^2-y^2): (6xy,3dxy,0)
      const float g11 = 2.0f * G[11];
      const float a13 = 3.0f * G[13], a14 = 3.0f * G[14];
      gx = fmaf(p5, G[9], fmaf(xz, g11, fmaf(yz, G[12], fmaf(dxy, a13, fmaf(2.0f * xy, a14, gx)))));
      gy = fmaf(p5, G[10], fmaf(-yz, g11, fmaf(xz, G[12], fmaf(-2.0f * xy, a13, fmaf(dxy, a14, gy)))));
      gz = fmaf(fmaf(15.0f, z2, -3.0f), G[8],
                fmaf(10.0f * xz, G[9], fmaf(10.0f * yz, G[10], fmaf(dxy, G[11], fmaf(xy, G[12], gz)))));
      if constexpr (L >= 4) {
        const float q7 = fmaf(7.0f, z2, -3.0f), r7 = q7 + 2.0f;
        const float x3 = x * (dxy - 2.0f * y * y), y3 = y * (dxy + 2.0f * x * x);
        const float zq = z * q7;                       // 7z^3 - 3z
        const float w21 = fmaf(21.0f, z2, -3.0f);      // 21 z^2 - 3
        const float xyz = xy * z;
        // 35z^4-30z^2+3: (0,0,z(140z^2-60))
        // xz(7z^2-3): (zq,0,x w21)     yz(7z^2-3): (0,zq,y w21)
        // dxy r7: (2x r7,-2y r7,14 z dxy)   xy r7: (y r7, x r7, 14 xyz)
        // z x3: (3 z dxy, -6 xyz, x3)   z y3: (6 xyz, 3 z dxy, y3)
        // dxy^2-4x^2y^2: (4 x3, -4 y3, 0)   xy dxy: (y3, x3, 0)
        const float g18 = 2.0f * r7 * G[18];
        const float zd3 = 3.0f * z * dxy, xyz6 = 6.0f * xyz;
        const float g22 = 4.0f * G[22];
        gx = fmaf(zq, G[16], fmaf(x, g18, fmaf(y * r7, G[19], fmaf(zd3, G[20], fmaf(xyz6, G[21],
             fmaf(x3, g22, fmaf(y3, G[23], gx)))))));
        gy = fmaf(zq, G[17], fmaf(-y, g18, fmaf(x * r7, G[19], fmaf(-xyz6, G[20], fmaf(zd3, G[21],
             fmaf(-y3, g22, fmaf(x3, G[23], gy)))))));
        gz = fmaf(z * fmaf(140.0f, z2, -60.0f), G[15],
                  fmaf(x * w21, G[16], fmaf(y * w21, G[17], fmaf(14.0f * z * dxy, G[18], fmaf(14.0f * xyz, G[19],
                  fmaf(x3, G[20], fmaf(y3, G[21], gz)))))));
      }
    }
  }
}

// ------------------------------------------------------------- host helpers

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

}  // namespace nepmi

#define NEPMI_HIP(call)                                             \
  do {                                                              \
    hipError_t _e = (call);                                         \
    if (_e != hipSuccess) return ::nepmi::hip_fail(_e, #call);      \
  } while (0)
