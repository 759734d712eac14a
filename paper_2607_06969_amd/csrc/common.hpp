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

// ------------------------------------------------- precision-generic helpers

// The float32 kernels and the float64 variants share the templated helpers
// below; each call resolves to the single- or double-precision function.
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float tanh_(float x) { return tanhf(x); }
__device__ __forceinline__ double tanh_(double x) { return tanh(x); }
__device__ __forceinline__ float cospi_(float x) { return cospif(x); }
__device__ __forceinline__ double cospi_(double x) { return cospi(x); }
__device__ __forceinline__ void sincospi_(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_(double x, double* s, double* c) { sincospi(x, s, c); }

// Position (x, y, z) and species of a slot: float4 with the species bits in w,
// or double4 with the species value in w.
template <class R>
struct Vec4T;
template <>
struct Vec4T<float> {
  using type = float4;
};
template <>
struct Vec4T<double> {
  using type = double4;
};
template <class R>
using Vec4 = typename Vec4T<R>::type;
__device__ __forceinline__ int species_of(const float4& x) { return __float_as_int(x.w); }
__device__ __forceinline__ int species_of(const double4& x) { return (int)x.w; }
template <class R>
__device__ __forceinline__ Vec4<R> make_v4(R x, R y, R z, R w);
template <>
__device__ __forceinline__ float4 make_v4<float>(float x, float y, float z, float w) {
  return make_float4(x, y, z, w);
}
template <>
__device__ __forceinline__ double4 make_v4<double>(double x, double y, double z, double w) {
  return make_double4(x, y, z, w);
}

template <class R>
struct ShC;  // constants of the real spherical harmonics, per precision

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

// Register copy the compiler cannot see through.  A ring slot is read through
// it before the slot is reloaded, so the old value is dead when the load
// issues and the load lands in the slot's own register.  Otherwise the load
// goes to a fresh register and the loop latch copies it back, which waits for
// the load just issued and drains the prefetch ring once per trip.
__device__ __forceinline__ uint32_t take_slot(uint32_t v) {
  uint32_t r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v) : "memory");
  return r;
}

// No per-pair loads ahead of the ring's prefetches.
struct NoPre {
  __device__ __forceinline__ int operator()(int, uint32_t) const { return 0; }
};

// Pair lists (the Verlet list, its reverse index and the compact lists) are
// stored in groups of four entries: group g (entries 4g .. 4g+3) of slot p is
// the uint4 at [g * n_slots + p].  A writer that appends entries one lane at
// a time then stores once per four entries (each such store touches one cache
// line per lane, so their number is what costs), and a reader loads four
// entries with one coalesced 16-byte load.
template <int G = 4>
constexpr int list_groups(int entries) {
  return (entries + G - 1) / G;
}

__device__ __forceinline__ uint32_t comp4(const uint4& v, int u) {
  return u == 0 ? v.x : (u == 1 ? v.y : (u == 2 ? v.z : v.w));
}

// Opaque copy of a group (see take_slot).
__device__ __forceinline__ uint4 take_group(const uint4& v) {
  return make_uint4(take_slot(v.x), take_slot(v.y), take_slot(v.z), take_slot(v.w));
}

// Software-pipelined walk over one atom's pair list (groups of four), calling
// f(k, entry, neighbour position, aux entry, pre(k, entry)) for k = 0 .. n-1
// in order.  A pair needs two dependent loads: the list entry (a stream from
// HBM), then the neighbour's position (a gather, mostly from L2).  Groups are
// loaded two at a time (A = group 2i, B = group 2i+1), the next pair of
// groups three to four pairs before their first position is needed, and
// neighbour positions two pairs ahead; with AUX, a second list of the same
// shape (aux) is loaded alongside and its entry reaches f as the fourth
// argument.  The loop is unrolled by eight so that every ring slot is a fixed
// register; groups past the last are clamped to it, so every load is in
// bounds, and an empty list loads nothing.
//
// Loads complete in issue order as far as the wait counter is concerned:
// waiting for a load waits for every load issued before it.  So pair k's own
// loads (pre, e.g. a row of the neighbour) are issued before the prefetches
// of this step, and waiting for them leaves the prefetches in flight; pre runs
// on every step, also past the end of a short list (k >= n), where f is not
// called.
template <bool AUX = false, class P, class Pre, class F>
__device__ __forceinline__ void walk_groups(const uint4* __restrict__ list, int64_t ns, int64_t p, int n,
                                            const P* __restrict__ pos4, Pre&& pre, F&& f,
                                            const uint4* __restrict__ aux = nullptr) {
  if (n <= 0) return;
  const int ng = list_groups(n);
  // group g of this slot, clamped to the last group
  auto at = [&](const uint4* l, int g) { return l[(int64_t)(g < ng ? g : ng - 1) * ns + p]; };
  uint4 A = at(list, 0), B = at(list, 1);
  uint4 XA = make_uint4(0u, 0u, 0u, 0u), XB = XA;
  if constexpr (AUX) {
    XA = at(aux, 0);
    XB = at(aux, 1);
  }
  P x[2];
  x[0] = pos4[A.x & kNbrMask];
  x[1] = pos4[A.y & kNbrMask];
  __builtin_amdgcn_sched_barrier(0);
  for (int g = 0; g < ng; g += 2) {
    const int k0 = 4 * g;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      const uint32_t ek = take_slot(comp4(u < 4 ? A : B, u & 3));
      const uint32_t ak = AUX ? take_slot(comp4(u < 4 ? XA : XB, u & 3)) : 0u;
      const P xk = x[u & 1];
      const auto pk = pre(k, ek);
      asm volatile("" ::: "memory");  // keeps pre's loads ahead of the prefetches
      // the entry of pair k + 2 (from A, B or the next A), then its position
      uint32_t en;
      if (u < 2) {
        en = comp4(A, u + 2);
      } else if (u < 6) {
        en = comp4(B, u - 2);
      } else {
        en = comp4(A, u - 6);
      }
      x[u & 1] = pos4[en & kNbrMask];
      if (u == 3) {  // A is used up: the next even group
        A = at(list, g + 2);
        if constexpr (AUX) XA = at(aux, g + 2);
      }
      if (u == 7) {  // B is used up: the next odd group
        B = at(list, g + 3);
        if constexpr (AUX) XB = at(aux, g + 3);
      }
      if (k < n) f(k, ek, xk, ak, pk);
    }
  }
}

// Entry k of slot p of a list stored in groups of four.
__device__ __forceinline__ int64_t group_index(int64_t ns, int64_t p, int k) {
  return (((int64_t)(k >> 2) * ns + p) << 2) + (k & 3);
}

// One periodic configuration as the kernels see it.
struct CfgDev {
  float H[9];       // lattice vectors as rows, float32
  double Hd[9];     // same, float64
  double Hinv[9];   // inverse, float64 (fractional = x . Hinv)
  int nb[3];        // bins per direction
  int bin_off;      // first global bin of this configuration
  int64_t atom_off; // first atom (caller's order)
  int n_atoms;
  int periodic;     // bit a set: periodic along lattice vector a
};

// Runtime (non-shape) parameters of a launch.
template <class R>
struct CutoffsT {
  R rcR, rcA;        // cutoffs of the potential
  R rcR2, rcA2;      // squared
  R rclR2, rclA2;    // squared list cutoffs (cutoff + skin)
};
using Cutoffs = CutoffsT<float>;

// ------------------------------------------------------------ device helpers

// Image code = 9 (w0 + 1) + 3 (w1 + 1) + (w2 + 1), w in {-1, 0, 1}; the shift is
// w0 a + w1 b + w2 c for lattice rows a, b, c.  Digits by multiply-shift
// (exact for code < 27: floor(57 c / 512) = floor(c / 9), floor(11 r / 32) =
// floor(r / 3) for r < 9).  Every w_a is -1, 0 or 1, so the shift of code
// 26 - code is the exact negative of the shift of code.
template <class R>
__device__ __forceinline__ void image_shift(const R* __restrict__ H, uint32_t code, R& sx, R& sy, R& sz) {
  // 24-bit products (full-rate multiplies; every operand is below 2^9)
  const uint32_t d0 = __umul24(code, 57u) >> 9;
  const uint32_t r = code - __umul24(9u, d0);
  const uint32_t d1 = __umul24(r, 11u) >> 5;
  const uint32_t d2 = r - __umul24(3u, d1);
  const R w0 = (R)((int)d0 - 1);
  const R w1 = (R)((int)d1 - 1);
  const R w2 = (R)((int)d2 - 1);
  sx = w0 * H[0] + w1 * H[3] + w2 * H[6];
  sy = w0 * H[1] + w1 * H[4] + w2 * H[7];
  sz = w0 * H[2] + w1 * H[5] + w2 * H[8];
}

// Chebyshev radial basis of Eq. 12-15 and its radial derivative dQ_k/dd:
//   x = 2 (d/rc - 1)^2 - 1,  f_c = (1 + cos(pi d/rc)) / 2,  Q_k = (T_k(x) + 1)/2 f_c.
// Valid for d < rc (the caller tests the cutoff).
template <int B, class R>
__device__ __forceinline__ void cheb_basis_d(R d, R rc_inv, R (&Q)[B], R (&dQ)[B]) {
  using C = ShC<R>;
  const R t = d * rc_inv;
  const R y = t - R(1.0);
  const R x = R(2.0) * y * y - R(1.0);
  const R dx = R(4.0) * y * rc_inv;
  R sn, cs;
  sincospi_(t, &sn, &cs);
  const R fc = R(0.5) * (R(1.0) + cs);
  const R dfc = -R(0.5) * C::pi * rc_inv * sn;
  R tm = R(1.0), tk = x, dtm = R(0.0), dtk = R(1.0);
  Q[0] = fc;
  dQ[0] = dfc;
  if (B > 1) {
    Q[1] = R(0.5) * (x + R(1.0)) * fc;
    dQ[1] = R(0.5) * (dx * fc + (x + R(1.0)) * dfc);
  }
#pragma unroll
  for (int k = 2; k < B; ++k) {
    const R tn = R(2.0) * x * tk - tm;
    const R dtn = R(2.0) * tk + R(2.0) * x * dtk - dtm;
    tm = tk;
    tk = tn;
    dtm = dtk;
    dtk = dtn;
    Q[k] = R(0.5) * (tn + R(1.0)) * fc;
    dQ[k] = R(0.5) * (dtn * dx * fc + (tn + R(1.0)) * dfc);
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
template <class R>
__device__ __forceinline__ R pair_d2(R rx, R ry, R rz) {
  return fma_(rz, rz, fma_(ry, ry, rx * rx));
}

// Lattice rows of a configuration in the precision of the caller.
__device__ __forceinline__ const float* cell_rows(const CfgDev& C, float) { return C.H; }
__device__ __forceinline__ const double* cell_rows(const CfgDev& C, double) { return C.Hd; }

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

// Precision traits of the templated helpers: the float members are the float
// constants above, the double members the same quantities to double precision.
template <class R>
struct ShC;
template <>
struct ShC<float> {
  static constexpr float c1 = sh::c1;
  static constexpr float k20 = sh::k20;
  static constexpr float k21 = sh::k21;
  static constexpr float k22 = sh::k22;
  static constexpr float k30 = sh::k30;
  static constexpr float k31 = sh::k31;
  static constexpr float k32 = sh::k32;
  static constexpr float k32s = sh::k32s;
  static constexpr float k33 = sh::k33;
  static constexpr float k40 = sh::k40;
  static constexpr float k41 = sh::k41;
  static constexpr float k42 = sh::k42;
  static constexpr float k42s = sh::k42s;
  static constexpr float k43 = sh::k43;
  static constexpr float k44 = sh::k44;
  static constexpr float k44s = sh::k44s;
  static constexpr float pi = 3.14159265358979323846f;
};
template <>
struct ShC<double> {
  static constexpr double c1 = 0.48860251190291992158;
  static constexpr double k20 = 0.31539156525252000603;
  static constexpr double k21 = 1.09254843059207907054;
  static constexpr double k22 = 0.54627421529603953527;
  static constexpr double k30 = 0.37317633259011539141;
  static constexpr double k31 = 0.45704579946446573615;
  static constexpr double k32 = 1.44530572132027702769;
  static constexpr double k32s = 2.89061144264055405538;
  static constexpr double k33 = 0.59004358992664351034;
  static constexpr double k40 = 0.10578554691520430380;
  static constexpr double k41 = 0.66904654355728916795;
  static constexpr double k42 = 0.47308734787878000904;
  static constexpr double k42s = 0.94617469575756001809;
  static constexpr double k43 = 1.77013076977993053103;
  static constexpr double k44 = 0.62583573544917613458;
  static constexpr double k44s = 2.50334294179670453834;
  static constexpr double pi = 3.14159265358979323846;
};

template <int L, class R>
__device__ __forceinline__ void real_sph(R x, R y, R z, R (&Y)[L * L + 2 * L]) {
  using C = ShC<R>;
  Y[0] = C::c1 * z;
  Y[1] = C::c1 * x;
  Y[2] = C::c1 * y;
  if constexpr (L >= 2) {
    const R z2 = z * z;
    Y[3] = C::k20 * (R(3.0) * z2 - R(1.0));
    Y[4] = C::k21 * x * z;
    Y[5] = C::k21 * y * z;
    Y[6] = C::k22 * (x * x - y * y);
    Y[7] = C::k21 * x * y;
    if constexpr (L >= 3) {
      const R x2my2 = x * x - y * y;
      const R p = R(5.0) * z2 - R(1.0);
      Y[8] = C::k30 * z * (R(5.0) * z2 - R(3.0));
      Y[9] = C::k31 * x * p;
      Y[10] = C::k31 * y * p;
      Y[11] = C::k32 * z * x2my2;
      Y[12] = C::k32s * x * y * z;
      Y[13] = C::k33 * x * (x * x - R(3.0) * y * y);
      Y[14] = C::k33 * y * (R(3.0) * x * x - y * y);
      if constexpr (L >= 4) {
        const R q = R(7.0) * z2 - R(3.0);
        const R r = R(7.0) * z2 - R(1.0);
        Y[15] = C::k40 * (R(35.0) * z2 * z2 - R(30.0) * z2 + R(3.0));
        Y[16] = C::k41 * x * z * q;
        Y[17] = C::k41 * y * z * q;
        Y[18] = C::k42 * x2my2 * r;
        Y[19] = C::k42s * x * y * r;
        Y[20] = C::k43 * x * z * (x * x - R(3.0) * y * y);
        Y[21] = C::k43 * y * z * (R(3.0) * x * x - y * y);
        Y[22] = C::k44 * (x2my2 * x2my2 - R(4.0) * x * x * y * y);
        Y[23] = C::k44s * x * y * x2my2;
      }
    }
  }
}

// g = sum_lm G_lm grad_u P_lm(u), where P_lm is the polynomial of real_sph
// (extended off the unit sphere).  The gradient of Y_lm(r/|r|) with respect to
// r is (I - u u^T) grad_u P_lm / |r|; the caller applies that projection.
template <int L, class R>
__device__ __forceinline__ void real_sph_grad_dot(R x, R y, R z, const R (&G)[L * L + 2 * L],
                                                  R& gx, R& gy, R& gz) {
  using C = ShC<R>;
  gx = C::c1 * G[1];
  gy = C::c1 * G[2];
  gz = C::c1 * G[0];
  if constexpr (L >= 2) {
    gz += R(6.0) * C::k20 * z * G[3];
    gx += C::k21 * z * G[4];
    gz += C::k21 * x * G[4];
    gy += C::k21 * z * G[5];
    gz += C::k21 * y * G[5];
    gx += R(2.0) * C::k22 * x * G[6];
    gy -= R(2.0) * C::k22 * y * G[6];
    gx += C::k21 * y * G[7];
    gy += C::k21 * x * G[7];
    if constexpr (L >= 3) {
      const R z2 = z * z, x2 = x * x, y2 = y * y;
      const R p = R(5.0) * z2 - R(1.0);
      gz += C::k30 * (R(15.0) * z2 - R(3.0)) * G[8];
      gx += C::k31 * p * G[9];
      gz += R(10.0) * C::k31 * x * z * G[9];
      gy += C::k31 * p * G[10];
      gz += R(10.0) * C::k31 * y * z * G[10];
      gx += R(2.0) * C::k32 * x * z * G[11];
      gy -= R(2.0) * C::k32 * y * z * G[11];
      gz += C::k32 * (x2 - y2) * G[11];
      gx += C::k32s * y * z * G[12];
      gy += C::k32s * x * z * G[12];
      gz += C::k32s * x * y * G[12];
      gx += R(3.0) * C::k33 * (x2 - y2) * G[13];
      gy -= R(6.0) * C::k33 * x * y * G[13];
      gx += R(6.0) * C::k33 * x * y * G[14];
      gy += R(3.0) * C::k33 * (x2 - y2) * G[14];
      if constexpr (L >= 4) {
        const R q = R(7.0) * z2 - R(3.0);
        const R r = R(7.0) * z2 - R(1.0);
        gz += C::k40 * (R(140.0) * z2 * z - R(60.0) * z) * G[15];
        gx += C::k41 * z * q * G[16];
        gz += C::k41 * x * (R(21.0) * z2 - R(3.0)) * G[16];
        gy += C::k41 * z * q * G[17];
        gz += C::k41 * y * (R(21.0) * z2 - R(3.0)) * G[17];
        gx += R(2.0) * C::k42 * x * r * G[18];
        gy -= R(2.0) * C::k42 * y * r * G[18];
        gz += R(14.0) * C::k42 * z * (x2 - y2) * G[18];
        gx += C::k42s * y * r * G[19];
        gy += C::k42s * x * r * G[19];
        gz += R(14.0) * C::k42s * x * y * z * G[19];
        gx += R(3.0) * C::k43 * z * (x2 - y2) * G[20];
        gy -= R(6.0) * C::k43 * x * y * z * G[20];
        gz += C::k43 * x * (x2 - R(3.0) * y2) * G[20];
        gx += R(6.0) * C::k43 * x * y * z * G[21];
        gy += R(3.0) * C::k43 * z * (x2 - y2) * G[21];
        gz += C::k43 * y * (R(3.0) * x2 - y2) * G[21];
        gx += R(4.0) * C::k44 * x * (x2 - R(3.0) * y2) * G[22];
        gy += R(4.0) * C::k44 * y * (y2 - R(3.0) * x2) * G[22];
        gx += C::k44s * y * (R(3.0) * x2 - y2) * G[23];
        gy += C::k44s * x * (x2 - R(3.0) * y2) * G[23];
      }
    }
  }
}

// Dl[lm] = w . grad_u P_lm(u) for every component (P_lm as in real_sph).
template <int L, class R>
__device__ __forceinline__ void real_sph_dir(R x, R y, R z, R wx, R wy, R wz,
                                             R (&Dl)[L * L + 2 * L]) {
  using C = ShC<R>;
  Dl[0] = C::c1 * wz;
  Dl[1] = C::c1 * wx;
  Dl[2] = C::c1 * wy;
  if constexpr (L >= 2) {
    Dl[3] = R(6.0) * C::k20 * z * wz;
    Dl[4] = C::k21 * (z * wx + x * wz);
    Dl[5] = C::k21 * (z * wy + y * wz);
    Dl[6] = R(2.0) * C::k22 * (x * wx - y * wy);
    Dl[7] = C::k21 * (y * wx + x * wy);
    if constexpr (L >= 3) {
      const R z2 = z * z, x2 = x * x, y2 = y * y;
      const R p = R(5.0) * z2 - R(1.0);
      Dl[8] = C::k30 * (R(15.0) * z2 - R(3.0)) * wz;
      Dl[9] = C::k31 * (p * wx + R(10.0) * x * z * wz);
      Dl[10] = C::k31 * (p * wy + R(10.0) * y * z * wz);
      Dl[11] = C::k32 * (R(2.0) * x * z * wx - R(2.0) * y * z * wy + (x2 - y2) * wz);
      Dl[12] = C::k32s * (y * z * wx + x * z * wy + x * y * wz);
      Dl[13] = C::k33 * (R(3.0) * (x2 - y2) * wx - R(6.0) * x * y * wy);
      Dl[14] = C::k33 * (R(6.0) * x * y * wx + R(3.0) * (x2 - y2) * wy);
      if constexpr (L >= 4) {
        const R q = R(7.0) * z2 - R(3.0);
        const R r = R(7.0) * z2 - R(1.0);
        Dl[15] = C::k40 * (R(140.0) * z2 * z - R(60.0) * z) * wz;
        Dl[16] = C::k41 * (z * q * wx + x * (R(21.0) * z2 - R(3.0)) * wz);
        Dl[17] = C::k41 * (z * q * wy + y * (R(21.0) * z2 - R(3.0)) * wz);
        Dl[18] = C::k42 * (R(2.0) * x * r * wx - R(2.0) * y * r * wy + R(14.0) * z * (x2 - y2) * wz);
        Dl[19] = C::k42s * (y * r * wx + x * r * wy + R(14.0) * x * y * z * wz);
        Dl[20] = C::k43 * (R(3.0) * z * (x2 - y2) * wx - R(6.0) * x * y * z * wy + x * (x2 - R(3.0) * y2) * wz);
        Dl[21] = C::k43 * (R(6.0) * x * y * z * wx + R(3.0) * z * (x2 - y2) * wy + y * (R(3.0) * x2 - y2) * wz);
        Dl[22] = C::k44 * (R(4.0) * x * (x2 - R(3.0) * y2) * wx + R(4.0) * y * (y2 - R(3.0) * x2) * wy);
        Dl[23] = C::k44s * (y * (R(3.0) * x2 - y2) * wx + x * (x2 - R(3.0) * y2) * wy);
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
