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

// Lattice-vector multiples (w0, w1, w2) of the 27 image codes (see
// image_shift), in LDS: one read per pair instead of the integer decode.
struct ImageTable {
  float4 w[32];
  __device__ void fill() {
    if (threadIdx.x < 27) {
      const int c = threadIdx.x;
      w[c] = make_float4((float)(c / 9 - 1), (float)((c / 3) % 3 - 1), (float)(c % 3 - 1), 0.f);
    }
  }
};

__device__ __forceinline__ PairVec pair_vec(uint32_t e, float4 xq, float4 xi, const float (&H)[9],
                                            const ImageTable& it) {
  PairVec v;
  v.q = (int)(e & kNbrMask);
  // the same expression as image_shift, so the shift of code 26 - c is again
  // exactly the negative of the shift of c
  const float4 w = it.w[e >> kNbrShift];
  const float sx = w.x * H[0] + w.y * H[3] + w.z * H[6];
  const float sy = w.x * H[1] + w.y * H[4] + w.z * H[7];
  const float sz = w.x * H[2] + w.y * H[5] + w.z * H[8];
  v.rx = (xq.x - xi.x) + sx;
  v.ry = (xq.y - xi.y) + sy;
  v.rz = (xq.z - xi.z) + sz;
  v.d2 = pair_d2(v.rx, v.ry, v.rz);
  v.zj = __float_as_int(xq.w);
  return v;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Groups of four list entries fill by shifting entries in from the top
// (register moves, no selects), so a full group holds them in order; a
// partly filled one holds its r entries in the top r components, which
// front4 moves to the front (the rest repeat the last entry, a real one).
__device__ __forceinline__ void shift_in4(uint4& v, uint32_t e) { v = make_uint4(v.y, v.z, v.w, e); }
__device__ __forceinline__ uint4 front4(uint4 g, int r) {
  return r == 1 ? make_uint4(g.w, g.w, g.w, g.w) : r == 2 ? make_uint4(g.z, g.w, g.w, g.w)
                                                           : make_uint4(g.y, g.z, g.w, g.w);
}

// One neighbour's radial adjoint row (B_R floats).
template <int BR>
struct AdjRow {
  float4 v[BR / 4];
};

// Network dimensions padded to the 4-wide groups of the matrix instructions.
template <class S>
struct MlpPad {
  static constexpr int HP = (S::H + 3) / 4 * 4;
  static constexpr int DP = (S::D + 3) / 4 * 4;
};

// tanh(x) = 1 - 2 / (1 + e^{2x}) with the hardware exp2 and reciprocal
// (absolute error a few 1e-7; saturates to +-1 for large |x|).
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 log2(e)
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
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

// S_nlm (l = 1..L) of one group of NH angular functions, summed over the
// angular pairs of the atom (Eq. 16): S = sum_j g_n(r_ij) Y_lm(u_ij) with
// g_n = sum_k c[Z_i][Z_j][n][k] Q_k = hf sum_k ctil_nk T_k (derived table).
template <class S, int NH>
__device__ __forceinline__ void angular_sums(const float4* __restrict__ pos4, const uint32_t* __restrict__ cnA,
                                             int64_t n_slots, int64_t p, int nA, float4 xi, const float (&Hc)[9],
                                             const ImageTable& it, const float* cl0, float rcA_inv,
                                             float (&Sg)[NH][S::K]) {
  constexpr int T = S::T, NA = S::NA, BA = S::BA, L = S::L, K = S::K;
#pragma unroll
  for (int nn = 0; nn < NH; ++nn)
#pragma unroll
    for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = 0.f;
  walk_groups(reinterpret_cast<const uint4*>(cnA), n_slots, p, nA, pos4, NoPre{},
              [&](int, uint32_t e, float4 xq, uint32_t, int) {
    const PairVec v = pair_vec(e, xq, xi, Hc, it);
    const float inv = rsqrt_hw(v.d2);
    const RadialF f = radial_f(v.d2 * inv * rcA_inv);
    float Tk[BA];
    cheb_t<BA>(f.x, Tk);
    const float* cl = cl0 + v.zj * (NA * BA);
    float g[NH];
#pragma unroll
    for (int nn = 0; nn < NH; ++nn) {
      float acc = 0.f;
#pragma unroll
      for (int kk = 0; kk < BA; ++kk) acc = fmaf(cl[nn * BA + kk], Tk[kk], acc);
      g[nn] = f.hf * acc;
    }
    float P[K];
    raw_sph<L>(v.rx * inv, v.ry * inv, v.rz * inv, P);
#pragma unroll
    for (int nn = 0; nn < NH; ++nn)
#pragma unroll
      for (int lm = 0; lm < K; ++lm) Sg[nn][lm] = fmaf(g[nn], P[lm], Sg[nn][lm]);
  });
  constexpr Kappa<L> kap;
#pragma unroll
  for (int nn = 0; nn < NH; ++nn)
#pragma unroll
    for (int lm = 0; lm < K; ++lm) Sg[nn][lm] *= kap.v[lm];
  (void)T;
}

// ------------------------------------------------------- network (Sec. 2.3)

// First-layer weights of the species this block's wavefronts hold (each
// wavefront is uniform) into LDS, zero padded, as [Z][h][d] and transposed
// [Z][d][h].  Every thread of the block must call it (it ends with a barrier).
template <class S, int BS>
__device__ __forceinline__ void load_weights(const float* __restrict__ params, const float4* __restrict__ pos4,
                                             int64_t n_slots, int64_t p, float* W0s, float* W0Ts) {
  constexpr int T = S::T, D = S::D, H = S::H;
  constexpr int HP = MlpPad<S>::HP, DP = MlpPad<S>::DP;
  const int64_t b0 = p - threadIdx.x;
  unsigned need = 0;
#pragma unroll
  for (int w = 0; w < BS / kWave; ++w) {
    const int64_t s0 = b0 + w * kWave;
    need |= 1u << __float_as_int(pos4[s0 < n_slots ? s0 : n_slots - 1].w);
  }
  for (int z = 0; z < T; ++z) {
    if (!(need >> z & 1u)) continue;
    const float* W0g = params + S::PCR + S::PCA + (int64_t)z * S::PMLP;
    for (int t = threadIdx.x; t < HP * DP; t += BS) {
      const int h = t / DP, d = t % DP;
      const float w = (h < H && d < D) ? W0g[h * D + d] : 0.0f;
      W0s[(z * HP + h) * DP + d] = w;
      W0Ts[(z * DP + d) * HP + h] = w;
    }
  }
  __syncthreads();
}

// The network of species Zs on the matrix cores, and what follows from it:
// site energy E_i, dE_i/dq for the angular descriptors (fp), the radial
// adjoint atil_i[b][k] = sum_n dE_i/dq_n ctil[Z_i][b][n][k] (aR), and the
// optional descriptor copy.  With the 16-block 4x4x1 fp32 MFMA, block b
// (lanes 4b..4b+3) forms C[i][j] += A[i] B[j] with A[i] from lane 4b+i and
// B[j] from lane 4b+j, and lane 4b+j keeps column j.  Every lane supplies its
// own atom's value as B and a weight row selected by lane % 4 as A, so each
// lane accumulates four entries of its own atom: no data moves between
// lanes.  Every lane of the wavefront must call it (inactive atoms included).
template <class S>
__device__ __forceinline__ void network(const float (&q)[MlpPad<S>::DP], int Zs, bool active, int64_t n_slots,
                                        int64_t p, const int* __restrict__ orig, const float* __restrict__ params,
                                        const float* W0s, const float* W0Ts, float* __restrict__ fp,
                                        float* __restrict__ aR, float* __restrict__ Ei, float* __restrict__ qout,
                                        float* __restrict__ Eproc, int want_adjoint) {
  constexpr int T = S::T, NR = S::NR, BR = S::BR, D = S::D, H = S::H;
  constexpr int HP = MlpPad<S>::HP, DP = MlpPad<S>::DP;
  const float* __restrict__ dco = params + S::P;
  const int lq = threadIdx.x & 3;
  const float* b0g = params + S::PCR + S::PCA + (int64_t)Zs * S::PMLP + H * D;
  const float* w1g = b0g + H;
  //  forward: a_h = b0_h + sum_d W0[h][d] q_d, four hidden units per group
  floatx4 acc[HP / 4];
#pragma unroll
  for (int hg = 0; hg < HP / 4; ++hg)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[hg][r] = (4 * hg + r < H) ? b0g[4 * hg + r] : 0.f;
  {
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
      }
    }
  }
  if (active && qout) {
    const int i = orig[p];
#pragma unroll
    for (int d = 0; d < D; ++d) qout[(int64_t)i * D + d] = q[d];
  }
  //  E = b1 + sum_h w1_h tanh(a_h);  z_h = dE/da_h = w1_h (1 - tanh^2)
  float E = w1g[H];
  float zt[HP];
#pragma unroll
  for (int hg = 0; hg < HP / 4; ++hg)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int h = 4 * hg + r;
      if (h < H) {
        const float t = tanh_fast(acc[hg][r]);
        E = fmaf(w1g[h], t, E);
        zt[h] = w1g[h] * fmaf(-t, t, 1.0f);
      } else {
        zt[h] = 0.f;
      }
    }
  //  backward: dE/dq_d = sum_h z_h W0[h][d], four descriptors per group
  floatx4 fpa[DP / 4];
#pragma unroll
  for (int dg = 0; dg < DP / 4; ++dg) fpa[dg] = floatx4{0.f, 0.f, 0.f, 0.f};
  {
    const float* WzT = W0Ts + (Zs * DP + lq) * HP;
#pragma unroll
    for (int hg = 0; hg < HP / 4; ++hg) {
#pragma unroll
      for (int dg = 0; dg < DP / 4; ++dg) {
        const float4 w = *reinterpret_cast<const float4*>(WzT + 4 * dg * HP + 4 * hg);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, zt[4 * hg + 0], fpa[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, zt[4 * hg + 1], fpa[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, zt[4 * hg + 2], fpa[dg], 0, 0, 0);
        fpa[dg] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, zt[4 * hg + 3], fpa[dg], 0, 0, 0);
      }
    }
  }
  float Fp[DP];
#pragma unroll
  for (int dg = 0; dg < DP / 4; ++dg)
#pragma unroll
    for (int r = 0; r < 4; ++r) Fp[4 * dg + r] = fpa[dg][r];
  if (!active) return;
  const int i = orig[p];
  Ei[i] = E;
  if (Eproc) Eproc[p] = E;
  if (!want_adjoint) return;
#pragma unroll
  for (int d = NR; d < D; ++d) fp[(int64_t)(d - NR) * n_slots + p] = Fp[d];
  // radial adjoint atil[b][k] = sum_n dE/dq_n ctil[Z_i][b][n][k], one row
  // of B_R floats per part, written as float4
  static_assert(BR % 4 == 0, "adjoint rows are written as float4");
  const float* cR = dco + (int64_t)Zs * (T * NR * BR);
#pragma unroll
  for (int b = 0; b < T; ++b) {
    float4* row = reinterpret_cast<float4*>(aR + ((int64_t)b * n_slots + p) * BR);
#pragma unroll
    for (int k4 = 0; k4 < BR / 4; ++k4) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float acc = 0.f;
#pragma unroll
        for (int nn = 0; nn < NR; ++nn) acc = fmaf(Fp[nn], cR[(b * NR + nn) * BR + 4 * k4 + u], acc);
        v[u] = acc;
      }
      row[k4] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// ------------------------------------------------------------------ k_desc

// NET: the network runs in this kernel (4x4x1 matrix instructions, one atom
// per lane); otherwise the descriptors are left for k_net in the buffers the
// network's outputs later take: radial q_n in the atom's aR rows (entry
// n % B_R of part n / B_R), the angular ones in fp.  The unfused form needs no
// network weights in LDS and fewer registers, so more wavefronts share a
// compute unit during the pair walks, and k_net runs the network as dense
// products; it pays one extra write and read of the descriptors.
template <class S, int NSPLIT, int WPE, bool NET, int BS = kBlock>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(WPE))) void k_desc(
    int64_t n_slots, int capA, const float4* __restrict__ pos4, const int* __restrict__ cfg_of,
    const int* __restrict__ orig, const CfgDev* __restrict__ cfgs, const uint32_t* __restrict__ nbrR,
    const int* __restrict__ cntR, const uint32_t* __restrict__ vrev, uint32_t* __restrict__ cnR, int* __restrict__ ccR,
    uint32_t* __restrict__ cnA, uint32_t* __restrict__ cpA, int* __restrict__ ccA, uint64_t* __restrict__ amask,
    int* __restrict__ flags, Cutoffs cut,
    const float* __restrict__ params, float* __restrict__ fp, float* __restrict__ aR, float* __restrict__ Ei,
    float* __restrict__ qout, float* __restrict__ Eproc, int want_adjoint) {
  constexpr int T = S::T, NR = S::NR, NA = S::NA, BR = S::BR, BA = S::BA, L = S::L, K = S::K, D = S::D, H = S::H;
  constexpr int NH = NA / NSPLIT;
  static_assert(NA % NSPLIT == 0, "NSPLIT must divide n_angular");
  constexpr int HP = MlpPad<S>::HP, DP = MlpPad<S>::DP;
  const float* __restrict__ dco = params + S::P;  // derived coefficients: radial, then angular
  __shared__ float cA_s[T * T * NA * BA];
  __shared__ ImageTable itab;
  __shared__ float W0s[NET ? T * HP * DP : 1];   // [Z][h][d] network weights, zero padded
  __shared__ float W0Ts[NET ? T * DP * HP : 1];  // [Z][d][h] the same, transposed

  // Every lane of a wavefront takes part in the matrix instructions of the
  // network, so lanes past the last slot stay alive as inactive atoms.
  const int64_t p = xcd_tile() * BS + threadIdx.x;
  const bool in_range = p < n_slots;
  const int64_t pc = in_range ? p : n_slots - 1;
  const float4 xi = pos4[pc];
  const int Zs = __builtin_amdgcn_readfirstlane(__float_as_int(xi.w));
  for (int t = threadIdx.x; t < T * T * NA * BA; t += BS) cA_s[t] = dco[S::PCR + t];
  itab.fill();
  if constexpr (NET) {
    load_weights<S, BS>(params, pos4, n_slots, p, W0s, W0Ts);
  } else {
    __syncthreads();
  }

  const int c = in_range ? cfg_of[p] : -1;
  const bool active = c >= 0;
  float Hc[9];
  load_cell(cfgs, c, Hc);
  const float rcR_inv = 1.0f / cut.rcR, rcA_inv = 1.0f / cut.rcA;

  // ---- filter the Verlet list into the pairs inside the two cutoffs, and
  //      accumulate PT_b[k] = sum over radial neighbours j of species b of
  //      hf_j T_k(x_j) on the way (Eq. 11-15)
  float PT[T][BR];
#pragma unroll
  for (int b = 0; b < T; ++b)
#pragma unroll
    for (int k = 0; k < BR; ++k) PT[b][k] = 0.f;
  int nR = 0, nA = 0;
  if (active) {
    const int n = cntR[p];
    bool bad = false;
    // compact lists in groups of four entries: each lane collects a group in
    // registers and stores it when full (one store per four kept pairs)
    uint4* wr = reinterpret_cast<uint4*>(cnR) + p;   // next group of the compact radial list
    uint4* wa = reinterpret_cast<uint4*>(cnA) + p;   // ... of the compact angular list
    uint4* wp = reinterpret_cast<uint4*>(cpA) + p;   // ... and of its row pairs
    uint4 gr = make_uint4(0u, 0u, 0u, 0u), ga = gr, gp = gr;
    uint64_t* mw = amask + p;
    // bit a % 64: entry a of the angular part of the Verlet list (the entries
    // with a reverse position) is in the compact angular list
    uint64_t mword = 0;
    int ka = 0;  // position in the angular part of the list
    walk_groups<true>(reinterpret_cast<const uint4*>(nbrR), n_slots, p, n, pos4, NoPre{},
                      [&](int, uint32_t e, float4 xq, uint32_t rvk, int) {
      const PairVec v = pair_vec(e, xq, xi, Hc, itab);
      const bool in_ang_part = rvk != 0xFFFFFFFFu;
      if (v.d2 < cut.rcR2) {
        shift_in4(gr, e);
        if ((++nR & 3) == 0) {
          *wr = gr;
          wr += n_slots;
        }
        if (v.d2 < cut.rcA2) {
          // within rc_angular now implies within rc_angular + skin at the
          // last build, so nA stays below capA and the reverse row exists
          if (rvk <= 0xFFFFu && nA < capA) {
            shift_in4(ga, e);
            shift_in4(gp, (uint32_t)ka | (rvk << 16));
            if ((++nA & 3) == 0) {
              *wa = ga;
              *wp = gp;
              wa += n_slots;
              wp += n_slots;
            }
            mword |= 1ull << (ka & 63);
          } else {
            bad = true;
          }
        }
        const float inv = rsqrt_hw(v.d2);
        const RadialF f = radial_f(v.d2 * inv * rcR_inv);
        float Tk[BR];
        cheb_t<BR>(f.x, Tk);
#pragma unroll
        for (int b = 0; b < T; ++b) {
          const float m = (T == 1 || v.zj == b) ? f.hf : 0.0f;
#pragma unroll
          for (int kk = 0; kk < BR; ++kk) PT[b][kk] = fmaf(m, Tk[kk], PT[b][kk]);
        }
      }
      if (in_ang_part && (++ka & 63) == 0) {
        *mw = mword;
        mw += n_slots;
        mword = 0;
      }
    }, reinterpret_cast<const uint4*>(vrev));
    // the last, partly filled mask word and groups
    if (ka & 63) *mw = mword;
    if (nR & 3) *wr = front4(gr, nR & 3);
    if (nA & 3) {
      *wa = front4(ga, nA & 3);
      *wp = front4(gp, nA & 3);
    }
    if (bad) atomicOr(&flags[kFlagAsym], 1);
  }
  if (in_range) {
    ccR[p] = nR;
    ccA[p] = nA;
  }

  float q[DP];
#pragma unroll
  for (int d = D; d < DP; ++d) q[d] = 0.f;
  // descriptor d: kept for the fused network, else stored at once for k_net
  // (so that no register holds it through the angular passes)
  auto put_q = [&](int d, float v) {
    if constexpr (NET) {
      q[d] = v;
    } else if (active) {
      if (d < NR)
        aR[((int64_t)(d / BR) * n_slots + p) * BR + d % BR] = v;
      else
        fp[(int64_t)(d - NR) * n_slots + p] = v;
    }
  };
  // ---- radial descriptors, Eq. 11: q_n = sum_b sum_k ctil[Z_i][b][n][k] PT_b[k]
  {
    const float* cR = dco + (int64_t)Zs * (T * NR * BR);
#pragma unroll
    for (int nn = 0; nn < NR; ++nn) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) acc = fmaf(cR[(b * NR + nn) * BR + kk], PT[b][kk], acc);
      put_q(nn, acc);
    }
  }

  // ---- angular descriptors, Eq. 16-17, in NSPLIT groups of n
#pragma unroll
  for (int h = 0; h < NSPLIT; ++h) {
    float Sg[NH][K];
    angular_sums<S, NH>(pos4, cnA, n_slots, p, nA, xi, Hc, itab, cA_s + (Zs * T * NA + h * NH) * BA, rcA_inv, Sg);
    // invariants of this group
#pragma unroll
    for (int nn = 0; nn < NH; ++nn) {
      const int n = h * NH + nn;
      float s1 = 0.f;
#pragma unroll
      for (int l = 1; l <= L; ++l) {
        float s = 0.f;
#pragma unroll
        for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) s = fmaf(Sg[nn][lm], Sg[nn][lm], s);
        put_q(NR + (l - 1) * NA + n, s);
        if (l == 1) s1 = s;
      }
      if constexpr (S::F4) {
        float A[6];
        a_from_s2(&Sg[nn][3], A);
        put_q(S::OFF4 + n, tr_cube(A));
      }
      if constexpr (S::F5) put_q(S::OFF5 + n, s1 * s1);
    }
  }

  if constexpr (NET) network<S>(q, Zs, active, n_slots, p, orig, params, W0s, W0Ts, fp, aR, Ei, qout, Eproc, want_adjoint);
  (void)H;
}

// ------------------------------------------------------------------- k_net

// The network for descriptors left by the unfused k_desc, as dense products
// on the 16x16x4 fp32 matrix instructions.  A wavefront's 64 atoms are the
// columns (four tiles of 16).  Forward, a[h][atom] = b0_h + sum_d W0[h][d]
// q[d][atom]: rows are hidden units, the reduction runs over descriptors.
// Backward, dE/dq[d][atom] = sum_h W0[h][d] z[h][atom] with
// z_h = w1_h (1 - tanh^2 a_h): rows are descriptors, the reduction runs over
// hidden units, and z is consumed in the register layout the forward product
// left it in (lane group g of a tile holds rows 4g..4g+3, so the reduction
// index h = 16 m + 4 g + r is taken in that order, for A and B alike).
// Operand layouts of v_mfma_f32_16x16x4f32: lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16], and D[4 (l / 16) + r][l % 16] in its r-th register.
// First-layer weights sit in LDS once, [h][d] with a row stride of 68 floats
// (4 mod 64), which keeps both read patterns free of bank conflicts.  Each
// wavefront reads the descriptors of its own 64 atoms and overwrites them
// with the adjoints only after its products are done.
template <class S>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_net(int64_t n_slots, const float4* __restrict__ pos4,
                                                const int* __restrict__ cfg_of, const int* __restrict__ orig,
                                                const float* __restrict__ params, float* __restrict__ fp,
                                                float* __restrict__ aR, float* __restrict__ Ei,
                                                float* __restrict__ qout, float* __restrict__ Eproc,
                                                int want_adjoint) {
  constexpr int T = S::T, NR = S::NR, BR = S::BR, D = S::D, H = S::H;
  constexpr int MT = (H + 15) / 16;   // tiles of hidden units
  constexpr int KS = (D + 3) / 4;     // reduction steps of the forward product
  constexpr int MD = (D + 15) / 16;   // tiles of descriptors
  constexpr int HR = 16 * MT;         // rows of the weight table (zero beyond H)
  constexpr int WSR = ((16 * MD > 4 * KS ? 16 * MD : 4 * KS) + 63) / 64 * 64 + 4;  // row stride
  static_assert(NR <= T * BR, "the radial descriptors must fit the radial adjoint rows");
  static_assert(NR <= 16, "the radial adjoints come from the first descriptor tile");
  static_assert(BR % 4 == 0, "adjoint rows are written as float4");
  __shared__ float W0s[T * HR * WSR];
  __shared__ float b0s[T * HR];
  __shared__ float w1s[T * HR];
  __shared__ float fr_s[kBlock / kWave][NR][kWave + 1];  // radial dE/dq, transposed to one atom per lane
  // The grid is at most two blocks per compute unit, each looping over tiles
  // of kBlock slots: the weights of every species enter LDS once per block.
  for (int t = threadIdx.x; t < T * HR * WSR; t += kBlock) {
    const int z = t / (HR * WSR), h = (t / WSR) % HR, d = t % WSR;
    W0s[t] = (h < H && d < D) ? params[S::PCR + S::PCA + (int64_t)z * S::PMLP + h * D + d] : 0.0f;
  }
  for (int t = threadIdx.x; t < T * HR; t += kBlock) {
    const int z = t / HR, h = t % HR;
    const float* b0g = params + S::PCR + S::PCA + (int64_t)z * S::PMLP + H * D;
    b0s[t] = h < H ? b0g[h] : 0.0f;
    w1s[t] = h < H ? b0g[H + h] : 0.0f;
  }
  const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, c = lane & 15, wv = threadIdx.x / kWave;
  const int64_t n_tiles = (n_slots + kBlock - 1) / kBlock;
#pragma unroll 1
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    __syncthreads();  // weights loaded; the previous tile's transposition read
    // the slot count as an opaque per-tile value: otherwise the compiler keeps
    // every row offset (d - n_R) n_slots live across the loop in registers
    int64_t ns = n_slots;
    __asm__ volatile("" : "+s"(ns));
    const int64_t p = tile * kBlock + threadIdx.x;
    const int64_t base = p - lane;
    const bool in_range = p < ns;
    const int64_t pc = in_range ? p : ns - 1;
    const int Zs = __builtin_amdgcn_readfirstlane(__float_as_int(pos4[pc].w));
    const bool active = in_range && cfg_of[p] >= 0;
    auto q_at = [&](int d, int64_t a) {
      return d < NR ? aR[((int64_t)(d / BR) * ns + a) * BR + d % BR] : fp[(int64_t)(d - NR) * ns + a];
    };
    if (active && qout) {
      const int i = orig[p];
#pragma unroll
      for (int d = 0; d < D; ++d) qout[(int64_t)i * D + d] = q_at(d, p);
    }
    // B operands of the forward product: q[4 ks + g][atom 16 nt + c] (zero
    // past the last descriptor; columns past the last slot read the last slot)
    float qb[KS][4];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int d = 4 * ks + g;
        const int64_t a = base + 16 * nt + c;
        qb[ks][nt] = d < D ? q_at(d, a < ns ? a : ns - 1) : 0.0f;
      }
    const float* Wz = W0s + Zs * HR * WSR;
    floatx4 C[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float bb = b0s[Zs * HR + 16 * mt + 4 * g + r];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) C[mt][nt][r] = bb;
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const float a = Wz[(16 * mt + c) * WSR + 4 * ks + g];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
          C[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, qb[ks][nt], C[mt][nt], 0, 0, 0);
      }
    //  E = b1 + sum_h w1_h tanh(a_h): per lane over its rows, then over the
    //  four lane groups of each column; z_h = w1_h (1 - tanh^2) replaces a_h
    float Ep[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float w = w1s[Zs * HR + 16 * mt + 4 * g + r];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const float t = tanh_fast(C[mt][nt][r]);
          Ep[nt] = fmaf(w, t, Ep[nt]);
          C[mt][nt][r] = w * fmaf(-t, t, 1.0f);
        }
      }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      Ep[nt] += __shfl_xor(Ep[nt], 16);
      Ep[nt] += __shfl_xor(Ep[nt], 32);
    }
    // lane 16 g + c is atom 16 g + c of the wavefront: column c of tile g
    const float Es = g == 0 ? Ep[0] : (g == 1 ? Ep[1] : (g == 2 ? Ep[2] : Ep[3]));
    const float E = params[S::PCR + S::PCA + (int64_t)Zs * S::PMLP + H * D + 2 * H] + Es;
    if (active) {
      const int i = orig[p];
      Ei[i] = E;
      if (Eproc) Eproc[p] = E;
    }
    if (!want_adjoint) continue;
    floatx4 C2[MD][4];
#pragma unroll
    for (int md = 0; md < MD; ++md)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) C2[md][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int md = 0; md < MD; ++md) {
          const float a = Wz[(16 * mt + 4 * g + r) * WSR + 16 * md + c];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt)
            C2[md][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, C[mt][nt][r], C2[md][nt], 0, 0, 0);
        }
    // dE/dq of the angular descriptors straight from the product's layout (16
    // consecutive atoms per lane group); the radial ones through LDS
#pragma unroll
    for (int md = 0; md < MD; ++md)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int d = 16 * md + 4 * g + r;
          const int64_t a = base + 16 * nt + c;
          if (d < NR)
            fr_s[wv][d][16 * nt + c] = C2[md][nt][r];
          else if (d < D && a < ns)
            fp[(int64_t)(d - NR) * ns + a] = C2[md][nt][r];
        }
    __syncthreads();
    if (active) {
      float Fr[NR];
#pragma unroll
      for (int nn = 0; nn < NR; ++nn) Fr[nn] = fr_s[wv][nn][lane];
      // radial adjoint atil[b][k] = sum_n dE/dq_n ctil[Z_i][b][n][k]
      const float* cR = params + S::P + (int64_t)Zs * (T * NR * BR);
#pragma unroll
      for (int b = 0; b < T; ++b) {
        float4* row = reinterpret_cast<float4*>(aR + ((int64_t)b * ns + p) * BR);
#pragma unroll
        for (int k4 = 0; k4 < BR / 4; ++k4) {
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float acc = 0.f;
#pragma unroll
            for (int nn = 0; nn < NR; ++nn) acc = fmaf(Fr[nn], cR[(b * NR + nn) * BR + 4 * k4 + u], acc);
            v[u] = acc;
          }
          row[k4] = make_float4(v[0], v[1], v[2], v[3]);
        }
      }
    }
  }
}

// ----------------------------------------------------------------- k_force

// Row stride (floats) of the per-thread radial adjoint rows in LDS: a multiple
// of 4 with an odd quotient, so that 128-bit reads of consecutive lanes fall
// on distinct banks.
template <int W>
constexpr int lds_row() {
  return ((W + 3) / 4) % 2 ? ((W + 3) / 4) * 4 : ((W + 3) / 4 + 1) * 4;
}

template <class S, int NSPLIT, int WPE, int BS = kBlock>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(WPE))) void k_force(
    int64_t n_slots, const float4* __restrict__ pos4, const int* __restrict__ cfg_of,
    const int* __restrict__ orig, const CfgDev* __restrict__ cfgs, const uint32_t* __restrict__ cnR,
    const int* __restrict__ ccR, const uint32_t* __restrict__ cnA, const int* __restrict__ ccA, Cutoffs cut, const float* __restrict__ params, const float* __restrict__ fp,
    const float* aR, float4* __restrict__ frad, float4* __restrict__ fA, float* __restrict__ Wi) {
  // aR is not declared restrict: loads through a restrict read-only pointer may
  // be sunk past the pair walker's barrier, into the pair body after the
  // prefetches, where waiting for them would drain the prefetch ring
  constexpr int T = S::T, NR = S::NR, NA = S::NA, BR = S::BR, BA = S::BA, L = S::L, K = S::K;
  constexpr int NH = NA / NSPLIT;
  constexpr int RW = lds_row<T * BR>();
  const float* __restrict__ dco = params + S::P;
  __shared__ float cA_s[T * T * NA * BA];
  __shared__ float aown_s[T > 1 ? BS * RW : 1];
  __shared__ ImageTable itab;
  for (int t = threadIdx.x; t < T * T * NA * BA; t += BS) cA_s[t] = dco[S::PCR + t];
  itab.fill();
  __syncthreads();

  const int64_t p = xcd_tile() * BS + threadIdx.x;
  if (p >= n_slots) return;
  const float4 xi = pos4[p];
  const int Zs = __builtin_amdgcn_readfirstlane(__float_as_int(xi.w));
  const int c = cfg_of[p];
  if (c < 0) return;
  float Hc[9];
  load_cell(cfgs, c, Hc);
  const float rcR_inv = 1.0f / cut.rcR, rcA_inv = 1.0f / cut.rcA;

  float Fx = 0.f, Fy = 0.f, Fz = 0.f;
  // radial virial is symmetric (f_ij parallel to r_ij): xx, yy, zz, xy, xz, yz
  float Wr[6];
#pragma unroll
  for (int x = 0; x < 6; ++x) Wr[x] = 0.f;

  // ---- radial pairs: f_ij - f_ji = (s_own + s_rev) u_ij with
  //      s = dE/dd = dxhf sum_k atil_k T'_k + dfc2 sum_k atil_k T_k
  {
    float a1[T == 1 ? BR : 1];
    float* mine = aown_s + (T > 1 ? threadIdx.x * RW : 0);
    if constexpr (T == 1) {
#pragma unroll
      for (int kk = 0; kk < BR; ++kk) a1[kk] = aR[p * BR + kk];
    } else {
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) mine[b * BR + kk] = aR[((int64_t)b * n_slots + p) * BR + kk];
    }
    const int n = ccR[p];
    // the neighbour's adjoint row atil_j[Z_i] (part Z_i of the adjoint, stored
    // part-major so that a wavefront reads one compact array), loaded ahead of
    // the ring's prefetches
    static_assert(BR % 4 == 0, "adjoint rows are read as float4");
    const float4* aRz = reinterpret_cast<const float4*>(aR + (int64_t)Zs * n_slots * BR);
    auto row = [&](int, uint32_t e) {
      AdjRow<BR> r;
      const float4* src = aRz + (int64_t)(e & kNbrMask) * (BR / 4);
#pragma unroll
      for (int c = 0; c < BR / 4; ++c) r.v[c] = src[c];
      return r;
    };
    walk_groups(reinterpret_cast<const uint4*>(cnR), n_slots, p, n, pos4, row,
                [&](int, uint32_t e, float4 xq, uint32_t, const AdjRow<BR>& arow) {
      const PairVec v = pair_vec(e, xq, xi, Hc, itab);
      const float* ar = reinterpret_cast<const float*>(arow.v);
      const float inv = rsqrt_hw(v.d2);
      const RadialFD f = radial_fd(v.d2 * inv * rcR_inv, rcR_inv);
      float Tk[BR], Dk[BR];
      cheb_tt<BR>(f.x, Tk, Dk);
      float ao[BR];
      if constexpr (T == 1) {
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) ao[kk] = a1[kk];
      } else {
        const float* src = mine + v.zj * BR;
#pragma unroll
        for (int kk = 0; kk < BR; ++kk) ao[kk] = src[kk];
      }
      float to = ao[0], dn = 0.f, tr = ar[0], dr = 0.f;
#pragma unroll
      for (int kk = 1; kk < BR; ++kk) {
        to = fmaf(ao[kk], Tk[kk], to);
        dn = fmaf(ao[kk], Dk[kk], dn);
        tr = fmaf(ar[kk], Tk[kk], tr);
        dr = fmaf(ar[kk], Dk[kk], dr);
      }
      const float s_own = fmaf(f.dxhf, dn, f.dfc2 * to);
      const float s_rev = fmaf(f.dxhf, dr, f.dfc2 * tr);
      const float st = (s_own + s_rev) * inv;
      Fx = fmaf(st, v.rx, Fx);
      Fy = fmaf(st, v.ry, Fy);
      Fz = fmaf(st, v.rz, Fz);
      const float so = s_own * inv;
      const float ax = so * v.rx, ay = so * v.ry, az = so * v.rz;
      Wr[0] = fmaf(-ax, v.rx, Wr[0]);
      Wr[1] = fmaf(-ay, v.ry, Wr[1]);
      Wr[2] = fmaf(-az, v.rz, Wr[2]);
      Wr[3] = fmaf(-ax, v.ry, Wr[3]);
      Wr[4] = fmaf(-ax, v.rz, Wr[4]);
      Wr[5] = fmaf(-ay, v.rz, Wr[5]);
    });
  }

  // ---- angular pairs, in NSPLIT groups of n (the virial continues from the
  //      radial part, rows xx xy xz / yx yy yz / zx zy zz)
  float W[9] = {Wr[0], Wr[3], Wr[4], Wr[3], Wr[1], Wr[5], Wr[4], Wr[5], Wr[2]};
  const int nA = ccA[p];
  constexpr Kappa<L> kap;
#pragma unroll
  for (int h = 0; h < NSPLIT; ++h) {
    const float* cl0 = cA_s + (Zs * T * NA + h * NH) * BA;
    // recompute S for this group
    float Sg[NH][K];
    angular_sums<S, NH>(pos4, cnA, n_slots, p, nA, xi, Hc, itab, cl0, rcA_inv, Sg);
    // sigma = dE_i/dS for this group (in place), then scaled by kappa so that
    // the pair loop works with the unnormalised polynomials
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
#pragma unroll
      for (int lm = 0; lm < K; ++lm) Sg[nn][lm] *= kap.v[lm];
    }
    // pair forces of this group: f = u sum_n g'_n Z_n + (I - u u^T) v / d,
    // Z_n = sum_lm sigma_nlm P_lm, v = sum_lm G_lm grad P_lm, G_lm = sum_n sigma_nlm g_n
    float4* own = fA + p;  // i's compact slot k of the pair-force buffer
    // the earlier groups' sum for slot k, loaded ahead of the ring's
    // prefetches (row clamped at the last pair)
    const float4* own_ld = fA + p;
    auto prev = [&](int k, uint32_t) {
      float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
      if (h > 0) {
        o = *own_ld;
        if (k + 1 < nA) own_ld += n_slots;
      }
      return o;
    };
    walk_groups(reinterpret_cast<const uint4*>(cnA), n_slots, p, nA, pos4, prev,
                [&](int, uint32_t e, float4 xq, uint32_t, float4 o) {
      const PairVec v = pair_vec(e, xq, xi, Hc, itab);
      const float inv = rsqrt_hw(v.d2);
      const float ux = v.rx * inv, uy = v.ry * inv, uz = v.rz * inv;
      const RadialFD f = radial_fd(v.d2 * inv * rcA_inv, rcA_inv);
      // g_n and g'_n of this group first, so that T and T' die early
      float g[NH], gp[NH];
      {
        float Tk[BA], Dk[BA];
        cheb_tt<BA>(f.x, Tk, Dk);
        const float* cl = cl0 + v.zj * (NA * BA);
#pragma unroll
        for (int nn = 0; nn < NH; ++nn) {
          float ct = cl[nn * BA], cd = 0.f;
#pragma unroll
          for (int kk = 1; kk < BA; ++kk) {
            const float cc = cl[nn * BA + kk];
            ct = fmaf(cc, Tk[kk], ct);
            cd = fmaf(cc, Dk[kk], cd);
          }
          g[nn] = f.hf * ct;
          gp[nn] = fmaf(f.dxhf, cd, f.dfc2 * ct);
        }
      }
      float P[K];
      raw_sph<L>(ux, uy, uz, P);
      float G[K];
#pragma unroll
      for (int lm = 0; lm < K; ++lm) G[lm] = 0.f;
      float s = 0.f;
#pragma unroll
      for (int nn = 0; nn < NH; ++nn) {
        float zn = 0.f;
#pragma unroll
        for (int lm = 0; lm < K; ++lm) {
          zn = fmaf(Sg[nn][lm], P[lm], zn);
          G[lm] = fmaf(Sg[nn][lm], g[nn], G[lm]);
        }
        s = fmaf(gp[nn], zn, s);
      }
      float vx, vy, vz;
      raw_sph_grad_dot<L>(ux, uy, uz, G, vx, vy, vz);
      const float uv = fmaf(ux, vx, fmaf(uy, vy, uz * vz));
      const float fx = fmaf(s, ux, (vx - uv * ux) * inv);
      const float fy = fmaf(s, uy, (vy - uv * uy) * inv);
      const float fz = fmaf(s, uz, (vz - uv * uz) * inv);
      Fx += fx;
      Fy += fy;
      Fz += fz;
      W[0] = fmaf(-fx, v.rx, W[0]); W[1] = fmaf(-fx, v.ry, W[1]); W[2] = fmaf(-fx, v.rz, W[2]);
      W[3] = fmaf(-fy, v.rx, W[3]); W[4] = fmaf(-fy, v.ry, W[4]); W[5] = fmaf(-fy, v.rz, W[5]);
      W[6] = fmaf(-fz, v.rx, W[6]); W[7] = fmaf(-fz, v.ry, W[7]); W[8] = fmaf(-fz, v.rz, W[8]);
      // dE_i/dr_ij (summed over the groups) stays in i's own compact slot,
      // where j's gather finds it
      *own = h == 0 ? make_float4(fx, fy, fz, 0.f) : make_float4(o.x + fx, o.y + fy, o.z + fz, 0.f);
      own += n_slots;
    });
  }
  frad[p] = make_float4(Fx, Fy, Fz, 0.f);
  const int i = orig[p];
  float* w = Wi + (int64_t)i * 9;
#pragma unroll
  for (int x = 0; x < 9; ++x) w[x] = W[x];
}

// ---------------------------------------------------------------- k_gather

// F_i = (radial part + sum_j f_ij) - sum_j f_ji (Eq. 3).  The own part was
// summed by k_force.  f_ji = dE_j/dr_ji sits in j's compact angular slot of
// i, whose index is the number of entries of the angular part of j's Verlet
// list before i's that are in j's compact angular list: a popcount of j's
// entry mask below i's reverse position.
//
// Each pair needs three dependent loads: its entry and row pair (from the
// grouped compact lists, four pairs per load), j's mask word, then j's pair
// force.  Groups are processed in a two-stage pipeline: while the pair
// forces of group g are loaded, the mask words of group g + 1 are, and the
// entries of group g + 2.
struct GatherStage {
  uint4 e, r;      // entries and row pairs of four pairs
  uint64_t m[4];   // j's mask word holding i's entry, per pair
};

// Pair u of a group at list position k0 + u: positions past the end of the
// list (the unused part of the last group) take the group's first pair, a real
// one, so that every load they cause stays inside the lists of real pairs.
__device__ __forceinline__ int real_pair(int k0, int u, int n) { return k0 + u < n ? u : 0; }

__device__ __forceinline__ void gather_masks(GatherStage& st, const uint64_t* __restrict__ amask, int64_t ns, int k0,
                                             int n) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int v = real_pair(k0, u, n);
    const uint32_t j = comp4(st.e, v) & kNbrMask;
    const uint32_t rv = comp4(st.r, v) >> 16;
    st.m[u] = amask[(int64_t)(rv >> 6) * ns + j];
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_gather(int64_t n_slots, const int* __restrict__ orig,
                                                   const uint32_t* __restrict__ cnA, const uint32_t* __restrict__ cpA,
                                                   const int* __restrict__ ccA, const uint64_t* __restrict__ amask,
                                                   const float4* __restrict__ frad, const float4* __restrict__ fA,
                                                   float* __restrict__ Fuser, float4* __restrict__ Fproc) {
  const int64_t p = xcd_tile() * BS + threadIdx.x;
  if (p >= n_slots) return;
  const int i = orig[p];
  if (i < 0) {
    if (Fproc) Fproc[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float4 F = frad[p];
  const int n = ccA[p];
  if (n > 0) {
    const int ng = list_groups(n);
    const uint4* ge = reinterpret_cast<const uint4*>(cnA) + p;
    const uint4* gr = reinterpret_cast<const uint4*>(cpA) + p;
    // groups past the last are clamped to it: their loads stay in bounds and
    // their pairs are skipped
    auto load_group = [&](GatherStage& st, int g) {
      const int64_t o = (int64_t)(g < ng ? g : ng - 1) * n_slots;
      st.e = ge[o];
      st.r = gr[o];
    };
    // one step: the pair forces of group g (stage cur, mask words loaded one
    // step earlier), the entries of group g + 2 (into stage nn) and the mask
    // words of group g + 1 (stage nxt); the loop is unrolled by three so that
    // the stages keep their registers
    auto step = [&](GatherStage& cur, GatherStage& nxt, GatherStage& nn, int g) {
      float4 fv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int v = real_pair(4 * g, u, n);
        const uint32_t rv = comp4(cur.r, v) >> 16;
        const int64_t j = comp4(cur.e, v) & kNbrMask;
        int jc = __popcll(cur.m[u] & ((1ull << (rv & 63)) - 1ull));
        for (uint32_t w = 0; w < (rv >> 6); ++w) jc += __popcll(amask[(int64_t)w * n_slots + j]);
        fv[u] = fA[(int64_t)jc * n_slots + j];
      }
      load_group(nn, g + 2);
      gather_masks(nxt, amask, n_slots, 4 * (g + 1 < ng ? g + 1 : ng - 1), n);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (4 * g + u < n) {
          F.x -= fv[u].x;
          F.y -= fv[u].y;
          F.z -= fv[u].z;
        }
      }
    };
    GatherStage sa, sb, sc;
    load_group(sa, 0);
    load_group(sb, 1);
    gather_masks(sa, amask, n_slots, 0, n);
    for (int g = 0; g < ng; g += 3) {
      step(sa, sb, sc, g);
      step(sb, sc, sa, g + 1);
      step(sc, sa, sb, g + 2);
    }
  }
  if (Fuser) {
    Fuser[(int64_t)i * 3 + 0] = F.x;
    Fuser[(int64_t)i * 3 + 1] = F.y;
    Fuser[(int64_t)i * 3 + 2] = F.z;
  }
  if (Fproc) Fproc[p] = F;
}

// Derived coefficient table: ctil[..][n][0] = c[..][n][0] + sum_k c[..][n][k],
// ctil[..][n][k] = c[..][n][k] for k >= 1, for every radial row (length BR)
// and angular row (length BA).  With Q_k = hf (T_k + 1) this gives
// sum_k c_nk Q_k = hf sum_k ctil_nk T_k.
template <class S>
__global__ void k_derive(const float* __restrict__ params, float* __restrict__ out) {
  constexpr int rowsR = S::T * S::T * S::NR, rowsA = S::T * S::T * S::NA;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rowsR + rowsA) return;
  const int B = r < rowsR ? S::BR : S::BA;
  const int64_t o = r < rowsR ? (int64_t)r * S::BR : S::PCR + (int64_t)(r - rowsR) * S::BA;
  double sum = 0.0;
  for (int k = 0; k < B; ++k) sum += (double)params[o + k];
  out[o] = (float)((double)params[o] + sum);
  for (int k = 1; k < B; ++k) out[o + k] = params[o + k];
}

// ------------------------------------------------------------- launchers

// Kernel variants: (passes over the angular pairs, each for n_A / passes of the
// angular functions; waves per SIMD the register allocation must allow; for
// the descriptors, network in k_desc or in k_net; block size, 256 threads
// unless stated).  Every variant computes
// the same result: descriptors are bitwise identical across descriptor
// variants, site energies within each network form (the two forms sum the
// network in different orders); force variants differ only in the order the
// per-group pair forces are added.
// Blocks of k_net: two per compute unit (its LDS holds two).
constexpr unsigned kNetBlocks = 2 * 256;

template <class S, int NS>
constexpr int groups() {
  return NS <= S::NA ? NS : S::NA;
}

template <class S, int NS, int W, bool NET, int BS = kBlock>
static int launch_desc(hipStream_t st, const NepIO& io, const float* params, bool want_adjoint) {
  const unsigned g = (unsigned)((io.n_slots + BS - 1) / BS);
  hipLaunchKernelGGL((k_desc<S, groups<S, NS>(), W, NET, BS>), dim3(g), dim3(BS), 0, st, io.n_slots, io.capA,
                     io.pos4, io.cfg_of, io.orig, io.cfgs, io.nbrR, io.cntR, io.vrev, io.cnR, io.ccR, io.cnA, io.cpA,
                     io.ccA, io.amask, io.flags, io.cut, params, io.fp, io.aR, io.Ei, io.qout, io.Eproc,
                     want_adjoint ? 1 : 0);
  if constexpr (!NET) {
    const unsigned gk = (unsigned)((io.n_slots + kBlock - 1) / kBlock);
    const unsigned gn = gk < kNetBlocks ? gk : kNetBlocks;
    hipLaunchKernelGGL(k_net<S>, dim3(gn), dim3(kBlock), 0, st, io.n_slots, io.pos4, io.cfg_of, io.orig, params,
                       io.fp, io.aR, io.Ei, io.qout, io.Eproc, want_adjoint ? 1 : 0);
  }
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S, int NS, int W, int BS = kBlock>
static int launch_force(hipStream_t st, const NepIO& io, const float* params) {
  const unsigned g = (unsigned)((io.n_slots + BS - 1) / BS);
  hipLaunchKernelGGL((k_force<S, groups<S, NS>(), W, BS>), dim3(g), dim3(BS), 0, st, io.n_slots, io.pos4,
                     io.cfg_of, io.orig, io.cfgs, io.cnR, io.ccR, io.cnA, io.ccA, io.cut, params, io.fp, io.aR,
                     io.frad, io.fA, io.Wi);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S>
int Launch<S>::desc(hipStream_t st, const NepIO& io, const float* params, bool want_adjoint, int variant) {
  switch (variant) {
    case 1: return launch_desc<S, 4, 3, true>(st, io, params, want_adjoint);
    case 2: return launch_desc<S, 4, 2, true>(st, io, params, want_adjoint);
    case 3: return launch_desc<S, 1, 1, true>(st, io, params, want_adjoint);
    case 4: return launch_desc<S, 4, 4, false>(st, io, params, want_adjoint);
    case 5: return launch_desc<S, 1, 2, false>(st, io, params, want_adjoint);
    case 6: return launch_desc<S, 2, 2, false>(st, io, params, want_adjoint);
    case 7: return launch_desc<S, 2, 3, false>(st, io, params, want_adjoint);
    case 8: return launch_desc<S, 2, 2, true, 128>(st, io, params, want_adjoint);
    case 9: return launch_desc<S, 2, 2, true, 512>(st, io, params, want_adjoint);
    default: return launch_desc<S, 2, 2, true>(st, io, params, want_adjoint);
  }
}

template <class S>
int Launch<S>::force(hipStream_t st, const NepIO& io, const float* params, int variant) {
  switch (variant) {
    case 1: return launch_force<S, 4, 2>(st, io, params);
    case 2: return launch_force<S, 4, 3>(st, io, params);
    case 3: return launch_force<S, 1, 1>(st, io, params);
    case 4: return launch_force<S, 2, 2, 128>(st, io, params);
    case 5: return launch_force<S, 2, 2, 512>(st, io, params);
    default: return launch_force<S, 2, 2>(st, io, params);
  }
}

template <int BS>
static int launch_gather(hipStream_t st, const NepIO& io) {
  const unsigned g = (unsigned)((io.n_slots + BS - 1) / BS);
  hipLaunchKernelGGL(k_gather<BS>, dim3(g), dim3(BS), 0, st, io.n_slots, io.orig, io.cnA, io.cpA, io.ccA, io.amask,
                     io.frad, io.fA, io.Fuser, io.Fproc);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template <class S>
int Launch<S>::gather(hipStream_t st, const NepIO& io, int variant) {
  switch (variant) {
    case 1: return launch_gather<128>(st, io);
    case 2: return launch_gather<512>(st, io);
    case 3: return launch_gather<1024>(st, io);
    default: return launch_gather<256>(st, io);
  }
}

template <class S>
int Launch<S>::derive(hipStream_t st, float* params) {
  constexpr int rows = S::T * S::T * (S::NR + S::NA);
  hipLaunchKernelGGL(k_derive<S>, dim3((rows + 127) / 128), dim3(128), 0, st, params, params + S::P);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

template struct Launch<ShapeSmall>;
template struct Launch<ShapeGST>;
template struct Launch<ShapeTable2>;

}  // namespace nepmi
