// reduce.hip -- float64 per-configuration sums of per-atom values.
//
// E_c = sum_i E_i (Eq. 1) and V_c = sum_i W_i (Eq. 4), plus optional
// kinetic energies, are summed in float64 in a fixed order: every
// configuration's caller-order atom range is cut into chunks, one block sums
// a chunk in a fixed shape (wavefront butterflies, then the wavefronts in
// order), and one block per configuration sums its chunk sums the same way.
// Results are bitwise reproducible run to run.
#include "reduce.hpp"

namespace nepmi {

constexpr int kRedBlock = 256;       // threads of a block of the final pass
constexpr int kRedChunkBlock = 256;  // threads of a block of the first pass (1024 measured slower)

// Sum of the block's acc[v] into thread v (v < NV), in a fixed shape: a
// butterfly over the 64 lanes of each wavefront, then the wavefront sums in
// order.
template <int BS>
__device__ __forceinline__ void block_sum(double (&acc)[kRedValues], double (&sh)[BS / 64][kRedValues]) {
  constexpr int NV = kRedValues;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += __shfl_xor(acc[v], o, 64);
  const int w = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) sh[w][v] = acc[v];
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double t = sh[0][threadIdx.x];
#pragma unroll
    for (int u = 1; u < BS / 64; ++u) t += sh[u][threadIdx.x];
    acc[0] = t;
  }
}

template <class T>
__global__ __launch_bounds__(kRedChunkBlock) void k_reduce_chunks(const RedItem* __restrict__ items,
                                                             const T* __restrict__ Ei,
                                                             const T* __restrict__ Wi,
                                                             const T* __restrict__ Ki,
                                                             double* __restrict__ part) {
  constexpr int NV = kRedValues;
  __shared__ double sh[kRedChunkBlock / 64][NV];
  const RedItem it = items[blockIdx.x];
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int64_t a = it.a0 + threadIdx.x; a < it.a1; a += kRedChunkBlock) {
    if (Ei) acc[0] += (double)Ei[a];
    if (Wi) {
#pragma unroll
      for (int x = 0; x < 9; ++x) acc[1 + x] += (double)Wi[a * 9 + x];
    }
    if (Ki) acc[10] += (double)Ki[a];
  }
  block_sum<kRedChunkBlock>(acc, sh);
  if (threadIdx.x < NV) part[(int64_t)blockIdx.x * NV + threadIdx.x] = acc[0];
}

// One block per configuration: its chunk sums in a fixed assignment to
// threads, then the same fixed-shape sum.
__global__ __launch_bounds__(kRedBlock) void k_reduce_final(int n_cfg, const int* __restrict__ item_start,
                                                            const double* __restrict__ part, double* __restrict__ E,
                                                            double* __restrict__ V, double* __restrict__ Kout) {
  constexpr int NV = kRedValues;
  __shared__ double sh[kRedBlock / 64][NV];
  const int c = blockIdx.x;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int w = item_start[c] + (int)threadIdx.x; w < item_start[c + 1]; w += kRedBlock)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += part[(int64_t)w * NV + v];
  block_sum<kRedBlock>(acc, sh);
  const int v = (int)threadIdx.x;
  if (v == 0 && E) E[c] = acc[0];
  if (v >= 1 && v <= 9 && V) V[(int64_t)c * 9 + v - 1] = acc[0];
  if (v == 10 && Kout) Kout[c] = acc[0];
}

int Reducer::setup(int n_cfg_, const int64_t* atom_off, hipStream_t st) {
  std::vector<RedItem>& items = host_items;
  std::vector<int>& start = host_start;
  items.clear();
  start.assign((size_t)n_cfg_ + 1, 0);
  for (int c = 0; c < n_cfg_; ++c) {
    start[(size_t)c] = (int)items.size();
    int64_t a = atom_off[c];
    const int64_t b = atom_off[c + 1];
    do {
      RedItem it;
      it.cfg = c;
      it.a0 = a;
      it.a1 = (b - a > kRedChunk) ? a + kRedChunk : b;
      items.push_back(it);
      a = it.a1;
    } while (a < b);
  }
  start[(size_t)n_cfg_] = (int)items.size();
  n_cfg = n_cfg_;
  n_items = (int)items.size();
  int rc;
  if ((rc = items_dev.ensure(sizeof(RedItem) * items.size())) || (rc = start_dev.ensure(4 * start.size())) ||
      (rc = part.ensure(sizeof(double) * kRedValues * items.size())))
    return rc;
  NEPMI_HIP(hipMemcpyAsync(items_dev.p, items.data(), sizeof(RedItem) * items.size(), hipMemcpyHostToDevice, st));
  NEPMI_HIP(hipMemcpyAsync(start_dev.p, start.data(), 4 * start.size(), hipMemcpyHostToDevice, st));
  return NEPMI_OK;
}

int Reducer::run(hipStream_t st, const float* Ei, const float* Wi, const float* Ki, double* E, double* V,
                 double* Kout) {
  hipLaunchKernelGGL(k_reduce_chunks<float>, dim3(n_items), dim3(kRedChunkBlock), 0, st, items_dev.ptr<RedItem>(), Ei, Wi,
                     Ki, part.ptr<double>());
  hipLaunchKernelGGL(k_reduce_final, dim3(n_cfg), dim3(kRedBlock), 0, st, n_cfg, start_dev.ptr<int>(),
                     part.ptr<double>(), E, V, Kout);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int Reducer::run64(hipStream_t st, const double* Ei, const double* Wi, double* E, double* V) {
  hipLaunchKernelGGL(k_reduce_chunks<double>, dim3(n_items), dim3(kRedChunkBlock), 0, st, items_dev.ptr<RedItem>(), Ei,
                     Wi, static_cast<const double*>(nullptr), part.ptr<double>());
  hipLaunchKernelGGL(k_reduce_final, dim3(n_cfg), dim3(kRedBlock), 0, st, n_cfg, start_dev.ptr<int>(),
                     part.ptr<double>(), E, V, static_cast<double*>(nullptr));
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

}  // namespace nepmi
