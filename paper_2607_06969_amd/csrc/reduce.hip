// reduce.hip -- float64 per-configuration sums of per-atom values.
//
// E_c = sum_i E_i (Eq. 1) and V_c = sum_i W_i (Eq. 4), plus optional
// kinetic energies, are summed in float64 in a fixed order: every
// configuration's caller-order atom range is cut into chunks, one block sums
// a chunk with a fixed-shape tree, and one block per configuration sums its
// chunk sums the same way.  Results are bitwise reproducible run to run.
#include "reduce.hpp"

namespace nepmi {

constexpr int kRedBlock = 256;

template <class T>
__global__ __launch_bounds__(kRedBlock) void k_reduce_chunks(const RedItem* __restrict__ items,
                                                             const T* __restrict__ Ei,
                                                             const T* __restrict__ Wi,
                                                             const T* __restrict__ Ki,
                                                             double* __restrict__ part) {
  constexpr int NV = kRedValues;
  __shared__ double sh[NV][kRedBlock];
  const RedItem it = items[blockIdx.x];
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int64_t a = it.a0 + threadIdx.x; a < it.a1; a += kRedBlock) {
    if (Ei) acc[0] += (double)Ei[a];
    if (Wi) {
#pragma unroll
      for (int x = 0; x < 9; ++x) acc[1 + x] += (double)Wi[a * 9 + x];
    }
    if (Ki) acc[10] += (double)Ki[a];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < NV) part[(int64_t)blockIdx.x * NV + threadIdx.x] = sh[threadIdx.x][0];
}

// One block per configuration: its chunk sums in a fixed assignment to
// threads, then the same fixed-shape tree.
__global__ __launch_bounds__(kRedBlock) void k_reduce_final(int n_cfg, const int* __restrict__ item_start,
                                                            const double* __restrict__ part, double* __restrict__ E,
                                                            double* __restrict__ V, double* __restrict__ Kout) {
  constexpr int NV = kRedValues;
  __shared__ double sh[NV][kRedBlock];
  const int c = blockIdx.x;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int w = item_start[c] + (int)threadIdx.x; w < item_start[c + 1]; w += kRedBlock)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += part[(int64_t)w * NV + v];
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (E) E[c] = sh[0][0];
    if (V)
      for (int x = 0; x < 9; ++x) V[(int64_t)c * 9 + x] = sh[1 + x][0];
    if (Kout) Kout[c] = sh[10][0];
  }
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
  hipLaunchKernelGGL(k_reduce_chunks<float>, dim3(n_items), dim3(kRedBlock), 0, st, items_dev.ptr<RedItem>(), Ei, Wi,
                     Ki, part.ptr<double>());
  hipLaunchKernelGGL(k_reduce_final, dim3(n_cfg), dim3(kRedBlock), 0, st, n_cfg, start_dev.ptr<int>(),
                     part.ptr<double>(), E, V, Kout);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int Reducer::run64(hipStream_t st, const double* Ei, const double* Wi, double* E, double* V) {
  hipLaunchKernelGGL(k_reduce_chunks<double>, dim3(n_items), dim3(kRedBlock), 0, st, items_dev.ptr<RedItem>(), Ei,
                     Wi, static_cast<const double*>(nullptr), part.ptr<double>());
  hipLaunchKernelGGL(k_reduce_final, dim3(n_cfg), dim3(kRedBlock), 0, st, n_cfg, start_dev.ptr<int>(),
                     part.ptr<double>(), E, V, static_cast<double*>(nullptr));
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

}  // namespace nepmi
