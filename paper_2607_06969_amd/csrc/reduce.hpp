// reduce.hpp -- deterministic float64 per-configuration reductions.
#pragma once

#include <vector>

#include "nbr.hpp"

namespace nepmi {

constexpr int kRedValues = 11;    // energy, 9 virial components, kinetic energy
constexpr int64_t kRedChunk = 2048;  // atoms per block of the first pass

struct RedItem {
  int cfg;
  int pad;
  int64_t a0, a1;  // caller-order atom range
};

struct Reducer {
  int n_cfg = 0, n_items = 0;
  DevBuf items_dev, start_dev, part;
  // host copies of the plan, the sources of setup's asynchronous uploads:
  // they stay alive until the next setup, and the caller synchronises the
  // stream before that
  std::vector<RedItem> host_items;
  std::vector<int> host_start;
  // Plan the sums of a batch and upload it on `st` (does not synchronise).
  int setup(int n_cfg, const int64_t* atom_off, hipStream_t st);
  void use_arena(Arena* a) {
    for (DevBuf* b : {&items_dev, &start_dev, &part}) {
      b->release();
      b->arena = a;
    }
  }
  // Any input or output may be null.
  int run(hipStream_t st, const float* Ei, const float* Wi, const float* Ki, double* E, double* V, double* Kout);
  // The same sums of float64 per-atom energies and virials.
  int run64(hipStream_t st, const double* Ei, const double* Wi, double* E, double* V);
};

}  // namespace nepmi
