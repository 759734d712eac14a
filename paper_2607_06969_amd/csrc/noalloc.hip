// noalloc.hip -- the allocation-free variant of nepmi_compute.
//
// Every buffer of the evaluation (neighbour lists, processing order, the
// per-slot arrays the kernels hand to each other, the reduction plan) is
// carved from one file-scope device array instead of hipMalloc.  Each GPU the
// library runs on holds its own copy of the array until the process ends.
// Host code never uses the array's name as an address: the address is taken
// once per device with hipGetSymbolAddress and kept.
#include <mutex>

#include "model.hpp"

namespace nepmi {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // the workspace limit
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAllocDevice {
  void* ptr = nullptr;  // device address of `scratch` on this device
  Arena arena;
  EvalWork work;
};

static std::mutex g_noalloc_mutex;
static NoAllocDevice* g_noalloc[kMaxDevices] = {};

// The workspace of the current device; the first call on a device takes the
// array's address with that device current.
static int noalloc_device(NoAllocDevice** out) {
  int dev = 0;
  NEPMI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the allocation-free table");
    return NEPMI_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  if (!g_noalloc[dev]) {
    void* ptr = nullptr;
    NEPMI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    NoAllocDevice* d = new (std::nothrow) NoAllocDevice();
    if (!d) {
      set_error("out of host memory");
      return NEPMI_INVALID_ARG;
    }
    d->ptr = ptr;
    d->arena.base = static_cast<char*>(ptr);
    d->arena.cap = kScratchBytes;
    g_noalloc[dev] = d;
  }
  *out = g_noalloc[dev];
  return NEPMI_OK;
}

}  // namespace nepmi

using namespace nepmi;

extern "C" int nepmi_compute_noalloc(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc,
                                     const float* dev_pos, const int32_t* dev_species, double* dev_energy,
                                     float* dev_forces, double* dev_virial, float* dev_atom_energy,
                                     float* dev_atom_virial, void* stream) {
  if (!m || !dev_pos || !dev_species) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  NoAllocDevice* d = nullptr;
  int rc = noalloc_device(&d);
  if (rc) return rc;
  // every call lays the workspace out afresh from the start of the array
  d->arena.used = 0;
  d->work.use_arena(&d->arena);
  if ((rc = prepare_eval(d->work, m->ops, m->hp, n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st, 0.0)))
    return rc;
  return run_eval(d->work, m, dev_forces, dev_energy, dev_virial, dev_atom_energy, dev_atom_virial, st);
}
