// nbr.hpp -- device buffers and the neighbour-list pipeline (host side).
#pragma once

#include <vector>

#include "common.hpp"

namespace nepmi {

// Slots of the device flag word array.
enum {
  kFlagOverflow = 0,   // a list exceeded its capacity
  kFlagMaxR = 1,       // largest radial list length seen
  kFlagMaxA = 2,       // largest angular list length seen
  kFlagNaN = 3,        // non-finite input position
  kFlagBadSpecies = 4, // species out of range
  kFlagAsym = 5,       // a pair found from one side only
  kFlagRebuild = 6,    // MD: rebuild the lists in this step
  kFlagCount = 16
};

// Largest Verlet list length: positions are kept in 16 bits.
constexpr int kMaxListRows = 65535;

// A fixed block of device memory handed out front to back (a bump
// allocator).  Buffers bound to an arena take their memory from it instead of
// hipMalloc, and never free it; the owner resets `used` to reuse the block.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

// Device allocation that grows on demand (contents are not preserved).  With
// an arena, growing takes a new region of the arena (NEPMI_INVALID_ARG when
// the arena is exhausted) and nothing is ever freed.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* arena = nullptr;
  template <class T>
  T* ptr() const {
    return static_cast<T*>(p);
  }
  int ensure(size_t n);
  void release();
  ~DevBuf() { release(); }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// State that a rebuild moves from caller order into the new slot order along
// with the positions (MD: float64 positions, velocities, and the positions the
// new lists are built from, as the drift reference).  Used when xd is not null.
struct SlotCarry {
  const double* xd_user = nullptr;  // [N][3] float64 positions, caller order
  const float4* x_user = nullptr;   // [N] the float32 positions the build staged
  const float4* v_user = nullptr;   // [N] velocities
  double* xd = nullptr;             // [n_slots][3]
  float4* vel4 = nullptr;           // [n_slots] (zero in padding slots)
  float4* ref4 = nullptr;           // [n_slots]
};

// Neighbour lists of one batch of configurations, in processing order.
struct NbrPipeline {
  int64_t N = 0;        // atoms
  int n_cfg = 0;
  int n_species = 0;
  int64_t n_slots = 0;  // N + n_species * wavefront (upper bound of used slots)
  int total_bins = 0;
  int capR = 0, capA = 0;
  float rclR2 = 0.f, rclA2 = 0.f;
  double skin = 0.0;
  std::vector<CfgDev> host_cfgs;
  std::vector<int64_t> host_off;

  DevBuf cfgs, atom_off_dev;
  DevBuf key, cnt, start, cursor, tile_sums, base, perm, pos_tmp, cfg_tmp, crd_tmp;
  DevBuf pos4, cfg_of, orig, bin_of, slot_of;
  DevBuf nbrR, cntR;             // Verlet list (rc_radial + skin)
  DevBuf cntAV;                  // entries within rc_angular + skin (the angular part of the list)
  DevBuf nbrTA;                  // the angular part of each list, row-major, rows of rowTA entries (reverse search)
  DevBuf angm;                   // uint32: bit k % 32 of word k / 32 ([word][slot]): entry k is in the angular part
  int rowTA = 0;
  DevBuf vrev;                   // reverse index of the Verlet list (see k_reverse)
  DevBuf cnbrR, ccntR, cnbrA, ccntA, cposA;  // per-evaluation compact lists (rc_radial, rc_angular),
                                             // in groups of four entries (see list_groups)
  DevBuf flags;

  // Host-side setup of a batch: validates the cells, computes bins, sizes
  // buffers and uploads the configuration table.  pbc: host int32[3 n_cfg]
  // (1 periodic, 0 not, per lattice vector) or null (all periodic).  Returns
  // NEPMI_* codes.
  int setup(int n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, int n_species, double rcR,
            double rcA, double skin, hipStream_t st);
  // Sizes the lists for capR x capA entries per slot.
  int ensure_lists(int capR_, int capA_);
  // Take every buffer from `a` from now on (releases what is held; the next
  // setup sizes the lists afresh).
  void use_arena(Arena* a);
  // Stage, bin and sort (pos: N x pos_stride floats).  gate: optional device
  // flag; every kernel returns at once when *gate == 0.  cnt_zeroed: the
  // caller has already cleared the n_species * total_bins + 1 key counts
  // (cnt) on the stream.  carry: state moved into slot order with the
  // positions (optional).
  int launch_sort(hipStream_t st, const float* pos, int pos_stride, const int32_t* species, int n_species,
                  const int* gate, bool cnt_zeroed = false, const SlotCarry* carry = nullptr);
  int launch_lists(hipStream_t st, int n_species, const int* gate);
  // Full build with capacity check and regrow (synchronises st once or twice).
  int build(hipStream_t st, const float* pos, const int32_t* species);
  int check_flags(hipStream_t st, int* host_flags);
};

// Fill an int array with a value on the stream (graph-safe, no memset node).
void fill_int(hipStream_t st, int* p, int64_t n, int v, const int* gate);

}  // namespace nepmi
