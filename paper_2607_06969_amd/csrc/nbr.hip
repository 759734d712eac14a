// nbr.hip -- cell-list binning, processing order and Verlet neighbour lists.
//
// The paper builds neighbour lists on the fly with linear complexity before
// every evaluation (Sec. 3.4, Sec. 3.5).  Here that is a counting sort of the
// atoms into cell bins, done on the GPU, followed by a 27-bin stencil search.
//
// Processing order.  Atoms are renumbered into "slots" sorted by
// (species, global bin, caller index).  Each species group starts at a
// multiple of the wavefront size, so every wavefront of the evaluation
// kernels holds atoms of a single species and reads that species'
// coefficients and network weights through the scalar unit.  Padding slots
// carry orig = -1.
//
// Neighbour entries are 32-bit: slot index (27 bits) | image code (5 bits),
// code = (w0+1)*9 + (w1+1)*3 + (w2+1) for the lattice shift w in {-1,0,1}^3.
// Lists are column-major, entry k of slot p at [k * n_slots + p].  The
// Verlet list holds pairs within rc_radial + skin; at every evaluation the
// descriptor kernel filters it into compact lists of the pairs within
// rc_radial and within rc_angular, which all later kernels iterate.
#include "nbr.hpp"

namespace nepmi {

// ------------------------------------------------------------------ staging

// Per caller-order atom: validate, wrap into the cell, find its bin and sort key.
// Global sort key of a cell bin.  Bins are numbered in 4 x 4 x 4 tiles (tile
// row-major, then row-major inside the tile), so that a contiguous range of
// slots covers a compact region of space: the atoms a GPU die processes at
// the same time, and their neighbours, then fit its L2 better than with
// row-major slabs.  Each configuration owns ceil(nb/4)^3 * 64 keys.
__device__ __forceinline__ int bin_key(const CfgDev& C, int b0, int b1, int b2) {
  const int nt1 = (C.nb[1] + 3) >> 2, nt2 = (C.nb[2] + 3) >> 2;
  const int t = ((b0 >> 2) * nt1 + (b1 >> 2)) * nt2 + (b2 >> 2);
  return C.bin_off + (t << 6) + (((b0 & 3) << 4) | ((b1 & 3) << 2) | (b2 & 3));
}

// Bin coordinates packed into one int (each below 1024).
__device__ __forceinline__ int pack_bin(int b0, int b1, int b2) { return b0 | (b1 << 10) | (b2 << 20); }

__global__ void k_stage(int64_t N, int n_cfg, const int64_t* __restrict__ atom_off, const CfgDev* __restrict__ cfgs,
                        const float* __restrict__ pos, int pos_stride, const int32_t* __restrict__ species,
                        int n_species, int total_bins, float4* __restrict__ pos_tmp, int* __restrict__ cfg_tmp,
                        int* __restrict__ crd_tmp, int* __restrict__ key, int* __restrict__ cnt, int* __restrict__ flags,
                        const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  // configuration of atom i: binary search in atom_off
  int lo = 0, hi = n_cfg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (atom_off[mid] <= i) lo = mid; else hi = mid;
  }
  const CfgDev& C = cfgs[lo];
  const int z = species[i];
  if (z < 0 || z >= n_species) {
    atomicOr(&flags[kFlagBadSpecies], 1);
    key[i] = -1;
    return;
  }
  const float x = pos[i * pos_stride + 0], y = pos[i * pos_stride + 1], w = pos[i * pos_stride + 2];
  if (!(isfinite(x) && isfinite(y) && isfinite(w))) {
    atomicOr(&flags[kFlagNaN], 1);
    key[i] = -1;
    return;
  }
  int b[3];
  double m[3];
  for (int a = 0; a < 3; ++a) {
    const double s = (double)x * C.Hinv[a] + (double)y * C.Hinv[3 + a] + (double)w * C.Hinv[6 + a];
    // along a non-periodic direction the atom is not wrapped, and one outside
    // the cell goes to the nearest bin: its neighbours within the list cutoff
    // lie in that bin or beyond the face as well (bins are wider than the
    // cutoff), so the stencil still finds every pair
    m[a] = (C.periodic >> a) & 1 ? floor(s) : 0.0;
    const double t = (s - m[a]) * C.nb[a];
    b[a] = t < 0.0 ? 0 : (t >= (double)C.nb[a] ? C.nb[a] - 1 : (int)t);
  }
  float o[3] = {x, y, w};
  if (m[0] != 0.0 || m[1] != 0.0 || m[2] != 0.0) {
    // wrap by whole lattice vectors (float64, then rounded once)
    for (int a = 0; a < 3; ++a)
      o[a] = (float)((double)o[a] - m[0] * C.Hd[a] - m[1] * C.Hd[3 + a] - m[2] * C.Hd[6 + a]);
  }
  const int k = z * total_bins + bin_key(C, b[0], b[1], b[2]);
  key[i] = k;
  pos_tmp[i] = make_float4(o[0], o[1], o[2], __int_as_float(z));
  cfg_tmp[i] = lo;
  crd_tmp[i] = pack_bin(b[0], b[1], b[2]);
  atomicAdd(&cnt[k], 1);
}

// ------------------------------------------------------------ exclusive scan

constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ int block_exclusive_scan(int v, int* sh, int& total) {
  // Hillis-Steele within a block of kScanBlock threads (deterministic).
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kScanBlock - 1];
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

// out[0..M] = exclusive prefix sum of in[0..M-1] (out[M] = total), tile level.
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const int* __restrict__ in, int M, int* __restrict__ out,
                                                           int* __restrict__ tile_sums, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems], s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < M) ? in[base + j] : 0;
    s += v[j];
  }
  int total;
  int ex = block_exclusive_scan(s, sh, total);
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < M) out[base + j] = ex;
    ex += v[j];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// Scan of the tile sums (one block; n_tiles <= kScanTile) and the final
// total, then the processing order's species bases: base[z] = first slot of
// species z, each species' group padded to the wavefront size.  out holds the
// tile-local prefixes of k_scan_tiles; the global prefix of key k is
// out[k] + (scanned tile sum of k's tile).
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int* __restrict__ tile_sums, int n_tiles,
                                                          int* __restrict__ out, int M, int total_bins,
                                                          int n_species, int* __restrict__ species_base,
                                                          const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int sh[kScanBlock];
  __shared__ int tile_ex[kScanTile];
  const int b0 = threadIdx.x * kScanItems;
  int v[kScanItems], s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (b0 + j < n_tiles) ? tile_sums[b0 + j] : 0;
    s += v[j];
  }
  int total;
  int ex = block_exclusive_scan(s, sh, total);
  for (int j = 0; j < kScanItems; ++j) {
    if (b0 + j < n_tiles) {
      tile_sums[b0 + j] = ex;
      tile_ex[b0 + j] = ex;
    }
    ex += v[j];
  }
  if (threadIdx.x == 0) out[M] = total;
  __syncthreads();
  if (threadIdx.x != 0) return;
  int acc = 0, lo = 0;  // lo: global prefix at z * total_bins
  for (int z = 0; z < n_species; ++z) {
    const int k = (z + 1) * total_bins;
    const int hi = k < M ? out[k] + tile_ex[k / kScanTile] : total;
    species_base[z] = acc;
    acc += (hi - lo + kWave - 1) / kWave * kWave;
    lo = hi;
  }
  species_base[n_species] = acc;
}

// Global prefixes, also copied into the scatter cursors.
__global__ void k_scan_add(int* __restrict__ out, int M, const int* __restrict__ tile_sums,
                           int* __restrict__ cursor, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) {
    const int v = out[i] + tile_sums[i / kScanTile];
    out[i] = v;
    cursor[i] = v;
  }
}

// ------------------------------------------------------- processing order

// Slot of every atom (order inside a key decided by an atomic; made
// deterministic by k_sort_keys).
__global__ void k_scatter(int64_t N, const int* __restrict__ key, const int* __restrict__ start,
                          int* __restrict__ cursor, const int* __restrict__ base, int total_bins,
                          int* __restrict__ perm, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = key[i];
  if (k < 0) return;
  const int z = k / total_bins;
  // cursor[k] starts at start[k]: the returned value is start[k] + rank in key
  const int r = atomicAdd(&cursor[k], 1);
  const int p = base[z] + (r - start[z * total_bins]);
  perm[p] = (int)i;
}

// Sort the slots of each key by caller index (insertion sort; keys hold few atoms).
__global__ void k_sort_keys(int M, const int* __restrict__ start, const int* __restrict__ base, int total_bins,
                            int* __restrict__ perm, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const int z = k / total_bins;
  const int n = start[k + 1] - start[k];
  if (n < 2) return;
  int* s = perm + base[z] + (start[k] - start[z * total_bins]);
  for (int a = 1; a < n; ++a) {
    const int v = s[a];
    int b = a - 1;
    while (b >= 0 && s[b] > v) {
      s[b + 1] = s[b];
      --b;
    }
    s[b + 1] = v;
  }
}

// Fill the slot arrays.  Padding slots get orig = -1 and their group's species.
// With carry.xd set, the carried state moves into the slot as well: the
// staging wraps again only in a last-ulp case at a cell face, and that shift
// (zero otherwise) is carried into the float64 position.
__global__ void k_fill_slots(int64_t n_slots, const int* __restrict__ base, const int* __restrict__ start,
                             int total_bins, int n_species, const int* __restrict__ perm,
                             const float4* __restrict__ pos_tmp, const int* __restrict__ cfg_tmp,
                             const int* __restrict__ crd_tmp,
                             const int* __restrict__ key, float4* __restrict__ pos4, int* __restrict__ cfg_of,
                             int* __restrict__ orig, int* __restrict__ bin_of, int* __restrict__ slot_of,
                             SlotCarry carry, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  int z = -1;
  for (int t = 0; t < n_species; ++t)
    if (p >= base[t] && p < base[t + 1]) z = t;
  if (z >= 0) {
    const int r = (int)(p - base[z]);
    const int c = start[(z + 1) * total_bins] - start[z * total_bins];
    if (r < c) {
      const int i = perm[p];
      const float4 xs = pos_tmp[i];
      pos4[p] = xs;
      cfg_of[p] = cfg_tmp[i];
      orig[p] = i;
      bin_of[p] = crd_tmp[i];  // packed bin coordinates
      if (slot_of) slot_of[i] = (int)p;
      if (carry.xd) {
        const float4 xu = carry.x_user[i];
        const double* r = carry.xd_user + 3 * (int64_t)i;
        double* o = carry.xd + 3 * p;
        o[0] = r[0] + ((double)xs.x - (double)xu.x);
        o[1] = r[1] + ((double)xs.y - (double)xu.y);
        o[2] = r[2] + ((double)xs.z - (double)xu.z);
        carry.vel4[p] = carry.v_user[i];
        carry.ref4[p] = xs;
      }
      return;
    }
  } else {
    z = 0;
  }
  if (carry.xd) carry.vel4[p] = make_float4(0.f, 0.f, 0.f, 0.f);
  pos4[p] = make_float4(0.f, 0.f, 0.f, __int_as_float(z));
  cfg_of[p] = -1;
  orig[p] = -1;
  bin_of[p] = -1;
}

// --------------------------------------------------------- Verlet lists

// For every active slot, scan the 27 stencil bins (with periodic images) and
// keep neighbours within the radial and angular list cutoffs.  Along a
// non-periodic direction a stencil bin beyond the cell has no atoms (no
// images): it is skipped.
__global__ __launch_bounds__(256) void k_build_lists(int64_t n_slots, int n_species, int total_bins,
                                                     const CfgDev* __restrict__ cfgs,
                                                     const float4* __restrict__ pos4, const int* __restrict__ cfg_of,
                                                     const int* __restrict__ bin_of, const int* __restrict__ start,
                                                     const int* __restrict__ base, float rclR2, float rclA2, int capR,
                                                     int capA, int rowTA, uint32_t* __restrict__ nbrR,
                                                     uint32_t* __restrict__ nbrTA, uint32_t* __restrict__ angm,
                                                     int* __restrict__ cntR, int* __restrict__ cntAV,
                                                     int* __restrict__ flags, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t p = xcd_tile() * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  const int c = cfg_of[p];
  if (c < 0) {
    cntR[p] = 0;
    cntAV[p] = 0;
    return;
  }
  const CfgDev& C = cfgs[c];
  const float4 xi = pos4[p];
  const int pb = bin_of[p];
  const int b0 = pb & 1023, b1 = (pb >> 10) & 1023, b2 = pb >> 20;
  // The 27 stencil bins in ascending bin key, visited per species: slots are
  // ordered by (species, bin key), so the list comes out in slot order.
  // Neighbouring atoms then tend to have their k-th neighbours in the same
  // cache lines, and a wavefront's gather of the k-th neighbours touches fewer
  // lines than with the stencil order.  Each bin is packed with its image code
  // (bin key << 5 | code: unique, so the order is total; bin keys are below
  // 2^27) and sorted by a compare-exchange network with fixed indices, which
  // stays in registers; the sorted bins wait in this thread's LDS column.
  // Skipped bins are kNoBin, which sorts last.
  constexpr uint32_t kNoBin = 0xFFFFFFFFu;
  __shared__ uint32_t sorted_bins[27 * 256];
  uint32_t sb[27];
  const int per = C.periodic;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    int t0 = b0 + o / 9 - 1, t1 = b1 + (o / 3) % 3 - 1, t2 = b2 + o % 3 - 1;
    const int w0 = t0 < 0 ? -1 : (t0 >= C.nb[0] ? 1 : 0);
    const int w1 = t1 < 0 ? -1 : (t1 >= C.nb[1] ? 1 : 0);
    const int w2 = t2 < 0 ? -1 : (t2 >= C.nb[2] ? 1 : 0);
    const bool skip = (w0 && !(per & 1)) || (w1 && !(per & 2)) || (w2 && !(per & 4));
    t0 -= w0 * C.nb[0];
    t1 -= w1 * C.nb[1];
    t2 -= w2 * C.nb[2];
    const uint32_t code = (uint32_t)((w0 + 1) * 9 + (w1 + 1) * 3 + (w2 + 1));
    sb[o] = skip ? kNoBin : (((uint32_t)bin_key(C, t0, t1, t2) << 5) | code);
  }
#pragma unroll
  for (int i = 1; i < 27; ++i)
#pragma unroll
    for (int j = i; j > 0; --j) {
      const uint32_t lo = sb[j - 1] < sb[j] ? sb[j - 1] : sb[j];
      const uint32_t hi = sb[j - 1] < sb[j] ? sb[j] : sb[j - 1];
      sb[j - 1] = lo;
      sb[j] = hi;
    }
#pragma unroll
  for (int o = 0; o < 27; ++o) sorted_bins[o * 256 + threadIdx.x] = sb[o];
  // Entries are collected four at a time and stored as one group: one store
  // per four entries instead of one per entry.  The entries within
  // rc_angular + skin (the angular part of the list, which the reverse index
  // searches) are also kept in their own row-major list, and marked in a bit
  // mask over the list (bit k % 32 of word k / 32: entry k is in that part).
  // Entries and mask bits shift in from the top, so a full group or word
  // holds them in list order; the store pointers advance one column at a time.
  const int capG = 4 * list_groups(capR);   // entries the groups can hold
  const int capGA = 4 * list_groups(capA);
  uint4 grp = make_uint4(0u, 0u, 0u, 0u), gra = grp;
  uint32_t mword = 0;
  uint4* colG = reinterpret_cast<uint4*>(nbrR) + p;         // next group, column-major
  uint4* rowA = reinterpret_cast<uint4*>(nbrTA + p * rowTA);  // angular part, row-major
  uint32_t* colM = angm + p;                                // next mask word, column-major
  int kR = 0, kA = 0;
  for (int z = 0; z < n_species; ++z) {
    for (int o = 0; o < 27; ++o) {
      const uint32_t sbo = sorted_bins[o * 256 + threadIdx.x];
      if (sbo == kNoBin) break;
      const int tb = (int)(sbo >> 5);
      const uint32_t code = sbo & 31u;
      float sx, sy, sz;
      image_shift(C.H, code, sx, sy, sz);
      const int k = z * total_bins + tb;
      const int q0 = base[z] + start[k] - start[z * total_bins];
      const int q1 = q0 + start[k + 1] - start[k];
      // four candidates per round, loaded together (indices clamped into the
      // bin's range, so every load is in bounds; the extra ones are skipped)
      for (int q4 = q0; q4 < q1; q4 += 4) {
        float4 xs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xs[u] = pos4[q4 + u < q1 ? q4 + u : q1 - 1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q4 + u;
          if (q >= q1 || (q == (int)p && code == 13u)) continue;
          const float rx = (xs[u].x - xi.x) + sx, ry = (xs[u].y - xi.y) + sy, rz = (xs[u].z - xi.z) + sz;
          const float d2 = pair_d2(rx, ry, rz);
          if (d2 < rclR2) {
            // entries shift into a group from the top (four register moves,
            // no selects); a full group holds them in list order
            const uint32_t e = (uint32_t)q | (code << kNbrShift);
            grp = make_uint4(grp.y, grp.z, grp.w, e);
            mword = (mword >> 1) | (d2 < rclA2 ? 0x80000000u : 0u);
            ++kR;
            if ((kR & 3) == 0 && kR <= capG) {
              *colG = grp;
              colG += n_slots;
            }
            if ((kR & 31) == 0 && kR <= capG) {
              *colM = mword;
              colM += n_slots;
            }
            if (d2 < rclA2) {
              gra = make_uint4(gra.y, gra.z, gra.w, e);
              ++kA;
              if ((kA & 3) == 0 && kA <= capGA) rowA[(kA >> 2) - 1] = gra;
            }
          }
        }
      }
    }
  }
  // the last, partly filled groups (their r entries sit in the top r
  // components: moved down to the front) and mask word
  auto front = [](uint4 g, int r) {
    return r == 1 ? make_uint4(g.w, g.w, g.w, g.w) : r == 2 ? make_uint4(g.z, g.w, g.w, g.w)
                                                           : make_uint4(g.y, g.z, g.w, g.w);
  };
  if ((kR & 3) && kR < capG) *colG = front(grp, kR & 3);
  if ((kR & 31) && kR < capG) *colM = mword >> (32 - (kR & 31));
  if ((kA & 3) && kA < capGA) rowA[kA >> 2] = front(gra, kA & 3);
  cntR[p] = kR < capR ? kR : capR;
  cntAV[p] = kA < capA ? kA : capA;
  // the angular pairs within rc_angular at any step between rebuilds are among
  // those within rc_angular + skin now, so kA bounds the per-step angular list
  if (kR > capR || kA > capA) atomicOr(&flags[kFlagOverflow], 1);
  atomicMax(&flags[kFlagMaxR], kR);
  atomicMax(&flags[kFlagMaxA], kA);
}

// Reverse index: for every entry k of i's Verlet list whose pair is within
// rc_angular + skin (the angular part of the list), the position of i in the
// angular part of the list of the neighbour j (the entry with i's slot and the
// opposite image code), else 0xFFFFFFFF; 0xFFFFFFFE marks an angular entry
// whose partner was not found, which also raises the asymmetry flag.  The
// pair-force buffer is indexed through these positions, so that each step's
// gather reads without searching.  The angular entries are known from the
// bit mask k_build_lists leaves, and the search reads the angular part of j's
// list only (about a third of the list).  The four entries of a group are
// searched together and their results stored together.  Grid (slot tiles, rows): row y takes the
// groups g = y, y + rows, ... of each list, so the searches of one atom run
// side by side.  The x extent is a multiple of the XCD count, so that every
// row maps a slot tile to the same XCD.  Small batches take kRevSplit rows;
// from kRevOneRow tiles on, the slot tiles alone fill the chip and one row is
// used (more rows there only add blocks, which cost time even when the
// rebuild gate sends them home at once).
constexpr int kRevSplit = 4;
constexpr unsigned kRevOneRow = 2048;
__global__ __launch_bounds__(256) void k_reverse(int64_t n_slots, const int* __restrict__ cfg_of,
                                                 const uint32_t* __restrict__ nbrR, const uint32_t* __restrict__ nbrTA,
                                                 int rowTA, const uint32_t* __restrict__ angm,
                                                 const int* __restrict__ cntR, const int* __restrict__ cntAV,
                                                 uint32_t* __restrict__ vrev, int* __restrict__ flags,
                                                 const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t p = xcd_tile() * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  const int c = cfg_of[p];
  if (c < 0) return;
  const int n = cntR[p];
  const int ng = list_groups(n);
  const uint4* grp = reinterpret_cast<const uint4*>(nbrR) + p;
  uint4* out = reinterpret_cast<uint4*>(vrev) + p;
  bool missing = false;
  // The four entries of a group are searched side by side: the angular ones
  // (marked by k_build_lists) have their neighbours' list lengths loaded
  // together, then the first kRevWin entries of every row that needs a search
  // (one memory latency for the group); longer rows are finished one at a time.
  constexpr int kRevWin = 8;  // uint4 per row read at once (32 entries)
  for (int g = (int)blockIdx.y; g < ng; g += (int)gridDim.y) {
    const uint4 eg = grp[(int64_t)g * n_slots];
    const uint32_t bits = (angm[(int64_t)(g >> 3) * n_slots + p] >> (4 * (g & 7))) & 15u;
    bool ang[4];
    int nq[4];
    uint32_t want[4];
    const uint4* row[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ang[u] = 4 * g + u < n && ((bits >> u) & 1u);
      const uint32_t e = comp4(eg, ang[u] ? u : 0);
      nq[u] = ang[u] ? cntAV[e & kNbrMask] : 0;
      want[u] = (uint32_t)p | ((26u - (e >> kNbrShift)) << kNbrShift);
      row[u] = reinterpret_cast<const uint4*>(nbrTA + (int64_t)(e & kNbrMask) * rowTA);
    }
    // the angular part of each neighbour's list, row-major, rows padded to a
    // multiple of 4 entries so that the 16-byte reads stay inside the row;
    // entries at or past nq are ignored
    uint4 w[4][kRevWin];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < kRevWin; ++t) w[u][t] = 4 * t < nq[u] ? row[u][t] : make_uint4(~0u, ~0u, ~0u, ~0u);
    uint32_t res[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      uint32_t r = 0xFFFFFFFEu;
#pragma unroll
      for (int t = kRevWin - 1; t >= 0; --t) {
        const int j = 4 * t;
        if (w[u][t].w == want[u] && j + 3 < nq[u]) r = (uint32_t)(j + 3);
        if (w[u][t].z == want[u] && j + 2 < nq[u]) r = (uint32_t)(j + 2);
        if (w[u][t].y == want[u] && j + 1 < nq[u]) r = (uint32_t)(j + 1);
        if (w[u][t].x == want[u] && j < nq[u]) r = (uint32_t)j;
      }
      for (int j0 = 4 * kRevWin; j0 < nq[u] && r == 0xFFFFFFFEu; j0 += 4) {
        const uint4 x = row[u][j0 >> 2];
        if (x.w == want[u] && j0 + 3 < nq[u]) r = (uint32_t)(j0 + 3);
        if (x.z == want[u] && j0 + 2 < nq[u]) r = (uint32_t)(j0 + 2);
        if (x.y == want[u] && j0 + 1 < nq[u]) r = (uint32_t)(j0 + 1);
        if (x.x == want[u]) r = (uint32_t)j0;
      }
      if (ang[u]) missing |= r == 0xFFFFFFFEu;
      res[u] = ang[u] ? r : 0xFFFFFFFFu;
    }
    out[(int64_t)g * n_slots] = make_uint4(res[0], res[1], res[2], res[3]);
  }
  if (missing) atomicOr(&flags[kFlagAsym], 1);
}

// ---------------------------------------------------------------- host side

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_fill_int(int* __restrict__ p, int64_t n, int v, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void fill_int(hipStream_t st, int* p, int64_t n, int v, const int* gate) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v, gate);
}

int DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return NEPMI_OK;
  if (arena) {
    const size_t want = ((n < 256 ? 256 : n) + 255) / 256 * 256;
    if (arena->used + want > arena->cap) {
      set_error("the batch needs more than the " + std::to_string(arena->cap >> 20) +
                " MiB of the allocation-free workspace");
      return NEPMI_INVALID_ARG;
    }
    p = arena->base + arena->used;
    arena->used += want;
    bytes = want;
    return NEPMI_OK;
  }
  release();
  const size_t want = n < 256 ? 256 : n;
  NEPMI_HIP(hipMalloc(&p, want));
  bytes = want;
  return NEPMI_OK;
}

void DevBuf::release() {
  if (p && !arena) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

static void cell_geometry(const double* H, double w[3], double Hi[9], double& det) {
  const double *a = H, *b = H + 3, *c = H + 6;
  const double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
  const double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
  const double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  det = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
  const double V = fabs(det);
  w[0] = V / sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  w[1] = V / sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
  w[2] = V / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
  // rows of Hinv^T are bc, ca, ab divided by det: fractional s_a = x . (col a of Hinv)
  for (int x = 0; x < 3; ++x) {
    Hi[3 * x + 0] = bc[x] / det;
    Hi[3 * x + 1] = ca[x] / det;
    Hi[3 * x + 2] = ab[x] / det;
  }
}

int NbrPipeline::setup(int n_cfg_, const int64_t* atom_off, const double* cells, const int32_t* pbc, int n_species_,
                       double rcR, double rcA, double skin_, hipStream_t st) {
  if (n_cfg_ < 1 || !atom_off || !cells) {
    set_error("n_cfg must be >= 1 and atom_off, cells non-null");
    return NEPMI_INVALID_ARG;
  }
  if (atom_off[0] != 0) {
    set_error("atom_off[0] must be 0");
    return NEPMI_INVALID_ARG;
  }
  for (int c = 0; c < n_cfg_; ++c)
    if (atom_off[c + 1] < atom_off[c]) {
      set_error("atom_off must be non-decreasing");
      return NEPMI_INVALID_ARG;
    }
  const int64_t N_ = atom_off[n_cfg_];
  if (N_ < 1) {
    set_error("the batch holds no atoms");
    return NEPMI_INVALID_ARG;
  }
  if (N_ > (int64_t)kMaxAtoms - 64 * n_species_) {
    set_error("too many atoms for 27-bit neighbour indices");
    return NEPMI_INVALID_ARG;
  }
  const double rcl = rcR + skin_;
  std::vector<CfgDev> hc((size_t)n_cfg_);
  int64_t bins = 0;
  for (int c = 0; c < n_cfg_; ++c) {
    CfgDev& C = hc[(size_t)c];
    const double* H = cells + 9 * (size_t)c;
    double w[3], det;
    cell_geometry(H, w, C.Hinv, det);
    if (!(fabs(det) > 0.0) || !std::isfinite(det)) {
      set_error("singular or non-finite cell");
      return NEPMI_INVALID_ARG;
    }
    C.periodic = 0;
    for (int a = 0; a < 3; ++a) {
      const int32_t pa = pbc ? pbc[3 * (size_t)c + a] : 1;
      if (pa != 0 && pa != 1) {
        set_error("pbc entries must be 0 or 1");
        return NEPMI_INVALID_ARG;
      }
      C.periodic |= pa << a;
      // only a periodic direction needs the width: no pair may meet two
      // images of one atom
      if (pa && w[a] < 2.0 * rcl) {
        set_error("cell width " + std::to_string(w[a]) + " of configuration " + std::to_string(c) +
                  " is below 2 * (rc_radial + skin) = " + std::to_string(2.0 * rcl));
        return NEPMI_CELL_TOO_SMALL;
      }
      // bins a little wider than the list cutoff, so that a position rounded
      // differently by 1e-3 A cannot move a neighbour out of the 27-bin stencil
      int nb = (int)floor(w[a] / (rcl * (1.0 + 1e-6) + 1e-3));
      C.nb[a] = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
    }
    for (int x = 0; x < 9; ++x) {
      C.Hd[x] = H[x];
      C.H[x] = (float)H[x];
    }
    C.bin_off = (int)bins;
    C.atom_off = atom_off[c];
    C.n_atoms = (int)(atom_off[c + 1] - atom_off[c]);
    bins += (int64_t)((C.nb[0] + 3) / 4) * ((C.nb[1] + 3) / 4) * ((C.nb[2] + 3) / 4) * 64;
  }
  // bin keys below 2^27: the list build packs a key and a 5-bit image code
  // into 32 bits
  if (bins >= (int64_t)1 << 27 || bins * n_species_ > (int64_t)1 << 30) {
    set_error("too many cell bins");
    return NEPMI_INVALID_ARG;
  }
  N = N_;
  n_cfg = n_cfg_;
  n_species = n_species_;
  n_slots = N + (int64_t)kWave * n_species_;
  total_bins = (int)bins;
  skin = skin_;
  const float rlR = (float)(rcR + skin_), rlA = (float)(rcA + skin_);
  rclR2 = rlR * rlR;
  rclA2 = rlA * rlA;
  host_cfgs = hc;
  host_off.assign(atom_off, atom_off + n_cfg_ + 1);
  const int64_t M = (int64_t)n_species_ * bins;
  const int64_t n_tiles = (M + kScanTile - 1) / kScanTile;
  if (n_tiles > kScanTile) {
    set_error("too many sort keys");
    return NEPMI_INVALID_ARG;
  }
  int rc;
  const size_t Na = (size_t)(N > 0 ? N : 1);
  if ((rc = cfgs.ensure(sizeof(CfgDev) * (size_t)n_cfg_)) || (rc = atom_off_dev.ensure(8 * (size_t)(n_cfg_ + 1))) ||
      (rc = key.ensure(4 * Na)) || (rc = cnt.ensure(4 * (size_t)(M + 1))) || (rc = start.ensure(4 * (size_t)(M + 1))) ||
      (rc = cursor.ensure(4 * (size_t)(M + 1))) || (rc = tile_sums.ensure(4 * (size_t)(n_tiles + 1))) ||
      (rc = base.ensure(4 * (size_t)(n_species_ + 1))) || (rc = perm.ensure(4 * (size_t)n_slots)) ||
      (rc = pos_tmp.ensure(16 * Na)) || (rc = cfg_tmp.ensure(4 * Na)) || (rc = crd_tmp.ensure(4 * Na)) || (rc = pos4.ensure(16 * (size_t)n_slots)) ||
      (rc = cfg_of.ensure(4 * (size_t)n_slots)) || (rc = orig.ensure(4 * (size_t)n_slots)) ||
      (rc = bin_of.ensure(4 * (size_t)n_slots)) || (rc = slot_of.ensure(4 * Na)) ||
      (rc = cntR.ensure(4 * (size_t)n_slots)) || (rc = cntAV.ensure(4 * (size_t)n_slots)) ||
      (rc = ccntR.ensure(4 * (size_t)n_slots)) ||
      (rc = ccntA.ensure(4 * (size_t)n_slots)) ||
      (rc = flags.ensure(4 * kFlagCount)))
    return rc;
  // uploaded from the members, which outlive the asynchronous copies (the
  // caller synchronises the stream before the next setup)
  NEPMI_HIP(hipMemcpyAsync(cfgs.p, host_cfgs.data(), sizeof(CfgDev) * (size_t)n_cfg_, hipMemcpyHostToDevice, st));
  NEPMI_HIP(hipMemcpyAsync(atom_off_dev.p, host_off.data(), 8 * (size_t)(n_cfg_ + 1), hipMemcpyHostToDevice, st));
  if (capR == 0) {
    // initial capacity from the densest configuration
    double dmax = 0.0;
    for (int c = 0; c < n_cfg_; ++c) {
      const double* H = cells + 9 * (size_t)c;
      double w[3], Hi[9], det;
      cell_geometry(H, w, Hi, det);
      const double dens = (double)hc[(size_t)c].n_atoms / fabs(det);
      dmax = dens > dmax ? dens : dmax;
    }
    const double vR = 4.18879020478639 * rlR * rlR * rlR, vA = 4.18879020478639 * rlA * rlA * rlA;
    capR = (int)(1.5 * dmax * vR) + 16;
    capA = (int)(1.5 * dmax * vA) + 16;
  }
  return ensure_lists(capR, capA);
}

void NbrPipeline::use_arena(Arena* a) {
  DevBuf* all[] = {&cfgs, &atom_off_dev, &key, &cnt, &start, &cursor, &tile_sums, &base, &perm, &pos_tmp,
                   &cfg_tmp, &crd_tmp, &pos4, &cfg_of, &orig, &bin_of, &slot_of, &nbrR, &cntR, &cntAV, &nbrTA, &angm, &vrev,
                   &cnbrR, &ccntR, &cnbrA, &ccntA, &cposA, &flags};
  for (DevBuf* b : all) {
    b->release();
    b->arena = a;
  }
  capR = capA = 0;
}

int NbrPipeline::ensure_lists(int capR_, int capA_) {
  if (capR_ > kMaxListRows) {
    // list positions are stored in 16 bits (reverse index, pair buffer rows)
    set_error("more than " + std::to_string(kMaxListRows) + " neighbours within rc_radial + skin");
    return NEPMI_NEIGHBOR_OVERFLOW;
  }
  capR = capR_;
  capA = capA_;
  int rc;
  const size_t ns = (size_t)n_slots;
  rowTA = 4 * list_groups(capA_);
  // the Verlet list, its reverse index and the compact lists are stored in
  // groups of four entries (see list_groups); the angular part of the Verlet
  // list, row-major, in rows of rowTA entries
  if ((rc = nbrR.ensure(16 * (size_t)list_groups(capR) * ns)) || (rc = nbrTA.ensure(4 * (size_t)rowTA * ns)) ||
      (rc = angm.ensure(4 * (size_t)((4 * list_groups(capR) + 31) / 32) * ns)) ||
      (rc = vrev.ensure(16 * (size_t)list_groups(capR) * ns)) ||
      (rc = cnbrR.ensure(16 * (size_t)list_groups(capR) * ns)) ||
      (rc = cnbrA.ensure(16 * (size_t)list_groups(capA) * ns)) ||
      (rc = cposA.ensure(16 * (size_t)list_groups(capA) * ns)))
    return rc;
  return NEPMI_OK;
}

int NbrPipeline::check_flags(hipStream_t st, int* hf) {
  NEPMI_HIP(hipMemcpyAsync(hf, flags.p, sizeof(int) * kFlagCount, hipMemcpyDeviceToHost, st));
  NEPMI_HIP(hipStreamSynchronize(st));
  if (hf[kFlagNaN]) {
    set_error("non-finite position");
    return NEPMI_NAN_DETECTED;
  }
  if (hf[kFlagBadSpecies]) {
    set_error("species index out of range");
    return NEPMI_INVALID_ARG;
  }
  return NEPMI_OK;
}

int NbrPipeline::build(hipStream_t st, const float* pos, const int32_t* species) {
  fill_int(st, flags.ptr<int>(), kFlagCount, 0, nullptr);
  int rc = launch_sort(st, pos, 3, species, n_species, nullptr);
  if (rc) return rc;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if ((rc = launch_lists(st, n_species, nullptr))) return rc;
    int hf[kFlagCount];
    if ((rc = check_flags(st, hf))) return rc;
    if (!hf[kFlagOverflow]) {
      if (hf[kFlagAsym]) {
        set_error("neighbour list is not symmetric");
        return NEPMI_INVALID_ARG;
      }
      return NEPMI_OK;
    }
    // grow to the largest list seen plus a margin and rebuild the lists
    if ((rc = ensure_lists(hf[kFlagMaxR] + 8, hf[kFlagMaxA] + 8))) return rc;
    fill_int(st, flags.ptr<int>(), kFlagCount, 0, nullptr);
  }
  set_error("neighbour capacity overflow after regrow");
  return NEPMI_NEIGHBOR_OVERFLOW;
}

int NbrPipeline::launch_sort(hipStream_t st, const float* pos, int pos_stride, const int32_t* species, int n_species,
                             const int* gate, bool cnt_zeroed, const SlotCarry* carry) {
  const int M = n_species * total_bins;
  if (!cnt_zeroed) fill_int(st, cnt.ptr<int>(), M + 1, 0, gate);
  if (N > 0)
  hipLaunchKernelGGL(k_stage, dim3(nblk(N, 256)), dim3(256), 0, st, N, n_cfg, atom_off_dev.ptr<int64_t>(),
                     cfgs.ptr<CfgDev>(), pos, pos_stride, species, n_species, total_bins, pos_tmp.ptr<float4>(),
                     cfg_tmp.ptr<int>(), crd_tmp.ptr<int>(), key.ptr<int>(), cnt.ptr<int>(), flags.ptr<int>(), gate);
  const int n_tiles = (M + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(n_tiles), dim3(kScanBlock), 0, st, cnt.ptr<int>(), M, start.ptr<int>(),
                     tile_sums.ptr<int>(), gate);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, st, tile_sums.ptr<int>(), n_tiles, start.ptr<int>(),
                     M, total_bins, n_species, base.ptr<int>(), gate);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk(M, 256)), dim3(256), 0, st, start.ptr<int>(), M, tile_sums.ptr<int>(),
                     cursor.ptr<int>(), gate);
  if (N > 0)
  hipLaunchKernelGGL(k_scatter, dim3(nblk(N, 256)), dim3(256), 0, st, N, key.ptr<int>(), start.ptr<int>(),
                     cursor.ptr<int>(), base.ptr<int>(), total_bins, perm.ptr<int>(), gate);
  hipLaunchKernelGGL(k_sort_keys, dim3(nblk(M, 256)), dim3(256), 0, st, M, start.ptr<int>(), base.ptr<int>(),
                     total_bins, perm.ptr<int>(), gate);
  hipLaunchKernelGGL(k_fill_slots, dim3(nblk(n_slots, 256)), dim3(256), 0, st, n_slots, base.ptr<int>(),
                     start.ptr<int>(), total_bins, n_species, perm.ptr<int>(), pos_tmp.ptr<float4>(),
                     cfg_tmp.ptr<int>(), crd_tmp.ptr<int>(), key.ptr<int>(), pos4.ptr<float4>(), cfg_of.ptr<int>(), orig.ptr<int>(),
                     bin_of.ptr<int>(), slot_of.ptr<int>(), carry ? *carry : SlotCarry{}, gate);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int NbrPipeline::launch_lists(hipStream_t st, int n_species, const int* gate) {
  hipLaunchKernelGGL(k_build_lists, dim3(nblk(n_slots, 256)), dim3(256), 0, st, n_slots, n_species, total_bins,
                     cfgs.ptr<CfgDev>(), pos4.ptr<float4>(), cfg_of.ptr<int>(), bin_of.ptr<int>(), start.ptr<int>(),
                     base.ptr<int>(), rclR2, rclA2, capR, capA, rowTA, nbrR.ptr<uint32_t>(), nbrTA.ptr<uint32_t>(),
                     angm.ptr<uint32_t>(), cntR.ptr<int>(), cntAV.ptr<int>(), flags.ptr<int>(), gate);
  const unsigned rev_tiles = (nblk(n_slots, 256) + kXcds - 1) / kXcds * kXcds;
  const unsigned rev_rows = rev_tiles >= kRevOneRow ? 1u : (unsigned)kRevSplit;
  hipLaunchKernelGGL(k_reverse, dim3(rev_tiles, rev_rows), dim3(256), 0, st, n_slots, cfg_of.ptr<int>(),
                     nbrR.ptr<uint32_t>(), nbrTA.ptr<uint32_t>(), rowTA, angm.ptr<uint32_t>(), cntR.ptr<int>(),
                     cntAV.ptr<int>(), vrev.ptr<uint32_t>(), flags.ptr<int>(), gate);
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

}  // namespace nepmi
