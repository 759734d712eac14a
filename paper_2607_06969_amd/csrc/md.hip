// md.hip -- velocity-Verlet NVE molecular dynamics replayed as a HIP graph.
//
// One step: half kick + drift (float64 positions, float32 copy for the force
// kernels) and a displacement check; a neighbour-list rebuild whose kernels
// all return at once unless an atom moved more than skin/2 since the last
// build; descriptor/network, pair-force and gather kernels; the second half
// kick; float64 sums of potential energy (Eq. 1), virial (Eq. 4) and kinetic
// energy.  The graph topology is fixed; only the rebuild flag decides whether
// the rebuild kernels do work.
#include <cmath>
#include <new>
#include <vector>

#include "model.hpp"

namespace nepmi {

constexpr float kAccUnit = 9.648533212e-3f;  // 1 eV/(A u) in A/fs^2
constexpr int kMaxSpecies = 8;

struct MdConst {
  float acc[kMaxSpecies];   // dt/2 * kAccUnit / m_s   (half kick per unit force)
  float kin[kMaxSpecies];   // m_s / (2 kAccUnit)       (eV per (A/fs)^2)
  float dt;
  float half_skin2;         // (skin/2)^2
};

struct Dbl3 {
  double x, y, z;
};

__global__ void k_md_kick_drift(int64_t n_slots, MdConst mc, const int* __restrict__ cfg_of,
                                const float4* __restrict__ F4, float4* __restrict__ vel4, Dbl3* __restrict__ xd,
                                float4* __restrict__ pos4, const float4* __restrict__ ref4, int* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots || cfg_of[p] < 0) return;
  float4 x = pos4[p];
  const int z = __float_as_int(x.w);
  const float4 f = F4[p];
  float4 v = vel4[p];
  v.x = fmaf(mc.acc[z], f.x, v.x);
  v.y = fmaf(mc.acc[z], f.y, v.y);
  v.z = fmaf(mc.acc[z], f.z, v.z);
  vel4[p] = v;
  Dbl3 r = xd[p];
  r.x += (double)mc.dt * v.x;
  r.y += (double)mc.dt * v.y;
  r.z += (double)mc.dt * v.z;
  xd[p] = r;
  x.x = (float)r.x;
  x.y = (float)r.y;
  x.z = (float)r.z;
  pos4[p] = x;
  const float4 o = ref4[p];
  const float dx = x.x - o.x, dy = x.y - o.y, dz = x.z - o.z;
  if (dx * dx + dy * dy + dz * dz > mc.half_skin2) atomicOr(&flags[kFlagRebuild], 1);
}

// Wrap r into the cell along its periodic directions in float64, and round it
// to f; if the rounding lands outside the cell (a last-ulp case at a face),
// wrap the rounded value once more.  Non-periodic directions are left alone.
__device__ void wrap_periodic(const CfgDev& C, double r[3], float f[3]) {
  for (int pass = 0; pass < 2; ++pass) {
    double m[3];
    for (int a = 0; a < 3; ++a) {
      const double s = r[0] * C.Hinv[a] + r[1] * C.Hinv[3 + a] + r[2] * C.Hinv[6 + a];
      m[a] = (C.periodic >> a) & 1 ? floor(s) : 0.0;
    }
    for (int a = 0; a < 3; ++a) r[a] -= m[0] * C.Hd[a] + m[1] * C.Hd[3 + a] + m[2] * C.Hd[6 + a];
    for (int a = 0; a < 3; ++a) f[a] = (float)r[a];
    // the float32 copy must also lie in the cell (as the staging kernel sees it)
    bool inside = true;
    for (int a = 0; a < 3; ++a) {
      const double s = (double)f[0] * C.Hinv[a] + (double)f[1] * C.Hinv[3 + a] + (double)f[2] * C.Hinv[6 + a];
      if ((C.periodic >> a) & 1 && floor(s) != 0.0) inside = false;
    }
    if (inside) break;
    for (int a = 0; a < 3; ++a) r[a] = (double)f[a];
  }
}

// Before a rebuild: state back to caller order, positions wrapped into the
// cell in float64 so that the float32 copy needs no further wrapping.  Also
// clears the n_clear key counts of the sort that follows (cnt may be null).
__global__ void k_md_unpermute(int64_t n_slots, const int* __restrict__ cfg_of, const int* __restrict__ orig,
                               const CfgDev* __restrict__ cfgs, const Dbl3* __restrict__ xd,
                               const float4* __restrict__ vel4, Dbl3* __restrict__ xd_user,
                               float4* __restrict__ x_user, float4* __restrict__ v_user, int* __restrict__ cnt,
                               int64_t n_clear, const int* __restrict__ gate) {
  if (*gate == 0) return;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cnt)
    for (int64_t k = p; k < n_clear; k += (int64_t)gridDim.x * blockDim.x) cnt[k] = 0;
  if (p >= n_slots) return;
  const int c = cfg_of[p];
  if (c < 0) return;
  double r[3] = {xd[p].x, xd[p].y, xd[p].z};
  float f[3];
  wrap_periodic(cfgs[c], r, f);
  const int i = orig[p];
  xd_user[i] = Dbl3{r[0], r[1], r[2]};
  x_user[i] = make_float4(f[0], f[1], f[2], 0.f);
  v_user[i] = vel4[p];
}

// Second half kick and per-atom kinetic energy.  The first thread also ends
// the step's bookkeeping: it counts the step (and the rebuild, if one ran)
// and clears the rebuild flag, which nothing later in the step reads.
__global__ void k_md_kick2(int64_t n_slots, MdConst mc, const int* __restrict__ orig, const float4* __restrict__ pos4,
                           const float4* __restrict__ F4, float4* __restrict__ vel4, float* __restrict__ Ki,
                           int* __restrict__ flags, long long* __restrict__ counters) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    if (flags[kFlagRebuild]) counters[1] += 1;
    counters[0] += 1;
    flags[kFlagRebuild] = 0;
  }
  if (p >= n_slots) return;
  const int i = orig[p];
  if (i < 0) return;
  const int z = __float_as_int(pos4[p].w);
  const float4 f = F4[p];
  float4 v = vel4[p];
  v.x = fmaf(mc.acc[z], f.x, v.x);
  v.y = fmaf(mc.acc[z], f.y, v.y);
  v.z = fmaf(mc.acc[z], f.z, v.z);
  vel4[p] = v;
  Ki[i] = mc.kin[z] * (v.x * v.x + v.y * v.y + v.z * v.z);
}

__global__ void k_md_kin(int64_t n_slots, MdConst mc, const int* __restrict__ orig, const float4* __restrict__ pos4,
                         const float4* __restrict__ vel4, float* __restrict__ Ki) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  const int i = orig[p];
  if (i < 0) return;
  const float4 v = vel4[p];
  Ki[i] = mc.kin[__float_as_int(pos4[p].w)] * (v.x * v.x + v.y * v.y + v.z * v.z);
}

__global__ void k_md_export(int64_t n_slots, const int* __restrict__ orig, const Dbl3* __restrict__ xd,
                            const float4* __restrict__ vel4, const float4* __restrict__ F4, float* __restrict__ x,
                            float* __restrict__ v, float* __restrict__ f) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots) return;
  const int i = orig[p];
  if (i < 0) return;
  if (x) {
    x[3 * (int64_t)i + 0] = (float)xd[p].x;
    x[3 * (int64_t)i + 1] = (float)xd[p].y;
    x[3 * (int64_t)i + 2] = (float)xd[p].z;
  }
  if (v) {
    v[3 * (int64_t)i + 0] = vel4[p].x;
    v[3 * (int64_t)i + 1] = vel4[p].y;
    v[3 * (int64_t)i + 2] = vel4[p].z;
  }
  if (f) {
    f[3 * (int64_t)i + 0] = F4[p].x;
    f[3 * (int64_t)i + 1] = F4[p].y;
    f[3 * (int64_t)i + 2] = F4[p].z;
  }
}

// Initial state: caller-order float32 positions/velocities to the wrapped
// float64 caller-order copies the rebuild consumes.
__global__ void k_md_init(int64_t N, int n_cfg, const int64_t* __restrict__ atom_off, const CfgDev* __restrict__ cfgs,
                          const float* __restrict__ pos, const float* __restrict__ vel, Dbl3* __restrict__ xd_user,
                          float4* __restrict__ x_user, float4* __restrict__ v_user) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int lo = 0, hi = n_cfg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (atom_off[mid] <= i) lo = mid; else hi = mid;
  }
  double r[3] = {(double)pos[3 * i], (double)pos[3 * i + 1], (double)pos[3 * i + 2]};
  float f[3];
  wrap_periodic(cfgs[lo], r, f);
  xd_user[i] = Dbl3{r[0], r[1], r[2]};
  x_user[i] = make_float4(f[0], f[1], f[2], 0.f);
  v_user[i] = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace nepmi

using namespace nepmi;

struct nepmi_md {
  nepmi_model* m = nullptr;
  NbrPipeline nbr;
  Reducer red;
  MdConst mc{};
  int n_species = 0;
  DevBuf species_user, xd_user, x_user, v_user, xd, vel4, ref4, F4;
  DevBuf fp, aR, Ei, frad, fA, amask, Wi, Ki, Eproc;
  DevBuf epot, ekin, vir, counters;
  // checkpoint of the last checked step (caller order, wrapped positions), its
  // device counters, and a device word holding 1 (an always-open gate)
  DevBuf snap_xd, snap_x, snap_v, snap_cnt, one;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;     // the step
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_t = nullptr;   // the same step with the timing nodes
  hipGraphExec_t exec_t = nullptr;
  int64_t host_steps = 0;
  int64_t regrows = 0;
  // timing: events recorded before k_desc, k_force, k_gather and after
  // k_gather in every replay of exec_t; their graph nodes; a pool of
  // per-step events
  hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphNode_t tnode[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timing = false, mark_failed = false;
  std::vector<hipEvent_t> tpool;

  NepIO io() {
    NepIO o;
    o.n_slots = nbr.n_slots;
    o.capR = nbr.capR;
    o.capA = nbr.capA;
    o.pos4 = nbr.pos4.ptr<float4>();
    o.cfg_of = nbr.cfg_of.ptr<int>();
    o.orig = nbr.orig.ptr<int>();
    o.cfgs = nbr.cfgs.ptr<CfgDev>();
    o.nbrR = nbr.nbrR.ptr<uint32_t>();
    o.cntR = nbr.cntR.ptr<int>();
    o.vrev = nbr.vrev.ptr<uint32_t>();
    o.cnR = nbr.cnbrR.ptr<uint32_t>();
    o.ccR = nbr.ccntR.ptr<int>();
    o.cnA = nbr.cnbrA.ptr<uint32_t>();
    o.cpA = nbr.cposA.ptr<uint32_t>();
    o.ccA = nbr.ccntA.ptr<int>();
    o.flags = nbr.flags.ptr<int>();
    const float rcR = (float)m->hp.rc_radial, rcA = (float)m->hp.rc_angular;
    o.cut.rcR = rcR;
    o.cut.rcA = rcA;
    o.cut.rcR2 = rcR * rcR;
    o.cut.rcA2 = rcA * rcA;
    o.cut.rclR2 = nbr.rclR2;
    o.cut.rclA2 = nbr.rclA2;
    o.fp = fp.ptr<float>();
    o.aR = aR.ptr<float>();
    o.Ei = Ei.ptr<float>();
    o.qout = nullptr;
    o.frad = frad.ptr<float4>();
    o.fA = fA.ptr<float4>();
    o.amask = amask.ptr<uint64_t>();
    o.Wi = Wi.ptr<float>();
    o.Fuser = nullptr;
    o.Fproc = F4.ptr<float4>();
    o.Eproc = nullptr;
    return o;
  }

  // mark: while the step is being captured, put an event-record node for
  // tev[0..3] before k_desc, k_force, k_gather and after k_gather.  The nodes
  // are added to the capture by hand (current dependencies -> node -> new
  // dependency).  Best effort: if the runtime refuses, the step is captured
  // without them and timed replays are unavailable.
  void mark(int i, hipStream_t st) {
    if (mark_failed) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    hipGraphNode_t node = nullptr;
    if (hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd) != hipSuccess || cs != hipStreamCaptureStatusActive ||
        hipGraphAddEventRecordNode(&node, g, deps, nd, tev[i]) != hipSuccess ||
        hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies) != hipSuccess) {
      (void)hipGetLastError();
      mark_failed = true;
      return;
    }
    tnode[i] = node;
  }

  int forces(hipStream_t st, bool timed = false) {
    NepIO o = io();
    const float* P = m->params.ptr<float>();
    int rc;
    if (timed) mark(0, st);
    if ((rc = m->ops->desc(st, o, P, true, m->vdesc))) return rc;
    if (timed) mark(1, st);
    if ((rc = m->ops->force(st, o, P, m->vforce))) return rc;
    if (timed) mark(2, st);
    if ((rc = m->ops->gather(st, o, m->vgather))) return rc;
    if (timed) mark(3, st);
    return NEPMI_OK;
  }

  int rebuild(hipStream_t st, const int* gate) {
    const int64_t ns = nbr.n_slots;
    hipLaunchKernelGGL(k_md_unpermute, dim3(nb256(ns)), dim3(256), 0, st, ns, nbr.cfg_of.ptr<int>(),
                       nbr.orig.ptr<int>(), nbr.cfgs.ptr<CfgDev>(), xd.ptr<Dbl3>(), vel4.ptr<float4>(),
                       xd_user.ptr<Dbl3>(), x_user.ptr<float4>(), v_user.ptr<float4>(), nbr.cnt.ptr<int>(),
                       (int64_t)n_species * nbr.total_bins + 1, gate);
    return after_unpermute(st, gate, true);
  }

  // Sort and lists from the caller-order state; the sort moves the state into
  // the new slot order.  cnt_zeroed: the key counts are already clear.
  int after_unpermute(hipStream_t st, const int* gate, bool cnt_zeroed) {
    SlotCarry carry;
    carry.xd_user = reinterpret_cast<const double*>(xd_user.ptr<Dbl3>());
    carry.x_user = x_user.ptr<float4>();
    carry.v_user = v_user.ptr<float4>();
    carry.xd = reinterpret_cast<double*>(xd.ptr<Dbl3>());
    carry.vel4 = vel4.ptr<float4>();
    carry.ref4 = ref4.ptr<float4>();
    int rc;
    if ((rc = nbr.launch_sort(st, x_user.ptr<float>(), 4, species_user.ptr<int32_t>(), n_species, gate, cnt_zeroed,
                              &carry)))
      return rc;
    return nbr.launch_lists(st, n_species, gate);
  }

  int step_launch(hipStream_t st, bool timed) {
    const int64_t ns = nbr.n_slots;
    int* flags = nbr.flags.ptr<int>();
    hipLaunchKernelGGL(k_md_kick_drift, dim3(nb256(ns)), dim3(256), 0, st, ns, mc, nbr.cfg_of.ptr<int>(),
                       F4.ptr<float4>(), vel4.ptr<float4>(), xd.ptr<Dbl3>(), nbr.pos4.ptr<float4>(),
                       ref4.ptr<float4>(), flags);
    int rc;
    if ((rc = rebuild(st, flags + kFlagRebuild))) return rc;
    if ((rc = forces(st, timed))) return rc;
    hipLaunchKernelGGL(k_md_kick2, dim3(nb256(ns)), dim3(256), 0, st, ns, mc, nbr.orig.ptr<int>(),
                       nbr.pos4.ptr<float4>(), F4.ptr<float4>(), vel4.ptr<float4>(), Ki.ptr<float>(), flags,
                       counters.ptr<long long>());
    if ((rc = red.run(st, Ei.ptr<float>(), Wi.ptr<float>(), Ki.ptr<float>(), epot.ptr<double>(), vir.ptr<double>(),
                      ekin.ptr<double>())))
      return rc;
    NEPMI_HIP(hipGetLastError());
    return NEPMI_OK;
  }

  void drop_graphs() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (exec_t) (void)hipGraphExecDestroy(exec_t);
    if (graph_t) (void)hipGraphDestroy(graph_t);
    exec = exec_t = nullptr;
    graph = graph_t = nullptr;
  }

  int capture_one(bool timed, hipGraph_t& graph_out, hipGraphExec_t& exec_out) {
    NEPMI_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = step_launch(cap_stream, timed);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    graph_out = g;
    NEPMI_HIP(hipGraphInstantiate(&exec_out, g, nullptr, nullptr, 0));
    return NEPMI_OK;
  }

  // Capture one step into the graphs (replacing any earlier ones): the plain
  // step, and the step with event nodes around k_desc, k_force and k_gather
  // that timed runs replay on a sample of their steps.
  int capture() {
    drop_graphs();
    for (hipGraphNode_t& n : tnode) n = nullptr;
    mark_failed = false;
    int rc;
    if ((rc = capture_one(false, graph, exec)) || (rc = capture_one(true, graph_t, exec_t))) return rc;
    timing = !mark_failed && tnode[0] && tnode[1] && tnode[2] && tnode[3];
    return NEPMI_OK;
  }

  // Checkpoint the current state (caller order) and the step counters.
  int snapshot(hipStream_t st) {
    const int64_t ns = nbr.n_slots;
    hipLaunchKernelGGL(k_md_unpermute, dim3(nb256(ns)), dim3(256), 0, st, ns, nbr.cfg_of.ptr<int>(),
                       nbr.orig.ptr<int>(), nbr.cfgs.ptr<CfgDev>(), xd.ptr<Dbl3>(), vel4.ptr<float4>(),
                       snap_xd.ptr<Dbl3>(), snap_x.ptr<float4>(), snap_v.ptr<float4>(), nullptr, (int64_t)0,
                       one.ptr<int>());
    NEPMI_HIP(hipGetLastError());
    NEPMI_HIP(hipMemcpyAsync(snap_cnt.p, counters.p, 16, hipMemcpyDeviceToDevice, st));
    return NEPMI_OK;
  }

  // Back to the checkpoint with lists of capR x capA entries: the lists are
  // rebuilt from the checkpoint's positions, the forces and sums recomputed,
  // and the step re-captured (the list buffers may have moved).
  int restore(hipStream_t st, int capR, int capA) {
    int rc;
    const int64_t N = nbr.N, ns = nbr.n_slots;
    const size_t Na = (size_t)(N > 0 ? N : 1);
    int* flags = nbr.flags.ptr<int>();
    for (int attempt = 0;; ++attempt) {
      if ((rc = nbr.ensure_lists(capR, capA)) || (rc = amask.ensure(8 * (size_t)ns * ((nbr.capA + 63) / 64))) ||
          (rc = fA.ensure(16 * (size_t)ns * nbr.capA)))
        return rc;
      NEPMI_HIP(hipMemcpyAsync(xd_user.p, snap_xd.p, 24 * Na, hipMemcpyDeviceToDevice, st));
      NEPMI_HIP(hipMemcpyAsync(x_user.p, snap_x.p, 16 * Na, hipMemcpyDeviceToDevice, st));
      NEPMI_HIP(hipMemcpyAsync(v_user.p, snap_v.p, 16 * Na, hipMemcpyDeviceToDevice, st));
      NEPMI_HIP(hipMemcpyAsync(counters.p, snap_cnt.p, 16, hipMemcpyDeviceToDevice, st));
      fill_int(st, flags, kFlagCount, 0, nullptr);
      hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, flags + kFlagRebuild, 1);
      if ((rc = after_unpermute(st, flags + kFlagRebuild, false))) return rc;
      int hf[kFlagCount];
      if ((rc = nbr.check_flags(st, hf))) return rc;
      if (!hf[kFlagOverflow]) break;
      // the checkpoint itself needs longer lists than asked for
      if (attempt == 1) {
        set_error("neighbour capacity overflow after regrowing the lists");
        return NEPMI_NEIGHBOR_OVERFLOW;
      }
      capR = hf[kFlagMaxR] + hf[kFlagMaxR] / 4 + 16;
      capA = hf[kFlagMaxA] + hf[kFlagMaxA] / 4 + 16;
    }
    // the longest lists seen stay in the flags; the rebuild request is spent
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, flags + kFlagRebuild, 0);
    if ((rc = forces(st))) return rc;
    hipLaunchKernelGGL(k_md_kin, dim3(nb256(ns)), dim3(256), 0, st, ns, mc, nbr.orig.ptr<int>(),
                       nbr.pos4.ptr<float4>(), vel4.ptr<float4>(), Ki.ptr<float>());
    if ((rc = red.run(st, Ei.ptr<float>(), Wi.ptr<float>(), Ki.ptr<float>(), epot.ptr<double>(), vir.ptr<double>(),
                      ekin.ptr<double>())))
      return rc;
    NEPMI_HIP(hipStreamSynchronize(st));
    return capture();
  }

  ~nepmi_md() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : tev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : tpool)
      if (e) (void)hipEventDestroy(e);
  }
};

extern "C" {

int nepmi_md_create(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, const float* dev_pos,
                    const float* dev_vel, const int32_t* dev_species, const double* masses, double dt_fs, double skin,
                    nepmi_md** out, void* stream) {
  if (!m || !dev_pos || !dev_vel || !dev_species || !masses || !out || !(dt_fs > 0) || !(skin >= 0)) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  if (m->ops->T > kMaxSpecies) {
    set_error("too many species for the MD path");
    return NEPMI_UNSUPPORTED;
  }
  hipStream_t st = (hipStream_t)stream;
  nepmi_md* md = new (std::nothrow) nepmi_md();
  if (!md) return NEPMI_INVALID_ARG;
  md->m = m;
  md->n_species = m->ops->T;
  int rc = NEPMI_OK;
  auto fail = [&](int code) {
    delete md;
    return code;
  };
  for (int s = 0; s < md->n_species; ++s) {
    if (!(masses[s] > 0)) {
      set_error("masses must be positive");
      return fail(NEPMI_INVALID_ARG);
    }
    md->mc.acc[s] = (float)(0.5 * dt_fs * kAccUnit / masses[s]);
    md->mc.kin[s] = (float)(0.5 * masses[s] / kAccUnit);
  }
  md->mc.dt = (float)dt_fs;
  md->mc.half_skin2 = (float)(0.25 * skin * skin);
  NbrPipeline& nb = md->nbr;
  if ((rc = nb.setup(n_cfg, atom_off, cells, pbc, md->n_species, m->hp.rc_radial, m->hp.rc_angular, skin, st)))
    return fail(rc);
  if ((rc = md->red.setup(n_cfg, atom_off, st))) return fail(rc);
  const int64_t N = nb.N, ns = nb.n_slots;
  const size_t Na = (size_t)(N > 0 ? N : 1);
  if ((rc = md->species_user.ensure(4 * Na)) || (rc = md->xd_user.ensure(24 * Na)) ||
      (rc = md->x_user.ensure(16 * Na)) || (rc = md->v_user.ensure(16 * Na)) || (rc = md->xd.ensure(24 * (size_t)ns)) ||
      (rc = md->vel4.ensure(16 * (size_t)ns)) || (rc = md->ref4.ensure(16 * (size_t)ns)) ||
      (rc = md->F4.ensure(16 * (size_t)ns)) || (rc = md->fp.ensure(4 * (size_t)ns * m->ops->NANG)) ||
      (rc = md->aR.ensure(4 * (size_t)ns * m->ops->T * m->ops->BR)) || (rc = md->Ei.ensure(4 * Na)) ||
      (rc = md->frad.ensure(16 * (size_t)ns)) || (rc = md->Wi.ensure(36 * Na)) || (rc = md->Ki.ensure(4 * Na)) ||
      (rc = md->epot.ensure(8 * (size_t)n_cfg)) || (rc = md->ekin.ensure(8 * (size_t)n_cfg)) ||
      (rc = md->vir.ensure(72 * (size_t)n_cfg)) || (rc = md->counters.ensure(16)) ||
      (rc = md->snap_xd.ensure(24 * Na)) || (rc = md->snap_x.ensure(16 * Na)) || (rc = md->snap_v.ensure(16 * Na)) ||
      (rc = md->snap_cnt.ensure(16)) || (rc = md->one.ensure(4)))
    return fail(rc);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, md->one.ptr<int>(), 1);
  if (hipMemcpyAsync(md->species_user.p, dev_species, 4 * (size_t)N, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(hip_fail(hipGetLastError(), "hipMemcpyAsync(species)"));
  hipLaunchKernelGGL(k_md_init, dim3(nb256(N > 0 ? N : 1)), dim3(256), 0, st, N, n_cfg, nb.atom_off_dev.ptr<int64_t>(),
                     nb.cfgs.ptr<CfgDev>(), dev_pos, dev_vel, md->xd_user.ptr<Dbl3>(), md->x_user.ptr<float4>(),
                     md->v_user.ptr<float4>());
  fill_int(st, nb.flags.ptr<int>(), kFlagCount, 0, nullptr);
  fill_int(st, md->counters.ptr<int>(), 4, 0, nullptr);
  // first build, with capacity growth and a margin for the density
  // fluctuations of the run
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, nb.flags.ptr<int>() + kFlagRebuild, 1);
  if ((rc = md->after_unpermute(st, nb.flags.ptr<int>() + kFlagRebuild, false))) return fail(rc);
  int hf[kFlagCount];
  if ((rc = nb.check_flags(st, hf))) return fail(rc);
  const int wantR = hf[kFlagMaxR] + hf[kFlagMaxR] / 4 + 16, wantA = hf[kFlagMaxA] + hf[kFlagMaxA] / 4 + 16;
  if (hf[kFlagOverflow] || nb.capR < wantR || nb.capA < wantA) {
    if ((rc = nb.ensure_lists(wantR > nb.capR ? wantR : nb.capR, wantA > nb.capA ? wantA : nb.capA))) return fail(rc);
    fill_int(st, nb.flags.ptr<int>(), kFlagCount, 0, nullptr);
    if ((rc = nb.launch_lists(st, md->n_species, nullptr))) return fail(rc);
    if ((rc = nb.check_flags(st, hf))) return fail(rc);
    if (hf[kFlagOverflow]) {
      set_error("neighbour capacity overflow");
      return fail(NEPMI_NEIGHBOR_OVERFLOW);
    }
  }
  if (hf[kFlagAsym]) {
    set_error("angular neighbour list is not symmetric");
    return fail(NEPMI_INVALID_ARG);
  }
  if ((rc = md->amask.ensure(8 * (size_t)ns * ((nb.capA + 63) / 64))) || (rc = md->fA.ensure(16 * (size_t)ns * nb.capA)))
    return fail(rc);
  // the longest lists seen stay in the flags; the rebuild request is spent
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, nb.flags.ptr<int>() + kFlagRebuild, 0);
  // kernel variants timed on this state, then the forces of the initial state
  if (!m->pinned && (rc = autotune_io(m, md->io(), st, 4))) return fail(rc);
  if ((rc = md->forces(st))) return fail(rc);
  hipLaunchKernelGGL(k_md_kin, dim3(nb256(ns)), dim3(256), 0, st, ns, md->mc, nb.orig.ptr<int>(), nb.pos4.ptr<float4>(),
                     md->vel4.ptr<float4>(), md->Ki.ptr<float>());
  if ((rc = md->red.run(st, md->Ei.ptr<float>(), md->Wi.ptr<float>(), md->Ki.ptr<float>(), md->epot.ptr<double>(),
                        md->vir.ptr<double>(), md->ekin.ptr<double>())))
    return fail(rc);
  if (hipStreamSynchronize(st) != hipSuccess) return fail(hip_fail(hipGetLastError(), "hipStreamSynchronize"));
  // capture one step
  for (int i = 0; i < 4; ++i)
    if (hipEventCreate(&md->tev[i]) != hipSuccess) return fail(hip_fail(hipGetLastError(), "hipEventCreate"));
  if (hipStreamCreateWithFlags(&md->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(hip_fail(hipGetLastError(), "hipStreamCreate"));
  if ((rc = md->capture())) return fail(rc);
  if (hipStreamSynchronize(st) != hipSuccess) return fail(hip_fail(hipGetLastError(), "hipStreamSynchronize"));
  *out = md;
  return NEPMI_OK;
}

// Steps between overflow checks.  Every chunk of this many graph replays ends
// with one stream synchronisation and a read of the device flags; a chunk in
// which a list build overflowed its capacity is undone (back to the
// checkpoint taken before it) and run again with larger lists.
constexpr int kMdCheckEvery = 32;
constexpr int kMdMaxRegrows = 3;

// Timed runs replay the graph with the event nodes on every kTimedEvery-th
// step (the first of each group) and the plain graph on the others: the
// kernel durations are averages over those steps, and the event nodes (a few
// microseconds each) stay out of most of the steps that the run times.
constexpr int kTimedEvery = 4;

// Advance n_steps replays with overflow recovery; with `ms`, the timed graph's
// event nodes record into per-step events and ms[0..2] get the average
// durations over the steps that ran it.
static int md_run(nepmi_md* md, int32_t n_steps, hipStream_t st, double* ms) {
  if (ms) {
    const size_t need = 4 * (size_t)n_steps;
    while (md->tpool.size() < need) {
      hipEvent_t e;
      NEPMI_HIP(hipEventCreate(&e));
      md->tpool.push_back(e);
    }
  }
  int rc;
  if ((rc = md->snapshot(st))) return rc;
  int done = 0, regrown = 0;
  while (done < n_steps) {
    const int k = n_steps - done < kMdCheckEvery ? n_steps - done : kMdCheckEvery;
    if (ms && !md->timing) {
      set_error("the step graph has no timing nodes");
      return NEPMI_UNSUPPORTED;
    }
    for (int s = done; s < done + k; ++s) {
      if (ms && s % kTimedEvery == 0) {
        // every launch is enqueued before the next change of its event nodes,
        // so each timed step records into its own four events
        for (int i = 0; i < 4; ++i)
          NEPMI_HIP(hipGraphExecEventRecordNodeSetEvent(md->exec_t, md->tnode[i], md->tpool[4 * (size_t)s + i]));
        NEPMI_HIP(hipGraphLaunch(md->exec_t, st));
      } else {
        NEPMI_HIP(hipGraphLaunch(md->exec, st));
      }
    }
    int hf[kFlagCount];
    if ((rc = md->nbr.check_flags(st, hf))) return rc;
    if (hf[kFlagOverflow]) {
      // a list build in this chunk truncated a list: undo the chunk, grow the
      // lists to the longest seen plus a margin and run the chunk again
      if (++regrown > kMdMaxRegrows) {
        set_error("neighbour capacity exceeded during MD after regrowing the lists");
        return NEPMI_NEIGHBOR_OVERFLOW;
      }
      const int wantR = hf[kFlagMaxR] + hf[kFlagMaxR] / 4 + 16, wantA = hf[kFlagMaxA] + hf[kFlagMaxA] / 4 + 16;
      if ((rc = md->restore(st, wantR > md->nbr.capR ? wantR : md->nbr.capR,
                            wantA > md->nbr.capA ? wantA : md->nbr.capA)))
        return rc;
      ++md->regrows;
      continue;
    }
    if (hf[kFlagAsym]) {
      set_error("angular neighbour list is not symmetric");
      return NEPMI_INVALID_ARG;
    }
    done += k;
    md->host_steps += k;
    if (done < n_steps && (rc = md->snapshot(st))) return rc;
  }
  if (ms) {
    double acc[3] = {0, 0, 0};
    int n_timed = 0;
    rc = NEPMI_OK;
    for (int s = 0; s < n_steps && !rc; s += kTimedEvery, ++n_timed)
      for (int i = 0; i < 3; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, md->tpool[4 * (size_t)s + i], md->tpool[4 * (size_t)s + i + 1]) != hipSuccess) {
          rc = hip_fail(hipGetLastError(), "hipEventElapsedTime");
          break;
        }
        acc[i] += t;
      }
    for (int i = 0; i < 4; ++i) (void)hipGraphExecEventRecordNodeSetEvent(md->exec_t, md->tnode[i], md->tev[i]);
    if (rc) return rc;
    for (int i = 0; i < 3; ++i) ms[i] = acc[i] / n_timed;
  }
  return NEPMI_OK;
}

int nepmi_md_step_timed(nepmi_md* md, int32_t n_steps, double* ms, void* stream) {
  if (!md || n_steps < 1 || !ms) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  return md_run(md, n_steps, (hipStream_t)stream, ms);
}

int nepmi_md_step(nepmi_md* md, int32_t n_steps, void* stream) {
  if (!md || n_steps < 0) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  return md_run(md, n_steps, (hipStream_t)stream, nullptr);
}

int nepmi_md_capacity(nepmi_md* md, int32_t capR, int32_t capA, int32_t* cur_capR, int32_t* cur_capA) {
  if (!md || capR < 0 || capA < 0) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  if (capR > 0 || capA > 0) {
    // never below the longest lists of the builds so far
    int hf[kFlagCount];
    int rc;
    if ((rc = md->nbr.check_flags(0, hf))) return rc;
    int r = capR > 0 ? capR : md->nbr.capR, a = capA > 0 ? capA : md->nbr.capA;
    r = r > hf[kFlagMaxR] ? r : hf[kFlagMaxR];
    a = a > hf[kFlagMaxA] ? a : hf[kFlagMaxA];
    // the lists of the new shape are built from the current state
    if ((rc = md->snapshot(0)) || (rc = md->restore(0, r, a))) return rc;
  }
  if (cur_capR) *cur_capR = md->nbr.capR;
  if (cur_capA) *cur_capA = md->nbr.capA;
  return NEPMI_OK;
}

int nepmi_md_get(nepmi_md* md, float* dev_pos, float* dev_vel, float* dev_forces, double* dev_epot, double* dev_ekin,
                 double* dev_virial, void* stream) {
  if (!md) {
    set_error("null handle");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t ns = md->nbr.n_slots;
  if (dev_pos || dev_vel || dev_forces)
    hipLaunchKernelGGL(k_md_export, dim3(nb256(ns)), dim3(256), 0, st, ns, md->nbr.orig.ptr<int>(),
                       md->xd.ptr<Dbl3>(), md->vel4.ptr<float4>(), md->F4.ptr<float4>(), dev_pos, dev_vel, dev_forces);
  const size_t nc = (size_t)md->nbr.n_cfg;
  if (dev_epot) NEPMI_HIP(hipMemcpyAsync(dev_epot, md->epot.p, 8 * nc, hipMemcpyDeviceToDevice, st));
  if (dev_ekin) NEPMI_HIP(hipMemcpyAsync(dev_ekin, md->ekin.p, 8 * nc, hipMemcpyDeviceToDevice, st));
  if (dev_virial) NEPMI_HIP(hipMemcpyAsync(dev_virial, md->vir.p, 72 * nc, hipMemcpyDeviceToDevice, st));
  NEPMI_HIP(hipGetLastError());
  return NEPMI_OK;
}

int nepmi_md_stats(nepmi_md* md, int64_t* steps, int64_t* rebuilds, int64_t* regrows) {
  if (!md) return NEPMI_INVALID_ARG;
  long long c[2];
  NEPMI_HIP(hipMemcpy(c, md->counters.p, sizeof c, hipMemcpyDeviceToHost));
  if (steps) *steps = c[0];
  if (rebuilds) *rebuilds = c[1] + 1;  // plus the build at creation
  if (regrows) *regrows = md->regrows;
  return NEPMI_OK;
}

void nepmi_md_destroy(nepmi_md* md) { delete md; }

int nepmi_md_time_kernels(nepmi_md* md, int32_t reps, double* ms, void* stream) {
  if (!md || reps < 1 || !ms) {
    set_error("invalid argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[8];
  for (int k = 0; k < 8; ++k) NEPMI_HIP(hipEventCreate(&ev[k]));
  double acc[4] = {0, 0, 0, 0};
  NepIO o = md->io();
  const float* P = md->m->params.ptr<float>();
  int rc = NEPMI_OK;
  for (int r = 0; r < reps && !rc; ++r) {
    NEPMI_HIP(hipEventRecord(ev[0], st));
    rc = md->m->ops->desc(st, o, P, true, md->m->vdesc);
    NEPMI_HIP(hipEventRecord(ev[1], st));
    if (!rc) rc = md->m->ops->force(st, o, P, md->m->vforce);
    NEPMI_HIP(hipEventRecord(ev[2], st));
    if (!rc) rc = md->m->ops->gather(st, o, md->m->vgather);
    NEPMI_HIP(hipEventRecord(ev[3], st));
    // a full list rebuild on the current state (sort + lists)
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, md->nbr.flags.ptr<int>() + kFlagRebuild, 1);
    NEPMI_HIP(hipEventRecord(ev[4], st));
    if (!rc) rc = md->rebuild(st, md->nbr.flags.ptr<int>() + kFlagRebuild);
    NEPMI_HIP(hipEventRecord(ev[5], st));
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, md->nbr.flags.ptr<int>() + kFlagRebuild, 0);
    NEPMI_HIP(hipStreamSynchronize(st));
    float t;
    for (int k = 0; k < 3; ++k) {
      NEPMI_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      acc[k] += t;
    }
    NEPMI_HIP(hipEventElapsedTime(&t, ev[4], ev[5]));
    acc[3] += t;
  }
  // forces of the rebuilt state, so the next step starts consistent
  if (!rc) rc = md->forces(st);
  NEPMI_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < 8; ++k) (void)hipEventDestroy(ev[k]);
  for (int k = 0; k < 4; ++k) ms[k] = acc[k] / reps;
  return rc;
}

}  // extern "C"
