// tune.hip -- choice of kernel variants by timing them on real inputs.
//
// k_desc and k_force are compiled in several variants (how many angular
// functions one pass over the pairs handles, and how many waves per SIMD the
// register allocation must leave room for; for k_desc also whether the
// network runs in it or in a kernel of its own).  The best one depends on the
// model shape and on the pair counts of the workload, so it is measured:
// every variant runs on the caller's batch (or MD state) with HIP events
// around it, and the fastest is kept in the model handle.
#include "model.hpp"

namespace nepmi {

int autotune_io(nepmi_model* m, const NepIO& io, hipStream_t st, int reps) {
  const float* P = m->params.ptr<float>();
  hipEvent_t e0, e1;
  NEPMI_HIP(hipEventCreate(&e0));
  NEPMI_HIP(hipEventCreate(&e1));
  int rc = NEPMI_OK;
  double best = 1e300;
  int bd = m->vdesc, bf = m->vforce;
  for (int v = 0; v < kDescVariants && !rc; ++v) {
    rc = m->ops->desc(st, io, P, true, v);  // warm-up (also code-object load)
    double t = 0.0;
    for (int r = 0; r < reps && !rc; ++r) {
      NEPMI_HIP(hipEventRecord(e0, st));
      rc = m->ops->desc(st, io, P, true, v);
      NEPMI_HIP(hipEventRecord(e1, st));
      NEPMI_HIP(hipEventSynchronize(e1));
      float ms;
      NEPMI_HIP(hipEventElapsedTime(&ms, e0, e1));
      t += ms;
    }
    if (t < best) {
      best = t;
      bd = v;
    }
  }
  if (!rc) rc = m->ops->desc(st, io, P, true, bd);
  best = 1e300;
  for (int v = 0; v < kForceVariants && !rc; ++v) {
    rc = m->ops->force(st, io, P, v);
    double t = 0.0;
    for (int r = 0; r < reps && !rc; ++r) {
      NEPMI_HIP(hipEventRecord(e0, st));
      rc = m->ops->force(st, io, P, v);
      NEPMI_HIP(hipEventRecord(e1, st));
      NEPMI_HIP(hipEventSynchronize(e1));
      float ms;
      NEPMI_HIP(hipEventElapsedTime(&ms, e0, e1));
      t += ms;
    }
    if (t < best) {
      best = t;
      bf = v;
    }
  }
  // gather block sizes, after the chosen force variant
  if (!rc) rc = m->ops->force(st, io, P, bf);
  int bg = m->vgather;
  best = 1e300;
  for (int v = 0; v < kGatherVariants && !rc; ++v) {
    rc = m->ops->gather(st, io, v);
    double t = 0.0;
    for (int r = 0; r < reps && !rc; ++r) {
      NEPMI_HIP(hipEventRecord(e0, st));
      rc = m->ops->gather(st, io, v);
      NEPMI_HIP(hipEventRecord(e1, st));
      NEPMI_HIP(hipEventSynchronize(e1));
      float ms;
      NEPMI_HIP(hipEventElapsedTime(&ms, e0, e1));
      t += ms;
    }
    if (t < best) {
      best = t;
      bg = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  m->vdesc = bd;
  m->vforce = bf;
  m->vgather = bg;
  // leave the outputs of the chosen variants behind
  if ((rc = m->ops->gather(st, io, bg))) return rc;
  return NEPMI_OK;
}

}  // namespace nepmi

using namespace nepmi;

extern "C" {

int nepmi_autotune(nepmi_model* m, int32_t n_cfg, const int64_t* atom_off, const double* cells, const int32_t* pbc, const float* dev_pos,
                   const int32_t* dev_species, int32_t* chosen, void* stream) {
  if (!m || !dev_pos || !dev_species) {
    set_error("null argument");
    return NEPMI_INVALID_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int rc = m->prepare(n_cfg, atom_off, cells, pbc, dev_pos, dev_species, st);
  if (rc) return rc;
  if ((rc = autotune_io(m, m->io(nullptr, nullptr, nullptr), st, 4))) return rc;
  if (chosen) {
    chosen[0] = m->vdesc;
    chosen[1] = m->vforce;
  }
  return NEPMI_OK;
}

int nepmi_set_gather_variant(nepmi_model* m, int32_t variant) {
  if (!m || variant < 0 || variant >= kGatherVariants) {
    set_error("variant out of range");
    return NEPMI_INVALID_ARG;
  }
  m->vgather = variant;
  m->pinned = true;
  return NEPMI_OK;
}

int nepmi_get_gather_variant(nepmi_model* m, int32_t* variant) {
  if (!m) return NEPMI_INVALID_ARG;
  if (variant) *variant = m->vgather;
  return NEPMI_OK;
}

int nepmi_set_variants(nepmi_model* m, int32_t desc_variant, int32_t force_variant) {
  if (!m || desc_variant < 0 || desc_variant >= kDescVariants || force_variant < 0 ||
      force_variant >= kForceVariants) {
    set_error("variant out of range");
    return NEPMI_INVALID_ARG;
  }
  m->vdesc = desc_variant;
  m->vforce = force_variant;
  m->pinned = true;
  return NEPMI_OK;
}

int nepmi_get_variants(nepmi_model* m, int32_t* desc_variant, int32_t* force_variant) {
  if (!m) return NEPMI_INVALID_ARG;
  if (desc_variant) *desc_variant = m->vdesc;
  if (force_variant) *force_variant = m->vforce;
  return NEPMI_OK;
}

}  // extern "C"
