/*
 * nepmi.h -- C ABI of the MI355X (gfx950) NEP evaluation library.
 *
 * The library evaluates a neuroevolution potential (NEP) as stated in the
 * AI2Pot paper, Sec. 2: the total energy is a sum of site energies (Eq. 1),
 * each the output of a per-element one-hidden-layer network (Sec. 2.3) on
 * radial descriptors (Eq. 11-15) and angular descriptors (Eq. 16-17, plus
 * 4-body and 5-body invariants); forces follow Eq. 3 and the virial Eq. 4.
 * A loss of the form of Eq. 18-21 and its gradient with respect to every
 * parameter serve training (Sec. 3.2: one operator backend for training and
 * inference; Sec. 3.4: neighbour lists rebuilt on every training step).
 *
 * Conventions (every entry point):
 *   - Units: Angstrom, eV, eV/Angstrom, atomic mass units, femtoseconds.
 *   - Species are 0..n_species-1.  The cell's rows are its lattice vectors
 *     a, b, c (row-major double[9] per configuration); the pair vectors use
 *     the cell rounded to float32.
 *   - Periodicity: pbc is a host int32[3*n_cfg] (pbc[3c+a] = 1 if
 *     configuration c is periodic along lattice vector a, 0 if not) or NULL
 *     (periodic in all three directions).  Eq. 3-4 sum over the neighbours
 *     inside the cutoff: along a periodic direction these include periodic
 *     images, along a non-periodic one there are none (a cluster, a slab).
 *     Every periodic direction must be at least 2 * (rc_radial + skin) wide
 *     (NEPMI_CELL_TOO_SMALL); a non-periodic one may have any width, and an
 *     atom may lie outside the cell along it (it is not wrapped; its list
 *     search then starts from the nearest bin of the cell).  Entries other
 *     than 0 and 1 give NEPMI_INVALID_ARG.
 *   - Positions and forces are float32, array-of-structs (N x 3, row-major),
 *     in the caller's atom order; configuration c owns atoms
 *     [atom_off[c], atom_off[c+1]).  A configuration may be empty (its E and
 *     V are 0); a batch with no atoms at all gives NEPMI_INVALID_ARG.
 *   - The virial is V_ab = - sum_i sum_j dE_i/dr_ij,a r_ij,b in eV (Eq. 4),
 *     not divided by the volume.
 *   - Arithmetic: float32 for descriptors, network and pair forces; float64
 *     for energy, virial and loss sums.
 *   - Pointers named dev_* are device pointers the caller owns (for example
 *     torch tensors) and that stay valid for the duration of the call, which
 *     is asynchronous on `stream` (a hipStream_t; NULL = default stream) unless
 *     stated.  Host pointers (atom_off, cells, pbc, masses, weights) are read
 *     before the call returns.  The library keeps no caller pointer past a
 *     call; handles own their workspace, which grows on demand.
 *   - Every call returns NEPMI_OK (0) or a negative code; nepmi_last_error()
 *     gives a message for the calling thread.  No C++ exception crosses the
 *     ABI.  A handle must not be used from two threads or streams at once.
 */
#ifndef NEPMI_H
#define NEPMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NEPMI_OK = 0,
  NEPMI_INVALID_ARG = -1,       /* bad size, pointer, species or hyper-parameter  */
  NEPMI_CELL_TOO_SMALL = -2,    /* a periodic width below 2 * (rc_radial + skin)  */
  NEPMI_NEIGHBOR_OVERFLOW = -3, /* neighbour capacity exceeded (MD only; compute
                                   calls grow the capacity and retry)            */
  NEPMI_HIP_ERROR = -4,         /* a HIP runtime call failed                      */
  NEPMI_NAN_DETECTED = -5,      /* a non-finite position was given               */
  NEPMI_UNSUPPORTED = -6        /* hyper-parameters with no compiled kernel set   */
};

/* Hyper-parameters, named as in Sec. 2.3: n_radial = n_max^radial and
 * n_angular = n_max^angular (counts of functions, n = 0..n-1); basis_* =
 * N_basis (Chebyshev orders 0..N_basis-1); l_max: the three-body term uses
 * l = 1..l_max; use_4body / use_5body add n_angular invariants each;
 * n_hidden = N_neurons; rc_* = r_max of the radial and angular terms
 * (rc_angular <= rc_radial). */
typedef struct {
  int32_t n_species, n_radial, n_angular, basis_radial, basis_angular;
  int32_t l_max, use_4body, use_5body, n_hidden, reserved;
  double rc_radial, rc_angular;
} nepmi_hparams;

typedef struct nepmi_model nepmi_model;
typedef struct nepmi_md nepmi_md;

/* Message of the last failed call on this thread ("" if none). */
const char *nepmi_last_error(void);

/* Number of trainable parameters (7899 for the model of Table 2). */
int nepmi_param_count(const nepmi_hparams *hp, int64_t *out);

/* Descriptor length D = n_radial + l_max n_angular (+ n_angular for each of
 * the 4-body and 5-body terms). */
int nepmi_descriptor_dim(const nepmi_hparams *hp, int32_t *out);

/* Create a model handle on the current HIP device.  NEPMI_UNSUPPORTED if the
 * hyper-parameters have no compiled kernel set (see nepmi_supported). */
int nepmi_model_create(const nepmi_hparams *hp, nepmi_model **out);

/* 1 if kernels for these hyper-parameters are compiled in, else 0. */
int nepmi_supported(const nepmi_hparams *hp);

/* Copy the flat float32 parameter vector (device memory, param_count values)
 * into the model.  Layout: [c_R: T*T*n_radial*basis_radial, order (Z_i, Z_j,
 * n, k)] [c_A: T*T*n_angular*basis_angular] then for each species s:
 * [W0: n_hidden x D row-major] [b0: n_hidden] [w1: n_hidden] [b1: 1].
 * The site energy is E_i = w1 . tanh(W0 q_i + b0) + b1 (Sec. 2.3). */
int nepmi_model_set_params(nepmi_model *m, const float *dev_params, void *stream);

/* Keep neighbour lists between calls on a fixed batch (off by default).
 * When enabled, a call of nepmi_compute, nepmi_descriptors, nepmi_neighbors,
 * nepmi_backward_params, nepmi_loss_grad or nepmi_autotune whose batch is
 * the previous such call's batch (same n_cfg, atom_off and cells, and the
 * same device addresses of positions and species) keeps the neighbour lists,
 * processing order and reduction plan of that call instead of rebuilding
 * them.  The caller guarantees that the positions and species at those
 * addresses have not changed, as for a training set of fixed configurations
 * (Sec. 3.3).  The float64 variant always rebuilds.  Enabling or disabling
 * clears what is kept.  NEPMI_INVALID_ARG on a null model. */
int nepmi_model_reuse_lists(nepmi_model *m, int32_t enable);

void nepmi_model_destroy(nepmi_model *m);

/* Energy, forces and virial of n_cfg configurations (Eq. 1, 3, 4).
 *   atom_off: host int64[n_cfg+1]; cells: host double[9*n_cfg]; pbc: host
 *   int32[3*n_cfg] or NULL (see the conventions above);
 *   dev_pos: float[N*3]; dev_species: int32[N];
 *   dev_energy: double[n_cfg]; dev_forces: float[N*3]; dev_virial:
 *   double[9*n_cfg]; dev_atom_energy: float[N] or NULL; dev_atom_virial:
 *   float[N*9] or NULL (row-major 3x3 per atom, -sum_j dE_i/dr_ij (x) r_ij).
 * Synchronises `stream` once to check the neighbour capacity (twice when the
 * lists must grow); the rest of the call is asynchronous. */
int nepmi_compute(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                  const float *dev_pos, const int32_t *dev_species, double *dev_energy, float *dev_forces,
                  double *dev_virial, float *dev_atom_energy, float *dev_atom_virial, void *stream);

/* Allocation-free variant of nepmi_compute, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as
 * nepmi_compute; neighbour lists are rebuilt on every call.  Every work
 * buffer (neighbour lists, processing order, per-atom arrays, reduction plan)
 * is carved from one static device array of 64 MiB per GPU, which each GPU
 * the library runs on holds until the process ends; no hipMalloc or hipFree
 * is called (the model's parameters were allocated by nepmi_model_create).
 * A batch whose work space exceeds 64 MiB (about 2.1 kB per atom with the
 * three-species Ge-Sb-Te model: some 30,000 atoms) returns NEPMI_INVALID_ARG.
 * All calls on one GPU share that array and it keeps the last call's
 * contents: calls that overlap on one GPU (from other streams or threads)
 * race and must not be made. */
int nepmi_compute_noalloc(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                          const float *dev_pos, const int32_t *dev_species, double *dev_energy, float *dev_forces,
                          double *dev_virial, float *dev_atom_energy, float *dev_atom_virial, void *stream);

/* Descriptors q_i (float[N*D], caller's atom order) of the same batch: the
 * radial q_n (Eq. 11), three-body q_nl (Eq. 17, l = 1..l_max, index
 * n_radial + (l-1) n_angular + n), then the 4-body and 5-body values. */
int nepmi_descriptors(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                      const float *dev_pos, const int32_t *dev_species, float *dev_q, void *stream);

/* Neighbour lists of the same batch, for inspection and tests.  which = 0:
 * radial list (pairs closer than rc_radial), 1: angular list (rc_angular).
 * For caller atom i, dev_count[i] (int32[N]) neighbours are written to
 * dev_nbr[i*cap + k] (int32, caller index of the neighbour) and
 * dev_rvec[(i*cap + k)*3 + a] (float32, r_ij = r_j - r_i + image shift);
 * entries beyond cap are dropped (dev_count still reports the full length).
 * The list order is the library's evaluation order.  which = 2: the angular
 * part of the library's own list (the entries within rc_angular, in the
 * order the force gather indexes them), written the same way.  which = 3: for
 * the same entries, dev_nbr receives the reverse index instead of the
 * neighbour (the position of atom i in the angular part of its neighbour's
 * list, or a negative value where no partner entry was found) and dev_rvec
 * the pair vector of the entry. */
int nepmi_neighbors(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                    const float *dev_pos, const int32_t *dev_species, int32_t which, int32_t cap,
                    int32_t *dev_count, int32_t *dev_nbr, float *dev_rvec, void *stream);

/* Kernel variants.  The descriptor and pair-force kernels are compiled in
 * several variants: angular functions handled per pass over the pairs, the
 * register budget they keep to, the block size (256 threads unless stated),
 * and for the descriptors whether the network runs in the same kernel or in
 * one of its own on dense 16x16x4 matrix products.  Descriptor variants:
 * 0..3 network in the kernel, 4..7 network apart, 8 and 9 variant 0 in
 * blocks of 128 and 512 threads.  Force variants: 0..3, and 4 and 5 variant 0
 * in blocks of 128 and 512.  The gather runs in blocks of 256, 128, 512 or
 * 1024 threads (gather variants 0..3).  All compute the same result:
 * descriptors bitwise across descriptor variants, energies bitwise within
 * each network form and up to float32 summation order across them, forces
 * up to float32 summation order across force variants and bitwise across
 * gather variants.  nepmi_autotune times every variant on the given batch
 * and keeps the fastest in the model; chosen = host int32[2] (descriptor,
 * force) or NULL.  Synchronises `stream`.  nepmi_set_variants and
 * nepmi_set_gather_variant pin a choice; nepmi_md_create autotunes on its
 * initial state unless a choice is pinned. */
int nepmi_autotune(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                   const float *dev_pos, const int32_t *dev_species, int32_t *chosen, void *stream);
int nepmi_set_variants(nepmi_model *m, int32_t desc_variant, int32_t force_variant);
int nepmi_get_variants(nepmi_model *m, int32_t *desc_variant, int32_t *force_variant);
int nepmi_set_gather_variant(nepmi_model *m, int32_t gather_variant);
int nepmi_get_gather_variant(nepmi_model *m, int32_t *gather_variant);

/* Vector-Jacobian product of (E, F, V) with respect to the parameters:
 *   dev_grad[p] = sum_c ebar_c dE_c/dtheta_p + sum_i lambda_i . dF_i/dtheta_p
 *               + sum_c mu_c : dV_c/dtheta_p
 * with dev_ebar double[n_cfg], dev_lambda float[N*3], dev_mu double[9*n_cfg];
 * dev_grad float[param_count] is overwritten.  The neighbour lists and
 * forward state are rebuilt for the batch given; descriptors are recomputed,
 * no per-pair state is cached. */
int nepmi_backward_params(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                          const float *dev_pos, const int32_t *dev_species, const double *dev_ebar,
                          const float *dev_lambda, const double *dev_mu, float *dev_grad, void *stream);

/* Loss of Eq. 18-21 and its parameter gradient in one call (forward, loss,
 * adjoint seeds, backward).  weights = host double[3] (w_E, w_F, w_V).
 * loss_form 0: L = w_E/B sum_c ((E_c - Eref_c)/N_c)^2
 *                + w_F/(3 sum_c N_c) sum_{c,i,a} (F - Fref)^2
 *                + w_V/(9B) sum_c sum_ab ((V_c - Vref_c)/N_c)^2;
 * loss_form 1: L = 1/B sum_c [w_E/N_c dE^2 + w_F/(3N_c) sum dF^2 + w_V/(9N_c) sum dV^2]
 * (Eq. 19-21 per configuration, averaged over the batch).
 * dev_E_ref double[n_cfg], dev_F_ref float[N*3], dev_V_ref double[9*n_cfg];
 * dev_loss double[4] = (total, energy, force, virial); dev_grad float[P] or
 * NULL (loss only). */
int nepmi_loss_grad(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                    const float *dev_pos, const int32_t *dev_species, const double *dev_E_ref,
                    const float *dev_F_ref, const double *dev_V_ref, const double *weights, int32_t loss_form,
                    double *dev_loss, float *dev_grad, void *stream);

/* Velocity-Verlet NVE molecular dynamics of n_cfg independent cells stepped
 * together (one time step for all).  The handle copies positions, velocities
 * (float[N*3], Angstrom/fs) and species; masses: host double[n_species] (u);
 * dt_fs: time step; skin: Verlet-list skin in Angstrom (lists are rebuilt
 * when an atom has moved more than skin/2 since the last build).  Positions
 * are wrapped into the cell along its periodic directions at each rebuild
 * (pbc as for nepmi_compute).  The step (half kick, drift,
 * displacement check, conditional rebuild, forces, half kick, float64
 * energy/virial/kinetic sums) is captured once in a HIP graph and replayed. */
int nepmi_md_create(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                    const float *dev_pos, const float *dev_vel, const int32_t *dev_species, const double *masses,
                    double dt_fs, double skin, nepmi_md **out, void *stream);

/* Advance n_steps time steps (graph replays) on `stream`.  The replays run in
 * chunks of 32 steps; after each chunk the call synchronises `stream` and
 * reads the device flags.  Before each chunk the state (positions, velocities,
 * step counters) is checkpointed on the device.  If a list build inside a
 * chunk needed more entries than the lists hold, the chunk is undone: the
 * checkpoint is restored, the lists are regrown to 1.25x the longest list seen
 * plus 16, rebuilt, the step graph re-captured and the chunk run again (the
 * trajectory is the same up to float32 summation order).  Returns
 * NEPMI_NEIGHBOR_OVERFLOW only if three regrows within one call do not
 * suffice, or if a list would exceed 65535 entries; the state is then the
 * last checkpoint.  Returns when the n_steps are done (stream synchronised). */
int nepmi_md_step(nepmi_md *md, int32_t n_steps, void *stream);

/* List capacities of the run.  capR, capA > 0 set the radial / angular list
 * capacity (entries per atom; raised to the longest list built so far, and 0
 * keeps the current value); the lists are rebuilt from the current state and
 * the step graph re-captured.  cur_capR, cur_capA (host, may be NULL) receive
 * the capacities in force.  Synchronises the null stream. */
int nepmi_md_capacity(nepmi_md *md, int32_t capR, int32_t capA, int32_t *cur_capR, int32_t *cur_capA);

/* Copy the current state out (any pointer may be NULL): positions and
 * velocities float[N*3] and forces float[N*3] in the caller's atom order;
 * potential energy, kinetic energy double[n_cfg] and virial double[9*n_cfg]
 * of the last step. */
int nepmi_md_get(nepmi_md *md, float *dev_pos, float *dev_vel, float *dev_forces, double *dev_epot,
                 double *dev_ekin, double *dev_virial, void *stream);

/* Host counters (any pointer may be NULL): steps taken, neighbour-list
 * builds (including the first) and list regrows after an overflow. */
int nepmi_md_stats(nepmi_md *md, int64_t *steps, int64_t *rebuilds, int64_t *regrows);

void nepmi_md_destroy(nepmi_md *md);

/* Advance n_steps (>= 1) like nepmi_md_step and time the hot kernels of
 * these steps: steps 0, 4, 8, ... of the call replay a copy of the step graph
 * that records HIP events before k_desc, k_force and k_gather and after
 * k_gather, each step into its own events; the other steps replay the plain
 * graph (the event nodes cost a few microseconds each).  ms_per_launch: host
 * double[3] = average duration (ms) of descriptors + network, pair forces +
 * virial, force gather over the timed replays.  Chunks, checkpoints and
 * overflow recovery as nepmi_md_step (a chunk run again records its steps
 * again).  Errors as nepmi_md_step, and NEPMI_UNSUPPORTED if the graph could
 * not be built with timing nodes. */
int nepmi_md_step_timed(nepmi_md *md, int32_t n_steps, double *ms_per_launch, void *stream);

/* Average duration of each hot kernel, measured with HIP events recorded on
 * `stream` around `reps` standalone launches of the force evaluation on the
 * current MD state (the same kernels and launch shapes the graph replays).
 * ms_per_launch: host double[4] = descriptors + network, pair forces +
 * virial, force gather, neighbour-list build.  Synchronises `stream`. */
int nepmi_md_time_kernels(nepmi_md *md, int32_t reps, double *ms_per_launch, void *stream);

/* ---------------------------------------------------------------------------
 * Float64 variant (Sec. 3.2: every operator exists in float32 and float64).
 *
 * Same quantities as nepmi_compute and nepmi_backward_params, with positions,
 * parameters and every result in float64 and all arithmetic in float64.
 * Parameters are passed per call (dev_params: device double[param_count], the
 * layout of nepmi_set_params), so a caller can differentiate with respect to
 * them; the model handle supplies the shape, the cutoffs and the work space.
 * Neighbour lists come from the float32 rounding of the positions with a
 * 0.01 A skin; every pair is then tested against the cutoffs in float64.
 * Periodic widths must be at least 2 (rc_radial + 0.01) (NEPMI_CELL_TOO_SMALL).
 * Asynchronous on `stream`.
 * ------------------------------------------------------------------------- */

/* Energy, forces and virial of a batch (Eq. 1-4) in float64.
 * atom_off host int64[n_cfg + 1], cells host double[9 * n_cfg] (rows a, b, c),
 * pbc host int32[3 * n_cfg] or NULL;
 * dev_pos double[N*3], dev_species int32[N] (caller order);
 * outputs: dev_energy double[n_cfg], dev_forces double[N*3],
 * dev_virial double[9 * n_cfg] (row-major, sum over atoms of
 * -dE_i/dr_ij (x) r_ij), dev_atom_energy double[N] or NULL. */
int nepmi_compute_f64(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                      const double *dev_pos, const int32_t *dev_species, const double *dev_params, double *dev_energy,
                      double *dev_forces, double *dev_virial, double *dev_atom_energy, void *stream);

/* Vector-Jacobian product of (E, F, V) with respect to the parameters, in
 * float64 (the float64 twin of nepmi_backward_params):
 *   dev_grad[p] = sum_c ebar_c dE_c/dtheta_p + sum_i lambda_i . dF_i/dtheta_p
 *               + sum_c mu_c : dV_c/dtheta_p
 * dev_ebar double[n_cfg], dev_lambda double[N*3], dev_mu double[9*n_cfg];
 * dev_grad double[param_count] is overwritten. */
int nepmi_backward_params_f64(nepmi_model *m, int32_t n_cfg, const int64_t *atom_off, const double *cells, const int32_t *pbc,
                              const double *dev_pos, const int32_t *dev_species, const double *dev_params,
                              const double *dev_ebar, const double *dev_lambda, const double *dev_mu,
                              double *dev_grad, void *stream);

/* ---------------------------------------------------------------------------
 * Optimisation protocol (Sec. 3.3).
 * ------------------------------------------------------------------------- */

/* One Adam step (Sec. 3.3.1) over n FP32 parameters on the device, with the
 * moments kept by the caller (dev_m, dev_v: n floats each, zero before the
 * first step; updated in place).  With g = dev_grad and t >= 1 the step count:
 *   m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
 *   p <- p - lr / (1 - beta1^t) * m / (sqrt(v) / sqrt(1 - beta2^t) + eps).
 * No weight decay.  The paper's setting is beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8.  Asynchronous on `stream`.  NEPMI_INVALID_ARG on bad sizes,
 * null pointers, t < 1 or coefficients out of range. */
int nepmi_adam_step(int64_t n, float *dev_params, const float *dev_grad, float *dev_m, float *dev_v, int64_t t,
                    double lr, double beta1, double beta2, double eps, void *stream);

/* Learning rate of training step `step` (0-based) under the two-stage
 * schedule of Sec. 3.3.2 (host only): linear warmup of the factor from
 * start_factor (1e-4 in the paper) to 1 over warmup_steps (one epoch in the
 * paper), then cosine annealing from lr_start to lr_end over the remaining
 * total_steps - warmup_steps steps (held at lr_end after them). */
int nepmi_lr_schedule(int64_t step, int64_t warmup_steps, int64_t total_steps, double lr_start, double lr_end,
                      double start_factor, double *lr_out);

/* Loss weights of one step (Sec. 3.3.3, host only):
 *   w_c = w_start[c] x + w_end[c] (1 - x),  c = energy, force, virial,
 * with x = lr (the formula as printed, normalised = 0) or x = lr / lr_start
 * (normalised = 1).  w_start, w_end, w_out: host double[3]. */
int nepmi_loss_weights(double lr, double lr_start, const double *w_start, const double *w_end, int32_t normalised,
                       double *w_out);

#ifdef __cplusplus
}
#endif
#endif /* NEPMI_H */
