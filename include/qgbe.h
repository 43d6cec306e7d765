/*
 * qgbe.h -- C ABI of libqgbe: Monte Carlo 2->2 collision term of the
 * relativistic Boltzmann equation for quarks and gluons, with its explicit
 * drift and time step, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Zhang, Wu, Pu, Qin, Wang, "Towards a full solution of relativistic
 * Boltzmann equation for quark-gluon matter on GPUs" (arXiv:1912.04457).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Species      0..6 = u, d, s, ubar, dbar, sbar, g.  Degeneracies N_q = 6,
 *              N_g = 16 (Eq. C_quark, Eq. C_gluon).
 * Grid         cell-centred.  Momentum node i of an axis sits at
 *              -p_half + (i + 1/2) * 2 p_half / n_p (GeV); spatial cells
 *              likewise with x_half (fm).  Boundaries are periodic in x and p
 *              for the drift (Sec. III).
 * Layout       distributions and collision terms are float64
 *              [species][cell][node], cell = (ix*ny + iy)*nz + iz,
 *              node = (ipx*npy + ipy)*npz + ipz (pz fastest).
 * A            the collision output A_Y(x,q) = N_Y C_Y(x,q) in GeV, i.e. the
 *              left-hand side of Eq. C_quark / Eq. C_gluon.
 * Channels     one per (reaction of Table I, species placed first), ordered by
 *              code = ((s1*7+s2)*7+s3)*7+s4 ascending; 70 for all 7 species.
 * Random draws Philox4x32-10 with key (seed_lo, seed_hi + step) and counter
 *              (sample, node, cell, code<<8 | block): every sample is a pure
 *              function of (seed, step, cell, channel, node, sample).
 * Pointers     "on_device" = 1: a device pointer on the context's device
 *              (e.g. a torch tensor's data_ptr), used on the context's stream;
 *              0: host memory.  The caller owns every buffer it passes and keeps
 *              device buffers alive until the stream has finished with them.
 *              The library owns the context and the device workspace it
 *              allocates in qgbe_init_grid (reported by qgbe_workspace_bytes).
 * Errors       every entry point returns a qgbe_status; nothing is thrown
 *              across the ABI.  Argument errors are reported before any device
 *              work.  qgbe_last_error() gives a message for the calling thread.
 * Streams      device work is enqueued on the context's stream.  Calls that
 *              return host data (stats, host outputs) synchronise that stream.
 */
#ifndef QGBE_H
#define QGBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qgbe_ctx qgbe_ctx;

typedef enum {
  QGBE_OK = 0,
  QGBE_EINVAL = -1,       /* bad argument (sizes, masks, null pointers)       */
  QGBE_ENOMEM = -2,       /* device allocation failed                          */
  QGBE_EDEVICE = -3,      /* a HIP call failed                                 */
  QGBE_ESTATE = -4,       /* call not valid in the context's current state     */
  QGBE_ENUMERIC = -5,     /* NaN/Inf found in the evolved distribution         */
  QGBE_EUNSUPPORTED = -6  /* configuration not supported by this build         */
} qgbe_status;

enum { QGBE_FP64 = 0, QGBE_FP32 = 1 };                 /* integrand precision   */
enum {
  QGBE_SAMPLER_UNIFORM = 0,   /* CM-angle parameterisation, uniform draws       */
  QGBE_SAMPLER_LEARNED = 1,   /* the proposal table's mixture, weight 1/q       */
  QGBE_SAMPLER_ROOTS = 2,     /* the paper's root parameterisation (FP64)       */
  QGBE_SAMPLER_ROOTS_ALT = 3  /* its alternative elimination (FP64)             */
};
enum { QGBE_DRIFT_UPWIND = 0, QGBE_DRIFT_CENTRAL = 1 };
enum { QGBE_MASS_DYNAMIC = 0, QGBE_MASS_CONSTANT = 1 };

/* stats flags */
enum { QGBE_FLAG_NEGATIVE_F = 1, QGBE_FLAG_PAULI = 2, QGBE_FLAG_NONFINITE = 4 };

typedef struct {
  int32_t n_x[3];          /* spatial cells per axis, >= 1                    */
  int32_t n_p[3];          /* momentum nodes per axis, >= 2                   */
  double x_half[3];        /* spatial box half-widths, fm, > 0                */
  double p_half[3];        /* momentum box half-widths, GeV, > 0              */
  uint32_t species_mask;   /* bit Y: species Y evolves; a reaction is included
                              when all four of its species evolve             */
  uint32_t row_mask;       /* bit r-1: Table I row r enabled                  */
  double alpha_s;          /* strong coupling, g^2 = 4 pi alpha_s             */
  int32_t precision;       /* QGBE_FP64 or QGBE_FP32 (FP32 integrand and f
                              interpolation, FP64 sample geometry and FP64
                              accumulation)                                   */
  int32_t symmetric;       /* 1: symmetric sampling (Sec. III B), 0: direct  */
  int32_t drift;           /* QGBE_DRIFT_UPWIND or QGBE_DRIFT_CENTRAL         */
  int32_t mass_mode;       /* QGBE_MASS_DYNAMIC (Eq. mg, Eq. mq) or CONSTANT  */
  double const_mass2[7];   /* GeV^2 per species, used when mass_mode=CONSTANT */
  uint64_t seed;           /* Philox seed                                     */
  int32_t device;          /* HIP device ordinal                              */
  void* stream;            /* hipStream_t; NULL = the default stream          */
} qgbe_grid_desc;

typedef struct {
  double N_total;          /* Eq. particle numbers summed over species        */
  double N[7];
  double E_total;          /* T^00 of Eq. energy momentum tensor, integrated   */
  double E[7];
  double P[3];             /* total momentum                                   */
  double mass2_avg[7];     /* cell-averaged thermal masses squared, GeV^2      */
  double min_f;            /* minimum of f over evolved species                */
  double max_fermion_f;    /* maximum of quark/antiquark f                     */
  double n_evals;          /* integrand evaluations in the collision term     */
  double t_collide_ms;     /* device time of the collision kernels             */
  double t_step_ms;        /* device time of the whole step                    */
  uint32_t flags;          /* QGBE_FLAG_*                                      */
  uint32_t step;           /* step index the stats belong to                   */
  double n_accepted;       /* evaluations above threshold and inside the box  */
  double mc_err_est;       /* relative MC error of the collision term's direct
                              sums, estimated from the samples themselves:
                              sqrt(V / (Q - V)) with V = sum_i Var S_i and
                              Q = sum_i S_i^2 over the work items i, S_i the
                              item's sum of N sample values, Var S_i =
                              N/(N-1) (sum v^2 - S_i^2/N); infinite when
                              Q <= V (the sums are noise)                     */
  /* Energy bookkeeping of a step (Eq. current conservation and the modified
   * tensor of Sec. IV, energy test), all integrated over the box, in GeV.
   * With f_k the field the step starts from, m_k^2 its masses and m_{k-1}^2
   * those of the step before:
   *   E_source  = sum over species, cells, nodes of N dV f_k (E(m_k^2) -
   *               E(m_{k-1}^2)): the kinetic-energy change that the mass
   *               change alone causes at fixed f (the integral of S_ex^0 over
   *               the step); 0 on a first step and with constant masses.
   *   E_collide = dt/(hbar c) sum dV E(m_k^2) A over evolved species: the
   *               energy the collision term adds (zero in the continuum; the
   *               grid leaves a residue).
   * so that E_total(k) - E_total(k-1) = E_source + E_collide + the drift's
   * part.  E_total_mod = E_total - 1/4 sum N dV m^2 f / E, T^00 of the
   * modified tensor (conserved for a single species, Sec. IV).  qgbe_step
   * fills E_source and E_collide; other calls leave them 0.                  */
  double E_source;
  double E_collide;
  double E_total_mod;
  /* Thermalisation diagnostics (Sec. IV C, D): the Boltzmann entropy
   * sum N dV [(1 + s f) ln(1 + s f)/s - f ln f] (s = +1 gluons, -1 quarks;
   * nodes with f <= 0 or 1 + s f <= 0 add nothing), which the collision term
   * does not decrease, and the diagonal of Eq. energy momentum tensor,
   * T_ii = sum N dV p_i^2 f / E (GeV), whose ratio T_zz / T_xx measures the
   * isotropisation.                                                          */
  double entropy;
  double T_ii[3];
  uint32_t n_collide_launches;  /* collision kernel launches of the term;
                                   t_collide_ms is their sum            */
  uint32_t reserved;
} qgbe_stats;

/* Optional outputs of the collision term (all may be NULL). */
typedef struct {
  double* scale;           /* [7][cells][nodes] sum of |deposit| of the
                              gain+loss magnitude, for error normalisation     */
  double* item_sums;       /* [cells][channels][nodes] sum of the sample values
                              of each work item (its direct part)              */
  int32_t on_device;       /* where scale and item_sums live                   */
} qgbe_collide_extras;

/* ---- context ------------------------------------------------------------ */

/* Create a context: validates the descriptor, builds the channel table of
 * Eq. C_quark / Eq. C_gluon, allocates the device workspace (f in FP64 and its
 * FP32 shadow, masses, accumulators) and zeroes f.  *out is NULL on failure. */
qgbe_status qgbe_init_grid(const qgbe_grid_desc* desc, qgbe_ctx** out);

/* Release the context and its workspace (waits for its stream). NULL is fine. */
void qgbe_destroy(qgbe_ctx* ctx);

/* Message describing the last failure on the calling thread ("" if none).
 * Valid until the next qgbe_* call on this thread. */
const char* qgbe_last_error(void);

/* Bytes of device memory the context owns. */
size_t qgbe_workspace_bytes(const qgbe_ctx* ctx);

/* ---- state -------------------------------------------------------------- */

/* Copy f of one species ([cells][nodes], float64) into the context (species
 * in 0..6), or all seven species at once with species = -1 ([7][cells][nodes]).
 * Resets the lagged masses, so the next mass evaluation uses E = |p|
 * (Sec. II, after Eq. mq). */
qgbe_status qgbe_set_distribution(qgbe_ctx* ctx, int32_t species, const double* f,
                                  int32_t on_device);

/* Copy f out (same shapes as qgbe_set_distribution). */
qgbe_status qgbe_get_distribution(qgbe_ctx* ctx, int32_t species, double* f,
                                  int32_t on_device);

/* Thermal masses squared [7][cells] (host) used by the last collision term or
 * step.  Eq. mg / Eq. mq as midpoint sums over the momentum grid. */
qgbe_status qgbe_get_masses(qgbe_ctx* ctx, double* mass2);

/* Step index used as the second Philox key word; advanced by qgbe_step. */
qgbe_status qgbe_set_step_index(qgbe_ctx* ctx, uint32_t step);
qgbe_status qgbe_get_step_index(const qgbe_ctx* ctx, uint32_t* step);

/* Serialise the evolving state into a host buffer: f, the step index, the
 * lagged masses the next mass evaluation will use, and the learned proposal
 * (network weights with their Adam moments, proposal table).  buf = NULL:
 * *bytes receives the size needed.  Otherwise *bytes is the buffer size on
 * entry (QGBE_EINVAL, with the size needed in *bytes, if too small) and the
 * size written on return.  The caller owns buf.  Synchronises the stream. */
qgbe_status qgbe_checkpoint(qgbe_ctx* ctx, void* buf, size_t* bytes);

/* Load a buffer written by qgbe_checkpoint into a context created with the
 * same descriptor (grid, species and rows, alpha_s, precision, symmetric,
 * drift, mass mode and seed; device and stream may differ).  QGBE_EINVAL for
 * a foreign, truncated or mismatching buffer, before any device work.  A run
 * continued from the restored state draws the same samples as the original
 * run would have. */
qgbe_status qgbe_restore(qgbe_ctx* ctx, const void* buf, size_t bytes);

/* ---- the hot path ------------------------------------------------------- */

/* The Monte Carlo collision term A = N_Y C_Y for every cell, species and node
 * (Eq. C_a_b summed as in Eq. C_quark / Eq. C_gluon).  Thermal masses are
 * evaluated first from the current f (lagged energies if a step has run).
 * n_samples samples per (cell, channel, node); sampler QGBE_SAMPLER_UNIFORM
 * draws p2 uniformly in the momentum box and the two CM angles uniformly
 * (Eq. MC C_gg with the CM-angle parameterisation), QGBE_SAMPLER_LEARNED
 * draws from the proposal table (qgbe_set_proposal_table, or the network's
 * table re-evaluated on the current masses after qgbe_proposal_build_table),
 * with weight 1/q, except on channels set back to the uniform sampler.
 * QGBE_SAMPLER_ROOTS is the paper's own parameterisation (Eq. work out delta
 * E, Eq. delta replace, Eq. ca): in channel order k1 + k2 <-> k3 + k4 with k1
 * observed, k2 uniform in the box, k3x and k3y uniform, k4 eliminated by
 * momentum conservation and k3z at each of the two roots of energy
 * conservation, weighted 1/|J|.  QGBE_SAMPLER_ROOTS_ALT eliminates k2 instead
 * (k4 uniform in the box), the alternative whose spread the paper compares
 * (Sec. IV A).  Both run in FP64 (f from the FP64 field) whatever the
 * context's precision, with Philox block 2 of the same counters.
 * Symmetric sampling (Eq. small c relation) adds each sample's value at the
 * observed node and at the trilinear stencils of the other three momenta with
 * signs (+,+,-,-), so sum_{Y,q} A = 0 per cell exactly.
 * A_out: [7][cells][nodes] float64, overwritten.  st may be NULL. */
qgbe_status qgbe_collision_term(qgbe_ctx* ctx, int32_t n_samples, int32_t sampler,
                                double* A_out, int32_t on_device, qgbe_stats* st);

/* User matrix elements (Sec. II: the tree-level Table I is the default and
 * users may supply their own).  Replaces row `row` (1..7) of Table I, for
 * every channel of that row, by
 *   |M|^2 = g^4 sum_{k < n_terms} coef[k] s^a t^b u^c / ((t - m_g^2)^d (u - m_g^2)^e s^f)
 * with g^2 = 4 pi alpha_s, the Mandelstam variables of the row's labelling
 * (Table I) and powers[6 k .. 6 k + 5] = {a, b, c, d, e, f}, each 0..4;
 * n_terms <= 8, and n_terms = 0 restores the Table I row.  Table I itself is
 * of this form (e.g. row 7 = 3456 - 1152 su/(t-m^2)^2 - 1152 st/(u-m^2)^2 -
 * 1152 tu/s^2).  Takes effect from the next collision term or step, in every
 * sampler and precision (the integrand's precision); waits for the work
 * already queued on the context's stream.  Not part of a checkpoint.
 * QGBE_EINVAL for a bad row, count, power, coefficient or NULL buffers. */
qgbe_status qgbe_set_matrix_element(qgbe_ctx* ctx, int32_t row, int32_t n_terms, const double* coef,
                                    const int32_t* powers);

/* Same with optional diagnostic outputs (extras may be NULL). */
qgbe_status qgbe_collision_term_ex(qgbe_ctx* ctx, int32_t n_samples, int32_t sampler,
                                   double* A_out, int32_t on_device,
                                   const qgbe_collide_extras* extras, qgbe_stats* st);

/* n_steps forward-Euler steps (Sec. III):
 *   masses -> collision term A -> drift D[f] of Eq. left handside (upwind or
 *   the central differences of Eq. descrete left hand, periodic) ->
 *   f += dt (A / (N_Y hbar c) - D[f]) -> observables.
 * dt_fm in fm/c, hbar c = 0.1973269804 GeV fm.  Non-evolving species are
 * frozen.  The sampler is as in qgbe_collision_term (a network-built table is
 * re-evaluated at every step).  per_step: n_steps entries (their t_step_ms
 * covers masses, table, collision term and update; each step then waits for
 * its statistics) or NULL (the steps run without the per-step reductions and
 * without synchronising the host).  With per_step, returns QGBE_ENUMERIC
 * (after finishing the step) if f became non-finite. */
qgbe_status qgbe_step(qgbe_ctx* ctx, double dt_fm, int32_t n_samples, int32_t sampler,
                      int32_t n_steps, qgbe_stats* per_step);

/* Observables of the current f with the current masses (Eq. particle numbers,
 * Eq. energy momentum tensor), FP64. */
qgbe_status qgbe_observables(qgbe_ctx* ctx, qgbe_stats* st);

/* ---- collision term without device allocation --------------------------- */

/* Device scratch of qgbe_collision_term_noalloc, in MiB: one statically sized
 * array per GPU, held until the process ends. */
#define QGBE_NOALLOC_SCRATCH_MIB 64

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the collision term of
 * qgbe_collision_term on a context freshly made from desc, with f set and the
 * step index at `step`, computed without a context and without any device
 * allocation.  Masses come from f with E = |p| (the first-call rule), or
 * desc->const_mass2 with QGBE_MASS_CONSTANT; Table I matrix elements.
 * f: [7][cells][nodes] float64 on desc->device (read only); A:
 * [7][cells][nodes] float64 on the same device, overwritten.  Both are owned
 * by the caller and must stay alive until desc->stream has finished the work.
 * sampler: QGBE_SAMPLER_UNIFORM (in desc->precision) or one of the root
 * samplers (FP64); QGBE_SAMPLER_LEARNED is refused (no proposal table).
 * Everything else the kernels need (channel table, masses, per-launch totals,
 * the FP32 copy of f and its node quads) lives in one device array of
 * QGBE_NOALLOC_SCRATCH_MIB MiB per GPU; a grid that needs more returns
 * QGBE_EINVAL before any device work.  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (other streams, other threads)
 * race; calls in sequence on one stream do not.  Asynchronous on desc->stream
 * except that the first call, and any call whose channel table differs from
 * the previous call's, waits for its upload of the table (a caller that
 * captures the stream makes one call with the same grid before capturing).
 * No statistics. */
qgbe_status qgbe_collision_term_noalloc(const qgbe_grid_desc* desc, const double* f, uint32_t step,
                                        int32_t n_samples, int32_t sampler, double* A);

/* Bytes of the array qgbe_collision_term_noalloc works in. */
size_t qgbe_noalloc_scratch_bytes(void);

/* ---- proposal table for the learned sampler ------------------------------ */

/* Install a mixture-of-logistic-normals proposal over the five unit-cube
 * variables (p2 in the box, cos theta*, phi*), one row per (channel, node):
 *   thr   [rows][K] uint32: thr[0] = defensive-uniform share alpha * 2^32;
 *         component k is drawn when thr[k] <= x < thr[k+1] (thr[K] = 2^32)
 *   mu    [rows][K][5] float32 location in logit space
 *   sigma [rows][K][5] float32 scale in logit space (> 0)
 * rows = channels * nodes.  K in 1..16.  Copied into the workspace.  An FP32
 * context's learned sampler takes K <= 8: with more components its collision
 * term and step return QGBE_EUNSUPPORTED before any device work. */
qgbe_status qgbe_set_proposal_table(qgbe_ctx* ctx, int32_t K, const uint32_t* thr,
                                    const float* mu, const float* sigma, int32_t on_device);

/* Per-channel sampler choice of the learned mode: use_learned[channels], 1 =
 * the channel draws from the proposal table, 0 = it falls back to the uniform
 * sampler (the same draws and weights as QGBE_SAMPLER_UNIFORM).  Installing a
 * table (qgbe_set_proposal_table, qgbe_proposal_build_table, training) sets
 * every channel to 1.  QGBE_ESTATE without a table. */
qgbe_status qgbe_set_channel_samplers(qgbe_ctx* ctx, const uint8_t* use_learned);
qgbe_status qgbe_get_channel_samplers(qgbe_ctx* ctx, uint8_t* use_learned);

/* The fallback judge of the learned proposal: n_reps pilot collision terms of
 * n_pilot samples per point with each sampler (on a key range of their own);
 * per channel, the variance of every (cell, node) estimate is estimated from
 * its own samples (as for mc_err_est), summed, and multiplied by the
 * sampler's pilot time; a channel keeps the learned sampler only if that
 * product is smaller than the uniform one.  Installs the decision and
 * returns it in use_learned[channels] (may be NULL); ratio[channels] (may be
 * NULL) receives learned / uniform variance x time.  The step index and f are
 * left as they were.  n_pilot >= 2, n_reps >= 1. */
qgbe_status qgbe_proposal_judge(qgbe_ctx* ctx, int32_t n_pilot, int32_t n_reps, uint8_t* use_learned,
                                double* ratio);

/* ---- the learned proposal (a network that writes the proposal table) ---- */
/*
 * Network: x (8 inputs) -> Linear 8x128 -> SiLU -> Linear 128x128 -> SiLU ->
 * Linear 128x88 = head (8 mixture logits, 8x5 locations, 8x5 log scales of a
 * logistic-normal mixture over the five unit-cube variables).  Products run
 * as BF16 x BF16 -> FP32 matrix-core GEMMs; master weights, Adam moments and
 * the head arithmetic are FP32.  The weights are the flat FP32 vector
 * W1 [8][128], b1 [128], W2 [128][128], b2 [128], W3 [128][88], b3 [88]
 * (row-major [in][out]), QGBE_MLP_PARAMS floats.
 * Inputs x of the work item (channel c, observed node p1, cell masses):
 *   p1x/Px, p1y/Py, p1z/Pz, |p1|/|P|, E1/|P|, m_g^2/|P|^2,
 *   species/3 - 1, 2c/(channels-1) - 1        (P = p_half, |P| its norm).
 * The proposal is unbiased for any weights (importance weights 1/q with a
 * defensive uniform share); training only lowers the variance.
 */
#define QGBE_MLP_PARAMS 29016
#define QGBE_MLP_BATCH 16384   /* maximum rows of one qgbe_mlp_loss_grad call */

typedef struct {
  int32_t epochs;          /* passes over the recorded rows                  */
  int32_t batch;           /* rows per Adam step (<= QGBE_MLP_BATCH)         */
  float lr;                /* initial learning rate                          */
  float lr_final;          /* learning rate at the end (cosine decay)        */
  float alpha;             /* defensive uniform share of the table, (0,1)    */
  uint64_t seed;           /* shuffling seed                                 */
} qgbe_train_cfg;

/* Copy the FP32 weights in (resets the Adam moments) or out. n must equal
 * QGBE_MLP_PARAMS.  Host pointers. */
qgbe_status qgbe_proposal_set_weights(qgbe_ctx* ctx, const float* w, int64_t n);
qgbe_status qgbe_proposal_get_weights(qgbe_ctx* ctx, float* w, int64_t n);

/* Network forward pass: X [rows][8] FP32 -> head Y [rows][88] FP32. */
qgbe_status qgbe_mlp_forward(qgbe_ctx* ctx, const float* X, int64_t rows, float* Y, int32_t on_device);

/* Weighted negative log-likelihood of the mixture head and its gradient:
 * X [rows][8], yw [rows][6] = (logit u (5), weight); loss = -sum w log q /
 * sum w; grad [QGBE_MLP_PARAMS] FP32; rows <= QGBE_MLP_BATCH. */
qgbe_status qgbe_mlp_loss_grad(qgbe_ctx* ctx, const float* X, const float* yw, int64_t rows, float* grad,
                               double* loss, int32_t on_device);

/* Conditioning inputs of every (channel, node) row, built from the masses of
 * the last collision term or step averaged over the cells (one table serves
 * every cell): X [channels*nodes][8]. */
qgbe_status qgbe_proposal_features(qgbe_ctx* ctx, float* X, int32_t on_device);

/* Record training rows from uniform samples of the current f: for every
 * item_stride-th work item (cell, channel, node; node fastest), n_per_item
 * samples, each row [x (8), logit u (5), |sample value|] (14 FP32).
 * *n_rows receives the row count; rows must hold max_rows rows. */
qgbe_status qgbe_record_samples(qgbe_ctx* ctx, int32_t n_per_item, int64_t item_stride, float* rows,
                                int64_t max_rows, int64_t* n_rows, int32_t on_device);

/* Train the network on recorded rows ([n][14], as qgbe_record_samples writes)
 * with Adam on device; epoch_loss [epochs] (may be NULL) receives the mean
 * training loss of each epoch.  Then builds the proposal table. */
qgbe_status qgbe_train_proposal(qgbe_ctx* ctx, const float* rows, int64_t n, const qgbe_train_cfg* cfg,
                                double* epoch_loss, int32_t on_device);

/* Evaluate the network on every (channel, node) row and install the result
 * as the proposal table (defensive share alpha).  From then on, every learned
 * collision term or step re-evaluates the network on the current masses
 * before sampling (the inference is part of that call's time), until
 * qgbe_set_proposal_table installs a fixed table. */
qgbe_status qgbe_proposal_build_table(qgbe_ctx* ctx, float alpha);

/* Copy the installed proposal table out (thr [rows][K], mu, sigma
 * [rows][K][5], rows = channels*nodes), K written to *K. */
qgbe_status qgbe_get_proposal_table(qgbe_ctx* ctx, int32_t* K, uint32_t* thr, float* mu, float* sigma);

/* ---- host-only helpers (no device needed) ------------------------------- */

/* The channel table the library builds for the masks: rows [n][5] =
 * (Table I row, s1, s2, s3, s4) and weights [n][2] = (w, sigma) where w is the
 * per-position symmetric weight and sigma the coefficient in Eq. C_quark /
 * Eq. C_gluon.  Returns the count, or a negative qgbe_status if max is too
 * small.  Either output may be NULL. */
int32_t qgbe_channel_table(uint32_t species_mask, uint32_t row_mask, int32_t* rows,
                           double* weights, int32_t max);

/* Philox4x32-10 block (Salmon et al., SC'11) as the device computes it; host
 * implementation for checks. */
void qgbe_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif /* QGBE_H */
