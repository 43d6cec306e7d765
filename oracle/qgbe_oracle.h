/*
 * qgbe_oracle.h -- FP64 CPU oracle for the Monte Carlo 2->2 collision term of
 * the relativistic Boltzmann equation for quarks and gluons (Zhang, Wu, Pu,
 * Qin, Wang, arXiv:1912.04457).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source with
 * the GPU library: every formula here is written out again from the paper.
 *
 * Conventions (all readings of the paper are listed in the design notes):
 *   species index   0..6 = u, d, s, ubar, dbar, sbar, g
 *   f, A layout     [species][cell][p_lin], cell = (ix*ny+iy)*nz+iz,
 *                   p_lin = (ipx*npy+ipy)*npz+ipz  (pz fastest)
 *   grid            cell-centred: q_i = -P + (i+1/2) * 2P/n per axis
 *   A               A_Y(x,q) = N_Y * C_Y(x,q) in GeV (left side of Eq. C_quark /
 *                   Eq. C_gluon), the collision term times the degeneracy
 *   mass2           [species][cell] thermal masses squared, GeV^2; the
 *                   regulator in every t/u pole of Table I is mass2[g][cell]
 */
#ifndef QGBE_ORACLE_H
#define QGBE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_x[3];        /* spatial cells per axis                       */
  int32_t n_p[3];        /* momentum nodes per axis                      */
  double x_half[3];      /* spatial box [-x_half, x_half] in fm          */
  double p_half[3];      /* momentum box [-p_half, p_half] in GeV        */
  uint32_t species_mask; /* bit Y set: species Y evolves                 */
  uint32_t row_mask;     /* bit r-1 set: Table I row r enabled           */
  double alpha_s;
} ref_grid;

/* one collision channel (reaction R, observed species at position 1) */
typedef struct {
  int32_t row;           /* Table I row 1..7                             */
  int32_t sp[4];         /* species at channel positions 1..4            */
  int32_t code;          /* ((sp1*7+sp2)*7+sp3)*7+sp4, the Philox tag    */
  double w;              /* per-position weight of the symmetric mode    */
  double sigma;          /* coefficient of this term in Eq. C_quark/C_gluon */
} ref_channel;

/* equilibrium parameters for the analytic-f test mode */
typedef struct {
  double T;              /* temperature, GeV                             */
  double mu[7];          /* chemical potential per species, GeV          */
} ref_equilibrium;

/* per-point evaluation record (test hooks) */
typedef struct {
  int32_t valid;         /* above threshold and inside the momentum box  */
  double k[4][4];        /* 4-momenta (E,px,py,pz) at positions 1..4      */
  double s, t, u;        /* Mandelstam invariants in Table I labelling    */
  double pstar;          /* |p*| of the final state in the CM frame       */
  double msq;            /* |M|^2 from Table I                            */
  double f[4];           /* occupation at the 4 momenta                   */
  double B;              /* f3 f4 F1 F2 - f1 f2 F3 F4                     */
  double GL;             /* f3 f4 F1 F2 + f1 f2 F3 F4                     */
  double g;              /* integrand per unit of the sampled 5-volume    */
  double gscale;         /* same with |msq| * GL in place of msq * B      */
} ref_point;

/* flags for the test hooks */
enum {
  REF_B_ONE = 1,          /* statistical bracket B replaced by 1           */
  REF_NO_BOXCUT = 2,      /* final momenta may leave the box               */
  REF_MASSLESS = 4,       /* kinematic masses 0 (regulator still mass2[g]) */
  REF_ANALYTIC_F = 8      /* f from Eq. fg / Eq. fq at the exact momenta   */
};

/* estimators of the uniform sampler.  In channel order k1 + k2 <-> k3 + k4,
   k1 the observed momentum (the paper's p):
     REF_EST_CM       CM-angle parameterisation (p2 in the box, two angles)
     REF_EST_ROOT     the paper's choice (Eq. work out delta E): k2 in the box,
                      k3x, k3y sampled, k3z from the roots, k4 eliminated
                      (the paper eliminates its k2, on the other side of p)
     REF_EST_ROOT_K3  the paper's alternative (Sec. III A, stability test):
                      k4 in the box, k3x, k3y sampled, k3z from the roots, k2
                      eliminated (the paper eliminates its k3, the partner of
                      p); the roots then depend on E1 - E4, which changes sign */
enum { REF_EST_CM = 0, REF_EST_ROOT = 1, REF_EST_ROOT_K3 = 2 };

/* Philox4x32-10 block (Salmon et al., SC'11) */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* the five unit-cube variables of sample s of work item (cell, channel code,
   p1) under the uniform sampler: Philox block 0 with key (seed_lo32,
   seed_hi32 + step), counter (s, p1_lin, cell, code << 8), five 23-bit fields
   mapped to the midpoints of their cells */
void ref_sample_uniforms(uint64_t seed, uint32_t step, uint32_t s, uint32_t p1_lin, uint32_t cell,
                         uint32_t code, double u_out[5]);

/* |M|^2 of Table I (summed over all colours and helicities), or the user's
   matrix element of that row (ref_set_matrix_element) */
double ref_msq(int32_t row, double s, double t, double u, double mg2, double alpha_s);

/* replace Table I row `row` (1..7) by g^4 sum_k c_k s^a t^b u^c /
   ((t - mg2)^d (u - mg2)^e s^f), powers[k] = {a, b, c, d, e, f} in
   0..REF_MSQ_MAX_POWER, n <= REF_MSQ_MAX_TERMS terms; n = 0 restores the
   row.  Returns -1 on bad arguments. */
enum { REF_MSQ_MAX_TERMS = 8, REF_MSQ_MAX_POWER = 4 };
int32_t ref_set_matrix_element(int32_t row, int32_t n, const double* coef, const int32_t* powers);

/* channel table for the species/row masks, in ascending order of code;
   returns the count (<= max) */
int32_t ref_channels(const ref_grid* g, ref_channel* out, int32_t max);

/* thermal masses, Eq. mg and Eq. mq; mass2_lag == NULL means E = |p| */
int32_t ref_masses(const ref_grid* g, const double* f, const double* mass2_lag,
                   double* mass2_out);

/* evaluate one configuration (CM-angle parameterisation) */
int32_t ref_eval_cm(const ref_grid* g, const ref_channel* ch, const double* f,
                    const double* mass2, int32_t cell, const double p1[3],
                    int32_t p1_lin, const double p2[3], double cos_th,
                    double phi, int32_t flags, const ref_equilibrium* eq,
                    ref_point* out);

/* the Monte Carlo collision term, uniform sampler.
 *   estimator  REF_EST_CM (CM-angle sampler), REF_EST_ROOT (the paper's
 *              own elimination with the k1z roots, Eq. work-out-delta-E) or
 *              REF_EST_ROOT_K3 (the alternative elimination)
 *   symmetric  1 = symmetric sampling, 0 = direct estimator
 *   A_out      [7][cells][nodes], overwritten
 *   S_out      same shape or NULL: sum of |deposit| of the gain+loss scale
 *   item_sum   [cells][channels][nodes] or NULL: per work item sum of v
 */
int32_t ref_collision(const ref_grid* g, const double* f, const double* mass2,
                      uint64_t seed, uint32_t step, int32_t n_samples,
                      int32_t estimator, int32_t symmetric, int32_t flags,
                      const ref_equilibrium* eq, double* A_out, double* S_out,
                      double* item_sum, int32_t n_threads);

/* direct sums (sum of sample values) of selected work items without any
   deposits: items[3i..3i+2] = (cell, channel ordinal, node); out[n_sel];
   out_scale[n_sel] (may be NULL) receives the sum of the samples' gain+loss
   magnitudes, the natural scale of each direct sum */
int32_t ref_item_sums(const ref_grid* g, const double* f, const double* mass2, uint64_t seed,
                      uint32_t step, int32_t n_samples, int32_t symmetric, int64_t n_sel,
                      const int64_t* items, double* out, double* out_scale, int32_t n_threads);
/* direct sums of selected items with the mixture proposal (table and flags
   as in ref_collision_learned) */
int32_t ref_item_sums_learned(const ref_grid* g, const double* f, const double* mass2, uint64_t seed,
                              uint32_t step, int32_t n_samples, int32_t K, const uint32_t* thr,
                              const float* mu, const float* sigma, int32_t table_per_cell,
                              const uint8_t* chan_learned, int64_t n_sel, const int64_t* items,
                              double* out, double* out_scale, int32_t n_threads);
/* the same for any estimator of the uniform sampler */
int32_t ref_item_sums_est(const ref_grid* g, const double* f, const double* mass2, uint64_t seed,
                          uint32_t step, int32_t n_samples, int32_t estimator, int32_t symmetric,
                          int64_t n_sel, const int64_t* items, double* out, double* out_scale,
                          int32_t n_threads);

/* the collision term with a mixture-of-logistic-normals proposal.
 *   K          mixture components
 *   thr        [rows][K] u32 boundaries: thr[0] = defensive-uniform share,
 *              component k drawn when thr[k] <= x < thr[k+1] (thr[K] = 2^32)
 *   mu, sigma  [rows][K][5] location and scale in logit space
 *   rows       = table_cells * channels * nodes (table_cells is 1 or cells)
 *   chan_learned [channels] 1: the channel samples from the mixture, 0: it
 *              falls back to the uniform sampler (its draws and weight 1);
 *              NULL: every channel uses the mixture
 */
int32_t ref_collision_learned(const ref_grid* g, const double* f, const double* mass2,
                              uint64_t seed, uint32_t step, int32_t n_samples,
                              int32_t K, const uint32_t* thr, const float* mu,
                              const float* sigma, int32_t table_per_cell,
                              const uint8_t* chan_learned,
                              double* A_out, double* S_out, double* item_sum,
                              int32_t n_threads);

/* the same operator by deterministic quadrature: pts[n][5] holds
   (p2x, p2y, p2z, cos theta, phi), wts[n] the quadrature weights */
int32_t ref_collision_points(const ref_grid* g, const double* f, const double* mass2,
                             int64_t n_pts, const double* pts, const double* wts,
                             int32_t symmetric, int32_t flags, double* A_out,
                             int32_t n_threads);

/* discrete drift operator D[f] (fm^-1): scheme 0 = upwind, 1 = central */
int32_t ref_drift(const ref_grid* g, const double* f, const double* mass2,
                  int32_t scheme, double* D_out);

/* the trilinear stencil every off-grid f read and every deposit uses, for
   n momenta pts[n][3]: node indices idx[n][8] and weights w[n][8] */
int32_t ref_stencil(const ref_grid* g, int64_t n, const double* pts, int64_t* idx, double* w);

/* number, energy and momentum per species (FP64 bookkeeping) */
int32_t ref_observables(const ref_grid* g, const double* f, const double* mass2,
                        double* N_out /*7*/, double* E_out /*7*/, double* P_out /*7x3*/);

#ifdef __cplusplus
}
#endif
#endif
