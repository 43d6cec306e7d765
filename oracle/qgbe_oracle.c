/*
 * qgbe_oracle.c -- plain FP64 CPU oracle for the Monte Carlo 2->2 collision
 * term of the quark-gluon Boltzmann equation (arXiv:1912.04457).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Slow on
 * purpose: one configuration at a time, written in the order of the paper's
 * formulas, every number in double precision.  It shares no code with the GPU
 * library.
 *
 * Paper sections followed:
 *   Sec. II     Eq. C_quark, Eq. C_gluon (channel coefficients), Eq. C_a_b
 *               (the 2->2 collision integral), Eq. fg / Eq. fq (equilibrium),
 *               Eq. mg / Eq. mq (thermal masses), Eq. particle numbers,
 *               Eq. energy momentum tensor
 *   Sec. III    Eq. left handside (flux form), Eq. descrete left hand
 *               (central differences), Eq. delta function / work out delta E /
 *               delta replace (the k1z roots), Eq. MC C_gg and Eq. ca (direct
 *               MC estimator), Eq. small c relation (symmetric sampling)
 *   Appendix    Table I (matrix elements squared)
 */
#include "qgbe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NSP 7
#define GLUON 6
static const double PI = 3.14159265358979323846264338328;

/* SU(3) with fundamental fermions (Table I caption) */
static const double D_F = 3.0, C_A = 3.0, C_F = 4.0 / 3.0, D_A = 8.0;

/* helicity x colour degeneracy: N_q = 2*3, N_g = 2*8 (Eq. C_quark, C_gluon) */
static double degeneracy(int sp) { return sp == GLUON ? 16.0 : 6.0; }
static int is_gluon(int sp) { return sp == GLUON; }

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon, Moraes, Dror, Shaw,   */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds   */
/* of two 32x32->64 multiplies with a Weyl-sequence key schedule.      */
/* ------------------------------------------------------------------ */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0; k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 23-bit integer -> uniform in (0,1), the midpoint of its 2^-23 cell */
static double unif23(uint32_t v) { return ((double)v + 0.5) / 8388608.0; }

/* ------------------------------------------------------------------ */
/* Table I: |M|^2 summed over colours and helicities, every t and u   */
/* pole regulated by the gluon thermal mass m_g^2.                     */
/* ------------------------------------------------------------------ */
/* User matrix elements (Sec. II: an interface for matrix elements of the
   user's own).  A row set here replaces Table I for every channel of that
   row: |M|^2 = g^4 sum_k c_k s^a t^b u^c / ((t - mg2)^d (u - mg2)^e s^f).
   Process-wide state of the test oracle; n = 0 restores Table I. */
static struct {
  int n;
  double c[REF_MSQ_MAX_TERMS];
  int p[REF_MSQ_MAX_TERMS][6];
} g_user_msq[8];

int32_t ref_set_matrix_element(int32_t row, int32_t n, const double* coef, const int32_t* powers) {
  if (row < 1 || row > 7 || n < 0 || n > REF_MSQ_MAX_TERMS) return -1;
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < 6; ++i)
      if (powers[6 * k + i] < 0 || powers[6 * k + i] > REF_MSQ_MAX_POWER) return -1;
  g_user_msq[row].n = n;
  for (int k = 0; k < n; ++k) {
    g_user_msq[row].c[k] = coef[k];
    for (int i = 0; i < 6; ++i) g_user_msq[row].p[k][i] = powers[6 * k + i];
  }
  return 0;
}

static double user_msq(int row, double s, double t, double u, double mg2) {
  double sum = 0.0;
  for (int k = 0; k < g_user_msq[row].n; ++k) {
    const int* e = g_user_msq[row].p[k];
    const double num = pow(s, e[0]) * pow(t, e[1]) * pow(u, e[2]);
    const double den = pow(t - mg2, e[3]) * pow(u - mg2, e[4]) * pow(s, e[5]);
    sum += g_user_msq[row].c[k] * num / den;
  }
  return sum;
}

double ref_msq(int32_t row, double s, double t, double u, double mg2, double alpha_s) {
  const double g2 = 4.0 * PI * alpha_s;
  const double g4 = g2 * g2;
  const double tm = t - mg2, um = u - mg2;
  if (row >= 1 && row <= 7 && g_user_msq[row].n > 0) return g4 * user_msq(row, s, t, u, mg2);
  const double c_qq = 8.0 * g4 * D_F * D_F * C_F * C_F / D_A;       /* 8 g^4 dF^2 CF^2 / dA */
  const double c_int = 16.0 * g4 * D_F * C_F * (C_F - C_A / 2.0);    /* interference         */
  switch (row) {
    case 1: /* q1 q2 -> q1 q2 (and the antiquark variants) */
      return c_qq * (s * s + u * u) / (tm * tm);
    case 2: /* q1 q1 -> q1 q1 */
      return c_qq * ((s * s + u * u) / (tm * tm) + (s * s + t * t) / (um * um))
             + c_int * s * s / (tm * um);
    case 3: /* q1 q1bar -> q1 q1bar */
      return c_qq * ((s * s + u * u) / (tm * tm) + (u * u + t * t) / (s * s))
             + c_int * u * u / (tm * s);
    case 4: /* q1 q1bar -> q2 q2bar */
      return c_qq * (t * t + u * u) / (s * s);
    case 5: /* q1 q1bar -> g g */
      return 8.0 * g4 * D_F * C_F * C_F * (u / tm + t / um)
             - 8.0 * g4 * D_F * C_F * C_A * (t * t + u * u) / (s * s);
    case 6: /* q1 g -> q1 g */
      return -8.0 * g4 * D_F * C_F * C_F * (u / s + s / um)
             + 8.0 * g4 * D_F * C_F * C_A * (s * s + u * u) / (tm * tm);
    case 7: /* g g -> g g */
      return 16.0 * g4 * D_A * C_A * C_A
             * (3.0 - s * u / (tm * tm) - s * t / (um * um) - t * u / (s * s));
    default:
      return 0.0;
  }
}

/* ------------------------------------------------------------------ */
/* Channel table.  The 34 reactions {a,b}<->{c,d} of Table I among     */
/* u,d,s,ubar,dbar,sbar,g, written a(k1) b(k2) -> c(k3) d(p).  Each     */
/* distinct species X of a reaction gives one channel, with the tuple  */
/* permuted (time reversal and/or swapping both pairs, which leave s,  */
/* t, u unchanged) so that X sits at position 1.                       */
/* ------------------------------------------------------------------ */
static int list_reactions(int rx[][5]) {
  int n = 0;
  /* row 1: q_i q_j, qbar_i qbar_j (i<j), q_i qbar_j (i != j) */
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j) { int r[5] = {1, i, j, i, j}; memcpy(rx[n++], r, sizeof r); }
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j) { int r[5] = {1, 3 + i, 3 + j, 3 + i, 3 + j}; memcpy(rx[n++], r, sizeof r); }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (i != j) { int r[5] = {1, i, 3 + j, i, 3 + j}; memcpy(rx[n++], r, sizeof r); }
  /* row 2: q_i q_i, qbar_i qbar_i */
  for (int i = 0; i < 3; ++i) { int r[5] = {2, i, i, i, i}; memcpy(rx[n++], r, sizeof r); }
  for (int i = 0; i < 3; ++i) { int r[5] = {2, 3 + i, 3 + i, 3 + i, 3 + i}; memcpy(rx[n++], r, sizeof r); }
  /* row 3: q_i qbar_i -> q_i qbar_i */
  for (int i = 0; i < 3; ++i) { int r[5] = {3, i, 3 + i, i, 3 + i}; memcpy(rx[n++], r, sizeof r); }
  /* row 4: q_i qbar_i -> q_j qbar_j, unordered flavour pair i<j */
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j) { int r[5] = {4, i, 3 + i, j, 3 + j}; memcpy(rx[n++], r, sizeof r); }
  /* row 5: q_i qbar_i -> g g */
  for (int i = 0; i < 3; ++i) { int r[5] = {5, i, 3 + i, GLUON, GLUON}; memcpy(rx[n++], r, sizeof r); }
  /* row 6: q_i g, qbar_i g */
  for (int i = 0; i < 3; ++i) { int r[5] = {6, i, GLUON, i, GLUON}; memcpy(rx[n++], r, sizeof r); }
  for (int i = 0; i < 3; ++i) { int r[5] = {6, 3 + i, GLUON, 3 + i, GLUON}; memcpy(rx[n++], r, sizeof r); }
  /* row 7: g g -> g g */
  { int r[5] = {7, GLUON, GLUON, GLUON, GLUON}; memcpy(rx[n++], r, sizeof r); }
  return n;
}

int32_t ref_channels(const ref_grid* g, ref_channel* out, int32_t max) {
  int rx[64][5];
  int nr = list_reactions(rx);
  int n = 0;
  for (int r = 0; r < nr; ++r) {
    const int row = rx[r][0];
    const int a = rx[r][1], b = rx[r][2], c = rx[r][3], d = rx[r][4];
    if (!(g->row_mask & (1u << (row - 1)))) continue;
    if (!((g->species_mask >> a) & 1u) || !((g->species_mask >> b) & 1u) ||
        !((g->species_mask >> c) & 1u) || !((g->species_mask >> d) & 1u))
      continue;
    const int tup[4] = {a, b, c, d};
    /* distinct species in order of first appearance */
    int dist[4], nd = 0, first[4];
    for (int p = 0; p < 4; ++p) {
      int seen = 0;
      for (int q = 0; q < nd; ++q) if (dist[q] == tup[p]) seen = 1;
      if (!seen) { first[nd] = p; dist[nd++] = tup[p]; }
    }
    const double S_in = (a == b) ? 2.0 : 1.0;
    const double S_out = (c == d) ? 2.0 : 1.0;
    /* {a,b} = {c,d} as multisets: summing every position counts each
       collision twice (forward and its time reverse are the same set) */
    const int elastic = ((a == c && b == d) || (a == d && b == c));
    const double kappa = elastic ? 0.5 : 1.0;
    for (int q = 0; q < nd; ++q) {
      if (n >= max) return -1;
      ref_channel* ch = &out[n++];
      int perm[4];
      switch (first[q]) {
        case 0: perm[0] = 0; perm[1] = 1; perm[2] = 2; perm[3] = 3; break; /* identity      */
        case 1: perm[0] = 1; perm[1] = 0; perm[2] = 3; perm[3] = 2; break; /* swap pairs    */
        case 2: perm[0] = 2; perm[1] = 3; perm[2] = 0; perm[3] = 1; break; /* time reversal */
        default: perm[0] = 3; perm[1] = 2; perm[2] = 1; perm[3] = 0; break;
      }
      ch->row = row;
      for (int p = 0; p < 4; ++p) ch->sp[p] = tup[perm[p]];
      ch->code = ((ch->sp[0] * 7 + ch->sp[1]) * 7 + ch->sp[2]) * 7 + ch->sp[3];
      int nX = 0;
      for (int p = 0; p < 4; ++p) if (tup[p] == dist[q]) ++nX;
      ch->w = kappa / (S_in * S_out * (double)nd);
      ch->sigma = (double)nX * kappa / (S_in * S_out);
    }
  }
  /* canonical order: ascending channel code */
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && out[j - 1].code > out[j].code; --j) {
      ref_channel tmp = out[j - 1]; out[j - 1] = out[j]; out[j] = tmp;
    }
  return n;
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */
static int64_t n_cells(const ref_grid* g) { return (int64_t)g->n_x[0] * g->n_x[1] * g->n_x[2]; }
static int64_t n_nodes(const ref_grid* g) { return (int64_t)g->n_p[0] * g->n_p[1] * g->n_p[2]; }
static double dp_of(const ref_grid* g, int a) { return 2.0 * g->p_half[a] / g->n_p[a]; }
static double dx_of(const ref_grid* g, int a) { return 2.0 * g->x_half[a] / g->n_x[a]; }

static void node_momentum(const ref_grid* g, int64_t lin, double p[3]) {
  int64_t iz = lin % g->n_p[2];
  int64_t iy = (lin / g->n_p[2]) % g->n_p[1];
  int64_t ix = lin / ((int64_t)g->n_p[2] * g->n_p[1]);
  const int64_t id[3] = {ix, iy, iz};
  for (int a = 0; a < 3; ++a) p[a] = -g->p_half[a] + ((double)id[a] + 0.5) * dp_of(g, a);
}

static double norm2(const double v[3]) { return v[0] * v[0] + v[1] * v[1] + v[2] * v[2]; }

/* trilinear (cloud-in-cell) stencil over the 8 surrounding cell centres,
   clamped at the box: a coordinate beyond the outermost centre uses that
   centre.  Interpolation and deposition share these weights. */
static void cic_stencil(const ref_grid* g, const double p[3], int64_t idx[8], double w[8]) {
  int i0[3], i1[3];
  double w1[3];
  for (int a = 0; a < 3; ++a) {
    const int n = g->n_p[a];
    if (n == 1) { i0[a] = 0; i1[a] = 0; w1[a] = 0.0; continue; }
    double t = (p[a] + g->p_half[a]) / dp_of(g, a) - 0.5;
    if (t < 0.0) t = 0.0;
    if (t > (double)(n - 1)) t = (double)(n - 1);
    int lo = (int)floor(t);
    if (lo > n - 2) lo = n - 2;
    i0[a] = lo; i1[a] = lo + 1; w1[a] = t - (double)lo;
  }
  for (int c = 0; c < 8; ++c) {
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const int ix = bx ? i1[0] : i0[0], iy = by ? i1[1] : i0[1], iz = bz ? i1[2] : i0[2];
    idx[c] = ((int64_t)ix * g->n_p[1] + iy) * g->n_p[2] + iz;
    w[c] = (bx ? w1[0] : 1.0 - w1[0]) * (by ? w1[1] : 1.0 - w1[1]) * (bz ? w1[2] : 1.0 - w1[2]);
  }
}

static double interp(const ref_grid* g, const double* f_sp_cell, const double p[3]) {
  int64_t idx[8];
  double w[8], v = 0.0;
  cic_stencil(g, p, idx, w);
  for (int c = 0; c < 8; ++c) v += w[c] * f_sp_cell[idx[c]];
  return v;
}

static int inside_box(const ref_grid* g, const double p[3]) {
  for (int a = 0; a < 3; ++a)
    if (p[a] < -g->p_half[a] || p[a] > g->p_half[a]) return 0;
  return 1;
}

/* Eq. fg / Eq. fq */
static double f_equilibrium(const ref_equilibrium* eq, int sp, double E) {
  const double x = (E - eq->mu[sp]) / eq->T;
  return is_gluon(sp) ? 1.0 / expm1(x) : 1.0 / (exp(x) + 1.0);
}

/* Minkowski square of a 4-vector, metric (+,-,-,-) */
static double mink2(const double k[4]) { return k[0] * k[0] - k[1] * k[1] - k[2] * k[2] - k[3] * k[3]; }

/* boost 4-vector k into the rest frame of the total momentum P (mass M) */
static void boost_to_rest(const double P[4], double M, const double k[4], double out[4]) {
  const double Pk = P[1] * k[1] + P[2] * k[2] + P[3] * k[3];
  out[0] = (P[0] * k[0] - Pk) / M;
  const double c = Pk / (M * (P[0] + M)) - k[0] / M;
  for (int a = 1; a < 4; ++a) out[a] = k[a] + P[a] * c;
}

/* inverse: from the rest frame of P back to the frame where P is given */
static void boost_from_rest(const double P[4], double M, const double k[4], double out[4]) {
  const double Pk = P[1] * k[1] + P[2] * k[2] + P[3] * k[3];
  out[0] = (P[0] * k[0] + Pk) / M;
  const double c = Pk / (M * (P[0] + M)) + k[0] / M;
  for (int a = 1; a < 4; ++a) out[a] = k[a] + P[a] * c;
}

/* orthonormal basis (b1, b2) completing the unit vector n, after Duff,
   Burgess, Christensen, Hery, Kensler, Liani, Villemin, "Building an
   orthonormal basis, revisited", JCGT 6(1), 2017 */
static void onb(const double n[3], double b1[3], double b2[3]) {
  const double sgn = copysign(1.0, n[2]);
  const double a = -1.0 / (sgn + n[2]);
  const double b = n[0] * n[1] * a;
  b1[0] = 1.0 + sgn * n[0] * n[0] * a; b1[1] = sgn * b; b1[2] = -sgn * n[0];
  b2[0] = b; b2[1] = sgn + n[1] * n[1] * a; b2[2] = -n[1];
}

static double mass2_of(const double* mass2, int64_t ncell, int sp, int64_t cell) {
  return mass2[(int64_t)sp * ncell + cell];
}

/* occupation and statistics factors, then the bracket of Eq. C_a_b with
   position 1 as the observed particle: gain = f3 f4 F1 F2, loss = f1 f2 F3 F4 */
static void bracket(const ref_grid* g, const ref_channel* ch, const double* f, int64_t cell,
                    int64_t p1_lin, const double k[4][4], int flags,
                    const ref_equilibrium* eq, ref_point* out) {
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  double fv[4];
  for (int i = 0; i < 4; ++i) {
    const int sp = ch->sp[i];
    if (flags & REF_ANALYTIC_F) {
      fv[i] = f_equilibrium(eq, sp, k[i][0]);
    } else {
      const double* fc = f + ((int64_t)sp * nc + cell) * nn;
      if (i == 0 && p1_lin >= 0) {
        fv[i] = fc[p1_lin];
      } else {
        const double p[3] = {k[i][1], k[i][2], k[i][3]};
        fv[i] = interp(g, fc, p);
      }
    }
  }
  double F[4];
  for (int i = 0; i < 4; ++i) F[i] = is_gluon(ch->sp[i]) ? 1.0 + fv[i] : 1.0 - fv[i];
  const double gain = fv[2] * fv[3] * F[0] * F[1];
  const double loss = fv[0] * fv[1] * F[2] * F[3];
  for (int i = 0; i < 4; ++i) out->f[i] = fv[i];
  if (flags & REF_B_ONE) { out->B = 1.0; out->GL = 1.0; }
  else { out->B = gain - loss; out->GL = gain + loss; }
}

int32_t ref_eval_cm(const ref_grid* g, const ref_channel* ch, const double* f,
                    const double* mass2, int32_t cell, const double p1[3],
                    int32_t p1_lin, const double p2[3], double cos_th,
                    double phi, int32_t flags, const ref_equilibrium* eq,
                    ref_point* out) {
  memset(out, 0, sizeof *out);
  const int64_t nc = n_cells(g);
  double m2[4];
  for (int i = 0; i < 4; ++i)
    m2[i] = (flags & REF_MASSLESS) ? 0.0 : mass2_of(mass2, nc, ch->sp[i], cell);
  const double mg2 = mass2_of(mass2, nc, GLUON, cell);

  double k1[4] = {sqrt(norm2(p1) + m2[0]), p1[0], p1[1], p1[2]};
  double k2[4] = {sqrt(norm2(p2) + m2[1]), p2[0], p2[1], p2[2]};
  /* the 1/(2E) measure of Eq. C_a_b is singular at a massless p = 0; that
     single point carries no weight (as in the thermal-mass sums) */
  if (!(k1[0] > 0.0) || !(k2[0] > 0.0)) return 0;
  double P[4];
  for (int a = 0; a < 4; ++a) P[a] = k1[a] + k2[a];
  const double s = mink2(P);
  const double m3 = sqrt(m2[2]), m4 = sqrt(m2[3]);
  for (int a = 0; a < 4; ++a) { out->k[0][a] = k1[a]; out->k[1][a] = k2[a]; }
  out->s = s;
  if (!(s > (m3 + m4) * (m3 + m4))) return 0; /* below threshold */
  const double M = sqrt(s);
  const double pstar = sqrt((s - (m3 + m4) * (m3 + m4)) * (s - (m3 - m4) * (m3 - m4))) / (2.0 * M);

  /* polar axis: direction of k1 in the CM frame */
  double k1s[4];
  boost_to_rest(P, M, k1, k1s);
  const double n1 = sqrt(k1s[1] * k1s[1] + k1s[2] * k1s[2] + k1s[3] * k1s[3]);
  const double e3[3] = {k1s[1] / n1, k1s[2] / n1, k1s[3] / n1};
  double e1[3], e2[3];
  onb(e3, e1, e2);
  const double sin_th = sqrt(fmax(0.0, 1.0 - cos_th * cos_th));
  double dir[3];
  for (int a = 0; a < 3; ++a)
    dir[a] = sin_th * cos(phi) * e1[a] + sin_th * sin(phi) * e2[a] + cos_th * e3[a];
  double k3s[4] = {sqrt(pstar * pstar + m2[2]), pstar * dir[0], pstar * dir[1], pstar * dir[2]};
  double k4s[4] = {sqrt(pstar * pstar + m2[3]), -pstar * dir[0], -pstar * dir[1], -pstar * dir[2]};
  double k3[4], k4[4];
  boost_from_rest(P, M, k3s, k3);
  boost_from_rest(P, M, k4s, k4);
  for (int a = 0; a < 4; ++a) { out->k[2][a] = k3[a]; out->k[3][a] = k4[a]; }
  out->pstar = pstar;

  const double p3[3] = {k3[1], k3[2], k3[3]}, p4[3] = {k4[1], k4[2], k4[3]};
  if (!(flags & REF_NO_BOXCUT) && (!inside_box(g, p3) || !inside_box(g, p4))) return 0;

  double d13[4], d14[4];
  for (int a = 0; a < 4; ++a) { d13[a] = k1[a] - k3[a]; d14[a] = k1[a] - k4[a]; }
  out->t = mink2(d13);
  out->u = mink2(d14);
  out->msq = ref_msq(ch->row, s, out->t, out->u, mg2, g->alpha_s);
  bracket(g, ch, f, cell, p1_lin, (const double(*)[4])out->k, flags, eq, out);

  /* dPhi_2 = |p*| dOmega / (16 pi^2 sqrt(s)); the k2 measure d^3k2/((2pi)^3 2E2);
     the 1/(2E1) of the observed particle (Eq. C_a_b) */
  const double norm = pstar / (pow(2.0 * PI, 3) * 2.0 * k1[0] * 2.0 * k2[0] * 16.0 * PI * PI * M);
  out->g = out->msq * out->B * norm;
  out->gscale = fabs(out->msq) * out->GL * norm;
  out->valid = 1;
  return 1;
}

/* ------------------------------------------------------------------ */
/* Deposits.  Symmetric sampling (Eq. small c relation): the value v   */
/* of one sample is added at positions 1 and 2 and subtracted at 3 and */
/* 4; off-grid momenta are spread over the 8 surrounding nodes.        */
/* ------------------------------------------------------------------ */
typedef struct {
  double* A;    /* [7][cells][nodes] */
  double* S;    /* same or NULL      */
} accum;

static void deposit_point(const ref_grid* g, accum* acc, int sp, int64_t cell,
                          const double p[3], double v, double vs) {
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  int64_t idx[8];
  double w[8];
  cic_stencil(g, p, idx, w);
  double* Ac = acc->A + ((int64_t)sp * nc + cell) * nn;
  for (int c = 0; c < 8; ++c) Ac[idx[c]] += v * w[c];
  if (acc->S) {
    double* Sc = acc->S + ((int64_t)sp * nc + cell) * nn;
    for (int c = 0; c < 8; ++c) Sc[idx[c]] += fabs(vs) * w[c];
  }
}

static void deposit_sample(const ref_grid* g, const ref_channel* ch, accum* acc, int64_t cell,
                           int64_t p1_lin, const double k[4][4], int symmetric, double v,
                           double vs, double v_direct, double vs_direct) {
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  const int64_t at1 = ((int64_t)ch->sp[0] * nc + cell) * nn + p1_lin;
  if (!acc->A) return; /* item sums only */
  if (!symmetric) {
    acc->A[at1] += v_direct;
    if (acc->S) acc->S[at1] += fabs(vs_direct);
    return;
  }
  acc->A[at1] += v;
  if (acc->S) acc->S[at1] += fabs(vs);
  const double p2[3] = {k[1][1], k[1][2], k[1][3]};
  const double p3[3] = {k[2][1], k[2][2], k[2][3]};
  const double p4[3] = {k[3][1], k[3][2], k[3][3]};
  deposit_point(g, acc, ch->sp[1], cell, p2, +v, vs);
  deposit_point(g, acc, ch->sp[2], cell, p3, -v, vs);
  deposit_point(g, acc, ch->sp[3], cell, p4, -v, vs);
}

/* ------------------------------------------------------------------ */
/* Second parameterisation: the paper's own elimination of one         */
/* momentum with the delta function (Eq. work out delta E, Eq. delta   */
/* replace).  In channel order: observed k1 on the grid, k2 in the box, */
/* k3x and k3y sampled, k3z from the two roots of energy conservation, */
/* k4 = k1 + k2 - k3.                                                  */
/* ------------------------------------------------------------------ */
static int eval_root(const ref_grid* g, const ref_channel* ch, const double* f,
                     const double* mass2, int64_t cell, const double p1[3], int64_t p1_lin,
                     const double p2[3], double p3x, double p3y, int flags,
                     const ref_equilibrium* eq, ref_point pts[2]) {
  const int64_t nc = n_cells(g);
  double m2[4];
  for (int i = 0; i < 4; ++i)
    m2[i] = (flags & REF_MASSLESS) ? 0.0 : mass2_of(mass2, nc, ch->sp[i], cell);
  const double mg2 = mass2_of(mass2, nc, GLUON, cell);
  const double E1 = sqrt(norm2(p1) + m2[0]), E2 = sqrt(norm2(p2) + m2[1]);
  const double W = E1 + E2;
  const double Q[3] = {p1[0] + p2[0], p1[1] + p2[1], p1[2] + p2[2]};
  const double a = p3x * p3x + p3y * p3y + m2[2];
  const double b = (Q[0] - p3x) * (Q[0] - p3x) + (Q[1] - p3y) * (Q[1] - p3y) + m2[3];
  const double c = W * W + a - b - Q[2] * Q[2];
  const double den = W * W - Q[2] * Q[2];
  const double H = c * c - 4.0 * a * den;
  int nv = 0;
  if (!(H >= 0.0) || !(den > 0.0)) return 0;
  const double sq = sqrt(H);
  for (int r = 0; r < 2; ++r) {
    const double z = (c * Q[2] + (r == 0 ? 1.0 : -1.0) * W * sq) / (2.0 * den);
    if (!(c + 2.0 * Q[2] * z > 0.0)) continue;
    const double E3 = sqrt(a + z * z);
    if (!(E3 < W)) continue;
    const double p3[3] = {p3x, p3y, z};
    const double p4[3] = {Q[0] - p3x, Q[1] - p3y, Q[2] - z};
    const double E4 = sqrt(norm2(p4) + m2[3]);
    ref_point* o = &pts[nv];
    memset(o, 0, sizeof *o);
    const double k1[4] = {E1, p1[0], p1[1], p1[2]};
    const double k2[4] = {E2, p2[0], p2[1], p2[2]};
    const double k3[4] = {E3, p3[0], p3[1], p3[2]};
    const double k4[4] = {E4, p4[0], p4[1], p4[2]};
    for (int q = 0; q < 4; ++q) { o->k[0][q] = k1[q]; o->k[1][q] = k2[q]; o->k[2][q] = k3[q]; o->k[3][q] = k4[q]; }
    if (!(flags & REF_NO_BOXCUT) && (!inside_box(g, p3) || !inside_box(g, p4))) continue;
    double P[4], d13[4], d14[4];
    for (int q = 0; q < 4; ++q) { P[q] = k1[q] + k2[q]; d13[q] = k1[q] - k3[q]; d14[q] = k1[q] - k4[q]; }
    o->s = mink2(P);
    o->t = mink2(d13);
    o->u = mink2(d14);
    o->msq = ref_msq(ch->row, o->s, o->t, o->u, mg2, g->alpha_s);
    bracket(g, ch, f, cell, p1_lin, (const double(*)[4])o->k, flags, eq, o);
    const double J = fabs(z / E3 - p4[2] / E4);
    const double norm = 1.0 / (pow(2.0 * PI, 5) * 16.0 * E1 * E2 * E3 * E4 * J);
    o->g = o->msq * o->B * norm;
    o->gscale = fabs(o->msq) * o->GL * norm;
    o->valid = 1;
    ++nv;
  }
  return nv;
}

/* ------------------------------------------------------------------ */
/* The alternative elimination (the paper's second choice): k4 and     */
/* k3x, k3y sampled, k2 = k3 + k4 - k1, and k3z from energy            */
/* conservation E3 - E2 = E1 - E4 =: D.  With Q = k4 - k1 and           */
/* a = k3x^2 + k3y^2 + m3^2, squaring |k3 + Q|^2 + m2^2 = (E3 - D)^2    */
/* gives C + 2 Qz k3z = -2 D E3, C = 2 (k3x Qx + k3y Qy) + Q^2 + m2^2  */
/* - m3^2 - D^2, and squaring again the quadratic                      */
/* (Qz^2 - D^2) z^2 + C Qz z + (C^2/4 - D^2 a) = 0.  A root counts when */
/* the unsquared equation holds (C + 2 Qz z and D of opposite signs,   */
/* E2 = E3 - D > 0).  Its coefficient Qz^2 - D^2 has no fixed sign,    */
/* unlike the W^2 - Qz^2 = s + Q_perp^2 > 0 of the paper's choice.      */
/* ------------------------------------------------------------------ */
static int eval_root_k3(const ref_grid* g, const ref_channel* ch, const double* f,
                        const double* mass2, int64_t cell, const double p1[3], int64_t p1_lin,
                        const double p4[3], double p3x, double p3y, int flags,
                        const ref_equilibrium* eq, ref_point pts[2]) {
  const int64_t nc = n_cells(g);
  double m2[4];
  for (int i = 0; i < 4; ++i)
    m2[i] = (flags & REF_MASSLESS) ? 0.0 : mass2_of(mass2, nc, ch->sp[i], cell);
  const double mg2 = mass2_of(mass2, nc, GLUON, cell);
  const double E1 = sqrt(norm2(p1) + m2[0]), E4 = sqrt(norm2(p4) + m2[3]);
  const double D = E1 - E4;
  const double Q[3] = {p4[0] - p1[0], p4[1] - p1[1], p4[2] - p1[2]};
  const double a = p3x * p3x + p3y * p3y + m2[2];
  const double C = 2.0 * (p3x * Q[0] + p3y * Q[1]) + norm2(Q) + m2[1] - m2[2] - D * D;
  const double den = Q[2] * Q[2] - D * D;
  const double H = C * C + 4.0 * a * den;
  int nv = 0;
  if (!(H >= 0.0) || den == 0.0 || D == 0.0) return 0;
  const double sq = fabs(D) * sqrt(H);
  for (int r = 0; r < 2; ++r) {
    const double z = (-C * Q[2] + (r == 0 ? 1.0 : -1.0) * sq) / (2.0 * den);
    if (!((C + 2.0 * Q[2] * z) * D < 0.0)) continue;
    const double E3 = sqrt(a + z * z);
    if (!(E3 - D > 0.0)) continue;
    const double p3[3] = {p3x, p3y, z};
    const double p2[3] = {p3[0] + Q[0], p3[1] + Q[1], p3[2] + Q[2]};
    const double E2 = sqrt(norm2(p2) + m2[1]);
    ref_point* o = &pts[nv];
    memset(o, 0, sizeof *o);
    const double k1[4] = {E1, p1[0], p1[1], p1[2]};
    const double k2[4] = {E2, p2[0], p2[1], p2[2]};
    const double k3[4] = {E3, p3[0], p3[1], p3[2]};
    const double k4[4] = {E4, p4[0], p4[1], p4[2]};
    for (int q = 0; q < 4; ++q) { o->k[0][q] = k1[q]; o->k[1][q] = k2[q]; o->k[2][q] = k3[q]; o->k[3][q] = k4[q]; }
    if (!(flags & REF_NO_BOXCUT) && (!inside_box(g, p2) || !inside_box(g, p3))) continue;
    double P[4], d13[4], d14[4];
    for (int q = 0; q < 4; ++q) { P[q] = k1[q] + k2[q]; d13[q] = k1[q] - k3[q]; d14[q] = k1[q] - k4[q]; }
    o->s = mink2(P);
    o->t = mink2(d13);
    o->u = mink2(d14);
    o->msq = ref_msq(ch->row, o->s, o->t, o->u, mg2, g->alpha_s);
    bracket(g, ch, f, cell, p1_lin, (const double(*)[4])o->k, flags, eq, o);
    /* d(E1 + E2 - E3 - E4)/dk3z with k2 = k3 + Q */
    const double J = fabs(p2[2] / E2 - z / E3);
    const double norm = 1.0 / (pow(2.0 * PI, 5) * 16.0 * E1 * E2 * E3 * E4 * J);
    o->g = o->msq * o->B * norm;
    o->gscale = fabs(o->msq) * o->GL * norm;
    o->valid = 1;
    ++nv;
  }
  return nv;
}

/* ------------------------------------------------------------------ */
/* Work items.  One (cell, channel, p1) item draws its N samples from   */
/* Philox4x32-10 with key (seed_lo, seed_hi + step) and counter         */
/* (s, p1_lin, cell, code<<8 | block).                                  */
/* ------------------------------------------------------------------ */
static void draw_block(uint64_t seed, uint32_t step, uint32_t s, uint32_t p1_lin, uint32_t cell,
                       uint32_t code, uint32_t block, uint32_t out[4]) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) + step};
  const uint32_t ctr[4] = {s, p1_lin, cell, (code << 8) | block};
  ref_philox4x32_10(ctr, key, out);
}

/* five 23-bit fields from one 128-bit block: the top 23 bits of each word
   give four, the low 9 bits of words 0 and 1 and bits 4..8 of word 2 give
   the fifth */
static void five_uniforms(const uint32_t x[4], double u[5]) {
  uint32_t v[5];
  for (int i = 0; i < 4; ++i) v[i] = x[i] >> 9;
  v[4] = ((x[0] & 0x1FFu) << 14) | ((x[1] & 0x1FFu) << 5) | ((x[2] & 0x1FFu) >> 4);
  for (int i = 0; i < 5; ++i) u[i] = unif23(v[i]);
}

/* the five unit-cube variables of sample s of a work item, uniform sampler
   (CM-angle estimator): block 0 of the item's Philox stream, five 23-bit
   fields.  Exported for the tests of recorded training rows. */
void ref_sample_uniforms(uint64_t seed, uint32_t step, uint32_t s, uint32_t p1_lin, uint32_t cell,
                         uint32_t code, double u_out[5]) {
  uint32_t x[4];
  draw_block(seed, step, s, p1_lin, cell, code, 0u, x);
  five_uniforms(x, u_out);
}

static double box_volume(const ref_grid* g) {
  return (2.0 * g->p_half[0]) * (2.0 * g->p_half[1]) * (2.0 * g->p_half[2]);
}

static void run_item_uniform(const ref_grid* g, const ref_channel* ch, const double* f,
                             const double* mass2, uint64_t seed, uint32_t step, int32_t N,
                             int estimator, int symmetric, int flags,
                             const ref_equilibrium* eq, int64_t cell, int64_t p1_lin,
                             accum* acc, double* item, double* item_scale) {
  double p1[3];
  node_momentum(g, p1_lin, p1);
  const double Vp = box_volume(g);
  double sum = 0.0, ssum = 0.0;
  for (int32_t s = 0; s < N; ++s) {
    uint32_t x[4];
    const uint32_t blk = (estimator == REF_EST_CM) ? 0u : 2u;
    draw_block(seed, step, (uint32_t)s, (uint32_t)p1_lin, (uint32_t)cell, (uint32_t)ch->code, blk, x);
    double u[5];
    five_uniforms(x, u);
    const double p2[3] = {-g->p_half[0] + 2.0 * g->p_half[0] * u[0],
                          -g->p_half[1] + 2.0 * g->p_half[1] * u[1],
                          -g->p_half[2] + 2.0 * g->p_half[2] * u[2]};
    if (estimator == REF_EST_CM) {
      const double V5 = Vp * 4.0 * PI;
      const double cth = 2.0 * u[3] - 1.0;
      const double phi = 2.0 * PI * u[4];
      ref_point pt;
      if (!ref_eval_cm(g, ch, f, mass2, (int32_t)cell, p1, (int32_t)p1_lin, p2, cth, phi, flags, eq, &pt))
        continue;
      const double v = ch->w * V5 * pt.g / N, vs = ch->w * V5 * pt.gscale / N;
      const double vd = ch->sigma * V5 * pt.g / N, vsd = ch->sigma * V5 * pt.gscale / N;
      deposit_sample(g, ch, acc, cell, p1_lin, (const double(*)[4])pt.k, symmetric, v, vs, vd, vsd);
      sum += symmetric ? v : vd;
      ssum += symmetric ? vs : vsd;
    } else {
      const double V5 = Vp * (2.0 * g->p_half[0]) * (2.0 * g->p_half[1]);
      const double p3x = -g->p_half[0] + 2.0 * g->p_half[0] * u[3];
      const double p3y = -g->p_half[1] + 2.0 * g->p_half[1] * u[4];
      ref_point pts[2];
      /* the box-uniform momentum is k2 for the paper's choice, k4 for the alternative */
      const int nv = (estimator == REF_EST_ROOT)
                         ? eval_root(g, ch, f, mass2, cell, p1, p1_lin, p2, p3x, p3y, flags, eq, pts)
                         : eval_root_k3(g, ch, f, mass2, cell, p1, p1_lin, p2, p3x, p3y, flags, eq, pts);
      for (int r = 0; r < nv; ++r) {
        const double v = ch->w * V5 * pts[r].g / N, vs = ch->w * V5 * pts[r].gscale / N;
        const double vd = ch->sigma * V5 * pts[r].g / N, vsd = ch->sigma * V5 * pts[r].gscale / N;
        deposit_sample(g, ch, acc, cell, p1_lin, (const double(*)[4])pts[r].k, symmetric, v, vs, vd, vsd);
        sum += symmetric ? v : vd;
        ssum += symmetric ? vs : vsd;
      }
    }
  }
  if (item) *item = sum;
  if (item_scale) *item_scale = ssum;
}

/* log of the mixture-of-logistic-normals density on the unit cube at the
   point with logit coordinates y (without the defensive share) */
static double log_q_mixture(int K, const uint32_t* thr, const float* mu, const float* sg,
                            const double y[5]) {
  double lw[64];
  double mx = -INFINITY;
  for (int k = 0; k < K; ++k) {
    const double hi = (k + 1 < K) ? (double)thr[k + 1] : 4294967296.0;
    const double pk = (hi - (double)thr[k]) / 4294967296.0;
    if (!(pk > 0.0)) { lw[k] = -INFINITY; continue; }
    double l = log(pk);
    for (int d = 0; d < 5; ++d) {
      const double sd = (double)sg[k * 5 + d];
      const double z = (y[d] - (double)mu[k * 5 + d]) / sd;
      l += -0.5 * z * z - log(sd) - 0.5 * log(2.0 * PI);
    }
    lw[k] = l;
    if (l > mx) mx = l;
  }
  if (mx == -INFINITY) return -INFINITY;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) if (lw[k] > -INFINITY) acc += exp(lw[k] - mx);
  double lq = mx + log(acc);
  /* Jacobian of u = sigmoid(y): du/dy = u (1 - u) */
  for (int d = 0; d < 5; ++d) lq -= log(1.0 / (1.0 + exp(-y[d]))) + log(1.0 / (1.0 + exp(y[d])));
  return lq;
}

static void run_item_learned(const ref_grid* g, const ref_channel* ch, const double* f,
                             const double* mass2, uint64_t seed, uint32_t step, int32_t N,
                             int K, const uint32_t* thr, const float* mu, const float* sg,
                             int64_t cell, int64_t p1_lin, accum* acc, double* item, double* item_scale) {
  double p1[3];
  node_momentum(g, p1_lin, p1);
  const double V5 = box_volume(g) * 4.0 * PI;
  const double alpha = (double)thr[0] / 4294967296.0;
  double sum = 0.0, ssum = 0.0;
  for (int32_t s = 0; s < N; ++s) {
    uint32_t x[8];
    draw_block(seed, step, (uint32_t)s, (uint32_t)p1_lin, (uint32_t)cell, (uint32_t)ch->code, 0u, x);
    draw_block(seed, step, (uint32_t)s, (uint32_t)p1_lin, (uint32_t)cell, (uint32_t)ch->code, 1u, x + 4);
    double u[5], y[5];
    if (x[0] < thr[0]) {
      /* defensive uniform component */
      for (int d = 0; d < 5; ++d) {
        u[d] = unif23(x[1 + d] >> 9);
        y[d] = log(u[d] / (1.0 - u[d]));
      }
    } else {
      int k = 0;
      for (int j = 1; j < K; ++j) if (x[0] >= thr[j]) k = j;
      double z[6];
      for (int pr = 0; pr < 3; ++pr) {
        const double a1 = unif23(x[1 + 2 * pr] >> 9), a2 = unif23(x[2 + 2 * pr] >> 9);
        const double r = sqrt(-2.0 * log(a1));
        z[2 * pr] = r * cos(2.0 * PI * a2);
        z[2 * pr + 1] = r * sin(2.0 * PI * a2);
      }
      for (int d = 0; d < 5; ++d) {
        y[d] = (double)mu[k * 5 + d] + (double)sg[k * 5 + d] * z[d];
        u[d] = 1.0 / (1.0 + exp(-y[d]));
      }
    }
    const double q = alpha + exp(log_q_mixture(K, thr, mu, sg, y));
    const double p2[3] = {-g->p_half[0] + 2.0 * g->p_half[0] * u[0],
                          -g->p_half[1] + 2.0 * g->p_half[1] * u[1],
                          -g->p_half[2] + 2.0 * g->p_half[2] * u[2]};
    const double cth = 2.0 * u[3] - 1.0;
    const double phi = 2.0 * PI * u[4];
    ref_point pt;
    if (!ref_eval_cm(g, ch, f, mass2, (int32_t)cell, p1, (int32_t)p1_lin, p2, cth, phi, 0, NULL, &pt))
      continue;
    const double v = ch->w * V5 * pt.g / (N * q), vs = ch->w * V5 * pt.gscale / (N * q);
    deposit_sample(g, ch, acc, cell, p1_lin, (const double(*)[4])pt.k, 1, v, vs, 0.0, 0.0);
    sum += v;
    ssum += fabs(vs);
  }
  if (item) *item = sum;
  if (item_scale) *item_scale = ssum;
}

static int check_grid(const ref_grid* g) {
  for (int a = 0; a < 3; ++a) {
    if (g->n_x[a] < 1 || g->n_p[a] < 1) return -1;
    if (!(g->x_half[a] > 0.0) || !(g->p_half[a] > 0.0)) return -1;
  }
  return 0;
}

int32_t ref_stencil(const ref_grid* g, int64_t n, const double* pts, int64_t* idx, double* w) {
  if (check_grid(g) || n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) cic_stencil(g, pts + 3 * i, idx + 8 * i, w + 8 * i);
  return 0;
}

typedef enum { ITEM_UNIFORM, ITEM_LEARNED } item_kind;

typedef struct {
  const ref_grid* g; const double* f; const double* mass2; uint64_t seed; uint32_t step;
  int32_t N; int estimator, symmetric, flags; const ref_equilibrium* eq;
  int K; const uint32_t* thr; const float* mu; const float* sg; int table_per_cell;
  const uint8_t* chan_learned;
} run_args;

static int32_t run_all(const run_args* ra, item_kind kind, double* A_out, double* S_out,
                       double* item_sum, int32_t n_threads) {
  const ref_grid* g = ra->g;
  if (check_grid(g)) return -1;
  if (ra->N <= 0) return -1;
  ref_channel chans[128];
  const int nch = ref_channels(g, chans, 128);
  if (nch < 0) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  const int64_t field = (int64_t)NSP * nc * nn;
  memset(A_out, 0, sizeof(double) * field);
  if (S_out) memset(S_out, 0, sizeof(double) * field);
  const int64_t n_items = nc * nch * nn;
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  (void)n_threads;
#endif
  double** bufA = (double**)calloc(nt, sizeof(double*));
  double** bufS = (double**)calloc(nt, sizeof(double*));
  for (int t = 0; t < nt; ++t) {
    bufA[t] = (double*)calloc(field, sizeof(double));
    bufS[t] = S_out ? (double*)calloc(field, sizeof(double)) : NULL;
  }
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
  for (int64_t it = 0; it < n_items; ++it) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    const int64_t cell = it / ((int64_t)nch * nn);
    const int64_t rem = it % ((int64_t)nch * nn);
    const int ci = (int)(rem / nn);
    const int64_t p1 = rem % nn;
    accum acc = {bufA[tid], bufS[tid]};
    double* item = item_sum ? &item_sum[(cell * nch + ci) * nn + p1] : NULL;
    if (kind == ITEM_UNIFORM || (ra->chan_learned && !ra->chan_learned[ci])) {
      run_item_uniform(g, &chans[ci], ra->f, ra->mass2, ra->seed, ra->step, ra->N, ra->estimator,
                       ra->symmetric, ra->flags, ra->eq, cell, p1, &acc, item, NULL);
    } else {
      const int64_t row = ((ra->table_per_cell ? cell : 0) * nch + ci) * nn + p1;
      run_item_learned(g, &chans[ci], ra->f, ra->mass2, ra->seed, ra->step, ra->N, ra->K,
                       ra->thr + row * ra->K, ra->mu + row * ra->K * 5, ra->sg + row * ra->K * 5,
                       cell, p1, &acc, item, NULL);
    }
  }
  for (int t = 0; t < nt; ++t) {
    for (int64_t i = 0; i < field; ++i) A_out[i] += bufA[t][i];
    if (S_out) for (int64_t i = 0; i < field; ++i) S_out[i] += bufS[t][i];
    free(bufA[t]);
    free(bufS[t]);
  }
  free(bufA);
  free(bufS);
  return nch;
}

/* direct sums of selected work items with the mixture proposal (the same
   table layout and fallback flags as ref_collision_learned) */
int32_t ref_item_sums_learned(const ref_grid* g, const double* f, const double* mass2, uint64_t seed,
                              uint32_t step, int32_t n_samples, int32_t K, const uint32_t* thr,
                              const float* mu, const float* sigma, int32_t table_per_cell,
                              const uint8_t* chan_learned, int64_t n_sel, const int64_t* items,
                              double* out, double* out_scale, int32_t n_threads) {
  if (check_grid(g) || n_samples <= 0 || K < 1 || K > 64) return -1;
  ref_channel chans[128];
  const int nch = ref_channels(g, chans, 128);
  if (nch < 0) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  for (int64_t i = 0; i < n_sel; ++i)
    if (items[3 * i] < 0 || items[3 * i] >= nc || items[3 * i + 1] < 0 || items[3 * i + 1] >= nch ||
        items[3 * i + 2] < 0 || items[3 * i + 2] >= nn)
      return -1;
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  (void)n_threads;
#endif
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic)
#endif
  for (int64_t i = 0; i < n_sel; ++i) {
    accum acc = {NULL, NULL};
    const int64_t cell = items[3 * i], p1 = items[3 * i + 2];
    const int ci = (int)items[3 * i + 1];
    if (chan_learned && !chan_learned[ci]) {
      run_item_uniform(g, &chans[ci], f, mass2, seed, step, n_samples, REF_EST_CM, 1, 0, NULL, cell, p1,
                       &acc, &out[i], out_scale ? &out_scale[i] : NULL);
    } else {
      const int64_t row = ((table_per_cell ? cell : 0) * nch + ci) * nn + p1;
      run_item_learned(g, &chans[ci], f, mass2, seed, step, n_samples, K, thr + row * K, mu + row * K * 5,
                       sigma + row * K * 5, cell, p1, &acc, &out[i], out_scale ? &out_scale[i] : NULL);
    }
  }
  return 0;
}

/* direct sums of selected work items (cell, channel ordinal, node), without
   deposits; items[3*i .. 3*i+2] */
int32_t ref_item_sums(const ref_grid* g, const double* f, const double* mass2, uint64_t seed,
                      uint32_t step, int32_t n_samples, int32_t symmetric, int64_t n_sel,
                      const int64_t* items, double* out, double* out_scale, int32_t n_threads) {
  return ref_item_sums_est(g, f, mass2, seed, step, n_samples, REF_EST_CM, symmetric, n_sel, items, out,
                           out_scale, n_threads);
}

int32_t ref_item_sums_est(const ref_grid* g, const double* f, const double* mass2, uint64_t seed,
                          uint32_t step, int32_t n_samples, int32_t estimator, int32_t symmetric,
                          int64_t n_sel, const int64_t* items, double* out, double* out_scale,
                          int32_t n_threads) {
  if (check_grid(g) || n_samples <= 0) return -1;
  if (estimator < REF_EST_CM || estimator > REF_EST_ROOT_K3) return -1;
  ref_channel chans[128];
  const int nch = ref_channels(g, chans, 128);
  if (nch < 0) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  for (int64_t i = 0; i < n_sel; ++i)
    if (items[3 * i] < 0 || items[3 * i] >= nc || items[3 * i + 1] < 0 || items[3 * i + 1] >= nch ||
        items[3 * i + 2] < 0 || items[3 * i + 2] >= nn)
      return -1;
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  (void)n_threads;
#endif
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic)
#endif
  for (int64_t i = 0; i < n_sel; ++i) {
    accum acc = {NULL, NULL};
    run_item_uniform(g, &chans[items[3 * i + 1]], f, mass2, seed, step, n_samples, estimator,
                     symmetric, 0, NULL, items[3 * i], items[3 * i + 2], &acc, &out[i],
                     out_scale ? &out_scale[i] : NULL);
  }
  return nch;
}

int32_t ref_collision(const ref_grid* g, const double* f, const double* mass2,
                      uint64_t seed, uint32_t step, int32_t n_samples,
                      int32_t estimator, int32_t symmetric, int32_t flags,
                      const ref_equilibrium* eq, double* A_out, double* S_out,
                      double* item_sum, int32_t n_threads) {
  if ((flags & REF_ANALYTIC_F) && !eq) return -1;
  if (estimator < REF_EST_CM || estimator > REF_EST_ROOT_K3) return -1;
  run_args ra = {g, f, mass2, seed, step, n_samples, estimator, symmetric, flags, eq,
                 0, NULL, NULL, NULL, 0, NULL};
  return run_all(&ra, ITEM_UNIFORM, A_out, S_out, item_sum, n_threads);
}

int32_t ref_collision_learned(const ref_grid* g, const double* f, const double* mass2,
                              uint64_t seed, uint32_t step, int32_t n_samples,
                              int32_t K, const uint32_t* thr, const float* mu,
                              const float* sigma, int32_t table_per_cell,
                              const uint8_t* chan_learned,
                              double* A_out, double* S_out, double* item_sum,
                              int32_t n_threads) {
  if (K < 1 || K > 64) return -1;
  run_args ra = {g, f, mass2, seed, step, n_samples, REF_EST_CM, 1, 0, NULL,
                 K, thr, mu, sigma, table_per_cell, chan_learned};
  return run_all(&ra, ITEM_LEARNED, A_out, S_out, item_sum, n_threads);
}

/* ------------------------------------------------------------------ */
/* Deterministic quadrature of the same box-truncated, CIC-deposited    */
/* operator: the sampled variables (p2, cos theta, phi) run over a      */
/* caller-given node set with weights instead of Philox draws.          */
/* ------------------------------------------------------------------ */
int32_t ref_collision_points(const ref_grid* g, const double* f, const double* mass2,
                             int64_t n_pts, const double* pts, const double* wts,
                             int32_t symmetric, int32_t flags, double* A_out, int32_t n_threads) {
  if (check_grid(g) || n_pts <= 0 || (flags & REF_ANALYTIC_F)) return -1;
  ref_channel chans[128];
  const int nch = ref_channels(g, chans, 128);
  if (nch < 0) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  const int64_t field = (int64_t)NSP * nc * nn;
  memset(A_out, 0, sizeof(double) * field);
  const int64_t n_items = nc * nch * nn;
  int nt = 1;
#ifdef _OPENMP
  nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#else
  (void)n_threads;
#endif
  double** buf = (double**)calloc(nt, sizeof(double*));
  for (int t = 0; t < nt; ++t) buf[t] = (double*)calloc(field, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
  for (int64_t it = 0; it < n_items; ++it) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    const int64_t cell = it / ((int64_t)nch * nn);
    const int64_t rem = it % ((int64_t)nch * nn);
    const int ci = (int)(rem / nn);
    const int64_t p1_lin = rem % nn;
    accum acc = {buf[tid], NULL};
    double p1[3];
    node_momentum(g, p1_lin, p1);
    for (int64_t i = 0; i < n_pts; ++i) {
      const double* q = pts + 5 * i;
      ref_point pt;
      if (!ref_eval_cm(g, &chans[ci], f, mass2, (int32_t)cell, p1, (int32_t)p1_lin, q, q[3], q[4],
                       flags, NULL, &pt))
        continue;
      const double v = chans[ci].w * wts[i] * pt.g;
      const double vd = chans[ci].sigma * wts[i] * pt.g;
      deposit_sample(g, &chans[ci], &acc, cell, p1_lin, (const double(*)[4])pt.k, symmetric, v, 0.0, vd, 0.0);
    }
  }
  for (int t = 0; t < nt; ++t) {
    for (int64_t i = 0; i < field; ++i) A_out[i] += buf[t][i];
    free(buf[t]);
  }
  free(buf);
  return nch;
}

/* ------------------------------------------------------------------ */
/* Thermal masses, Eq. mg and Eq. mq, as midpoint sums over the grid.  */
/* ------------------------------------------------------------------ */
int32_t ref_masses(const ref_grid* g, const double* f, const double* mass2_lag,
                   double* mass2_out) {
  if (check_grid(g)) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  const double dV = dp_of(g, 0) * dp_of(g, 1) * dp_of(g, 2);
  const double g2 = 4.0 * PI * g->alpha_s;
  const double meas = dV / pow(2.0 * PI, 3);
  for (int64_t x = 0; x < nc; ++x) {
    /* I_Y = sum_p dV/((2pi)^3 2E_Y) f_Y */
    double I[NSP];
    for (int sp = 0; sp < NSP; ++sp) {
      const double* fc = f + ((int64_t)sp * nc + x) * nn;
      const double m2 = mass2_lag ? mass2_lag[(int64_t)sp * nc + x] : 0.0;
      double acc = 0.0;
      for (int64_t p = 0; p < nn; ++p) {
        double q[3];
        node_momentum(g, p, q);
        const double E = sqrt(norm2(q) + m2);
        if (!(E > 0.0)) continue;
        acc += meas * fc[p] / (2.0 * E);
      }
      I[sp] = acc;
    }
    double sum_q = 0.0;
    for (int i = 0; i < 3; ++i) sum_q += degeneracy(i) * C_F * (I[i] + I[3 + i]);
    const double mg2 = (2.0 * g2 / D_A) * (degeneracy(GLUON) * C_A * I[GLUON] + sum_q);
    mass2_out[(int64_t)GLUON * nc + x] = mg2;
    for (int i = 0; i < 3; ++i) {
      const double mq2 = 2.0 * C_F * g2 * (2.0 * I[GLUON] + I[i] + I[3 + i]);
      mass2_out[(int64_t)i * nc + x] = mq2;
      mass2_out[(int64_t)(3 + i) * nc + x] = mq2;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Drift, Eq. left handside in flux form with periodic boundaries.     */
/* scheme 0: first-order upwind fluxes at the cell interfaces;          */
/* scheme 1: the central differences of Eq. descrete left hand.        */
/* ------------------------------------------------------------------ */
static int64_t cell_shift(const ref_grid* g, int64_t cell, int axis, int d) {
  int64_t iz = cell % g->n_x[2];
  int64_t iy = (cell / g->n_x[2]) % g->n_x[1];
  int64_t ix = cell / ((int64_t)g->n_x[2] * g->n_x[1]);
  int64_t id[3] = {ix, iy, iz};
  id[axis] = (id[axis] + d + g->n_x[axis]) % g->n_x[axis];
  return (id[0] * g->n_x[1] + id[1]) * g->n_x[2] + id[2];
}

static int64_t node_shift(const ref_grid* g, int64_t lin, int axis, int d) {
  int64_t iz = lin % g->n_p[2];
  int64_t iy = (lin / g->n_p[2]) % g->n_p[1];
  int64_t ix = lin / ((int64_t)g->n_p[2] * g->n_p[1]);
  int64_t id[3] = {ix, iy, iz};
  id[axis] = (id[axis] + d + g->n_p[axis]) % g->n_p[axis];
  return (id[0] * g->n_p[1] + id[1]) * g->n_p[2] + id[2];
}

static double energy(const ref_grid* g, const double* mass2, int sp, int64_t cell, int64_t node) {
  double q[3];
  node_momentum(g, node, q);
  return sqrt(norm2(q) + mass2[(int64_t)sp * n_cells(g) + cell]);
}

/* force component -dE/dx_axis by central difference over the periodic grid */
static double force(const ref_grid* g, const double* mass2, int sp, int64_t cell, int64_t node, int axis) {
  const int64_t cp = cell_shift(g, cell, axis, +1), cm = cell_shift(g, cell, axis, -1);
  return -(energy(g, mass2, sp, cp, node) - energy(g, mass2, sp, cm, node)) / (2.0 * dx_of(g, axis));
}

static double upwind_flux(double vel, double f_left, double f_right) {
  return vel > 0.0 ? vel * f_left : vel * f_right;
}

int32_t ref_drift(const ref_grid* g, const double* f, const double* mass2,
                  int32_t scheme, double* D_out) {
  if (check_grid(g)) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  for (int sp = 0; sp < NSP; ++sp) {
    for (int64_t x = 0; x < nc; ++x) {
      for (int64_t p = 0; p < nn; ++p) {
        const int64_t at = ((int64_t)sp * nc + x) * nn + p;
        if (!((g->species_mask >> sp) & 1u)) { D_out[at] = 0.0; continue; }
        double q[3];
        node_momentum(g, p, q);
        double D = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int64_t xp = cell_shift(g, x, a, +1), xm = cell_shift(g, x, a, -1);
          const int64_t pp = node_shift(g, p, a, +1), pm = node_shift(g, p, a, -1);
          const double* F = f + (int64_t)sp * nc * nn;
          if (scheme == 0) {
            /* x-advection with velocity p_a/E */
            const double vc = q[a] / energy(g, mass2, sp, x, p);
            const double vp = q[a] / energy(g, mass2, sp, xp, p);
            const double vm = q[a] / energy(g, mass2, sp, xm, p);
            const double fR = upwind_flux(0.5 * (vc + vp), F[x * nn + p], F[xp * nn + p]);
            const double fL = upwind_flux(0.5 * (vm + vc), F[xm * nn + p], F[x * nn + p]);
            D += (fR - fL) / dx_of(g, a);
            /* p-advection with the force -grad_x E */
            const double Fc = force(g, mass2, sp, x, p, a);
            const double Fp = force(g, mass2, sp, x, pp, a);
            const double Fm = force(g, mass2, sp, x, pm, a);
            const double gR = upwind_flux(0.5 * (Fc + Fp), F[x * nn + p], F[x * nn + pp]);
            const double gL = upwind_flux(0.5 * (Fm + Fc), F[x * nn + pm], F[x * nn + p]);
            D += (gR - gL) / dp_of(g, a);
          } else {
            const double ddx = 2.0 * dx_of(g, a), ddp = 2.0 * dp_of(g, a);
            D += (q[a] * F[xp * nn + p] / energy(g, mass2, sp, xp, p)
                  - q[a] * F[xm * nn + p] / energy(g, mass2, sp, xm, p)) / ddx;
            const double dEp = (energy(g, mass2, sp, xp, pp) - energy(g, mass2, sp, xm, pp)) / ddx;
            const double dEm = (energy(g, mass2, sp, xp, pm) - energy(g, mass2, sp, xm, pm)) / ddx;
            D -= (F[x * nn + pp] * dEp - F[x * nn + pm] * dEm) / ddp;
          }
        }
        D_out[at] = D;
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. particle numbers and T^{0mu} of Eq. energy momentum tensor      */
/* ------------------------------------------------------------------ */
int32_t ref_observables(const ref_grid* g, const double* f, const double* mass2,
                        double* N_out, double* E_out, double* P_out) {
  if (check_grid(g)) return -1;
  const int64_t nc = n_cells(g), nn = n_nodes(g);
  const double dVx = dx_of(g, 0) * dx_of(g, 1) * dx_of(g, 2);
  const double dVp = dp_of(g, 0) * dp_of(g, 1) * dp_of(g, 2);
  const double meas = dVx * dVp / pow(2.0 * PI, 3);
  for (int sp = 0; sp < NSP; ++sp) {
    double N = 0.0, E = 0.0, P[3] = {0.0, 0.0, 0.0};
    for (int64_t x = 0; x < nc; ++x) {
      for (int64_t p = 0; p < nn; ++p) {
        const double fv = f[((int64_t)sp * nc + x) * nn + p];
        double q[3];
        node_momentum(g, p, q);
        const double En = sqrt(norm2(q) + mass2[(int64_t)sp * nc + x]);
        N += fv;
        E += En * fv;
        for (int a = 0; a < 3; ++a) P[a] += q[a] * fv;
      }
    }
    const double dg = degeneracy(sp) * meas;
    N_out[sp] = dg * N;
    E_out[sp] = dg * E;
    for (int a = 0; a < 3; ++a) P_out[sp * 3 + a] = dg * P[a];
  }
  return 0;
}
