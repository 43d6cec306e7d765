// Operation counts of the oracle's per-sample arithmetic.
//
// TEST INFRASTRUCTURE ONLY, like the oracle itself: built by oracle.build(),
// run by tests/test_opcount.py, never by the product path.  The oracle's C
// source is compiled here once more with every `double` replaced by a type
// that counts the operations done on it.  The drivers below take the steps
// the oracle's item loops take around its evaluation functions (the map from
// the unit cube, the mixture draw, the value and its deposits) and call the
// oracle's functions for the rest.  The counts are taken per sample of the uniform sampler's
// collision estimator (Eq. C_a_b with the CM-angle parameterisation of
// Eq. MC C_gg, symmetric deposits of Eq. small c relation), per sample of the
// mixture draw and density, and per sample of the paper's root
// parameterisation (Eq. work out delta E, Eq. delta replace), each split into
// the classes the roofline of the GPU kernels weighs.
//
// Output (stdout): one JSON object.  Classes: add (add, sub), mul, fma, div,
// sqrt, trans (exp, log, sin, cos, pow, expm1), cmp (comparisons, min, max),
// misc (floor, copysign, conversions to integer or float).  Negation and
// absolute value are free source modifiers on the GPU and are not counted.
// Only operations that depend on the sample are counted (values computed from
// the grid, the work item or constants alone are per-item work, done once per
// item on the GPU), each distinct operation once per sample (the same
// operation on the same operands is common subexpression), and a division by
// a per-item value counts as the product with its reciprocal.

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <string>
#include <unordered_map>
#include <vector>

namespace opc {
// One counted operation of the current sample.
struct Op {
  char kind;      // 'a' add/sub, 'm' mul, 'd' div, 'r' sqrt, 't' transcendental, 'c' compare, 'x' misc
  int a = -1, b = -1;   // operand ops (-1: not a counted operation's result)
  int uses = 0;   // counted operations that take its result
};
static std::vector<Op> ops;
static std::unordered_map<std::string, int> seen;   // (operation, operand bits) -> op index
static bool on = false;
inline void reset() {
  ops.clear();
  seen.clear();
}
}  // namespace opc

// A double that records whether it depends on the sample being counted
// (id >= 0: the counted operation that produced it), or is an output
// accumulator (sink: additions into it are the deposits' atomic adds, not
// arithmetic of the sample).
struct Real {
  double v;
  int id;
  bool t, sink;
  Real() = default;
  constexpr Real(double x) : v(x), id(-1), t(false), sink(false) {}
  constexpr Real(double x, bool tainted) : v(x), id(-1), t(tainted), sink(false) {}
  explicit operator int() const;
  explicit operator long() const { return (long)(int)*this; }
  explicit operator long long() const { return (long long)(int)*this; }
  explicit operator unsigned() const { return (unsigned)(int)*this; }
  explicit operator float() const;
  explicit operator bool() const { return v != 0.0; }
};

namespace opc {
// Record one operation on operands a (and b); returns the result's id, or -1
// when it is not counted (no operand depends on the sample).
inline int record(char kind, char op, const Real& a, const Real* b, double result_v) {
  (void)result_v;
  const bool tainted = a.t || (b && b->t);
  if (!on || !tainted) return -1;
  std::string k(1 + 2 * sizeof(double), '\0');
  k[0] = op;
  memcpy(&k[1], &a.v, sizeof a.v);
  const double bv = b ? b->v : 0.0;
  memcpy(&k[1 + sizeof a.v], &bv, sizeof bv);
  auto it = seen.find(k);
  if (it != seen.end()) return it->second;   // the same operation once more: common subexpression
  if (a.id >= 0) ops[a.id].uses++;
  if (b && b->id >= 0) ops[b->id].uses++;
  ops.push_back(Op{kind, a.id, b ? b->id : -1});
  const int id = (int)ops.size() - 1;
  seen.emplace(k, id);
  return id;
}
inline Real make(char kind, char op, const Real& a, const Real* b, double v) {
  Real r(v, a.t || (b && b->t));
  r.id = record(kind, op, a, b, v);
  return r;
}
}  // namespace opc

inline Real::operator int() const { (void)opc::record('x', 'i', *this, nullptr, 0.0); return (int)v; }
inline Real::operator float() const { (void)opc::record('x', 'f', *this, nullptr, 0.0); return (float)v; }
inline Real operator+(Real a, Real b) {
  if (a.sink || b.sink) { Real r(a.v + b.v); r.sink = true; return r; }
  return opc::make('a', '+', a, &b, a.v + b.v);
}
inline Real operator-(Real a, Real b) {
  if (a.sink || b.sink) { Real r(a.v - b.v); r.sink = true; return r; }
  return opc::make('a', '-', a, &b, a.v - b.v);
}
inline Real operator*(Real a, Real b) { return opc::make('m', '*', a, &b, a.v * b.v); }
// a division by a per-item value is the product with its reciprocal
inline Real operator/(Real a, Real b) { return opc::make(b.t ? 'd' : 'm', '/', a, &b, a.v / b.v); }
inline Real& operator+=(Real& a, Real b) { a = a + b; return a; }
inline Real& operator-=(Real& a, Real b) { a = a - b; return a; }
inline Real& operator*=(Real& a, Real b) { a = a * b; return a; }
inline Real& operator/=(Real& a, Real b) { a = a / b; return a; }
inline Real operator-(Real a) { a.v = -a.v; return a; }
inline Real operator+(Real a) { return a; }
inline bool cmp_(char op, Real a, Real b) { (void)opc::record('c', op, a, &b, 0.0); return true; }
inline bool operator<(Real a, Real b) { cmp_('<', a, b); return a.v < b.v; }
inline bool operator>(Real a, Real b) { cmp_('<', b, a); return a.v > b.v; }
inline bool operator<=(Real a, Real b) { cmp_('l', a, b); return a.v <= b.v; }
inline bool operator>=(Real a, Real b) { cmp_('l', b, a); return a.v >= b.v; }
inline bool operator==(Real a, Real b) { cmp_('=', a, b); return a.v == b.v; }
inline bool operator!=(Real a, Real b) { cmp_('=', a, b); return a.v != b.v; }
inline bool operator!(Real a) { return a.v == 0.0; }
inline Real sqrt(Real a) { return opc::make('r', 'r', a, nullptr, std::sqrt(a.v)); }
inline Real exp(Real a) { return opc::make('t', 'e', a, nullptr, std::exp(a.v)); }
inline Real expm1(Real a) { return opc::make('t', 'E', a, nullptr, std::expm1(a.v)); }
inline Real log(Real a) { return opc::make('t', 'L', a, nullptr, std::log(a.v)); }
inline Real sin(Real a) { return opc::make('t', 's', a, nullptr, std::sin(a.v)); }
inline Real cos(Real a) { return opc::make('t', 'c', a, nullptr, std::cos(a.v)); }
inline Real pow(Real a, Real b) { return opc::make('t', 'p', a, &b, std::pow(a.v, b.v)); }
inline Real fabs(Real a) { a.v = std::fabs(a.v); return a; }
inline Real copysign(Real a, Real b) { return opc::make('x', 'C', a, &b, std::copysign(a.v, b.v)); }
inline Real floor(Real a) { return opc::make('x', 'F', a, nullptr, std::floor(a.v)); }
inline Real fmax(Real a, Real b) { return opc::make('c', 'M', a, &b, std::fmax(a.v, b.v)); }
inline Real fmin(Real a, Real b) { return opc::make('c', 'm', a, &b, std::fmin(a.v, b.v)); }

#define double Real
#include "qgbe_oracle.c"
#undef double

namespace {

// Class counts of one sample's operations.  fma: additions that take the
// result of a multiplication used by nothing else (the pair issues as one
// fused multiply-add).
struct Counts {
  double add = 0, mul = 0, fma = 0, div = 0, sqrt = 0, trans = 0, cmp = 0, misc = 0;
};

Counts summarize() {
  Counts c;
  std::vector<char> fused(opc::ops.size(), 0);
  for (size_t i = 0; i < opc::ops.size(); ++i) {
    const opc::Op& o = opc::ops[i];
    switch (o.kind) {
      case 'a': {
        c.add += 1;
        for (int src : {o.a, o.b})
          if (src >= 0 && opc::ops[src].kind == 'm' && opc::ops[src].uses == 1 && !fused[src]) {
            fused[src] = 1;
            c.fma += 1;
            break;
          }
        break;
      }
      case 'm': c.mul += 1; break;
      case 'd': c.div += 1; break;
      case 'r': c.sqrt += 1; break;
      case 't': c.trans += 1; break;
      case 'c': c.cmp += 1; break;
      default: c.misc += 1; break;
    }
  }
  return c;
}

struct Tally {
  double n = 0;
  Counts c;
  void add(const Counts& d) {
    n += 1;
    c.add += d.add; c.mul += d.mul; c.fma += d.fma; c.div += d.div; c.sqrt += d.sqrt;
    c.trans += d.trans; c.cmp += d.cmp; c.misc += d.misc;
  }
  void print(const char* name, bool last) const {
    const double k = n > 0 ? 1.0 / n : 0.0;
    printf("  \"%s\": {\"samples\": %.0f, \"add\": %.3f, \"mul\": %.3f, \"fma\": %.3f, \"div\": %.3f, "
           "\"sqrt\": %.3f, \"trans\": %.3f, \"cmp\": %.3f, \"misc\": %.3f}%s\n",
           name, n, c.add * k, c.mul * k, c.fma * k, c.div * k, c.sqrt * k, c.trans * k, c.cmp * k, c.misc * k,
           last ? "" : ",");
  }
};

// Output accumulators: additions into them are the deposits' atomic adds.
void mark_sink(Real* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i) a[i].sink = true;
}

// One uniform-sampler sample of a work item, the steps run_item_uniform
// takes (unit-cube map -> ref_eval_cm -> value -> symmetric deposits), the
// sample's five variates marked as the sample's own; returns its class
// (0 below threshold, 1 outside the box, 2 accepted) and its counts in *d.
int one_uniform(const ref_grid* g, const ref_channel* ch, const Real* f, const Real* mass2, uint64_t seed,
                int32_t N, int64_t cell, int64_t p1_lin, uint32_t s, accum* acc, Counts* d, int symmetric = 1) {
  Real p1[3];
  node_momentum(g, p1_lin, p1);
  const Real Vp = box_volume(g);
  uint32_t x[4];
  draw_block(seed, 0u, s, (uint32_t)p1_lin, (uint32_t)cell, (uint32_t)ch->code, 0u, x);
  Real u[5];
  five_uniforms(x, u);
  opc::reset();
  opc::on = true;
  for (int i = 0; i < 5; ++i) u[i].t = true;
  const Real p2[3] = {-g->p_half[0] + 2.0 * g->p_half[0] * u[0], -g->p_half[1] + 2.0 * g->p_half[1] * u[1],
                      -g->p_half[2] + 2.0 * g->p_half[2] * u[2]};
  const Real V5 = Vp * 4.0 * PI;
  const Real cth = 2.0 * u[3] - 1.0;
  const Real phi = 2.0 * PI * u[4];
  ref_point pt;
  const int ok = ref_eval_cm(g, ch, f, mass2, (int32_t)cell, p1, (int32_t)p1_lin, p2, cth, phi, 0, NULL, &pt);
  int cls = 2;
  if (!ok) {
    cls = (pt.k[2][0].v == 0.0 && pt.k[3][0].v == 0.0) ? 0 : 1;
  } else {
    // the value of the estimator in use (symmetric: w V5 g / N, direct: sigma V5 g / N)
    const Real v = (symmetric ? ch->w : ch->sigma) * V5 * pt.g / N;
    deposit_sample(g, ch, acc, cell, p1_lin, (const Real(*)[4])pt.k, symmetric, v, 0.0, v, 0.0);
  }
  opc::on = false;
  *d = summarize();
  return cls;
}

// One sample of the paper's root parameterisation (run_item_uniform with
// REF_EST_ROOT: k2 in the box, k3x and k3y sampled, k3z at the roots of energy
// conservation, each valid root with its value and deposits); returns the
// number of valid roots.
int one_root(const ref_grid* g, const ref_channel* ch, const Real* f, const Real* mass2, uint64_t seed, int32_t N,
             int64_t cell, int64_t p1_lin, uint32_t s, int symmetric, accum* acc, Counts* d) {
  Real p1[3];
  node_momentum(g, p1_lin, p1);
  const Real Vp = box_volume(g);
  uint32_t x[4];
  draw_block(seed, 0u, s, (uint32_t)p1_lin, (uint32_t)cell, (uint32_t)ch->code, 2u, x);
  Real u[5];
  five_uniforms(x, u);
  opc::reset();
  opc::on = true;
  for (int i = 0; i < 5; ++i) u[i].t = true;
  const Real p2[3] = {-g->p_half[0] + 2.0 * g->p_half[0] * u[0], -g->p_half[1] + 2.0 * g->p_half[1] * u[1],
                      -g->p_half[2] + 2.0 * g->p_half[2] * u[2]};
  const Real V5 = Vp * (2.0 * g->p_half[0]) * (2.0 * g->p_half[1]);
  const Real p3x = -g->p_half[0] + 2.0 * g->p_half[0] * u[3];
  const Real p3y = -g->p_half[1] + 2.0 * g->p_half[1] * u[4];
  ref_point pts[2];
  const int nv = eval_root(g, ch, f, mass2, cell, p1, p1_lin, p2, p3x, p3y, 0, NULL, pts);
  for (int r = 0; r < nv; ++r) {
    const Real v = (symmetric ? ch->w : ch->sigma) * V5 * pts[r].g / N;
    deposit_sample(g, ch, acc, cell, p1_lin, (const Real(*)[4])pts[r].k, symmetric, v, 0.0, v, 0.0);
  }
  opc::on = false;
  *d = summarize();
  return nv;
}

}  // namespace

int main() {
  // 7 species, 8^3 nodes on [-2,2]^3 GeV, two cells with smooth occupations
  ref_grid g;
  memset(&g, 0, sizeof g);
  for (int a = 0; a < 3; ++a) {
    g.n_x[a] = a == 0 ? 2 : 1;
    g.n_p[a] = 8;
    g.x_half[a] = 3.0;
    g.p_half[a] = 2.0;
  }
  g.species_mask = 0x7F;
  g.row_mask = 0x7F;
  g.alpha_s = 0.3;
  ref_channel ch[128];
  const int nch = ref_channels(&g, ch, 128);
  const int64_t cells = 2, nodes = 512, n = 7 * cells * nodes;
  std::vector<Real> f(n), A(n, Real(0.0)), m2(7 * cells, Real(0.0));
  for (int64_t i = 0; i < n; ++i) f[i] = 0.05 + 0.4 * (double)((i * 7919) % 1000) / 1000.0;
  ref_masses(&g, f.data(), NULL, m2.data());
  mark_sink(A.data(), n);
  accum acc{A.data(), NULL};
  Tally cls[3];
  const uint64_t seed = 0x5EED2019ull;
  for (int ci = 0; ci < nch; ++ci)
    for (int64_t item = 0; item < nodes; item += 37)
      for (uint32_t s = 0; s < 16; ++s) {
        Counts d;
        const int c = one_uniform(&g, &ch[ci], f.data(), m2.data(), seed, 16, item % cells, item, s, &acc, &d);
        cls[c].add(d);
      }
  // The mixture draw and density of one sample, the steps run_item_learned
  // takes before ref_eval_cm (component, three Box-Muller pairs, logistic map,
  // log_q_mixture), on a fixed 8-component table row; the defensive uniform
  // branch is the uniform sampler's map and is not counted here.
  Tally mix;
  {
    uint32_t thr[8];
    float mu[40], sg[40];
    for (int k = 0; k < 8; ++k) {
      thr[k] = (uint32_t)(0.1 * 4294967296.0) + (uint32_t)k * 400000000u;
      for (int d = 0; d < 5; ++d) {
        mu[k * 5 + d] = (float)(0.3 * (k - 4) + 0.1 * d);
        sg[k * 5 + d] = (float)(0.5 + 0.05 * k);
      }
    }
    const Real alpha = (Real)thr[0] / 4294967296.0;
    for (uint32_t s = 0; s < 4096; ++s) {
      uint32_t x[8];
      draw_block(seed, 0u, s, 7u, 0u, (uint32_t)ch[0].code, 0u, x);
      draw_block(seed, 0u, s, 7u, 0u, (uint32_t)ch[0].code, 1u, x + 4);
      if (x[0] < thr[0]) continue;
      opc::reset();
      opc::on = true;
      int k = 0;
      for (int j = 1; j < 8; ++j)
        if (x[0] >= thr[j]) k = j;
      Real z[6], y[5], u[5];
      for (int pr = 0; pr < 3; ++pr) {
        const Real a1(unif23(x[1 + 2 * pr] >> 9).v, true), a2(unif23(x[2 + 2 * pr] >> 9).v, true);
        const Real r = sqrt(-2.0 * log(a1));
        z[2 * pr] = r * cos(2.0 * PI * a2);
        z[2 * pr + 1] = r * sin(2.0 * PI * a2);
      }
      for (int d = 0; d < 5; ++d) {
        y[d] = (Real)mu[k * 5 + d] + (Real)sg[k * 5 + d] * z[d];
        u[d] = 1.0 / (1.0 + exp(-y[d]));
      }
      const Real q = alpha + exp(log_q_mixture(8, thr, mu, sg, y));
      (void)q;
      (void)u;
      opc::on = false;
      mix.add(summarize());
    }
  }
  // the same accepted samples with the direct estimator (no symmetric deposits)
  Tally direct;
  for (int ci = 0; ci < nch; ci += 7)
    for (int64_t item = 0; item < nodes; item += 37)
      for (uint32_t s = 0; s < 16; ++s) {
        Counts d;
        if (one_uniform(&g, &ch[ci], f.data(), m2.data(), seed, 16, item % cells, item, s, &acc, &d, 0) == 2)
          direct.add(d);
      }
  // the root parameterisation, direct and symmetric, by number of valid roots
  Tally roots[2][3];
  for (int sym = 0; sym < 2; ++sym)
    for (int ci = 0; ci < nch; ci += 3)
      for (int64_t item = 0; item < nodes; item += 37)
        for (uint32_t s = 0; s < 16; ++s) {
          Counts d;
          const int nv = one_root(&g, &ch[ci], f.data(), m2.data(), seed, 16, item % cells, item, s, sym, &acc, &d);
          roots[sym][nv].add(d);
        }
  printf("{\n  \"grid\": \"7 species, 2 cells, 8^3 nodes on [-2,2]^3 GeV, %d channels\",\n", nch);
  cls[0].print("uniform_below_threshold", false);
  cls[1].print("uniform_outside_box", false);
  cls[2].print("uniform_accepted", false);
  direct.print("uniform_accepted_direct", false);
  for (int sym = 0; sym < 2; ++sym)
    for (int nv = 0; nv < 3; ++nv) {
      char name[64];
      snprintf(name, sizeof name, "roots_%s_%d_valid", sym ? "symmetric" : "direct", nv);
      roots[sym][nv].print(name, false);
    }
  mix.print("mixture_draw_and_density", true);
  printf("}\n");
  return 0;
}
