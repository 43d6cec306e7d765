// Channel table of the collision term (Eq. C_quark, Eq. C_gluon, Table I).
//
// A reaction is an unordered pair of unordered species pairs {in} <-> {out}.
// Each distinct species X of a reaction gives one channel: the species tuple
// reordered so that X comes first, its collision partner second, and the
// particle on X's fermion/gluon line (the t-channel partner of Table I) third.
// The reorderings used (swap of both pairs, time reversal, or both) leave the
// Mandelstam s, t, u of Table I unchanged.
//
// Weights: with S_in, S_out = 2 for identical particles in a pair (else 1),
// kappa = 1/2 when {in} = {out} (each collision is then counted twice over the
// four positions) and M = the number of distinct species, the symmetric
// per-position weight is w = kappa / (S_in S_out M) and the coefficient of the
// reaction in the observed species' equation is sigma = n_X kappa / (S_in S_out)
// (n_X = positions holding X), which reproduces the factors 1/2 and 1 printed
// in Eq. C_quark and Eq. C_gluon.
#include <algorithm>
#include <vector>

#include "qgbe_common.h"

namespace qgbe {
namespace {

constexpr int G = kGluon;
inline bool is_quark(int s) { return s < 3; }
inline bool is_antiquark(int s) { return s >= 3 && s < 6; }
inline int flavour(int s) { return s % 3; }
inline int anti(int s) { return s == G ? G : (s < 3 ? s + 3 : s - 3); }

struct Reaction {
  int row;
  int a, b, c, d;  // Table I order a b -> c d
};

// Classify {a,b} -> {c,d}; returns the Table I row, or 0 if the pair of pairs
// is not a QCD 2->2 reaction of Table I (flavour or fermion number violated).
int classify(int a, int b, int c, int d) {
  const bool in_eq_out = (a == c && b == d) || (a == d && b == c);
  if (a == G && b == G && c == G && d == G) return 7;
  auto qg = [](int x, int y) { return (x == G) != (y == G); };
  if (in_eq_out && qg(a, b)) return 6;
  const bool in_qqbar = a != G && b == anti(a) && a != b;
  const bool out_qqbar = c != G && d == anti(c) && c != d;
  if (in_qqbar && c == G && d == G) return 5;
  if (!in_eq_out) {
    if (in_qqbar && out_qqbar && flavour(a) != flavour(c)) return 4;
    return 0;
  }
  if (a == G || b == G) return 0;
  if (in_qqbar) return 3;
  if (a == b) return 2;
  return 1;
}

std::vector<Reaction> all_reactions() {
  // enumerate unordered {in} <= {out} pairs of unordered species pairs
  std::vector<std::pair<int, int>> pairs;
  for (int x = 0; x < kSpecies; ++x)
    for (int y = x; y < kSpecies; ++y) pairs.push_back({x, y});
  std::vector<Reaction> out;
  for (size_t i = 0; i < pairs.size(); ++i)
    for (size_t j = i; j < pairs.size(); ++j) {
      int a = pairs[i].first, b = pairs[i].second, c = pairs[j].first, d = pairs[j].second;
      // Table I writes q qbar -> g g with the fermions incoming
      if (c != G && a == G && b == G) { std::swap(a, c); std::swap(b, d); }
      // put the quark before its antiquark and keep q-g with the fermion first
      if (a == G && b != G) std::swap(a, b);
      if (c == G && d != G) std::swap(c, d);
      const int row = classify(a, b, c, d);
      if (row) out.push_back({row, a, b, c, d});
    }
  return out;
}

}  // namespace

int build_channels(uint32_t species_mask, uint32_t row_mask, Channel* out, int max) {
  std::vector<Channel> chans;
  for (const Reaction& r : all_reactions()) {
    if (!((row_mask >> (r.row - 1)) & 1u)) continue;
    const int tup[4] = {r.a, r.b, r.c, r.d};
    bool present = true;
    for (int s : tup) present = present && ((species_mask >> s) & 1u);
    if (!present) continue;
    const bool in_eq_out = (r.a == r.c && r.b == r.d) || (r.a == r.d && r.b == r.c);
    const double kappa = in_eq_out ? 0.5 : 1.0;
    const double S = (r.a == r.b ? 2.0 : 1.0) * (r.c == r.d ? 2.0 : 1.0);
    std::vector<int> distinct;
    for (int s : tup)
      if (std::find(distinct.begin(), distinct.end(), s) == distinct.end()) distinct.push_back(s);
    for (int X : distinct) {
      Channel ch{};
      ch.row = r.row;
      // order: X, its partner, then the particle on X's line, then the last one
      int in_pos = -1;
      for (int p = 0; p < 4; ++p)
        if (tup[p] == X) { in_pos = p; break; }
      int o[4];
      if (in_pos < 2) {  // X incoming: keep the direction
        const int partner = in_pos == 0 ? 1 : 0;
        o[0] = in_pos; o[1] = partner; o[2] = 2 + in_pos; o[3] = 2 + partner;
      } else {           // X outgoing: reverse the reaction
        const int partner = in_pos == 2 ? 3 : 2;
        o[0] = in_pos; o[1] = partner; o[2] = in_pos - 2; o[3] = partner - 2;
      }
      for (int p = 0; p < 4; ++p) ch.sp[p] = tup[o[p]];
      ch.code = ((ch.sp[0] * 7 + ch.sp[1]) * 7 + ch.sp[2]) * 7 + ch.sp[3];
      int nX = 0;
      for (int s : tup) nX += (s == X);
      ch.w = kappa / (S * (double)distinct.size());
      ch.sigma = (double)nX * kappa / S;
      ch.nslot = 0;
      for (int p = 1; p < 4; ++p) {
        int slot = -1;
        for (int k = 0; k < ch.nslot; ++k)
          if (ch.slot_sp[k] == ch.sp[p]) slot = k;
        if (slot < 0) { slot = ch.nslot++; ch.slot_sp[slot] = ch.sp[p]; }
        ch.pos_slot[p - 1] = slot;
      }
      chans.push_back(ch);
    }
  }
  std::sort(chans.begin(), chans.end(), [](const Channel& x, const Channel& y) { return x.code < y.code; });
  if ((int)chans.size() > max) return -1;
  std::copy(chans.begin(), chans.end(), out);
  return (int)chans.size();
}

}  // namespace qgbe
