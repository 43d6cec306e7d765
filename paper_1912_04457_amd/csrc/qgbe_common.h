// Internal definitions of libqgbe shared by the host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qgbe {

constexpr int kSpecies = 7;
constexpr int kGluon = 6;
constexpr int kMaxChannels = 70;
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kHbarC = 0.1973269804;  // GeV fm

// Helicity x colour degeneracy (Eq. C_quark: N_q = 2*3, Eq. C_gluon: N_g = 2*8).
__host__ __device__ inline double degeneracy(int sp) { return sp == kGluon ? 16.0 : 6.0; }

// Momentum coordinate of node i on an axis of half-width ph and spacing dp:
// the centre of its momentum cell, -ph + (i + 1/2) dp, with the product
// rounded before the sum (no fused multiply-add).  The middle node of an odd
// axis then sits at exactly p = 0 (the fused form leaves ph times the
// rounding error of dp, about 1e-16), so a massless particle there has E = 0
// and the node zero measure in the mass integral and the collision term.
__host__ __device__ inline double node_coord(double ph, double dp, int i) {
#pragma clang fp contract(off)
  return -ph + (i + 0.5) * dp;
}

// One collision channel: a Table I reaction with the observed species at
// position 1.  Positions 2..4 map onto up to three distinct "slots" (species),
// which are the f tiles read by the interpolation and the accumulators that
// receive the symmetric deposits.
struct Channel {
  int row;          // Table I row 1..7
  int sp[4];        // species at positions 1..4
  int code;         // ((s1*7+s2)*7+s3)*7+s4
  double w;         // symmetric per-position weight
  double sigma;     // coefficient in Eq. C_quark / Eq. C_gluon
  int nslot;        // distinct species among positions 2..4
  int slot_sp[3];   // species of each slot
  int pos_slot[3];  // slot of positions 2, 3, 4
};

// User matrix elements: row r (1..7) of Table I replaced by
// sum_k c_k s^a t^b u^c / ((t - mu)^d (u - mu)^e s^f), in units of g^4.
constexpr int kMsqMaxTerms = 8;
constexpr int kMsqMaxPower = 4;
struct MsqTable {
  int n[8];                        // terms per row (index 1..7)
  double c[8][kMsqMaxTerms];
  int8_t p[8][kMsqMaxTerms][6];    // a, b, c, d, e, f
};

// Geometry of the phase-space grid, passed by value to every kernel.
struct Grid {
  int nx[3], np[3];
  int cells, nodes;
  int ox, oy;              // node strides of px and py (pz stride is 1)
  double xh[3], ph[3];     // half-widths
  double dx[3], dp[3];     // cell sizes
  double inv_dp[3];
  double pc[3];            // ph / dp - 1/2: grid coordinate t = p / dp + pc
  double Vp;               // momentum box volume
  double g2, g4;           // g^2 = 4 pi alpha_s
  uint32_t species_mask;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64 bit products with a Weyl key schedule.
__host__ __device__ inline void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t n0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
    const uint32_t n2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)b;
    x3 = (uint32_t)a;
    x0 = n0;
    x2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Host: build the channel table for the masks (ascending code).  Returns the
// count or -1 if max is exceeded.
int build_channels(uint32_t species_mask, uint32_t row_mask, Channel* out, int max);

}  // namespace qgbe
