// Monte Carlo collision term (Eq. C_a_b, Eq. MC C_gg, Eq. small c relation).
//
// Work item = (cell, channel, observed node p1).  One wavefront owns one item
// at a time, so everything that depends only on the item (p1, E1, f1, masses,
// channel) is wave-uniform; the 64 lanes draw samples s = lane, lane+64, ...
//
// Per sample (CM-angle parameterisation of the 5-D integral):
//   Philox4x32-10 block -> five 23-bit uniforms -> p2 in the box, cos theta*,
//   phi* -> E2, s, |p*| -> k1 boosted to the CM frame gives the polar axis ->
//   p3* on the sphere -> boost back, p4 = P - p3 -> box cut -> t, u ->
//   |M|^2 (Table I) -> trilinear f at p2, p3, p4 -> bracket
//   B = f3 f4 F1 F2 - f1 f2 F3 F4 -> value v.
// Symmetric sampling adds +v at (X, p1), +v W(p2) at species 2, -v W(p3) at
// species 3 and -v W(p4) at species 4 (W: trilinear stencil weights).
//
// Precision: the sample geometry (everything that decides the threshold,
// the box cut and the branch of the CM frame) is FP64 in both modes, so both
// precisions reject exactly the samples an FP64 evaluation rejects; on CDNA4
// FP64 add/mul/FMA issue at the rate of unpacked FP32.  The integrand
// (|M|^2, interpolation, bracket, value) is FP32 in QGBE_FP32 mode.  Direct
// sums are FP64; in FP32 mode the deposits go to FP32 LDS accumulators per
// workgroup and are flushed into the FP64 output.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "collide.h"

namespace qgbe {
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double unif23(uint32_t v) { return ((double)v + 0.5) * (1.0 / 8388608.0); }

// FP64 1/x and 1/sqrt(x) for finite x > 0: the hardware estimate (measured
// relative error below 2^-24 on gfx950) refined by one third-order step,
// which leaves ~2^-72 (below the last bit) without the scaling and
// special-case handling of a general division or square root.
//   1/x:       e = 1 - x r,          r (1 + e + e^2)
//   1/sqrt(x): t = (1 - x y^2) / 2,  y (1 + t + 3/2 t^2)
__device__ __forceinline__ double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

__device__ __forceinline__ double rsqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double t = fma(-0.5 * x * y, y, 0.5);
  return fma(y, fma(1.5 * t, t, t), y);
}

__device__ __forceinline__ double sqrt64(double x) { return x > 0.0 ? x * rsqrt64(x) : 0.0; }

// sin and cos of 2 pi u for u in [0, 1).  With x = 2u = q/2 + r, q the
// nearest multiple of 1/2 (exact: u has at most 24 significant bits) and
// |r| <= 1/4, sin(pi r) = r S(r^2) and cos(pi r) = C(r^2) with S and C of
// degree 6 (Chebyshev-node fits, gen_fp64_poly.py; fit errors 1e-17 and
// 5e-17), and the quadrant q mod 4 permutes and negates them.  Measured on
// the CPU over every 23-bit u: within 1.8e-16 of sin and cos (the Taylor
// series to r^15 and r^16 it replaces: 1.9e-16).
__device__ __forceinline__ void sincos_2pi(double u, double& sn, double& cs) {
  const double x = 2.0 * u;
  const double q = rint(2.0 * x);
  const double r = fma(-0.5, q, x);
  const double r2 = r * r;
  double ps = 0.0004615313805851339;
  ps = fma(ps, r2, -0.0073700215052934955);
  ps = fma(ps, r2, 0.08214586917478434);
  ps = fma(ps, r2, -0.5992645289394928);
  ps = fma(ps, r2, 2.550164039873374);
  ps = fma(ps, r2, -5.167712780049954);
  ps = fma(ps, r2, 3.141592653589793);
  ps *= r;
  double pc = 0.001906807054314109;
  pc = fma(pc, r2, -0.025804938121446575);
  pc = fma(pc, r2, 0.23533054718578558);
  pc = fma(pc, r2, -1.3352627670358546);
  pc = fma(pc, r2, 4.058712126397826);
  pc = fma(pc, r2, -4.934802200544605);
  pc = fma(pc, r2, 1.0);
  const int k = (int)q;
  const double a = (k & 1) ? pc : ps;   // sin before the sign
  const double b = (k & 1) ? ps : pc;   // cos before the sign
  sn = (k & 2) ? -a : a;
  cs = ((k + 1) & 2) ? -b : b;
}

// e^x: x = k ln2 + r with |r| <= ln2/2 (ln2 split so k*ln2_hi is exact for
// |k| < 2^11), e^r = 1 + r (1 + r g(r)) with g of degree 9 (a Chebyshev-node
// fit, gen_fp64_poly.py; relative error of e^r from the fit 2e-17), times
// 2^k.  Overflows to inf and underflows to 0 like exp.  Measured on the CPU:
// within 0.95 ulp over |x| < 700 (the Taylor series to r^13 it replaces: 0.89).
__device__ __forceinline__ double exp64(double x) {
  const double k = rint(x * 1.4426950408889634);
  double r = fma(-k, 0.6931471805598903, x);
  r = fma(-k, 5.497923018708371e-14, r);
  double p = 2.510038549551032e-08;
  p = fma(p, r, 2.7620088445409746e-07);
  p = fma(p, r, 2.7557268459997064e-06);
  p = fma(p, r, 2.4801521295954376e-05);
  p = fma(p, r, 0.00019841269863053618);
  p = fma(p, r, 0.0013888888917213717);
  p = fma(p, r, 0.008333333333330062);
  p = fma(p, r, 0.04166666666662413);
  p = fma(p, r, 0.16666666666666669);
  p = fma(p, r, 0.5000000000000001);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// ln a for finite a > 0: a = m 2^e with m in [1/sqrt2, sqrt2), ln m =
// 2 atanh(s) = 2 s P(s^2), s = (m-1)/(m+1), |s| <= 0.172, P of degree 7 (a
// Chebyshev-node fit of atanh(sqrt w)/sqrt w, gen_fp64_poly.py; relative
// fit error 1e-18).  Measured on the CPU: within 2.1 ulp of ln on the 23-bit
// uniforms, 2.7 ulp elsewhere (the series to s^21 it replaces: the same).
__device__ __forceinline__ double log64(double a) {
  int e;
  double m = frexp(a, &e);
  if (m < 0.7071067811865476) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) * rcp64(m + 1.0);
  const double s2 = s * s;
  double p = 0.07404933786156531;
  p = fma(p, s2, 0.0765625655736915);
  p = fma(p, s2, 0.09091816120808513);
  p = fma(p, s2, 0.11111098523202137);
  p = fma(p, s2, 0.1428571438036914);
  p = fma(p, s2, 0.19999999999650955);
  p = fma(p, s2, 0.33333333333333826);
  p = fma(p, s2, 1.0);
  const double de = (double)e;
  return fma(de, 0.6931471805598903, fma(de, 5.497923018708371e-14, 2.0 * s * p));
}


template <typename R>
__device__ __forceinline__ R rcp_r(R x);
template <>
__device__ __forceinline__ float rcp_r<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp_r<double>(double x) { return rcp64(x); }

// Table I |M|^2 in units of g^4, every t and u pole regulated by mu = m_g^2.
// Group factors (SU(3), fundamental quarks): 8 dF^2 CF^2/dA = 16,
// 16 dF CF (CF - CA/2) = -32/3, 8 dF CF^2 = 128/3, 8 dF CF CA = 96,
// 16 dA CA^2 = 1152.
template <typename R>
__device__ __forceinline__ R matrix_element(int row, R s, R t, R u, R mu) {
  const R rt = rcp_r<R>(t - mu);
  const R ru = rcp_r<R>(u - mu);
  const R rs = rcp_r<R>(s);
  const R s2 = s * s, t2 = t * t, u2 = u * u;
  switch (row) {
    case 1: return R(16) * (s2 + u2) * rt * rt;
    case 2: return R(16) * ((s2 + u2) * rt * rt + (s2 + t2) * ru * ru) - R(32.0 / 3.0) * s2 * rt * ru;
    case 3: return R(16) * ((s2 + u2) * rt * rt + (u2 + t2) * rs * rs) - R(32.0 / 3.0) * u2 * rt * rs;
    case 4: return R(16) * (t2 + u2) * rs * rs;
    case 5: return R(128.0 / 3.0) * (u * rt + t * ru) - R(96) * (t2 + u2) * rs * rs;
    case 6: return R(-128.0 / 3.0) * (u * rs + s * ru) + R(96) * (s2 + u2) * rt * rt;
    default: return R(1152) * (R(3) - s * u * rt * rt - s * t * ru * ru - t * u * rs * rs);
  }
}

// |M|^2 / g^4 of a row: the user's terms where the row was replaced (the
// row is uniform over a wavefront), else Table I.
// kUser = false: no user terms in this launch (the table's rows only).
template <typename R, bool kUser = true>
__device__ __forceinline__ R msq_row(uint32_t mask, const MsqTable* tab, int row, R s, R t, R u, R mu) {
  if (!kUser || !((mask >> row) & 1u)) return matrix_element<R>(row, s, t, u, mu);
  const R x[6] = {s, t, u, rcp_r<R>(t - mu), rcp_r<R>(u - mu), rcp_r<R>(s)};
  R sum = R(0);
  const int n = tab->n[row];
  for (int k = 0; k < n; ++k) {
    R term = (R)tab->c[row][k];
    for (int i = 0; i < 6; ++i)
      for (int e = 0; e < tab->p[row][k][i]; ++e) term *= x[i];
    sum += term;
  }
  return sum;
}

// Trilinear stencil over the 8 surrounding cell centres, clamped at the box.
template <typename R>
struct Stencil {
  int base;
  R wx, wy, wz;
};

// The grid coordinate and its fraction are formed in FP64 so the weights carry
// a relative (not an absolute 2^-24 * n) error when rounded to R.
template <typename R>
__device__ __forceinline__ R clamp_axis(double p, double pc, double inv_dp, int n, int& i0) {
  const double t = fmin(fmax(fma(p, inv_dp, pc), 0.0), (double)(n - 1));
  const int i = min((int)t, n - 2);
  i0 = i;
  return (R)(t - (double)i);
}

template <typename R>
__device__ __forceinline__ Stencil<R> make_stencil(const double p[3], const Grid& G) {
  Stencil<R> st;
  int ix, iy, iz;
  st.wx = clamp_axis<R>(p[0], G.pc[0], G.inv_dp[0], G.np[0], ix);
  st.wy = clamp_axis<R>(p[1], G.pc[1], G.inv_dp[1], G.np[1], iy);
  st.wz = clamp_axis<R>(p[2], G.pc[2], G.inv_dp[2], G.np[2], iz);
  st.base = ix * G.ox + iy * G.oy + iz;
  return st;
}

template <typename R, typename T>
__device__ __forceinline__ R interpolate(const T* __restrict__ tile, const Stencil<R>& st, int ox, int oy) {
  const T* q = tile + st.base;
  const R f000 = q[0], f001 = q[1], f010 = q[oy], f011 = q[oy + 1];
  const R f100 = q[ox], f101 = q[ox + 1], f110 = q[ox + oy], f111 = q[ox + oy + 1];
  const R a00 = f000 + st.wz * (f001 - f000);
  const R a01 = f010 + st.wz * (f011 - f010);
  const R a10 = f100 + st.wz * (f101 - f100);
  const R a11 = f110 + st.wz * (f111 - f110);
  const R b0 = a00 + st.wy * (a01 - a00);
  const R b1 = a10 + st.wy * (a11 - a10);
  return b0 + st.wx * (b1 - b0);
}

// Scatter v with the stencil weights (the transpose of interpolate): values
// in precision R, accumulators of type T.  kScope selects the atomic's memory
// scope: workgroup for accumulators in LDS, agent for global memory (the two
// kinds stay distinct instructions, so each keeps its address space).
template <typename R, typename T, int kScope = __HIP_MEMORY_SCOPE_AGENT>
__device__ __forceinline__ void deposit(T* acc, const Stencil<R>& st, R v, int ox, int oy) {
  T* q = acc + st.base;
  const R vx1 = v * st.wx, vx0 = v - vx1;
  const R v01 = vx0 * st.wy, v00 = vx0 - v01;
  const R v11 = vx1 * st.wy, v10 = vx1 - v11;
  __hip_atomic_fetch_add(q, (T)(v00 - v00 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + 1, (T)(v00 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + oy, (T)(v01 - v01 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + oy + 1, (T)(v01 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + ox, (T)(v10 - v10 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + ox + 1, (T)(v10 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + ox + oy, (T)(v11 - v11 * st.wz), __ATOMIC_RELAXED, kScope);
  __hip_atomic_fetch_add(q + ox + oy + 1, (T)(v11 * st.wz), __ATOMIC_RELAXED, kScope);
}

// The same deposit into accumulators that cover only the nodes [lo, lo + n)
// (acc[0] is node lo): the same corner values; a corner outside the window
// is left to the launch whose window holds it.
__device__ __forceinline__ void deposit_window(double* acc, const Stencil<double>& st, double v, int ox, int oy,
                                               int lo, int n) {
  const int b = st.base - lo;
  const double vx1 = v * st.wx, vx0 = v - vx1;
  const double v01 = vx0 * st.wy, v00 = vx0 - v01;
  const double v11 = vx1 * st.wy, v10 = vx1 - v11;
  const int off[8] = {0, 1, oy, oy + 1, ox, ox + 1, ox + oy, ox + oy + 1};
  const double val[8] = {v00 - v00 * st.wz, v00 * st.wz, v01 - v01 * st.wz, v01 * st.wz,
                         v10 - v10 * st.wz, v10 * st.wz, v11 - v11 * st.wz, v11 * st.wz};
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if ((unsigned)(b + off[c]) < (unsigned)n)
      __hip_atomic_fetch_add(acc + b + off[c], val[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// 1 / ((2 pi)^3 * 2 * 2 * 16 pi^2): two-body phase space |p*|/(16 pi^2 sqrt s),
// k2 measure d^3k2/((2 pi)^3 2 E2) and 1/(2 E1) of Eq. C_a_b
constexpr double kNorm = 1.0 / (8.0 * kPi * kPi * kPi * 4.0 * 16.0 * kPi * kPi);

// Quantities of a work item, identical for all lanes of the wave.
struct Item {
  int cell, p1_lin;
  double p1[3];
  double E1;
  double m1sq, m2sq, m3sq, m4sq;
  double dm34;              // m3^2 - m4^2
  double sum2, dif2;        // (m3 + m4)^2 (the threshold of s), (m3 - m4)^2
  double mu;                // regulator m_g^2
  double f1;
  double coef;              // w V5 / N (symmetric) or sigma V5 / N (direct)
  double pref;              // coef g^4 / ((2pi)^3 4 16 pi^2 E1): item part of the value
};

// The sampled configuration (FP64 geometry).
struct Geo {
  double p2[3], p3[3], p4[3];
  double E2, s, t, u, rs, pstar;
};

// Sample geometry from the five uniforms; false if below threshold or outside the box.
__device__ __forceinline__ bool geometry(const Item& it, const Grid& G, const double u[5], Geo& g) {
  for (int a = 0; a < 3; ++a) g.p2[a] = fma(2.0 * G.ph[a], u[a], -G.ph[a]);
  g.E2 = sqrt64(g.p2[0] * g.p2[0] + g.p2[1] * g.p2[1] + g.p2[2] * g.p2[2] + it.m2sq);
  const double E = it.E1 + g.E2;
  const double P[3] = {it.p1[0] + g.p2[0], it.p1[1] + g.p2[1], it.p1[2] + g.p2[2]};
  const double s = E * E - (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
  g.s = s;
  if (!(s > it.sum2)) return false;  // threshold (m3 + m4)^2
  const double rs = rsqrt64(s);
  const double sq = s * rs;
  g.rs = rs;
  g.pstar = 0.5 * rs * sqrt64((s - it.sum2) * (s - it.dif2));
  // k1 in the CM frame: p1* = p1 + P ((P.p1)/(sqrt s (E + sqrt s)) - E1/sqrt s)
  const double inv_E = rcp64(E + sq);
  const double Pp1 = P[0] * it.p1[0] + P[1] * it.p1[1] + P[2] * it.p1[2];
  const double c1 = (Pp1 * inv_E - it.E1) * rs;
  double n[3] = {it.p1[0] + P[0] * c1, it.p1[1] + P[1] * c1, it.p1[2] + P[2] * c1};
  const double rn = rsqrt64(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  n[0] *= rn; n[1] *= rn; n[2] *= rn;
  // orthonormal completion of n (Duff et al., JCGT 6(1), 2017)
  const double sgn = copysign(1.0, n[2]);
  const double a = -rcp64(sgn + n[2]);
  const double b = n[0] * n[1] * a;
  const double e1[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
  const double e2[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
  const double cth = 2.0 * u[3] - 1.0;
  const double sth = 2.0 * sqrt64(u[3] * (1.0 - u[3]));
  double sphi, cphi;
  sincos_2pi(u[4], sphi, cphi);
  const double sc = sth * cphi, ss = sth * sphi;
  double p3s[3];
  for (int k = 0; k < 3; ++k) p3s[k] = g.pstar * (sc * e1[k] + ss * e2[k] + cth * n[k]);
  const double E3s = 0.5 * (s + it.dm34) * rs;
  const double Pp3 = P[0] * p3s[0] + P[1] * p3s[1] + P[2] * p3s[2];
  const double c3 = (Pp3 * inv_E + E3s) * rs;
  for (int k = 0; k < 3; ++k) {
    g.p3[k] = p3s[k] + P[k] * c3;
    g.p4[k] = P[k] - g.p3[k];
  }
  const double E3 = (E * E3s + Pp3) * rs;
  const double E4 = E - E3;
  for (int k = 0; k < 3; ++k) {
    if (!(fabs(g.p3[k]) <= G.ph[k]) || !(fabs(g.p4[k]) <= G.ph[k])) return false;
  }
  const double d13[3] = {it.p1[0] - g.p3[0], it.p1[1] - g.p3[1], it.p1[2] - g.p3[2]};
  const double d14[3] = {it.p1[0] - g.p4[0], it.p1[1] - g.p4[1], it.p1[2] - g.p4[2]};
  g.t = (it.E1 - E3) * (it.E1 - E3) - (d13[0] * d13[0] + d13[1] * d13[1] + d13[2] * d13[2]);
  g.u = (it.E1 - E4) * (it.E1 - E4) - (d14[0] * d14[0] + d14[1] * d14[1] + d14[2] * d14[2]);
  return true;
}

// Five 23-bit uniforms from one Philox block: the top 23 bits of each word,
// and for the fifth the low 9 bits of words 0 and 1 and bits 4..8 of word 2.
__device__ __forceinline__ void five_uniforms(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, double u[5]) {
  u[0] = unif23(x0 >> 9);
  u[1] = unif23(x1 >> 9);
  u[2] = unif23(x2 >> 9);
  u[3] = unif23(x3 >> 9);
  u[4] = unif23(((x0 & 0x1FFu) << 14) | ((x1 & 0x1FFu) << 5) | ((x2 & 0x1FFu) >> 4));
}

// Order a wave's LDS accesses across its lanes (the LDS executes one wave's
// instructions in order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront sums.  The FP64 and root kernels, with one short item per
// wavefront, use DPP: two quad permutations and two rotations within
// each 16-lane row leave every lane with its row's sum; the four row sums
// are read from lanes 0, 16, 32, 48 and added in a fixed order.  Every lane
// must be active.
template <int kCtrl>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, false);
}

template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_i32<kCtrl>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_i32<kCtrl>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Butterfly sums through lane permutes, for the FP32 kernel (long items).
__device__ __forceinline__ int wave_count(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int wave_count_dpp(int v) {
  v += dpp_i32<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_i32<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_i32<0x124>(v);  // row_ror:4
  v += dpp_i32<0x128>(v);  // row_ror:8
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x124>(v);
  v += dpp_f64<0x128>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// ---------------------------------------------------------------------------
// Mixture proposal (learned sampler).  Row = (channel, observed node).
// thr[0] = alpha 2^32 selects the defensive uniform component; component k is
// drawn when thr[k] <= x < thr[k+1].  Its five coordinates are logistic-normal:
// y = mu + sigma z (z from Box-Muller), u = 1/(1 + exp(-y)).  The sample
// location is formed in FP64 (it decides the threshold and the box cut); the
// density q(u) = alpha + sum_k pi_k prod_d N(y_d; mu, sigma)/(u_d(1-u_d)) is
// evaluated in the kernel's precision.
// ---------------------------------------------------------------------------
constexpr double kTwo32 = 4294967296.0;
constexpr double kHalfLog2Pi = 0.91893853320467274178;

// Draw u (and y = logit u) for one sample from the 8 words of two Philox blocks.
__device__ __forceinline__ void mix_draw(const uint32_t x[8], const uint32_t* __restrict__ thr,
                                         const float* __restrict__ mu, const float* __restrict__ sg, int K,
                                         double u[5], double y[5]) {
  if (x[0] < thr[0]) {
    for (int d = 0; d < 5; ++d) {
      u[d] = unif23(x[1 + d] >> 9);
      y[d] = log64(u[d] * rcp64(1.0 - u[d]));
    }
    return;
  }
  int k = 0;
  for (int j = 1; j < K; ++j) k = x[0] >= thr[j] ? j : k;
  double z[6];
  for (int pr = 0; pr < 3; ++pr) {
    const double a1 = unif23(x[1 + 2 * pr] >> 9), a2 = unif23(x[2 + 2 * pr] >> 9);
    const double r = sqrt64(-2.0 * log64(a1));
    double sn, cs;
    sincos_2pi(a2, sn, cs);
    z[2 * pr] = r * cs;
    z[2 * pr + 1] = r * sn;
  }
  for (int d = 0; d < 5; ++d) {
    y[d] = (double)mu[k * 5 + d] + (double)sg[k * 5 + d] * z[d];
    u[d] = rcp64(1.0 + exp64(-y[d]));
  }
}

// Per-item constants of the FP32 sampler, one row per wave in LDS: mu (40),
// 1/sigma (40), log pi_k - sum_d log sigma_kd - 5/2 log 2 pi (8), alpha,
// sigma (40).
constexpr int kMixSigma = 89;
constexpr int kMixRow = kMixSigma + 40;
static_assert(5 * kMixKF32 == 40 && kMixKF32 <= 8, "row layout: 8 components");

// The same draw for the FP32 kernel: component parameters from the wave's
// LDS row (see mix_prepare_f32), thresholds from the (wave-uniform) table
// row; u in FP64 (it feeds the FP64 geometry), y in FP32 (it feeds only the
// FP32 density).
__device__ __forceinline__ void mix_draw_row(const uint32_t x[8], const uint32_t* __restrict__ thr, const float* row,
                                             int K, double u[5], float y[5]) {
  if (x[0] < thr[0]) {
    for (int d = 0; d < 5; ++d) {
      const uint32_t v = x[1 + d] >> 9;
      u[d] = unif23(v);
      const float uf = ((float)v + 0.5f) * (1.0f / 8388608.0f);  // = u[d] exactly, >= 2^-24
      // logit u = ln 2 (log2 u - log2 (1 - u)); v_log_f32 is log2 (no denormals here)
      y[d] = 0.6931471805599453f * (__builtin_amdgcn_logf(uf) - __builtin_amdgcn_logf(1.0f - uf));
    }
    return;
  }
  // component: the last threshold at or below x[0] (unrolled to the 8
  // components this row layout holds, so the threshold loads issue together)
  int k = 0;
#pragma unroll
  for (int j = 1; j < kMixKF32; ++j)
    if (j < K) k = x[0] >= thr[j] ? j : k;
  double z[6];
  for (int pr = 0; pr < 3; ++pr) {
    const double a1 = unif23(x[1 + 2 * pr] >> 9), a2 = unif23(x[2 + 2 * pr] >> 9);
    const double r = sqrt64(-2.0 * log64(a1));
    double sn, cs;
    sincos_2pi(a2, sn, cs);
    z[2 * pr] = r * cs;
    z[2 * pr + 1] = r * sn;
  }
  for (int d = 0; d < 5; ++d) {
    const double yd = (double)row[k * 5 + d] + (double)row[kMixSigma + k * 5 + d] * z[d];
    u[d] = rcp64(1.0 + exp64(-yd));
    y[d] = (float)yd;
  }
}

// log of u(1-u) from y = logit(u), written stably
template <typename R>
__device__ __forceinline__ R log_u1mu(R y) {
  const R a = y < R(0) ? -y : y;
  return -a - R(2) * log1p(exp(-a));
}

// q(u) in FP64 straight from the table row (reference-precision path)
__device__ __forceinline__ double mix_density_f64(const uint32_t* thr, const float* mu, const float* sg, int K,
                                                  const double y[5]) {
  double lk[16];
  double mx = -1e300;
  for (int k = 0; k < K; ++k) {
    const double hi = k + 1 < K ? (double)thr[k + 1] : kTwo32;
    const double pk = (hi - (double)thr[k]) / kTwo32;
    if (!(pk > 0.0)) { lk[k] = -1e300; continue; }
    double l = log(pk);
    for (int d = 0; d < 5; ++d) {
      const double s = (double)sg[k * 5 + d];
      const double z = (y[d] - (double)mu[k * 5 + d]) / s;
      l += -0.5 * z * z - log(s) - kHalfLog2Pi;
    }
    lk[k] = l;
    mx = fmax(mx, l);
  }
  double acc = 0.0;
  for (int k = 0; k < K; ++k) acc += exp(lk[k] - mx);
  double lq = mx + log(acc);
  for (int d = 0; d < 5; ++d) lq -= log_u1mu<double>(y[d]);
  return (double)thr[0] / kTwo32 + exp(lq);
}


__device__ __forceinline__ void mix_prepare_f32(const uint32_t* thr, const float* mu, const float* sg, int K,
                                                float* row, int lane) {
  for (int i = lane; i < K * 5; i += kWave) {
    row[i] = mu[i];
    row[40 + i] = (float)(rcp64((double)sg[i]) * 0.70710678118654752);
    row[kMixSigma + i] = sg[i];
  }
  // log pi_k - sum_d log sigma_kd - 5/2 log 2pi: the K x 6 logarithms one per
  // lane (lane 6k holds log pi_k, lanes 6k+1..6k+5 -log sigma_kd), gathered
  // by lane k; the wave waits for one logarithm instead of six in a row
  double lg = 0.0;
  const int kc = lane / 6, jc = lane - 6 * kc;
  if (lane < 6 * K) {
    if (jc == 0) {
      const double hi = kc + 1 < K ? (double)thr[kc + 1] : kTwo32;
      const double pk = (hi - (double)thr[kc]) * (1.0 / kTwo32);
      lg = pk > 0.0 ? log64(pk) : -1e30;
    } else {
      lg = -log64((double)sg[kc * 5 + jc - 1]);
    }
  }
  double c = -5.0 * kHalfLog2Pi;
#pragma unroll
  for (int t = 0; t < 6; ++t) c += __shfl(lg, min(6 * lane + t, kWave - 1), kWave);
  if (lane < K) row[80 + lane] = (float)c;
  if (lane == 0) row[88] = (float)((double)thr[0] / kTwo32);
}

// e^x and ln x from the hardware base-2 instructions (about one ulp; no
// special-case handling: the arguments here are finite, and a zero or
// subnormal sum of exponentials gives -inf or a large negative log, which
// leaves q = alpha through the final exponential)
__device__ __forceinline__ float exp_f32(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float log_f32(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }

__device__ __forceinline__ float mix_density_f32(const float* row, int K, const float yf[5]) {
  // l_k <= log pi_k - sum_d log sigma_kd - 5/2 log 2pi <= 35 (sigma >= e^-7), so the
  // exponentials need no max shift; all of them underflowing leaves q = alpha.
  // Unrolled over the 8 components the row holds, so the LDS reads of later
  // components are issued before the arithmetic of earlier ones waits.
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kMixKF32; ++k) {
    if (k < K) {
      float l = row[80 + k];
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        const float z = (yf[d] - row[k * 5 + d]) * row[40 + k * 5 + d];
        l = fmaf(-z, z, l);
      }
      acc += exp_f32(l);
    }
  }
  float lq = log_f32(acc);
  // log(u (1 - u)) = -|y| - 2 log(1 + e^-|y|); the five factors 1 + e^-|y|
  // lie in [1, 2], so their product takes one logarithm
  float prod = 1.0f;
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    const float a = fabsf(yf[d]);
    lq += a;
    prod *= 1.0f + exp_f32(-a);
  }
  lq += 2.0f * log_f32(prod);
  return row[88] + exp_f32(lq);
}

// Set up the wave-uniform item constants.
// The item constants of a (cell, channel) pair: masses, threshold terms and
// the channel coefficient (the same for every observed node of the pair).
__device__ __forceinline__ void item_pair(Item& it, const CollideArgs& A, const Channel& ch, int cell) {
  const Grid& G = A.G;
  it.cell = cell;
  it.m1sq = A.mass2[ch.sp[0] * G.cells + cell];
  it.m2sq = A.mass2[ch.sp[1] * G.cells + cell];
  it.m3sq = A.mass2[ch.sp[2] * G.cells + cell];
  it.m4sq = A.mass2[ch.sp[3] * G.cells + cell];
  it.mu = A.mass2[kGluon * G.cells + cell];
  const double m3 = sqrt(it.m3sq), m4 = sqrt(it.m4sq);
  it.sum2 = (m3 + m4) * (m3 + m4);
  it.dif2 = (m3 - m4) * (m3 - m4);
  it.dm34 = it.m3sq - it.m4sq;
  const double V5 = G.Vp * 4.0 * kPi;
  it.coef = (A.symmetric ? ch.w : ch.sigma) * V5 / (double)A.n_samples;
}

// The observed node's part of the item constants (p1, E1, f1, prefactor).
__device__ __forceinline__ void item_node(Item& it, const CollideArgs& A, const Channel& ch, int p1_lin) {
  const Grid& G = A.G;
  it.p1_lin = p1_lin;
  const int iz = p1_lin % G.np[2];
  const int iy = (p1_lin / G.np[2]) % G.np[1];
  const int ix = p1_lin / (G.np[2] * G.np[1]);
  it.p1[0] = node_coord(G.ph[0], G.dp[0], ix);
  it.p1[1] = node_coord(G.ph[1], G.dp[1], iy);
  it.p1[2] = node_coord(G.ph[2], G.dp[2], iz);
  it.E1 = sqrt(it.p1[0] * it.p1[0] + it.p1[1] * it.p1[1] + it.p1[2] * it.p1[2] + it.m1sq);
  it.f1 = A.f64[((size_t)ch.sp[0] * G.cells + it.cell) * G.nodes + p1_lin];
  it.pref = it.coef * G.g4 * kNorm / it.E1;
}

__device__ __forceinline__ void load_item(Item& it, const CollideArgs& A, const Channel& ch, int cell, int p1_lin) {
  item_pair(it, A, ch, cell);
  item_node(it, A, ch, p1_lin);
}


// Per-sample value without the bracket, in precision R: |M|^2 times the
// phase-space prefactor.
template <typename R>
__device__ __forceinline__ R prefactor(const Item& it, const Geo& g) {
  return (R)it.pref * (R)g.pstar * (R)g.rs * rcp_r<R>((R)g.E2);
}

template <typename R, bool kUser = true>
__device__ __forceinline__ R weight_no_bracket(const CollideArgs& A, const Item& it, const Geo& g, int row) {
  const R m = msq_row<R, kUser>(A.msq_mask, A.msq, row, (R)g.s, (R)g.t, (R)g.u, (R)it.mu);
  return m * prefactor<R>(it, g);
}

__device__ __forceinline__ bool is_gluon(int sp) { return sp == kGluon; }

// Unbiased estimate of the variance of an item's direct sum S = sum_s v_s
// over N samples: N/(N-1) (sum v^2 - S^2/N).
__device__ __forceinline__ double item_variance(double s, double sq, int n) {
  if (n < 2) return 0.0;
  return fmax(0.0, (sq - s * s / n) * ((double)n / (n - 1)));
}

}  // namespace

// Per-workgroup totals of the accepted count, the two error sums and the
// per-channel variance sums: the waves add into LDS and the workgroup adds
// its totals into global memory at the end, into stripe b mod kStripes (one
// global atomic per workgroup and value instead of one per item on a single
// address).
struct BlockTotals {
  unsigned long long* ok;
  double* mc;   // [2]
  double* var;  // [kMaxChannels]
  __device__ void init() {
    if (threadIdx.x == 0) {
      *ok = 0ull;
      mc[0] = 0.0;
      mc[1] = 0.0;
    }
    for (int i = threadIdx.x; i < kMaxChannels; i += blockDim.x) var[i] = 0.0;
    __syncthreads();
  }
  __device__ void add(int n_ok, double item_var, double sq, int ci) {
    __hip_atomic_fetch_add(ok, (unsigned long long)n_ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&mc[0], item_var, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&mc[1], sq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&var[ci], item_var, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ void flush(const CollideArgs& A) {
    __syncthreads();
    const int stripe = blockIdx.x % kStripes;
    if (threadIdx.x == 0) {
      if (A.n_accepted) atomicAdd(A.n_accepted + stripe, *ok);
      if (A.mc_acc) {
        atomicAdd(&A.mc_acc[2 * stripe], mc[0]);
        atomicAdd(&A.mc_acc[2 * stripe + 1], mc[1]);
      }
    }
    if (A.chan_var)
      for (int i = threadIdx.x; i < A.n_channels; i += blockDim.x)
        if (var[i] != 0.0) atomicAdd(&A.chan_var[(size_t)stripe * A.n_channels + i], var[i]);
  }
};

// ---------------------------------------------------------------------------
// FP64 kernel: f read from the FP64 field in global memory, deposits as FP64
// atomics into the output.  This is the reference-precision path.  kPriv (a
// grid whose whole output fits in LDS): the symmetric deposits go to a
// workgroup-private FP64 copy of the output in LDS, in the output's layout,
// flushed once per workgroup, instead of every workgroup's atomics
// contending for the same few global addresses.
// ---------------------------------------------------------------------------
template <bool kLearned, bool kPriv>
__global__ __launch_bounds__(256) void collide_f64_kernel(CollideArgs A) {
  const Grid& G = A.G;
  extern __shared__ double f64_acc[];  // kPriv: [7][cells][nodes], as the output
  const int n_out = kPriv ? kSpecies * G.cells * G.nodes : 0;
  for (int i = threadIdx.x; i < n_out; i += blockDim.x) f64_acc[i] = 0.0;
  __shared__ unsigned long long blk_ok;
  __shared__ double blk_mc[2];
  __shared__ double blk_var[kMaxChannels];
  BlockTotals blk{&blk_ok, blk_mc, blk_var};
  __shared__ Channel s_ch[kMaxChannels];
  __shared__ int s_group[kMaxChannels];
  for (int i = threadIdx.x; i < A.n_group; i += blockDim.x) s_group[i] = A.group[i];
  for (int i = threadIdx.x; i < A.n_channels; i += blockDim.x) s_ch[i] = A.chans[i];
  blk.init();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = gridDim.x * blockDim.x / kWave;
  const long long n_items = (long long)G.cells * A.n_group * G.nodes;
  for (long long w = wave; w < n_items; w += nwaves) {
    const int p1_lin = (int)(w % G.nodes);
    const int gi = (int)((w / G.nodes) % A.n_group);
    const int cell = (int)(w / ((long long)G.nodes * A.n_group));
    const int ci = s_group[gi];
    const Channel ch = s_ch[ci];
    Item it;
    load_item(it, A, ch, cell, p1_lin);
    if (!(it.E1 > 0.0)) {  // massless p = 0 node: zero measure
      if (lane == 0 && A.items) A.items[((size_t)cell * A.n_channels + ci) * G.nodes + p1_lin] = 0.0;
      continue;
    }
    const double* fc[4];
    double* Ac[4];
    double* Sc[4];
    for (int p = 0; p < 4; ++p) {
      fc[p] = A.f64 + ((size_t)ch.sp[p] * G.cells + cell) * G.nodes;
      Ac[p] = A.A + ((size_t)ch.sp[p] * G.cells + cell) * G.nodes;
      Sc[p] = A.scale ? A.scale + ((size_t)ch.sp[p] * G.cells + cell) * G.nodes : nullptr;
    }
    const bool g1 = is_gluon(ch.sp[0]), g2 = is_gluon(ch.sp[1]);
    const bool g3 = is_gluon(ch.sp[2]), g4 = is_gluon(ch.sp[3]);
    const double F1 = g1 ? 1.0 + it.f1 : 1.0 - it.f1;
    double dsum = 0.0, ssum = 0.0, dsq = 0.0;
    int n_ok = 0;
    const size_t mrow = (size_t)ci * G.nodes + p1_lin;
    const bool mix = kLearned && (!A.mix_on || A.mix_on[ci]);
    for (int s = lane; s < A.n_samples; s += kWave) {
      uint32_t x0 = (uint32_t)s, x1 = (uint32_t)p1_lin, x2 = (uint32_t)cell, x3 = ((uint32_t)ch.code << 8);
      philox4x32_10(x0, x1, x2, x3, A.key0, A.key1);
      double u[5];
      double inv_q = 1.0;
      if (mix) {
        uint32_t y0 = (uint32_t)s, y1 = (uint32_t)p1_lin, y2 = (uint32_t)cell, y3 = ((uint32_t)ch.code << 8) | 1u;
        philox4x32_10(y0, y1, y2, y3, A.key0, A.key1);
        const uint32_t xw[8] = {x0, x1, x2, x3, y0, y1, y2, y3};
        double yl[5];
        const uint32_t* thr = A.mix_thr + mrow * A.mix_K;
        const float* mu = A.mix_mu + mrow * A.mix_K * 5;
        const float* sg = A.mix_sigma + mrow * A.mix_K * 5;
        mix_draw(xw, thr, mu, sg, A.mix_K, u, yl);
        inv_q = 1.0 / mix_density_f64(thr, mu, sg, A.mix_K, yl);
      } else {
        five_uniforms(x0, x1, x2, x3, u);
      }
      Geo g;
      if (!geometry(it, G, u, g)) continue;
      ++n_ok;
      const double wnb = weight_no_bracket<double>(A, it, g, ch.row) * inv_q;
      const Stencil<double> s2 = make_stencil<double>(g.p2, G);
      const Stencil<double> s3 = make_stencil<double>(g.p3, G);
      const Stencil<double> s4 = make_stencil<double>(g.p4, G);
      const double f2 = interpolate<double>(fc[1], s2, G.ox, G.oy);
      const double f3 = interpolate<double>(fc[2], s3, G.ox, G.oy);
      const double f4 = interpolate<double>(fc[3], s4, G.ox, G.oy);
      const double F2 = g2 ? 1.0 + f2 : 1.0 - f2;
      const double F3 = g3 ? 1.0 + f3 : 1.0 - f3;
      const double F4 = g4 ? 1.0 + f4 : 1.0 - f4;
      const double gain = f3 * f4 * F1 * F2, loss = it.f1 * f2 * F3 * F4;
      const double v = wnb * (gain - loss);
      dsum += v;
      dsq = fma(v, v, dsq);
      const double vs = fabs(wnb) * (gain + loss);
      ssum += vs;
      if (kPriv) {
        deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(f64_acc + (Ac[1] - A.A), s2, v, G.ox, G.oy);
        deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(f64_acc + (Ac[2] - A.A), s3, -v, G.ox, G.oy);
        deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(f64_acc + (Ac[3] - A.A), s4, -v, G.ox, G.oy);
        if (A.scale) {
          deposit<double, double>(Sc[1], s2, vs, G.ox, G.oy);
          deposit<double, double>(Sc[2], s3, vs, G.ox, G.oy);
          deposit<double, double>(Sc[3], s4, vs, G.ox, G.oy);
        }
      } else if (A.symmetric) {
        deposit<double, double>(Ac[1], s2, v, G.ox, G.oy);
        deposit<double, double>(Ac[2], s3, -v, G.ox, G.oy);
        deposit<double, double>(Ac[3], s4, -v, G.ox, G.oy);
        if (A.scale) {
          deposit<double, double>(Sc[1], s2, vs, G.ox, G.oy);
          deposit<double, double>(Sc[2], s3, vs, G.ox, G.oy);
          deposit<double, double>(Sc[3], s4, vs, G.ox, G.oy);
        }
      }
    }
    dsum = wave_sum_dpp(dsum);
    if (A.scale) ssum = wave_sum_dpp(ssum);
    dsq = wave_sum_dpp(dsq);
    const int ok_total = wave_count_dpp(n_ok);
    if (lane == 0) {
      blk.add(ok_total, item_variance(dsum, dsq, A.n_samples), dsum * dsum, ci);
      atomicAdd(Ac[0] + p1_lin, dsum);
      if (A.scale) atomicAdd(Sc[0] + p1_lin, ssum);
      if (A.items) A.items[((size_t)cell * A.n_channels + ci) * G.nodes + p1_lin] = dsum;
    }
  }
  blk.flush(A);  // (begins with a barrier: every wave's deposits are in)
  for (int i = threadIdx.x; i < n_out; i += blockDim.x)  // kPriv: the same layout as the output
    if (f64_acc[i] != 0.0) atomicAdd(A.A + i, f64_acc[i]);
}

// ---------------------------------------------------------------------------
// The paper's own parameterisation (Eq. work out delta E, Eq. delta replace):
// momentum conservation eliminates one momentum, energy conservation fixes
// one z component at the two roots of a quadratic, and each root carries
// 1/|J|.  In channel order k1 + k2 <-> k3 + k4 with k1 observed (the
// paper's p):
//   kAlt = false, the paper's choice: k2 uniform in the box, k3x and k3y
//     uniform, k4 = k1 + k2 - k3; E1 + E2 = E3 + E4 has the roots
//     z = (c Qz +- W sqrt(c^2 - 4 a (W^2 - Qz^2))) / (2 (W^2 - Qz^2)) with
//     W = E1 + E2 > 0, Q = k1 + k2, a = k3x^2 + k3y^2 + m3^2,
//     c = W^2 + a - (Qx - k3x)^2 - (Qy - k3y)^2 - m4^2 - Qz^2; a root holds
//     when c + 2 Qz z > 0 and E3 < W;
//   kAlt = true, the alternative the paper tests (Sec. IV A): k4 uniform in
//     the box, k3x and k3y uniform, k2 = k3 + k4 - k1; E3 - E2 = D = E1 - E4
//     gives z = (-C Qz +- |D| sqrt(C^2 + 4 a (Qz^2 - D^2))) / (2 (Qz^2 - D^2))
//     with Q = k4 - k1, C = 2 (k3x Qx + k3y Qy) + Q^2 + m2^2 - m3^2 - D^2; a
//     root holds when (C + 2 Qz z) D < 0 and E3 > D.  Its leading
//     coefficient has no fixed sign: the instability the paper reports.
// The value of a root is w V5 / N |M|^2 B / ((2 pi)^5 16 E1 E2 E3 E4 |J|),
// V5 = (2 P)^3 (2 Px) (2 Py), J the z derivative of the energy sum.  FP64
// throughout (f from the FP64 field, FP64 atomics): the reference method.
// Every lane draws a sample and solves for its roots; samples with a valid
// root go to a per-wavefront queue in LDS, and whenever 64 are queued (and
// at the end of the item) the wavefront evaluates them on full lanes, so the
// value, f and deposits run once per valid sample, not on every lane.
// ---------------------------------------------------------------------------
constexpr double kRootNorm = 1.0 / (32.0 * kPi * kPi * kPi * kPi * kPi * 16.0);

constexpr int kRootWaves = 4;      // wavefronts per workgroup of the root kernel
constexpr int kRootQueueLen = 128;  // queued samples per wavefront (< 64 left + 64 new)

template <bool kAlt, bool kPriv>
__global__ __launch_bounds__(kRootWaves * kWave) void collide_roots_kernel(CollideArgs A) {
  const Grid& G = A.G;
  extern __shared__ double root_acc[];  // kPriv: [7][cells][nodes], as the output (see the FP64 kernel)
  const int n_out = kPriv ? kSpecies * G.cells * G.nodes : 0;
  for (int i = threadIdx.x; i < n_out; i += blockDim.x) root_acc[i] = 0.0;
  __shared__ unsigned long long blk_ok;
  __shared__ double blk_mc[2];
  __shared__ double blk_var[kMaxChannels];
  BlockTotals blk{&blk_ok, blk_mc, blk_var};
  __shared__ Channel s_ch[kMaxChannels];
  __shared__ int s_group[kMaxChannels];
  // Samples with at least one valid root, queued per wavefront: the uniform
  // momentum (k2 or k4), k3x, k3y, the two roots, and which roots hold.
  __shared__ double rq[kRootWaves][7][kRootQueueLen];
  __shared__ uint32_t rm[kRootWaves][kRootQueueLen];
  for (int i = threadIdx.x; i < A.n_group; i += blockDim.x) s_group[i] = A.group[i];
  for (int i = threadIdx.x; i < A.n_channels; i += blockDim.x) s_ch[i] = A.chans[i];
  blk.init();
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = gridDim.x * blockDim.x / kWave;
  const long long n_items = (long long)G.cells * A.n_group * G.nodes;
  for (long long w = wave; w < n_items; w += nwaves) {
    const int p1_lin = (int)(w % G.nodes);
    const int gi = (int)((w / G.nodes) % A.n_group);
    const int cell = (int)(w / ((long long)G.nodes * A.n_group));
    const int ci = s_group[gi];
    const Channel ch = s_ch[ci];
    Item it;
    load_item(it, A, ch, cell, p1_lin);
    if (!(it.E1 > 0.0)) {  // massless p = 0 node: zero measure
      if (lane == 0 && A.items) A.items[((size_t)cell * A.n_channels + ci) * G.nodes + p1_lin] = 0.0;
      continue;
    }
    const double* fc[4];
    double* Ac[4];
    double* Sc[4];
    for (int p = 0; p < 4; ++p) {
      fc[p] = A.f64 + ((size_t)ch.sp[p] * G.cells + cell) * G.nodes;
      Ac[p] = A.A + ((size_t)ch.sp[p] * G.cells + cell) * G.nodes;
      Sc[p] = A.scale ? A.scale + ((size_t)ch.sp[p] * G.cells + cell) * G.nodes : nullptr;
    }
    const bool g1 = is_gluon(ch.sp[0]), g2 = is_gluon(ch.sp[1]);
    const bool g3 = is_gluon(ch.sp[2]), g4 = is_gluon(ch.sp[3]);
    const double F1 = g1 ? 1.0 + it.f1 : 1.0 - it.f1;
    const double V5 = G.Vp * (2.0 * G.ph[0]) * (2.0 * G.ph[1]);
    const double coef = (A.symmetric ? ch.w : ch.sigma) * V5 / (double)A.n_samples * G.g4 * kRootNorm / it.E1;
    double dsum = 0.0, ssum = 0.0, dsq = 0.0;
    int n_ok = 0;
    // The value of one queued sample: the sum over its valid roots, with
    // their deposits.
    auto finish = [&](unsigned slot) {
      const double q[3] = {rq[wid][0][slot], rq[wid][1][slot], rq[wid][2][slot]};
      const double k3x = rq[wid][3][slot], k3y = rq[wid][4][slot];
      const uint32_t roots = rm[wid][slot];
      const double a3 = k3x * k3x + k3y * k3y + it.m3sq;
      const double Eq = sqrt64(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + (kAlt ? it.m4sq : it.m2sq));
      double vsample = 0.0;
#pragma unroll 1
      for (int r = 0; r < 2; ++r) {
        if (!((roots >> r) & 1u)) continue;
        const double z = rq[wid][5 + r][slot];
        const double E3 = sqrt64(a3 + z * z);
        double p2[3], p3[3] = {k3x, k3y, z}, p4[3], E2, E4, J;
        if (!kAlt) {
          for (int a = 0; a < 3; ++a) {
            p2[a] = q[a];
            p4[a] = it.p1[a] + q[a] - p3[a];
          }
          E2 = Eq;
          E4 = sqrt64(p4[0] * p4[0] + p4[1] * p4[1] + p4[2] * p4[2] + it.m4sq);
          J = fabs(z * rcp64(E3) - p4[2] * rcp64(E4));
        } else {
          for (int a = 0; a < 3; ++a) {
            p4[a] = q[a];
            p2[a] = p3[a] + (q[a] - it.p1[a]);
          }
          E4 = Eq;
          E2 = sqrt64(p2[0] * p2[0] + p2[1] * p2[1] + p2[2] * p2[2] + it.m2sq);
          J = fabs(p2[2] * rcp64(E2) - z * rcp64(E3));
        }
        ++n_ok;
        double Pq[3], d13[3], d14[3];
        for (int a = 0; a < 3; ++a) {
          Pq[a] = it.p1[a] + p2[a];
          d13[a] = it.p1[a] - p3[a];
          d14[a] = it.p1[a] - p4[a];
        }
        const double E12 = it.E1 + E2, E13 = it.E1 - E3, E14 = it.E1 - E4;
        const double ms = E12 * E12 - (Pq[0] * Pq[0] + Pq[1] * Pq[1] + Pq[2] * Pq[2]);
        const double mt = E13 * E13 - (d13[0] * d13[0] + d13[1] * d13[1] + d13[2] * d13[2]);
        const double mu = E14 * E14 - (d14[0] * d14[0] + d14[1] * d14[1] + d14[2] * d14[2]);
        const double wnb = coef * msq_row<double>(A.msq_mask, A.msq, ch.row, ms, mt, mu, it.mu) *
                           rcp64(E2 * E3 * E4 * J);
        const Stencil<double> s2 = make_stencil<double>(p2, G);
        const Stencil<double> s3 = make_stencil<double>(p3, G);
        const Stencil<double> s4 = make_stencil<double>(p4, G);
        const double f2 = interpolate<double>(fc[1], s2, G.ox, G.oy);
        const double f3 = interpolate<double>(fc[2], s3, G.ox, G.oy);
        const double f4 = interpolate<double>(fc[3], s4, G.ox, G.oy);
        const double F2 = g2 ? 1.0 + f2 : 1.0 - f2;
        const double F3 = g3 ? 1.0 + f3 : 1.0 - f3;
        const double F4 = g4 ? 1.0 + f4 : 1.0 - f4;
        const double gain = f3 * f4 * F1 * F2, loss = it.f1 * f2 * F3 * F4;
        const double v = wnb * (gain - loss);
        const double vs = fabs(wnb) * (gain + loss);
        vsample += v;
        ssum += vs;
        if (kPriv) {
          deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(root_acc + (Ac[1] - A.A), s2, v, G.ox, G.oy);
          deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(root_acc + (Ac[2] - A.A), s3, -v, G.ox, G.oy);
          deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(root_acc + (Ac[3] - A.A), s4, -v, G.ox, G.oy);
          if (A.scale) {
            deposit<double, double>(Sc[1], s2, vs, G.ox, G.oy);
            deposit<double, double>(Sc[2], s3, vs, G.ox, G.oy);
            deposit<double, double>(Sc[3], s4, vs, G.ox, G.oy);
          }
        } else if (A.symmetric) {
          deposit<double, double>(Ac[1], s2, v, G.ox, G.oy);
          deposit<double, double>(Ac[2], s3, -v, G.ox, G.oy);
          deposit<double, double>(Ac[3], s4, -v, G.ox, G.oy);
          if (A.scale) {
            deposit<double, double>(Sc[1], s2, vs, G.ox, G.oy);
            deposit<double, double>(Sc[2], s3, vs, G.ox, G.oy);
            deposit<double, double>(Sc[3], s4, vs, G.ox, G.oy);
          }
        }
      }
      dsum += vsample;
      dsq = fma(vsample, vsample, dsq);
    };
    unsigned head = 0, tail = 0;  // ring positions (wave-uniform)
    for (int base = 0; base < A.n_samples; base += kWave) {
      const int s = base + lane;
      uint32_t roots = 0;
      double q[3], k3x = 0.0, k3y = 0.0, zr[2] = {0.0, 0.0};
      if (s < A.n_samples) {
        uint32_t x0 = (uint32_t)s, x1 = (uint32_t)p1_lin, x2 = (uint32_t)cell, x3 = ((uint32_t)ch.code << 8) | 2u;
        philox4x32_10(x0, x1, x2, x3, A.key0, A.key1);
        double u[5];
        five_uniforms(x0, x1, x2, x3, u);
        for (int a = 0; a < 3; ++a) q[a] = fma(2.0 * G.ph[a], u[a], -G.ph[a]);
        k3x = fma(2.0 * G.ph[0], u[3], -G.ph[0]);
        k3y = fma(2.0 * G.ph[1], u[4], -G.ph[1]);
        const double a3 = k3x * k3x + k3y * k3y + it.m3sq;
        const double Eq = sqrt64(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + (kAlt ? it.m4sq : it.m2sq));
        double Q[3], lin, half, den, W = 0.0, D = 0.0, C = 0.0;
        bool any;
        if (!kAlt) {
          W = it.E1 + Eq;
          for (int a = 0; a < 3; ++a) Q[a] = it.p1[a] + q[a];
          const double b = (Q[0] - k3x) * (Q[0] - k3x) + (Q[1] - k3y) * (Q[1] - k3y) + it.m4sq;
          C = W * W + a3 - b - Q[2] * Q[2];
          den = W * W - Q[2] * Q[2];
          const double H = C * C - 4.0 * a3 * den;
          any = H >= 0.0 && den > 0.0;
          lin = C * Q[2];
          half = any ? W * sqrt64(H) : 0.0;
        } else {
          D = it.E1 - Eq;
          for (int a = 0; a < 3; ++a) Q[a] = q[a] - it.p1[a];
          C = 2.0 * (k3x * Q[0] + k3y * Q[1]) + (Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]) + it.m2sq - it.m3sq - D * D;
          den = Q[2] * Q[2] - D * D;
          const double H = C * C + 4.0 * a3 * den;
          any = H >= 0.0 && den != 0.0 && D != 0.0;
          lin = -C * Q[2];
          half = any ? fabs(D) * sqrt64(H) : 0.0;
        }
        const double inv_2den = any ? rcp64(2.0 * den) : 0.0;
        for (int r = 0; r < 2 && any; ++r) {
          const double z = (lin + (r == 0 ? half : -half)) * inv_2den;
          const double E3 = sqrt64(a3 + z * z);
          bool ok;
          if (!kAlt) ok = (C + 2.0 * Q[2] * z > 0.0) && (E3 < W);
          else ok = ((C + 2.0 * Q[2] * z) * D < 0.0) && (E3 - D > 0.0);
          const double p3[3] = {k3x, k3y, z};
          for (int a = 0; a < 3; ++a) {
            const double other = kAlt ? p3[a] + Q[a] : Q[a] - p3[a];  // p2 or p4
            ok = ok && fabs(p3[a]) <= G.ph[a] && fabs(other) <= G.ph[a];
          }
          if (ok) {
            roots |= 1u << r;
            zr[r] = z;
          }
        }
      }
      const unsigned long long mask = __ballot(roots != 0u);
      if (roots) {
        const unsigned slot = (tail + (unsigned)__popcll(mask & ((1ull << lane) - 1ull))) & (kRootQueueLen - 1);
        for (int a = 0; a < 3; ++a) rq[wid][a][slot] = q[a];
        rq[wid][3][slot] = k3x;
        rq[wid][4][slot] = k3y;
        rq[wid][5][slot] = zr[0];
        rq[wid][6][slot] = zr[1];
        rm[wid][slot] = roots;
      }
      tail += (unsigned)__popcll(mask);
      if (tail - head >= (unsigned)kWave) {
        wave_lds_sync();
        finish((head + lane) & (kRootQueueLen - 1));
        head += kWave;
        wave_lds_sync();
      }
    }
    if (tail != head) {  // the last, partial batch
      wave_lds_sync();
      if ((unsigned)lane < tail - head) finish((head + lane) & (kRootQueueLen - 1));
      wave_lds_sync();
    }
    dsum = wave_sum_dpp(dsum);
    if (A.scale) ssum = wave_sum_dpp(ssum);
    dsq = wave_sum_dpp(dsq);
    const int ok_total = wave_count_dpp(n_ok);
    if (lane == 0) {
      blk.add(ok_total, item_variance(dsum, dsq, A.n_samples), dsum * dsum, ci);
      atomicAdd(Ac[0] + p1_lin, dsum);
      if (A.scale) atomicAdd(Sc[0] + p1_lin, ssum);
      if (A.items) A.items[((size_t)cell * A.n_channels + ci) * G.nodes + p1_lin] = dsum;
    }
  }
  blk.flush(A);  // (begins with a barrier: every wave's deposits are in)
  for (int i = threadIdx.x; i < n_out; i += blockDim.x)
    if (root_acc[i] != 0.0) atomicAdd(A.A + i, root_acc[i]);
}

// ---------------------------------------------------------------------------
// FP32 kernel.  A workgroup owns (cell, channel, a chunk of observed nodes).
// LDS holds FP64 accumulators for the first `lds_acc` deposit slots of the
// channel and FP32 f tiles for the first `lds_tiles` slots; slots beyond those
// deposit with FP64 atomics into the output / read f from global memory.  The
// accumulators are flushed into the FP64 output once per workgroup.
// ---------------------------------------------------------------------------
// Trilinear read from the node quads: the same corners and the same
// arithmetic as interpolate, in two 16-byte loads.
template <typename R>
__device__ __forceinline__ R interpolate_quads(const float4* __restrict__ q4, const Stencil<R>& st, int ox) {
  typedef float V4 __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(1))) const V4 GlobalV4;
  const V4 lo = ((GlobalV4*)q4)[st.base];
  const V4 hi = ((GlobalV4*)q4)[st.base + ox];
  const R a00 = (R)lo.x + st.wz * ((R)lo.y - (R)lo.x);
  const R a01 = (R)lo.z + st.wz * ((R)lo.w - (R)lo.z);
  const R a10 = (R)hi.x + st.wz * ((R)hi.y - (R)hi.x);
  const R a11 = (R)hi.z + st.wz * ((R)hi.w - (R)hi.z);
  const R b0 = a00 + st.wy * (a01 - a00);
  const R b1 = a10 + st.wy * (a11 - a10);
  return b0 + st.wx * (b1 - b0);
}

template <bool kAllLds, typename R>
__device__ __forceinline__ R interp_slot(int k, int n_tiles, const float* tiles, const float4* __restrict__ f32q,
                                         size_t off, const Stencil<R>& st, int nodes, int ox, int oy) {
  // an address-space-qualified view keeps the LDS reads ds_read instructions
  // instead of generic flat loads
  typedef __attribute__((address_space(3))) const float LdsF32;
  if (kAllLds || k < n_tiles) return interpolate<R>((LdsF32*)(tiles + k * nodes), st, ox, oy);
  return interpolate_quads<R>(f32q + off, st, ox);
}

// The corner values are split in FP64 from the FP32 value and weights (both
// convert exactly), so the deposits of a sample cancel to FP64 rounding.
__device__ __forceinline__ Stencil<double> widen(const Stencil<float>& st) {
  return Stencil<double>{st.base, (double)st.wx, (double)st.wy, (double)st.wz};
}

template <bool kAllLds, bool kWin = true>
__device__ __forceinline__ void deposit_slot(int k, int slot_lo, int slot_hi, int n_acc, double* acc,
                                             double* __restrict__ out, size_t off, const Stencil<float>& st,
                                             float v, int nodes, int ox, int oy, int win_lo, int win_n) {
  if (k < slot_lo || k >= slot_hi) return;  // deposited by another launch
  const int j = k - slot_lo;
  if (kAllLds || j < n_acc) {
    if (!kWin || win_n == nodes)  // (wave-uniform) the whole grid in LDS
      deposit<double, double, __HIP_MEMORY_SCOPE_WORKGROUP>(acc + j * win_n, widen(st), (double)v, ox, oy);
    else
      deposit_window(acc + j * win_n, widen(st), (double)v, ox, oy, win_lo, win_n);
  } else {
    deposit<double, double>(out + off, widen(st), (double)v, ox, oy);
  }
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b mod
// 8), and each XCD has its own L2.  The logical index hands each XCD a
// contiguous range of (cell, channel, chunk) work, so the workgroups that
// read a cell's f quads and flush into its output rows share one L2.
__device__ __forceinline__ int xcd_local_block(int b, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd, x = b % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// Workgroup size: 12 waves, 3 per SIMD (the register budget is then 168
// VGPRs; the learned variant spills a few to scratch and still runs faster
// than with 8 waves), for both samplers.
constexpr int kF32Threads = 768;
// The compacting variant (below) keeps a sample queue per wave in LDS (52 B
// per entry) next to the accumulators and reads f from the global node quads.
constexpr int kQueueWaves = 12;
constexpr int kQueueLen = 128;  // ring entries per wave (>= 63 pending + 64 new)
constexpr int f32_block(bool queue) { return queue ? kQueueWaves * 64 : kF32Threads; }
// Compacting and learned variants: observed nodes go to the waves of a
// workgroup in blocks of 4 consecutive nodes; a wave stages the direct sums
// of its block in LDS and adds them to the output with one atomic
// instruction over one 32-byte sector, instead of one single-lane atomic
// (counted as a whole sector) per node.  The other variants keep one node
// per wave in turn and one atomic per node: there the block order cost 5%
// (the three-slot variant's sample loop compiled to more instructions).
constexpr int kNodeBlock = 4;

// kQueue (uniform sampler, every deposit slot in LDS, f from the global node
// quads): each wave first runs the sample geometry for 64 samples, appends
// the accepted ones (the three 23-bit uniforms of p2, p3 in FP64, s, t, u and
// the prefactor in FP32) to its ring in LDS, and evaluates |M|^2, f, bracket
// and deposits 64 queued samples at a time, so that long path runs on full
// wavefronts.  The deposits of one such batch are issued while the geometry
// of the next 64 samples runs, a third before, between and after it, so the
// LDS works off the atomics behind VALU work.  Same arithmetic per sample as
// the direct loop.
// kUser: some row of the matrix-element table is replaced by user terms; the
// variants without them carry no code for the user-term evaluation (which
// otherwise holds registers across the sample loop: 6% of the 7-species term).
template <bool kSym, bool kScale, bool kAllLds, bool kLearned, bool kQueue, bool kUser>
__global__ __launch_bounds__(f32_block(kQueue)) void collide_f32_kernel(CollideArgs A) {
  static_assert(!kQueue || (kSym && kAllLds && !kLearned), "the queue serves the uniform sampler, slots in LDS");
  // kAllLds: every f tile and accumulator in LDS (the queue variant: every
  // accumulator; f from the quads)
  constexpr bool kTilesLds = kAllLds && !kQueue;
  constexpr bool kAccLds = kAllLds;
  extern __shared__ double lds[];
  __shared__ float mix_rows[kLearned ? kF32Threads / kWave : 1][kLearned ? kMixRow : 1];
  __shared__ uint32_t q_v[kQueue ? kQueueWaves : 1][3][kQueue ? kQueueLen : 1];  // 23-bit uniforms of p2
  __shared__ double q_p3[kQueue ? kQueueWaves : 1][3][kQueue ? kQueueLen : 1];
  __shared__ float q_f[kQueue ? kQueueWaves : 1][4][kQueue ? kQueueLen : 1];    // s, t, u, prefactor
  __shared__ double mc_wg[2];  // this workgroup's item variances and squared item sums
  __shared__ unsigned long long ok_wg;  // and its accepted samples
  constexpr int kNB = kQueue || kLearned ? kNodeBlock : 1;  // nodes per block (as collide_f32_node_block)
  __shared__ double d_stage[kNB > 1 ? kF32Threads / kWave : 1][kNB];  // direct sums of a wave's current block
  static_assert(f32_block(kQueue) % (kWave * kNB) == 0, "a multiple of the waves is one of the block");
  const Grid& G = A.G;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int lb = xcd_local_block(blockIdx.x, gridDim.x);
  const int chunk = lb % A.n_chunks;
  // Uniform sampler: the chunks and channels of one cell follow each other
  // (they share its f quads and output rows in the XCD's L2).  Learned
  // sampler: blocks of 32 cells (the workgroups one XCD holds at a time),
  // and within a block the cells of one channel follow each other, so the
  // channel's proposal rows, shared by all cells, are read from HBM about
  // once per block instead of once per cell, and the block's f rows serve
  // every channel.
  int gi, cell;
  if (kLearned) {
    constexpr int kCellBlock = 32;
    const int u = lb / A.n_chunks;
    const int per = A.n_group * kCellBlock;
    const int cb = u / per;
    const int S = min(kCellBlock, G.cells - cb * kCellBlock);  // the last block may be short
    const int r = u - cb * per;
    gi = r / S;
    cell = cb * kCellBlock + r % S;
  } else {
    gi = (lb / A.n_chunks) % A.n_group;
    cell = lb / (A.n_chunks * A.n_group);
  }
  const int ci = A.group[gi];
  const Channel ch = A.chans[ci];
  const int nslot = ch.nslot;
  const int nodes = G.nodes;
  const int n_acc = kSym ? min(A.slot_hi - A.slot_lo, A.lds_acc) : 0;
  const int n_tiles = min(nslot, A.lds_tiles);
  const int win_lo = A.win_lo, win_n = A.win_n;
  double* acc = lds;                                          // [n_acc][win_n], slots slot_lo..
  float* tiles = reinterpret_cast<float*>(lds + (size_t)n_acc * win_n);  // [n_tiles][nodes]
  size_t goff[3];  // offsets of the slots' (species, cell) rows in f32 and A
  for (int k = 0; k < 3; ++k) {
    const int sp = k < nslot ? ch.slot_sp[k] : ch.slot_sp[0];
    goff[k] = ((size_t)sp * G.cells + cell) * nodes;
  }
  for (int i = threadIdx.x; i < n_acc * win_n; i += blockDim.x) acc[i] = 0.0;
  if (threadIdx.x < 2) mc_wg[threadIdx.x] = 0.0;
  if (threadIdx.x == 0) ok_wg = 0ull;
  if (kNB > 1 && lane < kNB) d_stage[wid][lane] = 0.0;
  for (int k = 0; k < n_tiles; ++k)
    for (int i = threadIdx.x; i < nodes; i += blockDim.x) tiles[k * nodes + i] = A.f32[goff[k] + i];
  __syncthreads();
  const int k2 = ch.pos_slot[0], k3 = ch.pos_slot[1], k4 = ch.pos_slot[2];
  // row offsets of positions 2, 3, 4 (scalars: no dynamically indexed array in the loop)
  const size_t off2 = goff[k2], off3 = goff[k3], off4 = goff[k4];
  const bool g1 = is_gluon(ch.sp[0]), g2 = is_gluon(ch.sp[1]);
  const bool g3 = is_gluon(ch.sp[2]), g4 = is_gluon(ch.sp[3]);
  const int first = chunk * A.chunk_items;
  const int last = min(first + A.chunk_items, nodes);
  // Learned sampler (short items): the (cell, channel) constants once per
  // workgroup.  The uniform sampler's long items recompute them per item:
  // held across its item loop they cost more spilled registers in the
  // sample loop than they save.
  Item pair;
  if (kLearned) item_pair(pair, A, ch, cell);
  // After the item at node p, the last of its node block (or of the chunk):
  // the wave adds the block's staged direct sums to the output, the lanes of
  // one atomic instruction covering consecutive nodes.
  auto flush_block = [&](int p) {
    if (kNB == 1 || !A.direct || ((p & (kNB - 1)) != kNB - 1 && p + 1 < last)) return;
    wave_lds_sync();
    if (lane < kNB) {
      const double d = d_stage[wid][lane];
      if (d != 0.0) atomicAdd(A.A + ((size_t)ch.sp[0] * G.cells + cell) * nodes + (p & ~(kNB - 1)) + lane, d);
      d_stage[wid][lane] = 0.0;
    }
    wave_lds_sync();
  };
  // Wave w takes the node blocks w, w + nw, w + 2 nw, ... of the chunk (the
  // chunk starts on a block boundary), the nodes of a block in turn.
  for (int p1_lin = first + kNB * wid; p1_lin < last; p1_lin += (p1_lin & (kNB - 1)) == kNB - 1 ? kNB * (nw - 1) + 1 : 1) {
    Item it;
    if (kLearned) {
      it = pair;
      item_node(it, A, ch, p1_lin);
    } else {
      load_item(it, A, ch, cell, p1_lin);
    }
    if (!(it.E1 > 0.0)) {  // massless p = 0 node: zero measure
      if (lane == 0 && A.items && A.direct) A.items[((size_t)cell * A.n_channels + ci) * nodes + p1_lin] = 0.0;
      flush_block(p1_lin);
      continue;
    }
    const float f1 = (float)it.f1;
    const float F1 = g1 ? 1.0f + f1 : 1.0f - f1;
    double dsum = 0.0, ssum = 0.0, dsq = 0.0;
    int n_ok = 0;
    const size_t mrow = (size_t)ci * nodes + p1_lin;
    const bool mix = kLearned && (!A.mix_on || A.mix_on[ci]);
    if (mix) {
      mix_prepare_f32(A.mix_thr + mrow * A.mix_K, A.mix_mu + mrow * A.mix_K * 5, A.mix_sigma + mrow * A.mix_K * 5,
                      A.mix_K, mix_rows[wid], lane);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // Queue mode: the deposits of the last evaluated batch, issued while the
    // next samples' geometry runs (lanes without a sample in a partial batch
    // deposit zeros).
    Stencil<float> pd2{}, pd3{}, pd4{};
    float pdv = 0.0f;
    bool pending = false;
    // Integrand, direct sum and deposits of an accepted sample (wnb = value
    // without the bracket).
    auto finish = [&](const Geo& g, float wnb) {
      ++n_ok;
      const Stencil<float> s2 = make_stencil<float>(g.p2, G);
      const Stencil<float> s3 = make_stencil<float>(g.p3, G);
      const Stencil<float> s4 = make_stencil<float>(g.p4, G);
      const float f2 = interp_slot<kTilesLds, float>(k2, n_tiles, tiles, A.f32q, off2, s2, nodes, G.ox, G.oy);
      const float f3 = interp_slot<kTilesLds, float>(k3, n_tiles, tiles, A.f32q, off3, s3, nodes, G.ox, G.oy);
      const float f4 = interp_slot<kTilesLds, float>(k4, n_tiles, tiles, A.f32q, off4, s4, nodes, G.ox, G.oy);
      const float F2 = g2 ? 1.0f + f2 : 1.0f - f2;
      const float F3 = g3 ? 1.0f + f3 : 1.0f - f3;
      const float F4 = g4 ? 1.0f + f4 : 1.0f - f4;
      const float gain = f3 * f4 * F1 * F2, loss = f1 * f2 * F3 * F4;
      const float v = wnb * (gain - loss);
      dsum += (double)v;
      dsq = fma((double)v, (double)v, dsq);
      if (kScale) ssum += (double)(fabsf(wnb) * (gain + loss));
      if (kSym) {
        if (kQueue) {
          pd2 = s2; pd3 = s3; pd4 = s4; pdv = v;
        } else {
          deposit_slot<kAccLds>(k2, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off2, s2, v,
                                nodes, G.ox, G.oy, win_lo, win_n);
          deposit_slot<kAccLds>(k3, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off3, s3, -v,
                                nodes, G.ox, G.oy, win_lo, win_n);
          deposit_slot<kAccLds>(k4, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off4, s4, -v,
                                nodes, G.ox, G.oy, win_lo, win_n);
        }
        if (kScale && A.direct) {
          const float vs = fabsf(wnb) * (gain + loss);
          deposit<double, double>(A.scale + ((size_t)ch.sp[1] * G.cells + cell) * nodes, widen(s2), (double)vs, G.ox, G.oy);
          deposit<double, double>(A.scale + ((size_t)ch.sp[2] * G.cells + cell) * nodes, widen(s3), (double)vs, G.ox, G.oy);
          deposit<double, double>(A.scale + ((size_t)ch.sp[3] * G.cells + cell) * nodes, widen(s4), (double)vs, G.ox, G.oy);
        }
      }
    };
    auto evaluate = [&](const double u[5], float inv_q) {
      Geo g;
      if (!geometry(it, G, u, g)) return;
      finish(g, weight_no_bracket<float, kUser>(A, it, g, ch.row) * inv_q);
    };
    if (kQueue) {
      // queued record -> the accepted sample's geometry, as geometry() left it
      auto finish_queued = [&](int slot) {
        Geo g;
        const uint32_t v0 = q_v[wid][0][slot], v1 = q_v[wid][1][slot], v2 = q_v[wid][2][slot];
        const double uu[3] = {unif23(v0), unif23(v1), unif23(v2)};
        for (int a = 0; a < 3; ++a) {
          g.p2[a] = fma(2.0 * G.ph[a], uu[a], -G.ph[a]);
          g.p3[a] = q_p3[wid][a][slot];
          g.p4[a] = (it.p1[a] + g.p2[a]) - g.p3[a];
        }
        const float m = msq_row<float, kUser>(A.msq_mask, A.msq, ch.row, q_f[wid][0][slot], q_f[wid][1][slot],
                                       q_f[wid][2][slot], (float)it.mu);
        finish(g, m * q_f[wid][3][slot]);
      };
      unsigned head = 0, tail = 0;  // ring positions (wave-uniform)
      for (int base = 0; base < A.n_samples; base += kWave) {
        const int s = base + lane;
        uint32_t x0 = (uint32_t)s, x1 = (uint32_t)p1_lin, x2 = (uint32_t)cell, x3 = ((uint32_t)ch.code << 8);
        philox4x32_10(x0, x1, x2, x3, A.key0, A.key1);
        if (pending) deposit_slot<true, false>(k2, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off2, pd2, pdv,
                                        nodes, G.ox, G.oy, win_lo, win_n);
        double u[5];
        five_uniforms(x0, x1, x2, x3, u);
        Geo g;
        const bool ok = s < A.n_samples && geometry(it, G, u, g);
        if (pending) deposit_slot<true, false>(k3, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off3, pd3, -pdv,
                                        nodes, G.ox, G.oy, win_lo, win_n);
        const unsigned long long mask = __ballot(ok);
        if (ok) {
          const unsigned slot = (tail + (unsigned)__popcll(mask & ((1ull << lane) - 1ull))) & (kQueueLen - 1);
          q_v[wid][0][slot] = x0 >> 9;
          q_v[wid][1][slot] = x1 >> 9;
          q_v[wid][2][slot] = x2 >> 9;
          for (int a = 0; a < 3; ++a) q_p3[wid][a][slot] = g.p3[a];
          q_f[wid][0][slot] = (float)g.s;
          q_f[wid][1][slot] = (float)g.t;
          q_f[wid][2][slot] = (float)g.u;
          q_f[wid][3][slot] = prefactor<float>(it, g);
        }
        if (pending) deposit_slot<true, false>(k4, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off4, pd4, -pdv,
                                        nodes, G.ox, G.oy, win_lo, win_n);
        pending = false;
        tail += (unsigned)__popcll(mask);
        if (tail - head >= (unsigned)kWave) {
          wave_lds_sync();
          pdv = 0.0f;
          finish_queued((head + lane) & (kQueueLen - 1));
          pending = true;
          head += kWave;
          wave_lds_sync();
        }
      }
      auto flush = [&]() {
        deposit_slot<true, false>(k2, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off2, pd2, pdv,
                           nodes, G.ox, G.oy, win_lo, win_n);
        deposit_slot<true, false>(k3, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off3, pd3, -pdv,
                           nodes, G.ox, G.oy, win_lo, win_n);
        deposit_slot<true, false>(k4, A.slot_lo, A.slot_hi, n_acc, acc, A.A, off4, pd4, -pdv,
                           nodes, G.ox, G.oy, win_lo, win_n);
      };
      if (pending) flush();  // the last full batch
      if (tail != head) {    // the last, partial batch
        wave_lds_sync();
        pdv = 0.0f;
        if ((unsigned)lane < tail - head) finish_queued((head + lane) & (kQueueLen - 1));
        flush();
        wave_lds_sync();
      }
      pending = false;
    } else
    for (int s = lane; s < A.n_samples; s += kWave) {
      uint32_t x0 = (uint32_t)s, x1 = (uint32_t)p1_lin, x2 = (uint32_t)cell, x3 = ((uint32_t)ch.code << 8);
      philox4x32_10(x0, x1, x2, x3, A.key0, A.key1);
      double u[5];
      float inv_q = 1.0f;
      if (mix) {
        uint32_t y0 = (uint32_t)s, y1 = (uint32_t)p1_lin, y2 = (uint32_t)cell, y3 = ((uint32_t)ch.code << 8) | 1u;
        philox4x32_10(y0, y1, y2, y3, A.key0, A.key1);
        const uint32_t xw[8] = {x0, x1, x2, x3, y0, y1, y2, y3};
        float yl[5];
        mix_draw_row(xw, A.mix_thr + mrow * A.mix_K, mix_rows[wid], A.mix_K, u, yl);
        inv_q = __builtin_amdgcn_rcpf(mix_density_f32(mix_rows[wid], A.mix_K, yl));  // about 1 ulp; q >= alpha
      } else {
        five_uniforms(x0, x1, x2, x3, u);
      }
      evaluate(u, inv_q);
    }
    if (!A.direct) continue;
    int ok_total;
    if (kLearned) {  // short items (few hundred samples): DPP sums, no LDS round trips
      dsum = wave_sum_dpp(dsum);
      if (kScale) ssum = wave_sum_dpp(ssum);
      dsq = wave_sum_dpp(dsq);
      ok_total = wave_count_dpp(n_ok);
    } else {
      dsum = wave_sum(dsum);
      if (kScale) ssum = wave_sum(ssum);
      dsq = wave_sum(dsq);
      ok_total = wave_count(n_ok);
    }
    if (lane == 0) {
      __hip_atomic_fetch_add(&ok_wg, (unsigned long long)ok_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(&mc_wg[0], item_variance(dsum, dsq, A.n_samples), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_fetch_add(&mc_wg[1], dsum * dsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (kNB > 1)
        d_stage[wid][p1_lin & (kNB - 1)] = dsum;
      else
        atomicAdd(A.A + ((size_t)ch.sp[0] * G.cells + cell) * nodes + p1_lin, dsum);
      if (kScale) atomicAdd(A.scale + ((size_t)ch.sp[0] * G.cells + cell) * nodes + p1_lin, ssum);
      if (A.items) A.items[((size_t)cell * A.n_channels + ci) * nodes + p1_lin] = dsum;
    }
    flush_block(p1_lin);
  }
  __syncthreads();
  const int stripe = blockIdx.x % kStripes;
  if (threadIdx.x < 2 && A.mc_acc && A.direct) atomicAdd(&A.mc_acc[2 * stripe + threadIdx.x], mc_wg[threadIdx.x]);
  if (threadIdx.x == 0 && A.n_accepted && A.direct) atomicAdd(A.n_accepted + stripe, ok_wg);
  if (threadIdx.x == 0 && A.chan_var && A.direct)  // one channel per workgroup
    atomicAdd(&A.chan_var[(size_t)stripe * A.n_channels + ci], mc_wg[0]);
  if (n_acc > 0) {
    for (int i = threadIdx.x; i < n_acc * win_n; i += blockDim.x) {
      const double v = acc[i];
      if (v != 0.0) {
        const int j = i / win_n;
        atomicAdd(A.A + goff[A.slot_lo + j] + win_lo + (i - j * win_n), v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Training data for the proposal: for every item_stride-th work item
// (cell, channel, node; node fastest), n_per_item uniform samples are drawn
// exactly as the uniform sampler draws them and recorded as rows
// [x (8 features), y = logit(u) (5), |value|].  FP64 evaluation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void record_kernel(CollideArgs A, int n_per_item, long long item_stride,
                                                     long long n_sel, float* __restrict__ rows) {
  const Grid& G = A.G;
  const long long total = n_sel * n_per_item;
  const double pn = sqrt(G.ph[0] * G.ph[0] + G.ph[1] * G.ph[1] + G.ph[2] * G.ph[2]);
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < total;
       r += (long long)gridDim.x * blockDim.x) {
    const long long j = r / n_per_item;
    const int s = (int)(r % n_per_item);
    const long long w = j * item_stride;
    const int p1_lin = (int)(w % G.nodes);
    const int ci = (int)((w / G.nodes) % A.n_channels);
    const int cell = (int)(w / ((long long)G.nodes * A.n_channels));
    const Channel ch = A.chans[ci];
    Item it;
    load_item(it, A, ch, cell, p1_lin);
    float* out = rows + (size_t)r * 14;
    const double a = sqrt(it.p1[0] * it.p1[0] + it.p1[1] * it.p1[1] + it.p1[2] * it.p1[2]);
    out[0] = (float)(it.p1[0] / G.ph[0]);
    out[1] = (float)(it.p1[1] / G.ph[1]);
    out[2] = (float)(it.p1[2] / G.ph[2]);
    out[3] = (float)(a / pn);
    out[4] = (float)(it.E1 / pn);
    out[5] = (float)(it.mu / (pn * pn));
    out[6] = (float)(ch.sp[0] / 3.0 - 1.0);
    out[7] = A.n_channels > 1 ? (float)(2.0 * ci / (A.n_channels - 1) - 1.0) : 0.0f;
    uint32_t x0 = (uint32_t)s, x1 = (uint32_t)p1_lin, x2 = (uint32_t)cell, x3 = ((uint32_t)ch.code << 8);
    philox4x32_10(x0, x1, x2, x3, A.key0, A.key1);
    double u[5];
    five_uniforms(x0, x1, x2, x3, u);
    for (int d = 0; d < 5; ++d) out[8 + d] = (float)log(u[d] / (1.0 - u[d]));
    double v = 0.0;
    Geo g;
    if (it.E1 > 0.0 && geometry(it, G, u, g)) {
      const double wnb = weight_no_bracket<double>(A, it, g, ch.row);
      const Stencil<double> s2 = make_stencil<double>(g.p2, G);
      const Stencil<double> s3 = make_stencil<double>(g.p3, G);
      const Stencil<double> s4 = make_stencil<double>(g.p4, G);
      const double* f = A.f64;
      const double f2 = interpolate<double>(f + ((size_t)ch.sp[1] * G.cells + cell) * G.nodes, s2, G.ox, G.oy);
      const double f3 = interpolate<double>(f + ((size_t)ch.sp[2] * G.cells + cell) * G.nodes, s3, G.ox, G.oy);
      const double f4 = interpolate<double>(f + ((size_t)ch.sp[3] * G.cells + cell) * G.nodes, s4, G.ox, G.oy);
      const double F1 = is_gluon(ch.sp[0]) ? 1.0 + it.f1 : 1.0 - it.f1;
      const double F2 = is_gluon(ch.sp[1]) ? 1.0 + f2 : 1.0 - f2;
      const double F3 = is_gluon(ch.sp[2]) ? 1.0 + f3 : 1.0 - f3;
      const double F4 = is_gluon(ch.sp[3]) ? 1.0 + f4 : 1.0 - f4;
      v = wnb * (f3 * f4 * F1 * F2 - it.f1 * f2 * F3 * F4);
    }
    out[13] = (float)fabs(v);
  }
}

hipError_t launch_record(const CollideArgs& a, int n_per_item, long long item_stride, long long n_sel, float* rows,
                         hipStream_t stream) {
  const long long total = n_sel * n_per_item;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(record_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a, n_per_item, item_stride, n_sel,
                     rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_collide_roots(const CollideArgs& a, bool alt, hipStream_t stream) {
  const long long items = (long long)a.G.cells * a.n_group * a.G.nodes;
  const int threads = kRootWaves * kWave;  // the per-wavefront queues are sized for this
  long long blocks = (items * kWave + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;  // 16 waves per CU; the rest by the grid-stride loop
  if (blocks < 1) blocks = 1;
  // a whole output that fits in 64 KB of dynamic LDS: workgroup-private deposits
  const size_t priv_b = (size_t)kSpecies * a.G.cells * a.G.nodes * sizeof(double);
  const bool priv = a.symmetric && priv_b <= 65536;
  const dim3 grid((unsigned)blocks), block(threads);
  if (priv) {
    if (alt) hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_roots_kernel<true, true>), grid, block, priv_b, stream, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_roots_kernel<false, true>), grid, block, priv_b, stream, a);
  } else {
    if (alt) hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_roots_kernel<true, false>), grid, block, 0, stream, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_roots_kernel<false, false>), grid, block, 0, stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_collide_f64(const CollideArgs& a, hipStream_t stream) {
  const long long items = (long long)a.G.cells * a.n_group * a.G.nodes;
  const int threads = 256;
  long long blocks = (items * kWave + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;  // 16 waves per CU; the rest by the grid-stride loop
  if (blocks < 1) blocks = 1;
  // a whole output that fits in the default dynamic LDS: workgroup-private deposits
  const size_t priv_b = (size_t)kSpecies * a.G.cells * a.G.nodes * sizeof(double);
  const bool priv = a.symmetric && priv_b <= 65536;
  const dim3 grid((unsigned)blocks), block(threads);
  if (priv) {
    if (a.learned) hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_f64_kernel<true, true>), grid, block, priv_b, stream, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_f64_kernel<false, true>), grid, block, priv_b, stream, a);
  } else {
    if (a.learned) hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_f64_kernel<true, false>), grid, block, 0, stream, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(collide_f64_kernel<false, false>), grid, block, 0, stream, a);
  }
  return hipGetLastError();
}

template <bool kSym, bool kScale, bool kAllLds, bool kLearned, bool kQueue>
void launch_f32_user(const CollideArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  if (a.msq_mask)
    hipLaunchKernelGGL((collide_f32_kernel<kSym, kScale, kAllLds, kLearned, kQueue, true>), grid, block, lds, st, a);
  else
    hipLaunchKernelGGL((collide_f32_kernel<kSym, kScale, kAllLds, kLearned, kQueue, false>), grid, block, lds, st, a);
}

template <bool kSym, bool kScale, bool kLearned>
void launch_f32_variant(const CollideArgs& a, bool all_lds, bool queue, dim3 grid, dim3 block, size_t lds,
                        hipStream_t st) {
  if constexpr (kSym && !kLearned) {
    if (queue) {
      launch_f32_user<true, kScale, true, false, true>(a, grid, block, lds, st);
      return;
    }
  }
  if (all_lds) launch_f32_user<kSym, kScale, true, kLearned, false>(a, grid, block, lds, st);
  else launch_f32_user<kSym, kScale, false, kLearned, false>(a, grid, block, lds, st);
}

template <bool kSym, bool kScale>
void launch_f32_sampler(const CollideArgs& a, bool all_lds, bool queue, dim3 grid, dim3 block, size_t lds,
                        hipStream_t st) {
  if (a.learned) launch_f32_variant<kSym, kScale, true>(a, all_lds, false, grid, block, lds, st);
  else launch_f32_variant<kSym, kScale, false>(a, all_lds, queue, grid, block, lds, st);
}

int collide_f32_waves(bool queue) { return f32_block(queue) / kWave; }
int collide_f32_node_block(bool queue, bool learned) { return queue || learned ? kNodeBlock : 1; }

hipError_t launch_collide_f32(const CollideArgs& a, int nslot, bool queue, hipStream_t stream) {
  const int n_acc = a.symmetric ? std::min(a.slot_hi - a.slot_lo, a.lds_acc) : 0;
  const int n_tiles = std::min(nslot, a.lds_tiles);
  // every tile and every accumulator of this launch's slots in LDS: the
  // variant without global-memory paths
  const bool all_acc = !a.symmetric || n_acc == a.slot_hi - a.slot_lo;
  const bool all_lds = n_tiles == nslot && all_acc;
  queue = queue && all_acc && a.symmetric && !a.learned && a.win_n == a.G.nodes;
  const int threads = f32_block(queue);
  const size_t lds = (size_t)n_acc * a.win_n * sizeof(double) + (size_t)n_tiles * a.G.nodes * sizeof(float);
  const long long blocks = (long long)a.G.cells * a.n_group * a.n_chunks;
  if (blocks <= 0) return hipSuccess;
  if (a.chunk_items % kNodeBlock != 0) return hipErrorInvalidValue;  // chunks start on node blocks
  const dim3 grid((unsigned)blocks), block(threads);
  if (a.symmetric) {
    if (a.scale) launch_f32_sampler<true, true>(a, all_lds, queue, grid, block, lds, stream);
    else launch_f32_sampler<true, false>(a, all_lds, queue, grid, block, lds, stream);
  } else {
    if (a.scale) launch_f32_sampler<false, true>(a, all_lds, false, grid, block, lds, stream);
    else launch_f32_sampler<false, false>(a, all_lds, false, grid, block, lds, stream);
  }
  return hipGetLastError();
}

hipError_t set_collide_lds_limit(size_t lds_max, size_t* budget_plain, size_t* budget_learned, size_t* budget_queue) {
  // Each FP32 variant may use what its static LDS leaves of lds_max.  Raising
  // the per-kernel dynamic limit is only needed (and only accepted) above the
  // runtime's default; after a refusal the budget is the limit in force.
  // Groups: 0 uniform sampler, 1 learned sampler, 2 the compacting variant.
  struct Fn { const void* fn; int group; };
#define QGBE_F32_PAIR(S, Sc, L, Le, Q, G) \
  {(const void*)collide_f32_kernel<S, Sc, L, Le, Q, false>, G}, {(const void*)collide_f32_kernel<S, Sc, L, Le, Q, true>, G}
  const Fn fns[36] = {
      QGBE_F32_PAIR(true, true, true, false, false, 0),   QGBE_F32_PAIR(true, false, true, false, false, 0),
      QGBE_F32_PAIR(false, true, true, false, false, 0),  QGBE_F32_PAIR(false, false, true, false, false, 0),
      QGBE_F32_PAIR(true, true, false, false, false, 0),  QGBE_F32_PAIR(true, false, false, false, false, 0),
      QGBE_F32_PAIR(false, true, false, false, false, 0), QGBE_F32_PAIR(false, false, false, false, false, 0),
      QGBE_F32_PAIR(true, true, true, true, false, 1),    QGBE_F32_PAIR(true, false, true, true, false, 1),
      QGBE_F32_PAIR(false, true, true, true, false, 1),   QGBE_F32_PAIR(false, false, true, true, false, 1),
      QGBE_F32_PAIR(true, true, false, true, false, 1),   QGBE_F32_PAIR(true, false, false, true, false, 1),
      QGBE_F32_PAIR(false, true, false, true, false, 1),  QGBE_F32_PAIR(false, false, false, true, false, 1),
      QGBE_F32_PAIR(true, true, true, false, true, 2),    QGBE_F32_PAIR(true, false, true, false, true, 2)};
#undef QGBE_F32_PAIR
  size_t budget[3] = {lds_max, lds_max, lds_max};
  for (const Fn& f : fns) {
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, f.fn) != hipSuccess) return hipGetLastError();
    const size_t stat = attr.sharedSizeBytes;
    size_t want = lds_max > stat ? lds_max - stat : 0;
    size_t have = attr.maxDynamicSharedSizeBytes > 0 ? (size_t)attr.maxDynamicSharedSizeBytes : 0;
    if (have < want) {
      if (hipFuncSetAttribute(f.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) == hipSuccess)
        have = want;
      else
        (void)hipGetLastError();
    }
    budget[f.group] = std::min(budget[f.group], std::min(have, want));
  }
  *budget_plain = budget[0];
  *budget_learned = budget[1];
  *budget_queue = budget[2];
  return hipSuccess;
}

}  // namespace qgbe
