// Field kernels around the collision term: thermal masses (Eq. mg, Eq. mq),
// the drift of Eq. left handside with the forward-Euler update (Sec. III),
// and the FP64 bookkeeping (Eq. particle numbers, Eq. energy momentum tensor).
// All of them are HBM-bound stencils or reductions in FP64.
#include <hip/hip_runtime.h>

#include "field.h"

namespace qgbe {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void node_p(const Grid& G, int node, double p[3]) {
  const int iz = node % G.np[2];
  const int iy = (node / G.np[2]) % G.np[1];
  const int ix = node / (G.np[2] * G.np[1]);
  p[0] = node_coord(G.ph[0], G.dp[0], ix);
  p[1] = node_coord(G.ph[1], G.dp[1], iy);
  p[2] = node_coord(G.ph[2], G.dp[2], iz);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) t += sh[i];
  return t;  // valid in thread 0
}

// I_Y = sum_p dV/(2pi)^3 f_Y / (2 E_Y) per cell, E_Y from the lagged masses
// (or |p| when there are none; a node at p = 0 then adds 0).  Stage 1: block
// (cell, chunk) sums kMassChunk nodes of every species; stage 2: one block
// per cell adds its chunks in a fixed order (deterministic) and applies
// Eq. mg / mq.
constexpr int kMassChunk = 256;  // nodes per block: a single cell of 30^3 nodes still fills 100+ CUs

__host__ __device__ inline int mass_chunks(const Grid& G) { return (G.nodes + kMassChunk - 1) / kMassChunk; }

__global__ __launch_bounds__(kBlock) void mass_partial(Grid G, const double* __restrict__ f,
                                                       const double* __restrict__ lag, double* part) {
  __shared__ double sh[kBlock / 64];
  const int chunks = mass_chunks(G);
  const int chunk = blockIdx.x % chunks, cell = blockIdx.x / chunks;
  const int lo = chunk * kMassChunk, hi = min(G.nodes, lo + kMassChunk);
  for (int sp = 0; sp < kSpecies; ++sp) {
    const double m2 = lag ? lag[sp * G.cells + cell] : 0.0;
    const double* fc = f + ((size_t)sp * G.cells + cell) * G.nodes;
    double acc = 0.0;
    for (int node = lo + threadIdx.x; node < hi; node += blockDim.x) {
      double p[3];
      node_p(G, node, p);
      const double E = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + m2);
      if (E > 0.0) acc += fc[node] / (2.0 * E);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[((size_t)cell * chunks + chunk) * kSpecies + sp] = t;
  }
}

__global__ __launch_bounds__(kBlock) void mass_final(Grid G, const double* __restrict__ part, int chunks,
                                                     double* mass2) {
  __shared__ double sh[kBlock / 64];
  const int cell = blockIdx.x;  // one block per cell; its threads stride over the chunks
  const double meas = G.dp[0] * G.dp[1] * G.dp[2] / (8.0 * kPi * kPi * kPi);
  double I[kSpecies];
  for (int sp = 0; sp < kSpecies; ++sp) {
    double t = 0.0;
    for (int c = threadIdx.x; c < chunks; c += blockDim.x) t += part[((size_t)cell * chunks + c) * kSpecies + sp];
    I[sp] = block_sum(t, sh) * meas;  // fixed order: deterministic
  }
  if (threadIdx.x != 0) return;
  // SU(3): dA = 8, CA = 3, CF = 4/3; N_g = 16, N_q = 6
  const double CF = 4.0 / 3.0;
  double q = 0.0;
  for (int i = 0; i < 3; ++i) q += 6.0 * CF * (I[i] + I[i + 3]);
  mass2[kGluon * G.cells + cell] = (2.0 * G.g2 / 8.0) * (16.0 * 3.0 * I[kGluon] + q);
  for (int i = 0; i < 3; ++i) {
    const double mq = 2.0 * CF * G.g2 * (2.0 * I[kGluon] + I[i] + I[i + 3]);
    mass2[i * G.cells + cell] = mq;
    mass2[(i + 3) * G.cells + cell] = mq;
  }
}

__global__ void const_mass_kernel(Grid G, Mass7 m, double* mass2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kSpecies * G.cells) mass2[i] = m.v[i / G.cells];
}

__device__ __forceinline__ int shift_cell(const Grid& G, int cell, int axis, int d) {
  int id[3] = {cell / (G.nx[1] * G.nx[2]), (cell / G.nx[2]) % G.nx[1], cell % G.nx[2]};
  id[axis] = (id[axis] + d + G.nx[axis]) % G.nx[axis];
  return (id[0] * G.nx[1] + id[1]) * G.nx[2] + id[2];
}

__device__ __forceinline__ int shift_node(const Grid& G, int node, int axis, int d) {
  int id[3] = {node / (G.np[1] * G.np[2]), (node / G.np[2]) % G.np[1], node % G.np[2]};
  id[axis] = (id[axis] + d + G.np[axis]) % G.np[axis];
  return (id[0] * G.np[1] + id[1]) * G.np[2] + id[2];
}

__device__ __forceinline__ double energy(const Grid& G, const double* mass2, int sp, int cell, int node) {
  double p[3];
  node_p(G, node, p);
  return sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + mass2[sp * G.cells + cell]);
}

__device__ __forceinline__ double upwind(double vel, double f_left, double f_right) {
  return vel > 0.0 ? vel * f_left : vel * f_right;
}

// D[f] at (sp, cell, node), flux form with periodic boundaries.
__device__ double drift_at(const Grid& G, const double* f, const double* mass2, int sp, int cell,
                           int node, int scheme) {
  const double* F = f + (size_t)sp * G.cells * G.nodes;
  double p[3];
  node_p(G, node, p);
  double D = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (G.nx[a] == 1) continue;  // a single periodic cell has no gradient
    const int xp = shift_cell(G, cell, a, +1), xm = shift_cell(G, cell, a, -1);
    const int pp = shift_node(G, node, a, +1), pm = shift_node(G, node, a, -1);
    const double Ec = energy(G, mass2, sp, cell, node);
    const double Exp = energy(G, mass2, sp, xp, node), Exm = energy(G, mass2, sp, xm, node);
    const double inv2dx = 0.5 / G.dx[a];
    if (scheme == 0) {
      const double vc = p[a] / Ec, vp = p[a] / Exp, vm = p[a] / Exm;
      const double fR = upwind(0.5 * (vc + vp), F[(size_t)cell * G.nodes + node], F[(size_t)xp * G.nodes + node]);
      const double fL = upwind(0.5 * (vm + vc), F[(size_t)xm * G.nodes + node], F[(size_t)cell * G.nodes + node]);
      D += (fR - fL) / G.dx[a];
      // p-advection with the force -dE/dx_a (central in x)
      const double Fc = -(Exp - Exm) * inv2dx;
      const double Fp = -(energy(G, mass2, sp, xp, pp) - energy(G, mass2, sp, xm, pp)) * inv2dx;
      const double Fm = -(energy(G, mass2, sp, xp, pm) - energy(G, mass2, sp, xm, pm)) * inv2dx;
      const double gR = upwind(0.5 * (Fc + Fp), F[(size_t)cell * G.nodes + node], F[(size_t)cell * G.nodes + pp]);
      const double gL = upwind(0.5 * (Fm + Fc), F[(size_t)cell * G.nodes + pm], F[(size_t)cell * G.nodes + node]);
      D += (gR - gL) / G.dp[a];
    } else {
      D += (p[a] * F[(size_t)xp * G.nodes + node] / Exp - p[a] * F[(size_t)xm * G.nodes + node] / Exm) * inv2dx;
      const double dEp = (energy(G, mass2, sp, xp, pp) - energy(G, mass2, sp, xm, pp)) * inv2dx;
      const double dEm = (energy(G, mass2, sp, xp, pm) - energy(G, mass2, sp, xm, pm)) * inv2dx;
      D -= (F[(size_t)cell * G.nodes + pp] * dEp - F[(size_t)cell * G.nodes + pm] * dEm) * (0.5 / G.dp[a]);
    }
  }
  return D;
}

// The evolving species, in order (the update touches only these; the frozen
// species hold the same values in both buffers of f, set together).
struct Evolving {
  int n;
  int sp[kSpecies];
};

// f_out = f + dt (A / (N_Y hbar c) - D[f]) for the evolving species.
__global__ __launch_bounds__(kBlock) void update_kernel(Grid G, Evolving ev, const double* __restrict__ f,
                                                        const double* __restrict__ A,
                                                        const double* __restrict__ mass2, double dt,
                                                        int scheme, double* __restrict__ f_out,
                                                        float* __restrict__ f32) {
  const size_t per = (size_t)G.cells * G.nodes;
  const size_t total = (size_t)ev.n * per;
  for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < total; j += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(j / per);
    const size_t rem = j - (size_t)k * per;
    const int sp = ev.sp[k];
    const size_t i = (size_t)sp * per + rem;
    const int cell = (int)(rem / G.nodes), node = (int)(rem % G.nodes);
    const double D = drift_at(G, f, mass2, sp, cell, node, scheme);
    const double v = f[i] + dt * (A[i] / (degeneracy(sp) * kHbarC) - D);
    f_out[i] = v;
    f32[i] = (float)v;
  }
}

// Observables: per species N, E, P (3), M = sum m^2 f / E (the mass term of
// the modified tensor), the entropy S = sum [(1 + s f) ln(1 + s f)/s - f ln f]
// (s = +1 for gluons, -1 for quarks; a node adds only while 0 < f and
// 1 + s f > 0) and the diagonal T^ii = sum p_i^2 f / E of Eq. energy momentum
// tensor, then min f and max fermion f, and a non-finite counter.  Stage 1:
// per-block partials; stage 2: one block.
constexpr int kObs = kSpecies * kObsPer;

__global__ __launch_bounds__(kBlock) void observables_partial(Grid G, const double* __restrict__ f,
                                                              const double* __restrict__ mass2,
                                                              double* partial) {
  __shared__ double sh[kBlock / 64];
  const size_t per = (size_t)G.cells * G.nodes;
  double minf = 1e300, maxq = -1e300, bad = 0.0;
  for (int sp = 0; sp < kSpecies; ++sp) {
    double N = 0.0, E = 0.0, P0 = 0.0, P1 = 0.0, P2 = 0.0, M = 0.0, S = 0.0, T0 = 0.0, T1 = 0.0, T2 = 0.0;
    const bool evolve = (G.species_mask >> sp) & 1u;
    const double sgn = sp == kGluon ? 1.0 : -1.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
      const int cell = (int)(i / G.nodes), node = (int)(i % G.nodes);
      const double fv = f[(size_t)sp * per + i];
      double p[3];
      node_p(G, node, p);
      const double m2 = mass2[sp * G.cells + cell];
      const double En = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + m2);
      N += fv;
      E += En * fv;
      if (En > 0.0) {
        const double w = fv / En;
        M += m2 * w;
        T0 += p[0] * p[0] * w;
        T1 += p[1] * p[1] * w;
        T2 += p[2] * p[2] * w;
      }
      const double one = 1.0 + sgn * fv;
      if (fv > 0.0 && one > 0.0) S += one * log(one) * sgn - fv * log(fv);
      P0 += p[0] * fv;
      P1 += p[1] * fv;
      P2 += p[2] * fv;
      if (evolve) {
        if (!isfinite(fv)) bad += 1.0;
        minf = fmin(minf, fv);
        if (sp != kGluon) maxq = fmax(maxq, fv);
      }
    }
    const double vals[kObsPer] = {N, E, P0, P1, P2, M, S, T0, T1, T2};
    for (int k = 0; k < kObsPer; ++k) {
      const double t = block_sum(vals[k], sh);
      if (threadIdx.x == 0) partial[(size_t)blockIdx.x * (kObs + 3) + sp * kObsPer + k] = t;
    }
  }
  // min / max over the block
  for (int off = 32; off > 0; off >>= 1) {
    minf = fmin(minf, __shfl_xor(minf, off, 64));
    maxq = fmax(maxq, __shfl_xor(maxq, off, 64));
  }
  const double nbad = block_sum(bad, sh);
  __shared__ double shmin[kBlock / 64], shmax[kBlock / 64];
  const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
  if (lane == 0) { shmin[w] = minf; shmax[w] = maxq; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x / 64); ++i) { minf = fmin(minf, shmin[i]); maxq = fmax(maxq, shmax[i]); }
    double* o = partial + (size_t)blockIdx.x * (kObs + 3);
    o[kObs] = minf;
    o[kObs + 1] = maxq;
    o[kObs + 2] = nbad;
  }
}

// Stage 2: one wave per value (min, max or sum over the block partials).
constexpr int kFinalThreads = 1024;

__global__ __launch_bounds__(kFinalThreads) void observables_final(Grid G, const double* partial, int nblocks,
                                                                   double* out) {
  const double meas = G.dx[0] * G.dx[1] * G.dx[2] * G.dp[0] * G.dp[1] * G.dp[2] / (8.0 * kPi * kPi * kPi);
  const int lane = threadIdx.x & 63, nw = blockDim.x / 64;
  for (int k = threadIdx.x / 64; k < kObs + 3; k += nw) {
    const bool is_min = k == kObs, is_max = k == kObs + 1;
    double v = is_min ? 1e300 : (is_max ? -1e300 : 0.0);
    for (int b = lane; b < nblocks; b += 64) {
      const double x = partial[(size_t)b * (kObs + 3) + k];
      v = is_min ? fmin(v, x) : (is_max ? fmax(v, x) : v + x);
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off, 64);
      v = is_min ? fmin(v, o) : (is_max ? fmax(v, o) : v + o);
    }
    if (lane == 0) out[k] = (k < kObs) ? v * degeneracy(k / kObsPer) * meas : v;
  }
}

// Energy bookkeeping of a step, per-block partials [source, collide]:
// source  = sum N f (E(m^2) - E(m_prev^2)), the difference taken as
//           (m^2 - m_prev^2) / (E + E_prev) so it keeps its relative accuracy;
// collide = sum over evolved species of E(m^2) A.
__global__ __launch_bounds__(kBlock) void energy_partial(Grid G, const double* __restrict__ f,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ mass2,
                                                         const double* __restrict__ mass2_prev, double* partial) {
  __shared__ double sh[kBlock / 64];
  const size_t per = (size_t)G.cells * G.nodes;
  double src = 0.0, col = 0.0;
  for (int sp = 0; sp < kSpecies; ++sp) {
    const bool evolve = (G.species_mask >> sp) & 1u;
    double s_sp = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
      const int cell = (int)(i / G.nodes), node = (int)(i % G.nodes);
      double p[3];
      node_p(G, node, p);
      const double pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      const double m2 = mass2[sp * G.cells + cell];
      const double E = sqrt(pp + m2);
      if (mass2_prev) {
        const double m2p = mass2_prev[sp * G.cells + cell];
        const double den = E + sqrt(pp + m2p);
        if (den > 0.0) s_sp += f[(size_t)sp * per + i] * (m2 - m2p) / den;
      }
      if (evolve) col += E * A[(size_t)sp * per + i];
    }
    src += degeneracy(sp) * s_sp;
  }
  const double t0 = block_sum(src, sh);
  const double t1 = block_sum(col, sh);
  if (threadIdx.x == 0) {
    partial[2 * (size_t)blockIdx.x] = t0;
    partial[2 * (size_t)blockIdx.x + 1] = t1;
  }
}

__global__ __launch_bounds__(kBlock) void energy_final(Grid G, const double* partial, int nblocks, double dt,
                                                       double* out) {
  __shared__ double sh[kBlock / 64];
  const double meas = G.dx[0] * G.dx[1] * G.dx[2] * G.dp[0] * G.dp[1] * G.dp[2] / (8.0 * kPi * kPi * kPi);
  for (int k = 0; k < 2; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[2 * (size_t)b + k];
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) out[k] = k == 0 ? t * meas : t * meas * dt / kHbarC;
  }
}

__global__ void to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void quads_kernel(Grid G, const float* __restrict__ f, float4* __restrict__ q, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int node = (int)(i % (size_t)G.nodes);
    const int iz = node % G.np[2], iy = (node / G.np[2]) % G.np[1];
    const size_t dz = iz + 1 < G.np[2] ? 1 : 0;
    const size_t dy = iy + 1 < G.np[1] ? (size_t)G.oy : 0;
    q[i] = make_float4(f[i], f[i + dz], f[i + dy], f[i + dy + dz]);
  }
}

__global__ void fill_kernel(double* __restrict__ dst, double v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

__global__ void zero_u64_kernel(unsigned long long* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = 0ull;
}

unsigned grid_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 16384) b = 16384;
  return (unsigned)(b ? b : 1);
}

}  // namespace

size_t mass_scratch(const Grid& G) { return (size_t)G.cells * mass_chunks(G) * kSpecies; }

hipError_t launch_masses(const Grid& G, const double* f, const double* lag, double* scratch, double* mass2,
                         hipStream_t st) {
  const int chunks = mass_chunks(G);
  hipLaunchKernelGGL(mass_partial, dim3(chunks * G.cells), dim3(kBlock), 0, st, G, f, lag, scratch);
  hipLaunchKernelGGL(mass_final, dim3(G.cells), dim3(kBlock), 0, st, G, scratch, chunks, mass2);
  return hipGetLastError();
}

hipError_t launch_const_masses(const Grid& G, const Mass7& m, double* mass2, hipStream_t st) {
  const int n = kSpecies * G.cells;
  hipLaunchKernelGGL(const_mass_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, G, m, mass2);
  return hipGetLastError();
}

hipError_t launch_update(const Grid& G, const double* f, const double* A, const double* mass2, double dt,
                         int scheme, double* f_out, float* f32, hipStream_t st) {
  Evolving ev{};
  for (int sp = 0; sp < kSpecies; ++sp)
    if ((G.species_mask >> sp) & 1u) ev.sp[ev.n++] = sp;
  const size_t n = (size_t)ev.n * G.cells * G.nodes;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, G, ev, f, A, mass2, dt, scheme, f_out,
                     f32);
  return hipGetLastError();
}

int observables_blocks(const Grid& G) {
  const size_t per = (size_t)G.cells * G.nodes;
  size_t b = (per + kBlock - 1) / kBlock;
  return (int)(b > 512 ? 512 : (b ? b : 1));
}

size_t observables_scratch(const Grid& G) { return (size_t)observables_blocks(G) * (kObs + 3); }

hipError_t launch_observables(const Grid& G, const double* f, const double* mass2, double* scratch,
                              double* out, hipStream_t st) {
  const int nb = observables_blocks(G);
  hipLaunchKernelGGL(observables_partial, dim3(nb), dim3(kBlock), 0, st, G, f, mass2, scratch);
  hipLaunchKernelGGL(observables_final, dim3(1), dim3(kFinalThreads), 0, st, G, scratch, nb, out);
  return hipGetLastError();
}

hipError_t launch_energy_budget(const Grid& G, const double* f, const double* A, const double* mass2,
                                const double* mass2_prev, double dt, double* scratch, double* out, hipStream_t st) {
  const int nb = observables_blocks(G);
  hipLaunchKernelGGL(energy_partial, dim3(nb), dim3(kBlock), 0, st, G, f, A, mass2, mass2_prev, scratch);
  hipLaunchKernelGGL(energy_final, dim3(1), dim3(kBlock), 0, st, G, scratch, nb, dt, out);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_f32_quads(const Grid& G, const float* f32, float4* q, hipStream_t st) {
  const size_t n = (size_t)kSpecies * G.cells * G.nodes;
  hipLaunchKernelGGL(quads_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, G, f32, q, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* dst, double v, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, dst, v, n);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, dst, n);
  return hipGetLastError();
}

}  // namespace qgbe
