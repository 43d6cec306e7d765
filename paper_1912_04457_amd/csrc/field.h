// Launch interface of the field kernels (masses, drift + update, observables).
#pragma once

#include "qgbe_common.h"

namespace qgbe {

struct Mass7 {
  double v[kSpecies];
};

// Observables layout in `out` (length observables_len): per species
// [N, E, Px, Py, Pz, M, S, Txx, Tyy, Tzz] (7 x 10) with M = sum N dV m^2 f / E,
// S the entropy and Tii = sum N dV p_i^2 f / E, then min f, max fermion f,
// non-finite count.
constexpr int kObsPer = 10;
constexpr int observables_len = kSpecies * kObsPer + 3;

// Thermal masses (Eq. mg, Eq. mq); scratch holds mass_scratch(G) doubles.
size_t mass_scratch(const Grid& G);
hipError_t launch_masses(const Grid& G, const double* f, const double* lag, double* scratch, double* mass2,
                         hipStream_t st);
hipError_t launch_const_masses(const Grid& G, const Mass7& m, double* mass2, hipStream_t st);
hipError_t launch_update(const Grid& G, const double* f, const double* A, const double* mass2, double dt,
                         int scheme, double* f_out, float* f32, hipStream_t st);
size_t observables_scratch(const Grid& G);
hipError_t launch_observables(const Grid& G, const double* f, const double* mass2, double* scratch,
                              double* out, hipStream_t st);
// out[0] = E_source, out[1] = E_collide of a step (mass2_prev NULL: no
// source term); scratch as for launch_observables.
hipError_t launch_energy_budget(const Grid& G, const double* f, const double* A, const double* mass2,
                                const double* mass2_prev, double dt, double* scratch, double* out, hipStream_t st);
hipError_t launch_to_f32(const double* src, float* dst, size_t n, hipStream_t st);
// Node quads of the FP32 field: q[i] = (f[i], f[i+1], f[i+oy], f[i+oy+1])
// within each (species, cell) block, so a trilinear read takes two 16-byte
// loads; entries on the last z or y layer (never a stencil base) repeat f[i].
hipError_t launch_f32_quads(const Grid& G, const float* f32, float4* q, hipStream_t st);
hipError_t launch_fill(double* dst, double v, size_t n, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* dst, int n, hipStream_t st);

}  // namespace qgbe
