// Context of libqgbe shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "collide.h"
#include "field.h"
#include "mlp.h"
#include "qgbe.h"
#include "qgbe_common.h"

namespace qgbe {

qgbe_status fail(qgbe_status s, const std::string& msg);
qgbe_status hip_fail(hipError_t e, const char* what);

#define HIP_TRY(expr, what)                                \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return ::qgbe::hip_fail(_e, what); \
  } while (0)

// Channels of the FP32 kernel grouped by their number of deposit slots.
struct Group {
  int start, count;   // range in the group index array
  int nslot;          // distinct species at positions 2..4
  int lds_acc[2];     // FP64 accumulators staged in LDS  [uniform, learned sampler]
  int lds_tiles[2];   // FP32 f tiles staged in LDS       [uniform, learned sampler]
  int win[2];         // nodes per accumulator window (= nodes unless one slot's FP64
                      // accumulators exceed LDS; then one launch per window and slot)
  bool queue;         // the uniform sampler's compacting variant fits
};

// Device buffers of the proposal network (allocated on first use).
struct MlpState {
  bool ready = false;
  bool has_weights = false;
  int adam_t = 0;
  float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  __bf16* pb = nullptr;
  float *X = nullptr, *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr, *dY = nullptr, *dH = nullptr, *dZ = nullptr;
  float* yw = nullptr;
  __bf16 *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *dZb = nullptr;
  double* scalars = nullptr;   // [0] loss, [1] weight sum
};

}  // namespace qgbe

struct qgbe_ctx {
  qgbe_grid_desc d{};
  qgbe::Grid G{};
  hipStream_t stream = nullptr;
  int nch = 0;
  std::vector<qgbe::Channel> chans;
  std::vector<int> group_index;
  std::vector<qgbe::Group> groups;
  qgbe::Channel* d_chans = nullptr;
  int* d_groups = nullptr;
  int* d_all = nullptr;            // identity channel list (FP64 kernel)
  double* d_f = nullptr;
  double* d_f_next = nullptr;
  float* d_f32 = nullptr;
  float4* d_f32q = nullptr;        // node quads of d_f32, for tiles read from global memory
  int n_launches = 0;                    // collision kernel launches of the last term
  bool need_quads[2] = {false, false};  // some group reads tiles globally [uniform, learned]
  double* d_mass2 = nullptr;
  double* d_lag = nullptr;
  bool has_lag = false;
  bool masses_valid = false;       // d_mass2 holds the masses of the current f
  double* d_A = nullptr;
  double* d_obs_scratch = nullptr;
  double* d_energy = nullptr;  // [E_source, E_collide] of the last step
  qgbe::MsqTable msq{};          // user matrix elements (host copy)
  uint32_t msq_mask = 0;         // rows replaced by them
  qgbe::MsqTable* d_msq = nullptr;  // device copy
  double* d_mass_part = nullptr;  // per (cell, chunk, species) partial mass integrals
  double* d_obs = nullptr;
  unsigned long long* d_count = nullptr;
  double* d_mc = nullptr;          // [2] MC error accumulators of the last collision term
  double* d_chan_var = nullptr;    // [kStripes][channels] per-channel variance sums of the last collision term
  uint32_t step = 0;
  int K = 0;                       // proposal table components (0 = none)
  uint32_t* d_thr = nullptr;
  float* d_mu = nullptr;
  float* d_sigma = nullptr;
  uint8_t* d_mix_on = nullptr;     // [channels] 1: learned sampler, 0: uniform fallback
  float* d_feat = nullptr;         // [nch * nodes][8] conditioning features
  double* d_mass7 = nullptr;       // cell-averaged masses behind d_feat
  bool table_net = false;          // table comes from the network: rebuilt whenever the masses change
  float table_alpha = 0.0f;        // defensive weight of that table
  qgbe::MlpState mlp;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t ws = 0;
  size_t lds_budget[2] = {0, 0};   // dynamic LDS per workgroup [uniform, learned sampler]
  size_t lds_budget_queue = 0;     // dynamic LDS of the compacting uniform-sampler variant
  int n_cu = 256;                  // compute units of the device
};

namespace qgbe {

size_t field_len(const qgbe_ctx* c);
// Descriptor checks (QGBE_EINVAL with a message), the grid it describes, and
// the LDS plan of the FP32 channel groups (needs c->G, c->d, c->chans and the
// LDS budgets).
qgbe_status validate(const qgbe_grid_desc* d);
void make_grid(const qgbe_grid_desc* d, Grid& G);
void plan_groups(qgbe_ctx* c);
// Enqueue the collision kernels of one collision term, accumulating into A
// (zeroed by the caller); zeroes the per-launch totals first.
qgbe_status run_collide(qgbe_ctx* c, int n_samples, int sampler, double* A, double* scale, double* items);
qgbe_status compute_masses(qgbe_ctx* c);
CollideArgs base_args(qgbe_ctx* c, int n_samples, double* A, double* scale, double* items);
// Enqueue features, network forward and table construction for the current
// masses (no allocation, no synchronisation).
qgbe_status refresh_proposal_table(qgbe_ctx* c);
// Device buffers of a K-component proposal table (reallocated if K changes).
qgbe_status install_proposal_table(qgbe_ctx* c, int K);
// Every channel back on the learned sampler (after a new table or network).
qgbe_status reset_channel_samplers(qgbe_ctx* c);
// Device buffers of the conditioning features.
qgbe_status ensure_proposal_features(qgbe_ctx* c);

template <typename T>
qgbe_status dev_alloc(qgbe_ctx* c, T** p, size_t n, const char* what) {
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, what);
  }
  c->ws += n * sizeof(T);
  return QGBE_OK;
}

}  // namespace qgbe
