// Launch interface of the collision kernels.
#pragma once

#include "qgbe_common.h"

namespace qgbe {

// Stripes of the per-launch totals: one global atomic per workgroup lands on
// one of kStripes addresses, so same-address atomics do not serialise.
constexpr int kStripes = 64;

// Mixture components the FP32 learned sampler takes (its per-wave LDS row of
// component constants is laid out for this many); the FP64 path takes 16.
constexpr int kMixKF32 = 8;

struct CollideArgs {
  Grid G;
  const Channel* chans;   // device channel table (all channels)
  const int* group;       // channel indices processed by this launch
  int n_group;
  int n_channels;         // total channels (layout of items)
  int n_chunks;           // workgroups per (cell, channel) (FP32 kernel)
  int chunk_items;        // observed nodes per workgroup (FP32 kernel)
  int lds_tiles;          // f tiles staged in LDS (FP32 kernel)
  int lds_acc;            // FP64 deposit accumulators in LDS (FP32 kernel)
  int slot_lo, slot_hi;   // deposit slots [lo, hi) written by this launch (FP32 kernel); the
                          // first lds_acc of them accumulate in LDS, the rest in global memory
  int win_lo, win_n;      // LDS accumulators cover nodes [win_lo, win_lo + win_n) (FP32 kernel);
                          // deposit corners outside belong to another launch
  int direct;             // this launch also writes the direct sums, items, scale and counts
  int n_samples;
  int symmetric;
  uint32_t key0, key1;    // Philox key
  const double* f64;      // [7][cells][nodes]
  const float* f32;       // FP32 shadow of f64
  const float4* f32q;     // node quads of f32 (global-memory tiles), see launch_f32_quads
  const double* mass2;    // [7][cells]
  double* A;              // [7][cells][nodes], accumulated into
  double* scale;          // optional, same shape
  double* items;          // optional [cells][n_channels][nodes]
  unsigned long long* n_accepted;  // [kStripes]: samples above threshold and inside the box
  double* mc_acc;         // [kStripes][2] (may be NULL): sum over items of the variance estimate
                          // of their direct sum, and of the squared direct sums
                          // (workgroup b adds into stripe b mod kStripes; the reader sums them)
  double* chan_var;       // [kStripes][n_channels] (may be NULL): variance sums per channel, striped
  uint32_t msq_mask;      // bit r: Table I row r replaced by the user terms in msq
  const MsqTable* msq;    // device copy of the user terms (NULL when msq_mask is 0)
  int learned;            // draw from the mixture table instead of uniformly
  int mix_K;              // mixture components
  const uint32_t* mix_thr;   // [channels*nodes][K]
  const float* mix_mu;       // [channels*nodes][K][5]
  const float* mix_sigma;    // [channels*nodes][K][5]
  const uint8_t* mix_on;     // [channels] 0: the channel falls back to the uniform sampler; NULL: all 1
};

hipError_t launch_collide_f64(const CollideArgs& a, hipStream_t stream);
// The paper's root parameterisation (FP64; alt: the alternative elimination).
hipError_t launch_collide_roots(const CollideArgs& a, bool alt, hipStream_t stream);
// queue: use the compacting variant if the launch qualifies (uniform sampler,
// symmetric, every tile and accumulator in LDS within the queue budget).
hipError_t launch_collide_f32(const CollideArgs& a, int nslot, bool queue, hipStream_t stream);
// Raise the FP32 kernels' dynamic LDS limit to what their static LDS leaves
// of lds_max; returns the dynamic budget of the uniform-sampler, the
// learned-sampler and the compacting variants.
hipError_t set_collide_lds_limit(size_t lds_max, size_t* budget_plain, size_t* budget_learned, size_t* budget_queue);
// Waves per workgroup of the FP32 kernel (chunks are multiples of it).
int collide_f32_waves(bool queue);
// Consecutive observed nodes a wave of the FP32 kernel takes at a time
// (chunks must be multiples of it; multiples of the waves are).
int collide_f32_node_block(bool queue, bool learned);
hipError_t launch_record(const CollideArgs& a, int n_per_item, long long item_stride, long long n_sel, float* rows,
                         hipStream_t stream);

}  // namespace qgbe
