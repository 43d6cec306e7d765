// C ABI of libqgbe: context management, validation and launch logic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

using namespace qgbe;

namespace {
thread_local std::string g_error;
}  // namespace

namespace qgbe {

qgbe_status fail(qgbe_status s, const std::string& msg) {
  g_error = msg;
  return s;
}

qgbe_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? QGBE_ENOMEM : QGBE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t field_len(const qgbe_ctx* c) { return (size_t)kSpecies * c->G.cells * c->G.nodes; }

}  // namespace qgbe

namespace qgbe {

qgbe_status compute_masses(qgbe_ctx* c) {
  if (c->d.mass_mode == QGBE_MASS_CONSTANT) {
    Mass7 m;
    for (int s = 0; s < kSpecies; ++s) m.v[s] = c->d.const_mass2[s];
    HIP_TRY(launch_const_masses(c->G, m, c->d_mass2, c->stream), "constant masses");
  } else {
    HIP_TRY(launch_masses(c->G, c->d_f, c->has_lag ? c->d_lag : nullptr, c->d_mass_part, c->d_mass2, c->stream),
            "masses");
  }
  c->masses_valid = true;
  return QGBE_OK;
}

CollideArgs base_args(qgbe_ctx* c, int n_samples, double* A, double* scale, double* items) {
  CollideArgs a{};
  a.G = c->G;
  a.chans = c->d_chans;
  a.n_channels = c->nch;
  a.n_samples = n_samples;
  a.symmetric = c->d.symmetric;
  a.key0 = (uint32_t)c->d.seed;
  a.key1 = (uint32_t)(c->d.seed >> 32) + c->step;
  a.f64 = c->d_f;
  a.f32 = c->d_f32;
  a.mass2 = c->d_mass2;
  a.win_lo = 0;
  a.win_n = c->G.nodes;
  a.msq_mask = c->msq_mask;
  a.msq = c->d_msq;
  a.A = A;
  a.scale = scale;
  a.items = items;
  a.n_accepted = c->d_count;
  a.mc_acc = c->d_mc;
  a.chan_var = c->d_chan_var;
  a.mix_K = c->K;
  a.mix_thr = c->d_thr;
  a.mix_mu = c->d_mu;
  a.mix_sigma = c->d_sigma;
  a.mix_on = c->d_mix_on;
  return a;
}


qgbe_status validate(const qgbe_grid_desc* d) {
  if (!d) return fail(QGBE_EINVAL, "descriptor is NULL");
  long long cells = 1, nodes = 1;
  for (int a = 0; a < 3; ++a) {
    if (d->n_x[a] < 1) return fail(QGBE_EINVAL, "n_x must be >= 1");
    if (d->n_p[a] < 2) return fail(QGBE_EINVAL, "n_p must be >= 2 on every axis");
    if (!(d->x_half[a] > 0.0) || !std::isfinite(d->x_half[a])) return fail(QGBE_EINVAL, "x_half must be > 0");
    if (!(d->p_half[a] > 0.0) || !std::isfinite(d->p_half[a])) return fail(QGBE_EINVAL, "p_half must be > 0");
    cells *= d->n_x[a];
    nodes *= d->n_p[a];
  }
  if (cells * nodes * kSpecies > (1LL << 31)) return fail(QGBE_EINVAL, "grid too large for 32-bit indexing");
  if (nodes > (1 << 23)) return fail(QGBE_EINVAL, "too many momentum nodes");
  if ((d->species_mask & ~0x7Fu) || d->species_mask == 0) return fail(QGBE_EINVAL, "species_mask must be in 1..0x7F");
  if (d->row_mask & ~0x7Fu) return fail(QGBE_EINVAL, "row_mask must be in 0..0x7F");
  if (!(d->alpha_s > 0.0) || !std::isfinite(d->alpha_s)) return fail(QGBE_EINVAL, "alpha_s must be > 0");
  if (d->precision != QGBE_FP64 && d->precision != QGBE_FP32) return fail(QGBE_EINVAL, "bad precision");
  if (d->symmetric != 0 && d->symmetric != 1) return fail(QGBE_EINVAL, "symmetric must be 0 or 1");
  if (d->drift != QGBE_DRIFT_UPWIND && d->drift != QGBE_DRIFT_CENTRAL) return fail(QGBE_EINVAL, "bad drift scheme");
  if (d->mass_mode != QGBE_MASS_DYNAMIC && d->mass_mode != QGBE_MASS_CONSTANT) return fail(QGBE_EINVAL, "bad mass_mode");
  if (d->mass_mode == QGBE_MASS_CONSTANT)
    for (int s = 0; s < kSpecies; ++s)
      if (!(d->const_mass2[s] >= 0.0) || !std::isfinite(d->const_mass2[s]))
        return fail(QGBE_EINVAL, "const_mass2 must be finite and >= 0");
  return QGBE_OK;
}

void make_grid(const qgbe_grid_desc* d, Grid& G) {
  G.cells = 1;
  G.nodes = 1;
  for (int a = 0; a < 3; ++a) {
    G.nx[a] = d->n_x[a];
    G.np[a] = d->n_p[a];
    G.xh[a] = d->x_half[a];
    G.ph[a] = d->p_half[a];
    G.dx[a] = 2.0 * d->x_half[a] / d->n_x[a];
    G.dp[a] = 2.0 * d->p_half[a] / d->n_p[a];
    G.inv_dp[a] = 1.0 / G.dp[a];
    G.pc[a] = G.ph[a] * G.inv_dp[a] - 0.5;
    G.cells *= d->n_x[a];
    G.nodes *= d->n_p[a];
  }
  G.oy = G.np[2];
  G.ox = G.np[1] * G.np[2];
  G.Vp = 8.0 * d->p_half[0] * d->p_half[1] * d->p_half[2];
  G.g2 = 4.0 * kPi * d->alpha_s;
  G.g4 = G.g2 * G.g2;
  G.species_mask = d->species_mask;
}

// LDS plan per sampler: FP64 accumulators first (they replace global
// atomics), then FP32 f tiles in what is left; slots that do not fit use
// global memory.
void plan_groups(qgbe_ctx* c) {
  const size_t acc_b = (size_t)c->G.nodes * sizeof(double);
  const size_t tile_b = (size_t)c->G.nodes * sizeof(float);
  c->group_index.clear();
  c->groups.clear();
  for (int nslot = 1; nslot <= 3; ++nslot) {
    Group g{(int)c->group_index.size(), 0, nslot, {0, 0}, {0, 0}, {c->G.nodes, c->G.nodes}, false};
    for (int l = 0; l < 2; ++l) {
      const size_t budget = c->lds_budget[l];
      if (c->d.symmetric && budget < acc_b) {
        // one slot's FP64 accumulators exceed LDS: node windows, one launch
        // per window holding every slot's accumulators for that window, the
        // same samples in each; f from the quads
        const int fit = (int)(budget / (sizeof(double) * nslot));
        const int n_win = (c->G.nodes + fit - 1) / fit;
        g.win[l] = (c->G.nodes + n_win - 1) / n_win;
        g.lds_acc[l] = nslot;
        g.lds_tiles[l] = 0;
        continue;
      }
      g.lds_acc[l] = c->d.symmetric ? (int)std::min<size_t>(nslot, budget / acc_b) : 0;
      g.lds_tiles[l] = (int)std::min<size_t>(nslot, (budget - g.lds_acc[l] * acc_b) / tile_b);
    }
    g.queue = c->d.symmetric && g.lds_acc[0] == nslot && nslot * acc_b <= c->lds_budget_queue;
    for (int i = 0; i < c->nch; ++i)
      if (c->chans[i].nslot == nslot) c->group_index.push_back(i);
    g.count = (int)c->group_index.size() - g.start;
    if (g.count) {
      c->groups.push_back(g);
      for (int l = 0; l < 2; ++l) c->need_quads[l] = c->need_quads[l] || g.lds_tiles[l] < nslot;
      c->need_quads[0] = c->need_quads[0] || g.queue;
    }
  }
}

// Enqueue the collision kernels accumulating into A (zeroed by the caller).
qgbe_status run_collide(qgbe_ctx* c, int n_samples, int sampler, double* A, double* scale, double* items) {
  const bool learned = sampler == QGBE_SAMPLER_LEARNED;
  HIP_TRY(launch_zero_u64(c->d_count, kStripes, c->stream), "zero counter");
  HIP_TRY(launch_fill(c->d_mc, 0.0, 2 * kStripes, c->stream), "zero error accumulators");
  HIP_TRY(launch_fill(c->d_chan_var, 0.0, kStripes * std::max(1, c->nch), c->stream), "zero channel variances");
  c->n_launches = 0;
  if (c->nch == 0) return QGBE_OK;
  CollideArgs a = base_args(c, n_samples, A, scale, items);
  a.learned = learned ? 1 : 0;
  a.slot_lo = 0;
  a.slot_hi = 3;
  a.direct = 1;
  if (sampler == QGBE_SAMPLER_ROOTS || sampler == QGBE_SAMPLER_ROOTS_ALT) {
    a.learned = 0;
    a.group = c->d_all;
    a.n_group = c->nch;
    HIP_TRY(launch_collide_roots(a, sampler == QGBE_SAMPLER_ROOTS_ALT, c->stream), "collide (roots)");
    ++c->n_launches;
    return QGBE_OK;
  }
  const bool f64_path = c->d.precision == QGBE_FP64;
  if (f64_path) {
    a.group = c->d_all;
    a.n_group = c->nch;
    HIP_TRY(launch_collide_f64(a, c->stream), "collide (fp64)");
    ++c->n_launches;
    return QGBE_OK;
  }
  const int l = learned ? 1 : 0;
  if (c->need_quads[l]) HIP_TRY(launch_f32_quads(c->G, c->d_f32, c->d_f32q, c->stream), "f32 quads");
  a.f32q = c->d_f32q;
  for (const Group& g : c->groups) {
    a.group = c->d_groups + g.start;
    a.n_group = g.count;
    // the compacting variant when the whole group fits in LDS next to its queues
    const bool queue = !learned && g.queue;
    const int waves = collide_f32_waves(queue);
    const long long items = (long long)c->G.cells * g.count * c->G.nodes;
    long long chunk = items / 2048;
    chunk = std::max<long long>(waves, std::min<long long>(512, chunk));
    // Every workgroup zeroes and flushes its LDS accumulators; with few
    // samples per point that costs as much as the samples themselves, so the
    // chunk grows until the flush entries are at most a quarter of the
    // workgroup's samples (measured: a quarter beats an eighth, a half and
    // one), keeping at least two workgroups per compute unit, or one where
    // even then the flush would outweigh the samples.
    const long long acc = c->d.symmetric ? (long long)std::min(g.nslot, std::max(g.lds_acc[l], 0)) * g.win[l] : 0;
    if (acc > 0 && chunk * n_samples < 4 * acc) {
      const long long want = (4 * acc + n_samples - 1) / n_samples;
      long long fill = items / (2LL * c->n_cu);
      if (fill * n_samples < acc) fill = items / c->n_cu;
      chunk = std::max(chunk, std::min(want, fill));
    }
    // With enough (cell, channel) pairs to give every compute unit one, the
    // nodes of a pair are split over at most two workgroups per compute unit
    // in all: fewer workgroups zero and flush their accumulators (on the
    // pure-gluon 16x16x1 grid: 4096 -> 512 workgroups, 71.0 -> 68.0 ms;
    // grids with fewer pairs than compute units keep the chunks above).
    const long long pairs = (long long)c->G.cells * g.count;
    if (pairs >= c->n_cu) {
      const long long per_pair = std::max(1LL, 2LL * c->n_cu / pairs);
      chunk = std::max(chunk, (c->G.nodes + per_pair - 1) / per_pair);
    }
    // A multiple of the waves; a small chunk of a variant that hands nodes to
    // its waves in blocks, whole blocks for every wave (36 nodes in blocks of 4
    // would leave 3 of 12 waves idle).  Large chunks keep the finer multiple:
    // C2's two chunks per cell of 4032 and 3968 nodes instead of 4008 and 3992
    // cost 0.5% (compute units that ran two long ones).
    const int nb = collide_f32_node_block(queue, learned);
    const int unit = chunk < 16LL * waves * nb ? waves * nb : waves;
    chunk = (chunk + unit - 1) / unit * unit;
    chunk = std::min<long long>(chunk, (c->G.nodes + unit - 1) / unit * unit);
    a.chunk_items = (int)chunk;
    a.n_chunks = (int)((c->G.nodes + chunk - 1) / chunk);
    // Deposit slots whose FP64 accumulators do not all fit in LDS are split
    // over launches that each keep their slots' accumulators in LDS: the
    // samples are recomputed (same draws), which costs far less than global
    // FP64 atomics on every deposit.  The first launch also writes the direct
    // sums.  Without room for even one accumulator, global atomics remain.
    const int per = g.lds_acc[l];
    const int n_pass = (c->d.symmetric && per >= 1 && per < g.nslot) ? (g.nslot + per - 1) / per : 1;
    const size_t acc_b = (size_t)c->G.nodes * sizeof(double), tile_b = (size_t)c->G.nodes * sizeof(float);
    const int win = g.win[l], n_win = (c->G.nodes + win - 1) / win;
    for (int pass = 0; pass < n_pass; ++pass) {
      for (int w = 0; w < n_win; ++w) {
        a.slot_lo = n_pass > 1 ? pass * per : 0;
        a.slot_hi = n_pass > 1 ? std::min(g.nslot, a.slot_lo + per) : g.nslot;
        a.win_lo = w * win;
        a.win_n = std::min(win, c->G.nodes - a.win_lo);
        a.direct = pass == 0 && w == 0 ? 1 : 0;
        a.lds_acc = g.lds_acc[l];
        a.lds_tiles = g.lds_tiles[l];
        if (n_pass > 1 && n_win == 1) {
          const size_t used = (size_t)(a.slot_hi - a.slot_lo) * acc_b;
          a.lds_tiles = (int)std::min<size_t>(g.nslot, (c->lds_budget[l] - used) / tile_b);
        }
        if (queue) a.lds_tiles = 0;  // the compacting variant reads f from the node quads
        HIP_TRY(launch_collide_f32(a, g.nslot, queue && n_pass == 1 && n_win == 1, c->stream), "collide (fp32)");
        ++c->n_launches;
      }
    }
  }
  return QGBE_OK;
}

}  // namespace qgbe

namespace {

void fill_stats(qgbe_ctx* c, const double* obs, const double* mass2_host, qgbe_stats* st) {
  std::memset(st, 0, sizeof *st);
  double mass_term = 0.0;
  for (int s = 0; s < kSpecies; ++s) {
    st->N[s] = obs[s * kObsPer];
    st->E[s] = obs[s * kObsPer + 1];
    st->N_total += st->N[s];
    st->E_total += st->E[s];
    for (int k = 0; k < 3; ++k) st->P[k] += obs[s * kObsPer + 2 + k];
    mass_term += obs[s * kObsPer + 5];
    st->entropy += obs[s * kObsPer + 6];
    for (int k = 0; k < 3; ++k) st->T_ii[k] += obs[s * kObsPer + 7 + k];
    double m = 0.0;
    for (int x = 0; x < c->G.cells; ++x) m += mass2_host[s * c->G.cells + x];
    st->mass2_avg[s] = m / c->G.cells;
  }
  st->E_total_mod = st->E_total - 0.25 * mass_term;
  st->min_f = obs[kSpecies * kObsPer];
  st->max_fermion_f = obs[kSpecies * kObsPer + 1];
  if (st->min_f < 0.0) st->flags |= QGBE_FLAG_NEGATIVE_F;
  if (st->max_fermion_f > 1.0) st->flags |= QGBE_FLAG_PAULI;
  if (obs[kSpecies * kObsPer + 2] > 0.0) st->flags |= QGBE_FLAG_NONFINITE;
  st->step = c->step;
}

qgbe_status read_stats(qgbe_ctx* c, qgbe_stats* st, bool energy = false) {
  HIP_TRY(launch_observables(c->G, c->d_f, c->d_mass2, c->d_obs_scratch, c->d_obs, c->stream), "observables");
  double obs[observables_len];
  unsigned long long counts[kStripes];
  HIP_TRY(hipMemcpyAsync(counts, c->d_count, sizeof counts, hipMemcpyDeviceToHost, c->stream), "copy counter");
  double mcs[2 * kStripes];
  HIP_TRY(hipMemcpyAsync(mcs, c->d_mc, sizeof mcs, hipMemcpyDeviceToHost, c->stream), "copy error accumulators");
  std::vector<double> m2((size_t)kSpecies * c->G.cells);
  HIP_TRY(hipMemcpyAsync(obs, c->d_obs, sizeof obs, hipMemcpyDeviceToHost, c->stream), "copy observables");
  HIP_TRY(hipMemcpyAsync(m2.data(), c->d_mass2, m2.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream),
          "copy masses");
  double budget[2] = {0.0, 0.0};
  if (energy)
    HIP_TRY(hipMemcpyAsync(budget, c->d_energy, sizeof budget, hipMemcpyDeviceToHost, c->stream), "copy energy budget");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  unsigned long long accepted = 0;
  double mc[2] = {0.0, 0.0};
  for (int i = 0; i < kStripes; ++i) {  // in stripe order: the same sum for the same stripes
    accepted += counts[i];
    mc[0] += mcs[2 * i];
    mc[1] += mcs[2 * i + 1];
  }
  fill_stats(c, obs, m2.data(), st);
  st->E_source = budget[0];
  st->E_collide = budget[1];
  st->n_accepted = (double)accepted;
  // sum S_i^2 estimates sum (E S_i)^2 + sum Var S_i; remove the variance part
  const double signal = mc[1] - mc[0];
  st->mc_err_est = mc[0] <= 0.0 ? 0.0 : (signal > 0.0 ? std::sqrt(mc[0] / signal) : INFINITY);
  return QGBE_OK;
}

bool species_ok(int s) { return s >= -1 && s < kSpecies; }

}  // namespace

extern "C" {

const char* qgbe_last_error(void) { return g_error.c_str(); }

size_t qgbe_workspace_bytes(const qgbe_ctx* ctx) { return ctx ? ctx->ws : 0; }

int32_t qgbe_channel_table(uint32_t species_mask, uint32_t row_mask, int32_t* rows, double* weights,
                           int32_t max) {
  Channel buf[kMaxChannels];
  const int n = build_channels(species_mask & 0x7Fu, row_mask & 0x7Fu, buf, kMaxChannels);
  if (n < 0) return QGBE_EINVAL;
  if (n > max) return fail(QGBE_EINVAL, "channel table larger than max");
  for (int i = 0; i < n; ++i) {
    if (rows) {
      rows[i * 5] = buf[i].row;
      for (int p = 0; p < 4; ++p) rows[i * 5 + 1 + p] = buf[i].sp[p];
    }
    if (weights) {
      weights[i * 2] = buf[i].w;
      weights[i * 2 + 1] = buf[i].sigma;
    }
  }
  return n;
}

void qgbe_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  philox4x32_10(x0, x1, x2, x3, key[0], key[1]);
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

qgbe_status qgbe_init_grid(const qgbe_grid_desc* desc, qgbe_ctx** out) {
  if (!out) return fail(QGBE_EINVAL, "out is NULL");
  *out = nullptr;
  qgbe_status st = validate(desc);
  if (st) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(QGBE_EDEVICE, "no HIP device");
  if (desc->device < 0 || desc->device >= ndev) return fail(QGBE_EINVAL, "device ordinal out of range");
  HIP_TRY(hipSetDevice(desc->device), "hipSetDevice");
  int lds_max = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, desc->device),
          "query LDS size");
  size_t lds_budget[3] = {0, 0, 0};
  HIP_TRY(set_collide_lds_limit((size_t)std::max(lds_max, 0), &lds_budget[0], &lds_budget[1], &lds_budget[2]),
          "raise the dynamic LDS limit");
  qgbe_ctx* c = new qgbe_ctx();
  c->d = *desc;
  c->stream = (hipStream_t)desc->stream;
  make_grid(desc, c->G);
  c->chans.resize(kMaxChannels);
  c->nch = build_channels(desc->species_mask, desc->row_mask, c->chans.data(), kMaxChannels);
  c->chans.resize(c->nch);
  c->lds_budget[0] = lds_budget[0];
  c->lds_budget[1] = lds_budget[1];
  c->lds_budget_queue = lds_budget[2];
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, desc->device) == hipSuccess && n_cu > 0)
    c->n_cu = n_cu;
  plan_groups(c);
  const size_t n = field_len(c);
  std::vector<int> all(std::max(1, c->nch));
  for (int i = 0; i < c->nch; ++i) all[i] = i;
#define ALLOC(p, cnt, what)                       \
  do {                                            \
    qgbe_status _s = dev_alloc(c, &(p), (cnt), what); \
    if (_s) { qgbe_destroy(c); return _s; }       \
  } while (0)
  ALLOC(c->d_chans, std::max(1, c->nch), "channel table");
  ALLOC(c->d_groups, std::max<size_t>(1, c->group_index.size()), "channel groups");
  ALLOC(c->d_all, all.size(), "channel list");
  ALLOC(c->d_f, n, "f");
  ALLOC(c->d_f_next, n, "f (next)");
  ALLOC(c->d_f32, n, "f (fp32)");
  if (c->d.precision == QGBE_FP32 && (c->need_quads[0] || c->need_quads[1])) ALLOC(c->d_f32q, n, "f (fp32 quads)");
  ALLOC(c->d_A, n, "collision term");
  ALLOC(c->d_mass2, (size_t)kSpecies * c->G.cells, "masses");
  ALLOC(c->d_lag, (size_t)kSpecies * c->G.cells, "lagged masses");
  ALLOC(c->d_obs_scratch, observables_scratch(c->G), "observables scratch");
  ALLOC(c->d_obs, (size_t)observables_len, "observables");
  ALLOC(c->d_energy, 2, "energy budget");
  ALLOC(c->d_msq, 1, "matrix element table");
  ALLOC(c->d_mass_part, mass_scratch(c->G), "mass partial sums");
  ALLOC(c->d_count, kStripes, "accepted counter");
  ALLOC(c->d_mc, 2 * kStripes, "error accumulators");
  ALLOC(c->d_chan_var, kStripes * std::max(1, c->nch), "channel variances");
#undef ALLOC
  const char* what = "copy channel table";
  hipError_t e = hipSuccess;
  if (c->nch) e = hipMemcpy(c->d_chans, c->chans.data(), c->nch * sizeof(Channel), hipMemcpyHostToDevice);
  if (e == hipSuccess && !c->group_index.empty()) {
    what = "copy channel groups";
    e = hipMemcpy(c->d_groups, c->group_index.data(), c->group_index.size() * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    what = "copy channel list";
    e = hipMemcpy(c->d_all, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice);
  }
  for (int i = 0; i < 4 && e == hipSuccess; ++i) {
    what = "create events";
    e = hipEventCreate(&c->ev[i]);
  }
  if (e == hipSuccess) {
    what = "zero f";
    e = launch_fill(c->d_f, 0.0, n, c->stream);
    // both buffers: the step updates only the evolving species
    if (e == hipSuccess) e = launch_fill(c->d_f_next, 0.0, n, c->stream);
  }
  if (e == hipSuccess) e = launch_to_f32(c->d_f, c->d_f32, n, c->stream);
  if (e == hipSuccess) {
    what = "synchronise";
    e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) {
    qgbe_status s = hip_fail(e, what);
    qgbe_destroy(c);
    return s;
  }
  *out = c;
  g_error.clear();
  return QGBE_OK;
}

void qgbe_destroy(qgbe_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->d.device);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->d_chans);
  (void)hipFree(c->d_groups);
  (void)hipFree(c->d_all);
  (void)hipFree(c->d_f);
  (void)hipFree(c->d_f_next);
  (void)hipFree(c->d_f32);
  (void)hipFree(c->d_f32q);
  (void)hipFree(c->d_A);
  (void)hipFree(c->d_mass2);
  (void)hipFree(c->d_lag);
  (void)hipFree(c->d_obs_scratch);
  (void)hipFree(c->d_energy);
  (void)hipFree(c->d_msq);
  (void)hipFree(c->d_mass_part);
  (void)hipFree(c->d_obs);
  (void)hipFree(c->d_count);
  (void)hipFree(c->d_mc);
  (void)hipFree(c->d_chan_var);
  (void)hipFree(c->d_thr);
  (void)hipFree(c->d_mu);
  (void)hipFree(c->d_sigma);
  (void)hipFree(c->d_feat);
  (void)hipFree(c->d_mix_on);
  (void)hipFree(c->d_mass7);
  {
    MlpState& m = c->mlp;
    void* bufs[] = {m.params, m.m, m.v, m.grad, m.pb, m.X, m.Xb, m.Z1, m.H1b, m.Z2, m.H2b, m.Y, m.dY, m.dYb,
                    m.dH, m.dZ, m.dZb, m.yw, m.scalars};
    for (void* b : bufs) (void)hipFree(b);
  }
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

qgbe_status qgbe_set_distribution(qgbe_ctx* c, int32_t species, const double* f, int32_t on_device) {
  if (!c || !f) return fail(QGBE_EINVAL, "NULL argument");
  if (!species_ok(species)) return fail(QGBE_EINVAL, "species must be -1 or 0..6");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  const size_t per = (size_t)c->G.cells * c->G.nodes;
  double* dst = species < 0 ? c->d_f : c->d_f + (size_t)species * per;
  const size_t cnt = species < 0 ? field_len(c) : per;
  HIP_TRY(hipMemcpyAsync(dst, f, cnt * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         c->stream), "copy f in");
  // the second buffer of f too: a step updates only the evolving species
  HIP_TRY(hipMemcpyAsync(c->d_f_next + (dst - c->d_f), dst, cnt * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
          "copy f to the second buffer");
  HIP_TRY(launch_to_f32(c->d_f, c->d_f32, field_len(c), c->stream), "f to fp32");
  if (!on_device) HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  c->has_lag = false;
  c->masses_valid = false;
  return QGBE_OK;
}

qgbe_status qgbe_get_distribution(qgbe_ctx* c, int32_t species, double* f, int32_t on_device) {
  if (!c || !f) return fail(QGBE_EINVAL, "NULL argument");
  if (!species_ok(species)) return fail(QGBE_EINVAL, "species must be -1 or 0..6");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  const size_t per = (size_t)c->G.cells * c->G.nodes;
  const double* src = species < 0 ? c->d_f : c->d_f + (size_t)species * per;
  const size_t cnt = species < 0 ? field_len(c) : per;
  HIP_TRY(hipMemcpyAsync(f, src, cnt * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         c->stream), "copy f out");
  if (!on_device) HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_get_masses(qgbe_ctx* c, double* mass2) {
  if (!c || !mass2) return fail(QGBE_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(mass2, c->d_mass2, (size_t)kSpecies * c->G.cells * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream), "copy masses");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_set_step_index(qgbe_ctx* c, uint32_t step) {
  if (!c) return fail(QGBE_EINVAL, "NULL context");
  c->step = step;
  return QGBE_OK;
}

qgbe_status qgbe_get_step_index(const qgbe_ctx* c, uint32_t* step) {
  if (!c || !step) return fail(QGBE_EINVAL, "NULL argument");
  *step = c->step;
  return QGBE_OK;
}

qgbe_status qgbe_collision_term_ex(qgbe_ctx* c, int32_t n_samples, int32_t sampler, double* A_out,
                                   int32_t on_device, const qgbe_collide_extras* ex, qgbe_stats* st) {
  if (!c || !A_out) return fail(QGBE_EINVAL, "NULL argument");
  if (n_samples < 1) return fail(QGBE_EINVAL, "n_samples must be >= 1");
  if (sampler < QGBE_SAMPLER_UNIFORM || sampler > QGBE_SAMPLER_ROOTS_ALT) return fail(QGBE_EINVAL, "bad sampler");
  if (sampler == QGBE_SAMPLER_LEARNED && !c->K) return fail(QGBE_ESTATE, "no proposal table installed");
  if (sampler == QGBE_SAMPLER_LEARNED && c->d.precision == QGBE_FP32 && c->K > kMixKF32)
    return fail(QGBE_EUNSUPPORTED, "the FP32 learned sampler takes at most 8 mixture components (FP64 takes 16)");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  const size_t n = field_len(c);
  double* A = on_device ? A_out : c->d_A;
  double* scale = nullptr;
  double* items = nullptr;
  const bool ex_host = ex && !ex->on_device;
  const size_t n_items = (size_t)c->G.cells * c->nch * c->G.nodes;
  if (ex && ex->scale) {
    if (ex_host) HIP_TRY(hipMalloc(&scale, n * sizeof(double)), "scale scratch");
    else scale = ex->scale;
  }
  if (ex && ex->item_sums && n_items) {
    if (ex_host) HIP_TRY(hipMalloc(&items, n_items * sizeof(double)), "item scratch");
    else items = ex->item_sums;
  }
  qgbe_status s = compute_masses(c);
  if (!s && sampler == QGBE_SAMPLER_LEARNED && c->table_net) s = refresh_proposal_table(c);
  if (!s) {
    hipError_t e = launch_fill(A, 0.0, n, c->stream);
    if (e == hipSuccess && scale) e = launch_fill(scale, 0.0, n, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[0], c->stream);
    if (e != hipSuccess) s = hip_fail(e, "zero outputs");
  }
  if (!s) s = run_collide(c, n_samples, sampler, A, scale, items);
  if (!s) {
    hipError_t e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess && !on_device)
      e = hipMemcpyAsync(A_out, A, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && ex_host && scale)
      e = hipMemcpyAsync(ex->scale, scale, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && ex_host && items)
      e = hipMemcpyAsync(ex->item_sums, items, n_items * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && (!on_device || ex_host || st)) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = hip_fail(e, "collision term");
  }
  if (ex_host) {
    (void)hipFree(scale);
    (void)hipFree(items);
  }
  if (s) return s;
  if (st) {
    s = read_stats(c, st);
    if (s) return s;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    st->t_collide_ms = ms;
    st->n_collide_launches = (uint32_t)c->n_launches;
    st->n_evals = (double)c->G.cells * c->nch * c->G.nodes * n_samples;
  }
  return QGBE_OK;
}

qgbe_status qgbe_set_matrix_element(qgbe_ctx* c, int32_t row, int32_t n_terms, const double* coef,
                                    const int32_t* powers) {
  if (!c) return fail(QGBE_EINVAL, "NULL context");
  if (row < 1 || row > 7) return fail(QGBE_EINVAL, "row must be 1..7");
  if (n_terms < 0 || n_terms > kMsqMaxTerms) return fail(QGBE_EINVAL, "0..8 terms per row");
  if (n_terms > 0 && (!coef || !powers)) return fail(QGBE_EINVAL, "NULL terms");
  for (int k = 0; k < n_terms; ++k) {
    if (!std::isfinite(coef[k])) return fail(QGBE_EINVAL, "non-finite coefficient");
    for (int i = 0; i < 6; ++i)
      if (powers[6 * k + i] < 0 || powers[6 * k + i] > kMsqMaxPower) return fail(QGBE_EINVAL, "powers must be 0..4");
  }
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  c->msq.n[row] = n_terms;
  for (int k = 0; k < kMsqMaxTerms; ++k) {
    c->msq.c[row][k] = k < n_terms ? coef[k] : 0.0;
    for (int i = 0; i < 6; ++i) c->msq.p[row][k][i] = (int8_t)(k < n_terms ? powers[6 * k + i] : 0);
  }
  if (n_terms > 0) c->msq_mask |= 1u << row;
  else c->msq_mask &= ~(1u << row);
  // the table is read by kernels already queued on the stream: wait for them
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  HIP_TRY(hipMemcpyAsync(c->d_msq, &c->msq, sizeof(MsqTable), hipMemcpyHostToDevice, c->stream),
          "copy matrix elements");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_collision_term(qgbe_ctx* c, int32_t n_samples, int32_t sampler, double* A_out, int32_t on_device,
                                qgbe_stats* st) {
  return qgbe_collision_term_ex(c, n_samples, sampler, A_out, on_device, nullptr, st);
}

qgbe_status qgbe_step(qgbe_ctx* c, double dt_fm, int32_t n_samples, int32_t sampler, int32_t n_steps,
                      qgbe_stats* per_step) {
  if (!c) return fail(QGBE_EINVAL, "NULL context");
  if (!(dt_fm > 0.0) || !std::isfinite(dt_fm)) return fail(QGBE_EINVAL, "dt must be > 0");
  if (n_samples < 1 || n_steps < 0) return fail(QGBE_EINVAL, "n_samples >= 1 and n_steps >= 0 required");
  if (sampler < QGBE_SAMPLER_UNIFORM || sampler > QGBE_SAMPLER_ROOTS_ALT) return fail(QGBE_EINVAL, "bad sampler");
  if (sampler == QGBE_SAMPLER_LEARNED && !c->K) return fail(QGBE_ESTATE, "no proposal table installed");
  if (sampler == QGBE_SAMPLER_LEARNED && c->d.precision == QGBE_FP32 && c->K > kMixKF32)
    return fail(QGBE_EUNSUPPORTED, "the FP32 learned sampler takes at most 8 mixture components (FP64 takes 16)");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  const size_t n = field_len(c);
  qgbe_status result = QGBE_OK;
  for (int k = 0; k < n_steps; ++k) {
    HIP_TRY(hipEventRecord(c->ev[2], c->stream), "event");
    qgbe_status s = compute_masses(c);
    if (!s && sampler == QGBE_SAMPLER_LEARNED && c->table_net) s = refresh_proposal_table(c);
    if (s) return s;
    HIP_TRY(launch_fill(c->d_A, 0.0, n, c->stream), "zero A");
    HIP_TRY(hipEventRecord(c->ev[0], c->stream), "event");
    s = run_collide(c, n_samples, sampler, c->d_A, nullptr, nullptr);
    if (s) return s;
    HIP_TRY(hipEventRecord(c->ev[1], c->stream), "event");
    if (per_step)  // before the update: f_k, its masses, the step before's masses
      HIP_TRY(launch_energy_budget(c->G, c->d_f, c->d_A, c->d_mass2, c->has_lag ? c->d_lag : nullptr, dt_fm,
                                   c->d_obs_scratch, c->d_energy, c->stream),
              "energy budget");
    HIP_TRY(launch_update(c->G, c->d_f, c->d_A, c->d_mass2, dt_fm, c->d.drift, c->d_f_next, c->d_f32, c->stream),
            "update");
    std::swap(c->d_f, c->d_f_next);
    c->masses_valid = false;
    HIP_TRY(hipMemcpyAsync(c->d_lag, c->d_mass2, (size_t)kSpecies * c->G.cells * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream), "lag masses");
    c->has_lag = c->d.mass_mode == QGBE_MASS_DYNAMIC;
    HIP_TRY(hipEventRecord(c->ev[3], c->stream), "event");
    c->step += 1;
    if (per_step) {
      s = read_stats(c, &per_step[k], true);
      if (s) return s;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
      per_step[k].t_collide_ms = ms;
      per_step[k].n_collide_launches = (uint32_t)c->n_launches;
      (void)hipEventElapsedTime(&ms, c->ev[2], c->ev[3]);
      per_step[k].t_step_ms = ms;
      per_step[k].n_evals = (double)c->G.cells * c->nch * c->G.nodes * n_samples;
      if (per_step[k].flags & QGBE_FLAG_NONFINITE) result = fail(QGBE_ENUMERIC, "non-finite f after step");
    }
  }
  return result;
}

qgbe_status qgbe_observables(qgbe_ctx* c, qgbe_stats* st) {
  if (!c || !st) return fail(QGBE_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  qgbe_status s = compute_masses(c);
  if (s) return s;
  return read_stats(c, st);
}


}  // extern "C"
