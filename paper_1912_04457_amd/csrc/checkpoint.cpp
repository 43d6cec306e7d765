// Checkpoint and restore of a context's evolving state: f (FP64), the step
// index (second Philox key word), the lagged masses that the next mass
// evaluation uses, the learned proposal (weights, Adam moments, table) and
// the user matrix elements that replace rows of Table I.
//
// Byte layout (host, native endianness): a fixed header, then the sections the
// header announces, each a plain array:
//   f          [7][cells][nodes]        double
//   lag        [7][cells]               double   (has_lag)
//   params, m, v [QGBE_MLP_PARAMS]      float    (has_weights)
//   thr        [channels*nodes][K]      uint32   (K > 0)
//   mu, sigma  [channels*nodes][K][5]   float    (K > 0)
//   samplers   [channels]               uint8    (K > 0; 0 = uniform fallback)
//   msq        one MsqTable (the user terms of every row)  (msq_mask != 0)
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "context.h"

using namespace qgbe;

namespace {

constexpr char kMagic[8] = {'Q', 'G', 'B', 'E', 'C', 'K', 'P', '1'};
constexpr uint32_t kVersion = 2;  // 2: user matrix elements

struct Header {
  char magic[8];
  uint32_t header_bytes;
  uint32_t version;
  // the grid the state belongs to
  int32_t n_x[3], n_p[3];
  double x_half[3], p_half[3];
  uint32_t species_mask, row_mask;
  double alpha_s;
  int32_t precision, symmetric, drift, mass_mode;
  double const_mass2[7];
  uint64_t seed;
  // the state
  uint32_t step;
  int32_t has_lag;
  int32_t has_weights;
  int32_t adam_t;
  int32_t K;
  int32_t table_net;
  float table_alpha;
  uint32_t msq_mask;  // bit r: Table I row r replaced by the stored user terms
  uint64_t n_field, n_lag, n_params, n_rows, n_chan;
};

bool same_grid(const Header& h, const qgbe_grid_desc& d) {
  bool ok = h.species_mask == d.species_mask && h.row_mask == d.row_mask && h.alpha_s == d.alpha_s &&
            h.precision == d.precision && h.symmetric == d.symmetric && h.drift == d.drift &&
            h.mass_mode == d.mass_mode && h.seed == d.seed;
  for (int a = 0; a < 3; ++a)
    ok = ok && h.n_x[a] == d.n_x[a] && h.n_p[a] == d.n_p[a] && h.x_half[a] == d.x_half[a] &&
         h.p_half[a] == d.p_half[a];
  for (int s = 0; s < 7; ++s) ok = ok && h.const_mass2[s] == d.const_mass2[s];
  return ok;
}

size_t payload_bytes(const Header& h) {
  size_t b = h.n_field * sizeof(double);
  if (h.has_lag) b += h.n_lag * sizeof(double);
  if (h.has_weights) b += 3 * h.n_params * sizeof(float);
  if (h.K > 0) b += h.n_rows * h.K * (sizeof(uint32_t) + 10 * sizeof(float)) + h.n_chan;
  if (h.msq_mask) b += sizeof(MsqTable);
  return b;
}

}  // namespace

extern "C" {

qgbe_status qgbe_checkpoint(qgbe_ctx* c, void* buf, size_t* bytes) {
  if (!c || !bytes) return fail(QGBE_EINVAL, "NULL argument");
  Header h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, sizeof kMagic);
  h.header_bytes = sizeof(Header);
  h.version = kVersion;
  const qgbe_grid_desc& d = c->d;
  for (int a = 0; a < 3; ++a) {
    h.n_x[a] = d.n_x[a];
    h.n_p[a] = d.n_p[a];
    h.x_half[a] = d.x_half[a];
    h.p_half[a] = d.p_half[a];
  }
  h.species_mask = d.species_mask;
  h.row_mask = d.row_mask;
  h.alpha_s = d.alpha_s;
  h.precision = d.precision;
  h.symmetric = d.symmetric;
  h.drift = d.drift;
  h.mass_mode = d.mass_mode;
  for (int s = 0; s < 7; ++s) h.const_mass2[s] = d.const_mass2[s];
  h.seed = d.seed;
  h.step = c->step;
  h.has_lag = c->has_lag ? 1 : 0;
  h.has_weights = (c->mlp.ready && c->mlp.has_weights) ? 1 : 0;
  h.adam_t = c->mlp.adam_t;
  h.K = c->K;
  h.table_net = c->table_net ? 1 : 0;
  h.table_alpha = c->table_alpha;
  h.msq_mask = c->msq_mask;
  h.n_field = field_len(c);
  h.n_lag = (uint64_t)kSpecies * c->G.cells;
  h.n_params = kMlpParams;
  h.n_rows = (uint64_t)c->nch * c->G.nodes;
  h.n_chan = (uint64_t)c->nch;
  const size_t need = sizeof(Header) + payload_bytes(h);
  if (!buf) {
    *bytes = need;
    return QGBE_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(QGBE_EINVAL, "checkpoint buffer too small");
  }
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  auto out = [&](const void* src, size_t n) -> hipError_t {
    hipError_t e = hipMemcpyAsync(p, src, n, hipMemcpyDeviceToHost, c->stream);
    p += n;
    return e;
  };
  HIP_TRY(out(c->d_f, h.n_field * sizeof(double)), "copy f");
  if (h.has_lag) HIP_TRY(out(c->d_lag, h.n_lag * sizeof(double)), "copy lagged masses");
  if (h.has_weights) {
    HIP_TRY(out(c->mlp.params, h.n_params * sizeof(float)), "copy weights");
    HIP_TRY(out(c->mlp.m, h.n_params * sizeof(float)), "copy adam m");
    HIP_TRY(out(c->mlp.v, h.n_params * sizeof(float)), "copy adam v");
  }
  if (h.K > 0) {
    const size_t rk = h.n_rows * h.K;
    HIP_TRY(out(c->d_thr, rk * sizeof(uint32_t)), "copy thresholds");
    HIP_TRY(out(c->d_mu, rk * 5 * sizeof(float)), "copy locations");
    HIP_TRY(out(c->d_sigma, rk * 5 * sizeof(float)), "copy scales");
    HIP_TRY(out(c->d_mix_on, h.n_chan), "copy channel samplers");
  }
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  if (h.msq_mask) std::memcpy(p, &c->msq, sizeof(MsqTable));
  *bytes = need;
  return QGBE_OK;
}

qgbe_status qgbe_restore(qgbe_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf) return fail(QGBE_EINVAL, "NULL argument");
  if (bytes < sizeof(Header)) return fail(QGBE_EINVAL, "checkpoint truncated");
  Header h;
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0 || h.header_bytes != sizeof(Header) ||
      h.version != kVersion)
    return fail(QGBE_EINVAL, "not a checkpoint of this library version");
  if (!same_grid(h, c->d)) return fail(QGBE_EINVAL, "checkpoint belongs to a different grid or configuration");
  if (h.n_field != field_len(c) || h.n_lag != (uint64_t)kSpecies * c->G.cells || h.n_params != kMlpParams ||
      h.n_rows != (uint64_t)c->nch * c->G.nodes || h.n_chan != (uint64_t)c->nch || h.K < 0 || h.K > 16)
    return fail(QGBE_EINVAL, "checkpoint sizes do not match the context");
  if (h.msq_mask & ~0xFEu) return fail(QGBE_EINVAL, "checkpoint has a bad matrix-element mask");
  if (bytes < sizeof(Header) + payload_bytes(h)) return fail(QGBE_EINVAL, "checkpoint truncated");
  MsqTable msq{};
  if (h.msq_mask) {
    std::memcpy(&msq, static_cast<const char*>(buf) + sizeof(Header) + payload_bytes(h) - sizeof(MsqTable),
                sizeof(MsqTable));
    for (int r = 1; r <= 7; ++r) {
      const int n = ((h.msq_mask >> r) & 1u) ? msq.n[r] : 0;
      if (n < 0 || n > kMsqMaxTerms || (((h.msq_mask >> r) & 1u) && n == 0))
        return fail(QGBE_EINVAL, "checkpoint has bad matrix-element terms");
    }
  }
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  if (h.has_weights) {
    qgbe_status s = qgbe_proposal_set_weights(c, reinterpret_cast<const float*>(
                                                     static_cast<const char*>(buf) + sizeof(Header) +
                                                     h.n_field * sizeof(double) +
                                                     (h.has_lag ? h.n_lag * sizeof(double) : 0)),
                                              (int64_t)h.n_params);
    if (s) return s;
  }
  const char* p = static_cast<const char*>(buf) + sizeof h;
  auto in = [&](void* dst, size_t n) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dst, p, n, hipMemcpyHostToDevice, c->stream);
    p += n;
    return e;
  };
  HIP_TRY(in(c->d_f, h.n_field * sizeof(double)), "copy f");
  // the second buffer of f too: a step updates only the evolving species
  HIP_TRY(hipMemcpyAsync(c->d_f_next, c->d_f, h.n_field * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
          "copy f to the second buffer");
  HIP_TRY(launch_to_f32(c->d_f, c->d_f32, h.n_field, c->stream), "f to fp32");
  if (h.has_lag) HIP_TRY(in(c->d_lag, h.n_lag * sizeof(double)), "copy lagged masses");
  if (h.has_weights) {
    p += h.n_params * sizeof(float);  // the master weights went in above (with their BF16 copy)
    HIP_TRY(in(c->mlp.m, h.n_params * sizeof(float)), "copy adam m");
    HIP_TRY(in(c->mlp.v, h.n_params * sizeof(float)), "copy adam v");
  }
  if (!h.has_weights) c->mlp.has_weights = false;
  if (h.K == 0) c->K = 0;
  if (h.K > 0) {
    qgbe_status s = install_proposal_table(c, h.K);
    if (s) return s;
    const size_t rk = h.n_rows * h.K;
    HIP_TRY(in(c->d_thr, rk * sizeof(uint32_t)), "copy thresholds");
    HIP_TRY(in(c->d_mu, rk * 5 * sizeof(float)), "copy locations");
    HIP_TRY(in(c->d_sigma, rk * 5 * sizeof(float)), "copy scales");
    HIP_TRY(in(c->d_mix_on, h.n_chan), "copy channel samplers");
  }
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  // the user matrix elements in force when the checkpoint was taken (rows
  // without user terms evaluate Table I)
  c->msq = msq;
  c->msq_mask = h.msq_mask;
  HIP_TRY(hipMemcpyAsync(c->d_msq, &c->msq, sizeof(MsqTable), hipMemcpyHostToDevice, c->stream),
          "copy matrix elements");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  c->step = h.step;
  c->has_lag = h.has_lag != 0;
  c->masses_valid = false;
  c->mlp.adam_t = h.has_weights ? h.adam_t : c->mlp.adam_t;
  c->table_net = h.K > 0 && h.table_net && h.has_weights;
  c->table_alpha = h.table_alpha;
  if (c->table_net) {
    qgbe_status s = ensure_proposal_features(c);
    if (s) return s;
  }
  return QGBE_OK;
}

}  // extern "C"
