// C ABI of the learned proposal: network weights, forward and backward
// passes, training with Adam, the proposal table, and the sample recorder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "context.h"

using namespace qgbe;

namespace {

constexpr int kBatch = QGBE_MLP_BATCH;
static_assert(QGBE_MLP_PARAMS == kMlpParams, "header and kernels disagree on the parameter count");

qgbe_status mlp_ensure(qgbe_ctx* c) {
  MlpState& m = c->mlp;
  if (m.ready) return QGBE_OK;
  qgbe_status s = QGBE_OK;
#define MA(p, n, what) \
  if (!s) s = dev_alloc(c, &(p), (size_t)(n), what)
  MA(m.params, kMlpParams, "mlp params");
  MA(m.m, kMlpParams, "adam m");
  MA(m.v, kMlpParams, "adam v");
  MA(m.grad, kMlpParams, "mlp grad");
  MA(m.pb, kMlpParams, "mlp bf16 params");
  MA(m.X, (size_t)kBatch * kMlpIn, "mlp X");
  MA(m.Xb, (size_t)kBatch * kMlpIn, "mlp X bf16");
  MA(m.Z1, (size_t)kBatch * kMlpHidden, "mlp Z1");
  MA(m.H1b, (size_t)kBatch * kMlpHidden, "mlp H1");
  MA(m.Z2, (size_t)kBatch * kMlpHidden, "mlp Z2");
  MA(m.H2b, (size_t)kBatch * kMlpHidden, "mlp H2");
  MA(m.Y, (size_t)kBatch * kMlpOut, "mlp Y");
  MA(m.dY, (size_t)kBatch * kMlpOut, "mlp dY");
  MA(m.dYb, (size_t)kBatch * kMlpOut, "mlp dY bf16");
  MA(m.dH, (size_t)kBatch * kMlpHidden, "mlp dH");
  MA(m.dZ, (size_t)kBatch * kMlpHidden, "mlp dZ");
  MA(m.dZb, (size_t)kBatch * kMlpHidden, "mlp dZ bf16");
  MA(m.yw, (size_t)kBatch * (kMixD + 1), "mlp yw");
  MA(m.scalars, 2, "mlp scalars");
#undef MA
  if (s) return s;
  m.ready = true;
  return QGBE_OK;
}

GemmArgs gemm(int M, int N, int K, const __bf16* A, long long ars, long long acs, const __bf16* B, long long brs,
              long long bcs) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.ars = ars; g.acs = acs;
  g.B = B; g.brs = brs; g.bcs = bcs;
  g.ldc = N;
  return g;
}

// Forward pass on rows already staged in m.Xb (BF16); head in m.Y (FP32).
qgbe_status forward_staged(qgbe_ctx* c, int rows) {
  MlpState& m = c->mlp;
  const float* P = m.params;
  GemmArgs g1 = gemm(rows, kMlpHidden, kMlpIn, m.Xb, kMlpIn, 1, m.pb + kOffW1, kMlpHidden, 1);
  g1.bias = P + kOffB1; g1.silu = 1; g1.Cz = m.Z1; g1.Cb = m.H1b;
  HIP_TRY(launch_gemm(g1, c->stream), "layer 1");
  GemmArgs g2 = gemm(rows, kMlpHidden, kMlpHidden, m.H1b, kMlpHidden, 1, m.pb + kOffW2, kMlpHidden, 1);
  g2.bias = P + kOffB2; g2.silu = 1; g2.Cz = m.Z2; g2.Cb = m.H2b;
  HIP_TRY(launch_gemm(g2, c->stream), "layer 2");
  GemmArgs g3 = gemm(rows, kMlpOut, kMlpHidden, m.H2b, kMlpHidden, 1, m.pb + kOffW3, kMlpOut, 1);
  g3.bias = P + kOffB3; g3.Cf = m.Y;
  HIP_TRY(launch_gemm(g3, c->stream), "layer 3");
  return QGBE_OK;
}

// The weight gradients reduce over the rows (K = rows, M x N <= 128 x 128):
// their K is split so that rows / 256 workgroups per tile share it.
constexpr int kGradChunk = 256;

// Loss and gradient for rows staged in m.Xb / m.yw; gradient in m.grad,
// loss in m.scalars[0] (accumulated).
qgbe_status loss_grad_staged(qgbe_ctx* c, int rows) {
  MlpState& m = c->mlp;
  qgbe_status s = forward_staged(c, rows);
  if (s) return s;
  HIP_TRY(hipMemsetAsync(m.scalars + 1, 0, sizeof(double), c->stream), "zero weight sum");
  HIP_TRY(launch_sum(m.yw + kMixD, kMixD + 1, rows, m.scalars + 1, c->stream), "weight sum");
  HIP_TRY(launch_nll(m.Y, m.yw, kMixD + 1, rows, m.scalars + 1, m.dY, m.dYb, m.scalars, c->stream), "nll");
  HIP_TRY(hipMemsetAsync(m.grad, 0, kMlpParams * sizeof(float), c->stream), "zero grad");
  // layer 3: dW3 = H2^T dY, db3 = colsum dY, dH2 = dY W3^T
  GemmArgs w3 = gemm(kMlpHidden, kMlpOut, rows, m.H2b, 1, kMlpHidden, m.dYb, kMlpOut, 1);
  w3.Cf = m.grad + kOffW3; w3.k_chunk = kGradChunk;
  HIP_TRY(launch_gemm(w3, c->stream), "dW3");
  HIP_TRY(launch_colsum(m.dY, rows, kMlpOut, m.grad + kOffB3, c->stream), "db3");
  GemmArgs h2 = gemm(rows, kMlpHidden, kMlpOut, m.dYb, kMlpOut, 1, m.pb + kOffW3, 1, kMlpOut);
  h2.Cf = m.dH;
  HIP_TRY(launch_gemm(h2, c->stream), "dH2");
  HIP_TRY(launch_silu_backward(m.dH, m.Z2, m.dZ, m.dZb, (size_t)rows * kMlpHidden, c->stream), "dZ2");
  // layer 2
  GemmArgs w2 = gemm(kMlpHidden, kMlpHidden, rows, m.H1b, 1, kMlpHidden, m.dZb, kMlpHidden, 1);
  w2.Cf = m.grad + kOffW2; w2.k_chunk = kGradChunk;
  HIP_TRY(launch_gemm(w2, c->stream), "dW2");
  HIP_TRY(launch_colsum(m.dZ, rows, kMlpHidden, m.grad + kOffB2, c->stream), "db2");
  GemmArgs h1 = gemm(rows, kMlpHidden, kMlpHidden, m.dZb, kMlpHidden, 1, m.pb + kOffW2, 1, kMlpHidden);
  h1.Cf = m.dH;
  HIP_TRY(launch_gemm(h1, c->stream), "dH1");
  HIP_TRY(launch_silu_backward(m.dH, m.Z1, m.dZ, m.dZb, (size_t)rows * kMlpHidden, c->stream), "dZ1");
  // layer 1
  GemmArgs w1 = gemm(kMlpIn, kMlpHidden, rows, m.Xb, 1, kMlpIn, m.dZb, kMlpHidden, 1);
  w1.Cf = m.grad + kOffW1; w1.k_chunk = kGradChunk;
  HIP_TRY(launch_gemm(w1, c->stream), "dW1");
  HIP_TRY(launch_colsum(m.dZ, rows, kMlpHidden, m.grad + kOffB1, c->stream), "db1");
  return QGBE_OK;
}

qgbe_status check_weights(qgbe_ctx* c) {
  if (!c->mlp.ready || !c->mlp.has_weights) return fail(QGBE_ESTATE, "proposal weights not set");
  return QGBE_OK;
}

qgbe_status ensure_masses(qgbe_ctx* c) {
  if (c->masses_valid) return QGBE_OK;
  return compute_masses(c);
}

}  // namespace

qgbe_status qgbe::install_proposal_table(qgbe_ctx* c, int K) {
  const size_t rows = (size_t)c->nch * c->G.nodes;
  if (c->d_thr && c->K == K) return QGBE_OK;
  (void)hipFree(c->d_thr);
  (void)hipFree(c->d_mu);
  (void)hipFree(c->d_sigma);
  c->d_thr = nullptr; c->d_mu = nullptr; c->d_sigma = nullptr; c->K = 0;
  qgbe_status s = dev_alloc(c, &c->d_thr, std::max<size_t>(1, rows * K), "proposal thresholds");
  if (!s) s = dev_alloc(c, &c->d_mu, std::max<size_t>(1, rows * K * 5), "proposal locations");
  if (!s) s = dev_alloc(c, &c->d_sigma, std::max<size_t>(1, rows * K * 5), "proposal scales");
  if (!s && !c->d_mix_on) s = dev_alloc(c, &c->d_mix_on, std::max(1, c->nch), "channel samplers");
  if (s) return s;
  c->K = K;
  return QGBE_OK;
}

qgbe_status qgbe::reset_channel_samplers(qgbe_ctx* c) {
  HIP_TRY(hipMemsetAsync(c->d_mix_on, 1, std::max(1, c->nch), c->stream), "channel samplers");
  return QGBE_OK;
}

qgbe_status qgbe::ensure_proposal_features(qgbe_ctx* c) {
  qgbe_status s = QGBE_OK;
  if (!c->d_feat) s = dev_alloc(c, &c->d_feat, std::max<size_t>(1, (size_t)c->nch * c->G.nodes) * kMlpIn, "features");
  if (!s && !c->d_mass7) s = dev_alloc(c, &c->d_mass7, kSpecies, "mean masses");
  return s;
}

// Features of the current (cell-averaged) masses -> network -> table, on the
// context's stream.  Needs the weights, the table buffers (K = kMixK) and the
// feature buffers in place.
qgbe_status qgbe::refresh_proposal_table(qgbe_ctx* c) {
  const int rows = c->nch * c->G.nodes;
  HIP_TRY(launch_features(c->G, c->d_chans, c->nch, c->d_mass2, c->d_mass7, c->d_feat, c->stream), "features");
  HIP_TRY(launch_mlp_table(c->d_feat, rows, c->mlp.pb, c->mlp.params, c->table_alpha, c->d_thr, c->d_mu, c->d_sigma,
                           c->stream), "proposal table");
  return QGBE_OK;
}

extern "C" {

qgbe_status qgbe_set_proposal_table(qgbe_ctx* c, int32_t K, const uint32_t* thr, const float* mu, const float* sigma,
                                    int32_t on_device) {
  if (!c || !thr || !mu || !sigma) return fail(QGBE_EINVAL, "NULL argument");
  if (K < 1 || K > 16) return fail(QGBE_EINVAL, "K must be in 1..16");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  qgbe_status s = install_proposal_table(c, K);
  if (s) return s;
  c->table_net = false;
  s = reset_channel_samplers(c);
  if (s) return s;
  const size_t rows = (size_t)c->nch * c->G.nodes;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(hipMemcpyAsync(c->d_thr, thr, rows * K * sizeof(uint32_t), kind, c->stream), "copy thresholds");
  HIP_TRY(hipMemcpyAsync(c->d_mu, mu, rows * K * 5 * sizeof(float), kind, c->stream), "copy locations");
  HIP_TRY(hipMemcpyAsync(c->d_sigma, sigma, rows * K * 5 * sizeof(float), kind, c->stream), "copy scales");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_get_proposal_table(qgbe_ctx* c, int32_t* K, uint32_t* thr, float* mu, float* sigma) {
  if (!c || !K) return fail(QGBE_EINVAL, "NULL argument");
  if (!c->K) return fail(QGBE_ESTATE, "no proposal table installed");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  *K = c->K;
  const size_t rows = (size_t)c->nch * c->G.nodes;
  if (thr) HIP_TRY(hipMemcpyAsync(thr, c->d_thr, rows * c->K * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream), "copy");
  if (mu) HIP_TRY(hipMemcpyAsync(mu, c->d_mu, rows * c->K * 5 * sizeof(float), hipMemcpyDeviceToHost, c->stream), "copy");
  if (sigma)
    HIP_TRY(hipMemcpyAsync(sigma, c->d_sigma, rows * c->K * 5 * sizeof(float), hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_proposal_set_weights(qgbe_ctx* c, const float* w, int64_t n) {
  if (!c || !w) return fail(QGBE_EINVAL, "NULL argument");
  if (n != kMlpParams) return fail(QGBE_EINVAL, "weight count must be QGBE_MLP_PARAMS");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  qgbe_status s = mlp_ensure(c);
  if (s) return s;
  MlpState& m = c->mlp;
  HIP_TRY(hipMemcpyAsync(m.params, w, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream), "copy weights");
  HIP_TRY(launch_f32_to_bf16(m.params, m.pb, kMlpParams, c->stream), "bf16 weights");
  HIP_TRY(hipMemsetAsync(m.m, 0, kMlpParams * sizeof(float), c->stream), "zero m");
  HIP_TRY(hipMemsetAsync(m.v, 0, kMlpParams * sizeof(float), c->stream), "zero v");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  m.adam_t = 0;
  m.has_weights = true;
  return QGBE_OK;
}

qgbe_status qgbe_proposal_get_weights(qgbe_ctx* c, float* w, int64_t n) {
  if (!c || !w) return fail(QGBE_EINVAL, "NULL argument");
  if (n != kMlpParams) return fail(QGBE_EINVAL, "weight count must be QGBE_MLP_PARAMS");
  qgbe_status s = check_weights(c);
  if (s) return s;
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(w, c->mlp.params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_mlp_forward(qgbe_ctx* c, const float* X, int64_t rows, float* Y, int32_t on_device) {
  if (!c || !X || !Y) return fail(QGBE_EINVAL, "NULL argument");
  if (rows < 0) return fail(QGBE_EINVAL, "rows must be >= 0");
  qgbe_status s = check_weights(c);
  if (s) return s;
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  MlpState& m = c->mlp;
  const hipMemcpyKind in = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind out = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int64_t r0 = 0; r0 < rows; r0 += kBatch) {
    const int nr = (int)std::min<int64_t>(kBatch, rows - r0);
    HIP_TRY(hipMemcpyAsync(m.X, X + r0 * kMlpIn, (size_t)nr * kMlpIn * sizeof(float), in, c->stream), "copy X");
    HIP_TRY(launch_f32_to_bf16(m.X, m.Xb, (size_t)nr * kMlpIn, c->stream), "X to bf16");
    s = forward_staged(c, nr);
    if (s) return s;
    HIP_TRY(hipMemcpyAsync(Y + r0 * kMlpOut, m.Y, (size_t)nr * kMlpOut * sizeof(float), out, c->stream), "copy Y");
  }
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_mlp_loss_grad(qgbe_ctx* c, const float* X, const float* yw, int64_t rows, float* grad, double* loss,
                               int32_t on_device) {
  if (!c || !X || !yw || !grad || !loss) return fail(QGBE_EINVAL, "NULL argument");
  if (rows < 1 || rows > kBatch) return fail(QGBE_EINVAL, "rows must be in 1..QGBE_MLP_BATCH");
  qgbe_status s = check_weights(c);
  if (s) return s;
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  MlpState& m = c->mlp;
  const hipMemcpyKind in = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(hipMemcpyAsync(m.X, X, (size_t)rows * kMlpIn * sizeof(float), in, c->stream), "copy X");
  HIP_TRY(hipMemcpyAsync(m.yw, yw, (size_t)rows * (kMixD + 1) * sizeof(float), in, c->stream), "copy yw");
  HIP_TRY(launch_f32_to_bf16(m.X, m.Xb, (size_t)rows * kMlpIn, c->stream), "X to bf16");
  HIP_TRY(hipMemsetAsync(m.scalars, 0, sizeof(double), c->stream), "zero loss");
  s = loss_grad_staged(c, (int)rows);
  if (s) return s;
  HIP_TRY(hipMemcpyAsync(grad, m.grad, kMlpParams * sizeof(float),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream), "copy grad");
  HIP_TRY(hipMemcpyAsync(loss, m.scalars, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy loss");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_proposal_features(qgbe_ctx* c, float* X, int32_t on_device) {
  if (!c || !X) return fail(QGBE_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  qgbe_status s = ensure_masses(c);
  if (!s) s = ensure_proposal_features(c);
  if (s) return s;
  const size_t rows = (size_t)c->nch * c->G.nodes;
  HIP_TRY(launch_features(c->G, c->d_chans, c->nch, c->d_mass2, c->d_mass7, c->d_feat, c->stream), "features");
  HIP_TRY(hipMemcpyAsync(X, c->d_feat, rows * kMlpIn * sizeof(float),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream), "copy features");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_record_samples(qgbe_ctx* c, int32_t n_per_item, int64_t item_stride, float* rows, int64_t max_rows,
                                int64_t* n_rows, int32_t on_device) {
  if (!c || !rows || !n_rows) return fail(QGBE_EINVAL, "NULL argument");
  if (n_per_item < 1 || item_stride < 1) return fail(QGBE_EINVAL, "n_per_item and item_stride must be >= 1");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  const long long items = (long long)c->G.cells * c->nch * c->G.nodes;
  const long long n_sel = (items + item_stride - 1) / item_stride;
  const long long total = n_sel * n_per_item;
  *n_rows = total;
  if (total > max_rows) return fail(QGBE_EINVAL, "rows buffer too small");
  if (total == 0) return QGBE_OK;
  qgbe_status s = ensure_masses(c);
  if (s) return s;
  float* dst = rows;
  if (!on_device) HIP_TRY(hipMalloc(&dst, (size_t)total * kRecordWidth * sizeof(float)), "record scratch");
  CollideArgs a = base_args(c, n_per_item, nullptr, nullptr, nullptr);
  hipError_t e = launch_record(a, n_per_item, item_stride, n_sel, dst, c->stream);
  if (e == hipSuccess && !on_device)
    e = hipMemcpyAsync(rows, dst, (size_t)total * kRecordWidth * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (!on_device) (void)hipFree(dst);
  if (e != hipSuccess) return hip_fail(e, "record samples");
  return QGBE_OK;
}

qgbe_status qgbe_proposal_build_table(qgbe_ctx* c, float alpha) {
  if (!c) return fail(QGBE_EINVAL, "NULL context");
  if (!(alpha > 0.0f && alpha < 1.0f)) return fail(QGBE_EINVAL, "alpha must be in (0,1)");
  qgbe_status s = check_weights(c);
  if (s) return s;
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  s = ensure_masses(c);
  if (!s) s = install_proposal_table(c, kMixK);
  if (!s) s = ensure_proposal_features(c);
  if (s) return s;
  c->table_alpha = alpha;
  c->table_net = true;
  s = reset_channel_samplers(c);
  if (!s) s = refresh_proposal_table(c);
  if (s) {
    c->table_net = false;
    return s;
  }
  HIP_TRY(hipStreamSynchronize(c->stream), "build proposal table");
  return QGBE_OK;
}

qgbe_status qgbe_set_channel_samplers(qgbe_ctx* c, const uint8_t* use_learned) {
  if (!c || !use_learned) return fail(QGBE_EINVAL, "NULL argument");
  if (!c->K) return fail(QGBE_ESTATE, "no proposal table installed");
  std::vector<uint8_t> v(std::max(1, c->nch), 1);
  for (int i = 0; i < c->nch; ++i) {
    if (use_learned[i] > 1) return fail(QGBE_EINVAL, "channel sampler flags must be 0 or 1");
    v[i] = use_learned[i];
  }
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(c->d_mix_on, v.data(), v.size(), hipMemcpyHostToDevice, c->stream), "copy flags");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_get_channel_samplers(qgbe_ctx* c, uint8_t* use_learned) {
  if (!c || !use_learned) return fail(QGBE_EINVAL, "NULL argument");
  if (!c->K) return fail(QGBE_ESTATE, "no proposal table installed");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(use_learned, c->d_mix_on, c->nch, hipMemcpyDeviceToHost, c->stream), "copy flags");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  return QGBE_OK;
}

qgbe_status qgbe_proposal_judge(qgbe_ctx* c, int32_t n_pilot, int32_t n_reps, uint8_t* use_learned,
                                double* ratio) {
  if (!c) return fail(QGBE_EINVAL, "NULL context");
  if (n_pilot < 2 || n_reps < 1) return fail(QGBE_EINVAL, "n_pilot >= 2 and n_reps >= 1 required");
  if (!c->K) return fail(QGBE_ESTATE, "no proposal table installed");
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  const int nch = std::max(1, c->nch);
  std::vector<double> var[2], h((size_t)kStripes * nch);
  double t_ms[2] = {0.0, 0.0};
  const uint32_t saved_step = c->step;
  qgbe_status s = reset_channel_samplers(c);
  for (int l = 0; l < 2 && !s; ++l) {
    var[l].assign(nch, 0.0);
    for (int r = 0; r < n_reps && !s; ++r) {
      // pilot draws use their own key range, apart from the run's steps
      c->step = 0xF0000000u + (uint32_t)r;
      qgbe_stats st;
      s = qgbe_collision_term_ex(c, n_pilot, l ? QGBE_SAMPLER_LEARNED : QGBE_SAMPLER_UNIFORM, c->d_A, 1, nullptr, &st);
      if (s) break;
      t_ms[l] += st.t_collide_ms;
      hipError_t e = hipMemcpyAsync(h.data(), c->d_chan_var, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                    c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) { s = hip_fail(e, "copy channel variances"); break; }
      for (int k = 0; k < kStripes; ++k)  // the stripes in order
        for (int ci = 0; ci < nch; ++ci) var[l][ci] += h[(size_t)k * nch + ci];
    }
  }
  c->step = saved_step;
  if (s) return s;
  // per channel: pooled variance of the item estimates x the sampler's pilot time
  std::vector<uint8_t> flags(nch, 1);
  for (int ci = 0; ci < c->nch; ++ci) {
    const double cost_u = var[0][ci] * t_ms[0], cost_l = var[1][ci] * t_ms[1];
    flags[ci] = (cost_u > 0.0 && cost_l < cost_u) ? 1 : 0;
    if (ratio) ratio[ci] = cost_u > 0.0 ? cost_l / cost_u : (cost_l > 0.0 ? INFINITY : 1.0);
  }
  HIP_TRY(hipMemcpyAsync(c->d_mix_on, flags.data(), flags.size(), hipMemcpyHostToDevice, c->stream), "copy flags");
  HIP_TRY(hipStreamSynchronize(c->stream), "synchronise");
  if (use_learned) std::memcpy(use_learned, flags.data(), c->nch);
  return QGBE_OK;
}

qgbe_status qgbe_train_proposal(qgbe_ctx* c, const float* rows, int64_t n, const qgbe_train_cfg* cfg,
                                double* epoch_loss, int32_t on_device) {
  if (!c || !rows || !cfg) return fail(QGBE_EINVAL, "NULL argument");
  if (n < 1) return fail(QGBE_EINVAL, "no training rows");
  if (cfg->epochs < 1 || cfg->batch < 1 || cfg->batch > kBatch) return fail(QGBE_EINVAL, "bad epochs or batch");
  if (!(cfg->lr > 0.0f) || !(cfg->lr_final >= 0.0f)) return fail(QGBE_EINVAL, "bad learning rate");
  if (!(cfg->alpha > 0.0f && cfg->alpha < 1.0f)) return fail(QGBE_EINVAL, "alpha must be in (0,1)");
  qgbe_status s = check_weights(c);
  if (s) return s;
  HIP_TRY(hipSetDevice(c->d.device), "hipSetDevice");
  MlpState& m = c->mlp;
  const float* d_rows = rows;
  float* owned = nullptr;
  if (!on_device) {
    HIP_TRY(hipMalloc(&owned, (size_t)n * kRecordWidth * sizeof(float)), "rows scratch");
    HIP_TRY(hipMemcpyAsync(owned, rows, (size_t)n * kRecordWidth * sizeof(float), hipMemcpyHostToDevice, c->stream),
            "copy rows");
    d_rows = owned;
  }
  // the epoch's row order goes to the device once per epoch (one copy, waited
  // for before the host shuffles again); each batch gathers its slice of it
  int* d_perm = nullptr;
  if (hipMalloc(&d_perm, (size_t)n * sizeof(int)) != hipSuccess) {
    if (owned) (void)hipFree(owned);
    return fail(QGBE_ENOMEM, "row order scratch");
  }
  std::mt19937_64 rng(cfg->seed);
  std::vector<int> perm((size_t)n);
  std::iota(perm.begin(), perm.end(), 0);
  const int steps_per_epoch = (int)((n + cfg->batch - 1) / cfg->batch);
  const long long total_steps = (long long)steps_per_epoch * cfg->epochs;
  long long step = 0;
  hipError_t e = hipSuccess;
  for (int ep = 0; ep < cfg->epochs && !s && e == hipSuccess; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    e = hipMemcpyAsync(d_perm, perm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m.scalars, 0, sizeof(double), c->stream);
    for (int b = 0; b < steps_per_epoch && !s && e == hipSuccess; ++b, ++step) {
      const int r0 = b * cfg->batch;
      const int nr = (int)std::min<int64_t>(cfg->batch, n - r0);
      e = launch_gather(d_rows, d_perm + r0, nr, m.X, m.Xb, m.yw, c->stream);
      if (e != hipSuccess) break;
      s = loss_grad_staged(c, nr);
      if (s) break;
      const double frac = total_steps > 1 ? (double)step / (double)(total_steps - 1) : 1.0;
      const float lr = (float)(cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + std::cos(kPi * frac)));
      m.adam_t += 1;
      e = launch_adam(m.params, m.grad, m.m, m.v, m.pb, kMlpParams, lr, 0.9f, 0.999f, 1e-8f, m.adam_t, c->stream);
    }
    if (!s && e == hipSuccess && epoch_loss) {
      double tot = 0.0;
      e = hipMemcpyAsync(&tot, m.scalars, sizeof(double), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      epoch_loss[ep] = tot / steps_per_epoch;
    }
  }
  // wait for the queued work before the scratch buffers go (also after an error)
  const hipError_t e_sync = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = e_sync;
  (void)hipFree(d_perm);
  if (owned) (void)hipFree(owned);
  if (s) return s;
  if (e != hipSuccess) return hip_fail(e, "train proposal");
  return qgbe_proposal_build_table(c, cfg->alpha);
}

}  // extern "C"
