// Launch interface of the proposal network kernels (BF16 MFMA GEMMs and the
// mixture head).
#pragma once

#include "qgbe_common.h"

namespace qgbe {

constexpr int kMlpIn = 8;
constexpr int kMlpHidden = 128;
constexpr int kMixK = 8;
constexpr int kMixD = 5;
constexpr int kMlpOut = kMixK * (1 + 2 * kMixD);    // 88
constexpr float kLsMin = -7.0f, kLsMax = 3.0f;       // clamp of the log scales
constexpr int kRecordWidth = kMlpIn + kMixD + 1;     // x[8], y[5], |g|
// flat parameter layout: W1 [8][128], b1, W2 [128][128], b2, W3 [128][88], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;

struct GemmArgs {
  int M, N, K;
  const __bf16* A;
  long long ars, acs;      // A(m,k) = A[m*ars + k*acs]
  const __bf16* B;
  long long brs, bcs;      // B(k,n) = B[k*brs + n*bcs]
  const float* bias;       // [N] or null
  int silu;                // apply SiLU in the epilogue
  int accumulate;          // add the existing Cf
  float* Cz;               // pre-activation (FP32) or null
  float* Cf;               // activation (FP32) or null
  __bf16* Cb;              // activation (BF16) or null
  long long ldc;
  int k_chunk;             // > 0: split K into chunks of this many (a multiple of 32), one
                           // workgroup per (tile, chunk), partial products added into Cf with
                           // FP32 atomics (Cf zeroed or holding what to add to; no epilogue)
};

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);
hipError_t launch_f32_to_bf16(const float* src, __bf16* dst, size_t n, hipStream_t st);
hipError_t launch_silu_backward(const float* dH, const float* Z, float* dZ, __bf16* dZb, size_t n, hipStream_t st);
hipError_t launch_colsum(const float* M, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_sum(const float* w, int stride, int rows, double* out, hipStream_t st);
hipError_t launch_nll(const float* Y, const float* yw, int yws, int rows, const double* wsum, float* dY, __bf16* dYb,
                      double* loss, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, __bf16* pb, int n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t st);
// Conditioning features of every (channel, node) row from the cell-averaged
// masses; mass7 receives those 7 averages.
hipError_t launch_features(const Grid& G, const Channel* chans, int nch, const double* mass2, double* mass7, float* X,
                           hipStream_t st);
// Network forward on X [rows][8] straight into the proposal table (thr, mu,
// sigma in the layout of qgbe_set_proposal_table), activations kept on chip.
hipError_t launch_mlp_table(const float* X, int rows, const __bf16* pb, const float* P, float alpha, uint32_t* thr,
                            float* mu, float* sigma, hipStream_t st);
hipError_t launch_gather(const float* rows, const int* idx, int n, float* X, __bf16* Xb, float* yw, hipStream_t st);

}  // namespace qgbe
