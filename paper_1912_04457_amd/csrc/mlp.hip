// The learned proposal's network on the matrix cores.
//
// x (8) -> Linear 8x128 -> SiLU -> Linear 128x128 -> SiLU -> Linear 128x88
// (head: 8 mixture logits, 8x5 locations, 8x5 log scales in logit space).
// Every product, forward and backward, is a BF16 x BF16 -> FP32 MFMA GEMM
// (v_mfma_f32_16x16x32_bf16) with strided operands, so transposed operands of
// the backward pass need no copies.  Master weights and Adam moments are FP32.
#include <hip/hip_runtime.h>

#include "mlp.h"

namespace qgbe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;    // block tile (M and N)
constexpr int kKStep = 32;   // K per MFMA
constexpr int kThreads = 256;

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C[M x N] = A[M x K] B[K x N] (+ bias[N]); A(m,k) = A[m*ars + k*acs],
// B(k,n) = B[k*brs + n*bcs].  Epilogue: z -> Cz (FP32, optional),
// act(z) -> Cb (BF16, optional) and/or Cf (FP32, optional), all with ldc.
// Wave w of the block owns the 32x32 sub-tile (w/2, w%2): 2x2 MFMA tiles.
__global__ __launch_bounds__(kThreads) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __bf16 As[kTile][kKStep];   // [m][k]
  __shared__ __bf16 Bs[kTile][kKStep];   // [n][k] (transposed for k-contiguous reads)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool split = g.k_chunk > 0;
  const int k_begin = split ? blockIdx.z * g.k_chunk : 0;
  const int k_end = split ? min(g.K, k_begin + g.k_chunk) : g.K;
  floatx4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = k_begin; k0 < k_end; k0 += kKStep) {
    // stage the tiles (zero outside the matrices)
    for (int e = tid; e < kTile * kKStep; e += kThreads) {
      const int r = e / kKStep, k = e % kKStep;
      const int gm = m0 + r, gn = n0 + r, gk = k0 + k;
      As[r][k] = (gm < g.M && gk < k_end) ? g.A[(size_t)gm * g.ars + (size_t)gk * g.acs] : (__bf16)0.0f;
      Bs[r][k] = (gn < g.N && gk < k_end) ? g.B[(size_t)gk * g.brs + (size_t)gn * g.bcs] : (__bf16)0.0f;
    }
    __syncthreads();
    // operand fragments: lane l holds row (l%16) and k = 8*(l/16) .. +7
    const int r = lane & 15, kq = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i)
      for (int q = 0; q < 8; ++q) {
        a[i][q] = As[wm + i * 16 + r][kq + q];
        b[i][q] = Bs[wn + i * 16 + r][kq + q];
      }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // result fragment: lane l holds column (l%16), rows 4*(l/16) .. +3
  const int c = lane & 15, rq = (lane >> 4) * 4;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + i * 16 + rq + q, gn = n0 + wn + j * 16 + c;
        if (gm >= g.M || gn >= g.N) continue;
        if (split) {  // a partial product over this workgroup's K chunk
          atomicAdd(&g.Cf[(size_t)gm * g.ldc + gn], acc[i][j][q]);
          continue;
        }
        float z = acc[i][j][q];
        if (g.bias) z += g.bias[gn];
        if (g.accumulate) z += g.Cf[(size_t)gm * g.ldc + gn];
        if (g.Cz) g.Cz[(size_t)gm * g.ldc + gn] = z;
        const float h = g.silu ? silu_f(z) : z;
        if (g.Cf) g.Cf[(size_t)gm * g.ldc + gn] = h;
        if (g.Cb) g.Cb[(size_t)gm * g.ldc + gn] = (__bf16)h;
      }
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ src, __bf16* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (__bf16)src[i];
}

// dZ = dH * silu'(Z), FP32 and BF16 copies
__global__ void silu_backward_kernel(const float* __restrict__ dH, const float* __restrict__ Z,
                                     float* __restrict__ dZ, __bf16* __restrict__ dZb, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float v = dH[i] * dsilu_f(Z[i]);
    dZ[i] = v;
    dZb[i] = (__bf16)v;
  }
}

// out[n] += sum over rows of M[row][n] (column sums for the bias gradients).
// A workgroup sums a chunk of kColsumRows rows of 64 columns: four row phases
// of 64 lanes, combined in LDS, one atomic per column.
constexpr int kColsumRows = 64;
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ M, int rows, int cols,
                                                     float* __restrict__ out) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * kColsumRows, r1 = min(rows, r0 + kColsumRows);
  float s = 0.f;
  if (n < cols)
    for (int r = r0 + ph; r < r1; r += 4) s += M[(size_t)r * cols + n];
  part[ph][lane] = s;
  __syncthreads();
  if (ph == 0 && n < cols) atomicAdd(&out[n], (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
}

__global__ void sum_kernel(const float* __restrict__ w, int stride, int rows, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) s += w[(size_t)r * stride];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, sh[0] + sh[1] + sh[2] + sh[3]);
}

// Weighted NLL of the mixture head per row: loss += -w L / W, dY.
// y and w are read from `yw` with row stride `yws` (y at 0..4, w at 5).
__global__ void nll_kernel(const float* __restrict__ Y, const float* __restrict__ yw, int yws, int rows,
                           const double* __restrict__ wsum, float* __restrict__ dY, __bf16* __restrict__ dYb,
                           double* loss) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  double part = 0.0;  // this row's loss term; summed over the wave before the atomic
  if (r < rows) {
    const float* h = Y + (size_t)r * kMlpOut;
    const float* yr = yw + (size_t)r * yws;
    const float s = (float)((double)yr[kMixD] / *wsum);
    float mx = -INFINITY;
    for (int k = 0; k < kMixK; ++k) mx = fmaxf(mx, h[k]);
    float se = 0.f;
    for (int k = 0; k < kMixK; ++k) se += __expf(h[k] - mx);
    const float lse_a = mx + __logf(se);
    float lk[kMixK];
    float z[kMixK][kMixD];
    float m2 = -INFINITY;
    for (int k = 0; k < kMixK; ++k) {
      float l = h[k] - lse_a;
      for (int d = 0; d < kMixD; ++d) {
        const float lr = h[kMixK + kMixK * kMixD + k * kMixD + d];
        const float ls = fminf(fmaxf(lr, kLsMin), kLsMax);
        const float zz = (yr[d] - h[kMixK + k * kMixD + d]) * __expf(-ls);
        z[k][d] = zz;
        l += -0.5f * zz * zz - ls - 0.91893853320467274f;
      }
      lk[k] = l;
      m2 = fmaxf(m2, l);
    }
    float se2 = 0.f;
    for (int k = 0; k < kMixK; ++k) se2 += __expf(lk[k] - m2);
    const float L = m2 + __logf(se2);
    part = -(double)s * (double)L;
    float* g = dY + (size_t)r * kMlpOut;
    __bf16* gb = dYb + (size_t)r * kMlpOut;
    for (int k = 0; k < kMixK; ++k) {
      const float resp = __expf(lk[k] - L);
      const float pi = __expf(h[k] - lse_a);
      const float ga = -s * (resp - pi);
      g[k] = ga;
      gb[k] = (__bf16)ga;
      for (int d = 0; d < kMixD; ++d) {
        const float lr = h[kMixK + kMixK * kMixD + k * kMixD + d];
        const float ls = fminf(fmaxf(lr, kLsMin), kLsMax);
        const float gmu = -s * resp * z[k][d] * __expf(-ls);
        float gls = -s * resp * (z[k][d] * z[k][d] - 1.0f);
        if (lr < kLsMin || lr > kLsMax) gls = 0.f;
        const int im = kMixK + k * kMixD + d, il = kMixK + kMixK * kMixD + k * kMixD + d;
        g[im] = gmu;
        gb[im] = (__bf16)gmu;
        g[il] = gls;
        gb[il] = (__bf16)gls;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, part);
}

// Adam (bias-corrected) on the FP32 master weights; refresh the BF16 copies.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, __bf16* __restrict__ pb, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mi = b1 * m[i] + (1.f - b1) * g[i];
  const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  const float w = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = w;
  pb[i] = (__bf16)w;
}

// Inference straight to the proposal table: each wave takes 16-row blocks of
// X through the network (layer 1 on the vector ALUs, K = 8; layers 2 and 3 on
// the matrix cores with the block's weights staged in LDS, transposed so the
// K index is contiguous) and turns its head rows into table rows; the
// activations never leave LDS.  Numerics as the staged GEMMs: BF16 inputs,
// weights and hidden activations, FP32 accumulation and head.
constexpr int kInfWaves = 4;
constexpr int kHPad = kMlpHidden + 8;     // row stride of the hidden tile (bank spread)
constexpr int kOutPad = 96;               // head columns rounded up to MFMA tiles
constexpr int kYPad = kMlpOut + 4;

__global__ __launch_bounds__(kInfWaves * 64) void mlp_table_kernel(const float* __restrict__ X, int rows,
                                                                    const __bf16* __restrict__ pb,
                                                                    const float* __restrict__ P, float alpha,
                                                                    uint32_t* __restrict__ thr, float* __restrict__ mu,
                                                                    float* __restrict__ sigma) {
  __shared__ __bf16 W2t[kMlpHidden][kHPad];   // [n][k]
  __shared__ __bf16 W3t[kOutPad][kHPad];      // [n][k], rows >= 88 zero
  __shared__ float W1s[kMlpIn][kMlpHidden];
  __shared__ float bias[2 * kMlpHidden + kMlpOut];
  __shared__ float Xs[kInfWaves][16][kMlpIn];
  __shared__ __bf16 H[kInfWaves][16][kHPad];
  __shared__ float Ys[kInfWaves][16][kYPad];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < kMlpHidden * kMlpHidden; e += blockDim.x) {
    const int k = e / kMlpHidden, n = e % kMlpHidden;
    W2t[n][k] = pb[kOffW2 + e];
  }
  for (int e = tid; e < kOutPad * kMlpHidden; e += blockDim.x) {
    const int n = e / kMlpHidden, k = e % kMlpHidden;
    W3t[n][k] = n < kMlpOut ? pb[kOffW3 + k * kMlpOut + n] : (__bf16)0.0f;
  }
  for (int e = tid; e < kMlpIn * kMlpHidden; e += blockDim.x) W1s[e / kMlpHidden][e % kMlpHidden] = (float)pb[kOffW1 + e];
  for (int e = tid; e < kMlpHidden; e += blockDim.x) {
    bias[e] = P[kOffB1 + e];
    bias[kMlpHidden + e] = P[kOffB2 + e];
  }
  for (int e = tid; e < kMlpOut; e += blockDim.x) bias[2 * kMlpHidden + e] = P[kOffB3 + e];
  __syncthreads();
  const int n_blocks = (rows + 15) / 16;
  const int r16 = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  for (int t = blockIdx.x * kInfWaves + w; t < n_blocks; t += gridDim.x * kInfWaves) {
    const int row0 = t * 16;
    // inputs, rounded to BF16 like the staged path
    for (int e = lane; e < 16 * kMlpIn; e += 64) {
      const int r = e / kMlpIn, c = e % kMlpIn;
      Xs[w][r][c] = row0 + r < rows ? (float)(__bf16)X[(size_t)(row0 + r) * kMlpIn + c] : 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 1: lane owns columns lane and lane + 64
    for (int h = 0; h < 2; ++h) {
      const int n = lane + 64 * h;
      float wcol[kMlpIn];
      for (int k = 0; k < kMlpIn; ++k) wcol[k] = W1s[k][n];
      for (int r = 0; r < 16; ++r) {
        float z = bias[n];
        for (int k = 0; k < kMlpIn; ++k) z = fmaf(Xs[w][r][k], wcol[k], z);
        H[w][r][n] = (__bf16)silu_f(z);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layers 2 and 3 on the matrix cores
    for (int layer = 0; layer < 2; ++layer) {
      bf16x8 a[kMlpHidden / kKStep];
      for (int ks = 0; ks < kMlpHidden / kKStep; ++ks)
        for (int q = 0; q < 8; ++q) a[ks][q] = H[w][r16][ks * kKStep + kq + q];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int n_tiles = layer == 0 ? kMlpHidden / 16 : kOutPad / 16;
      for (int j = 0; j < n_tiles; ++j) {
        floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < kMlpHidden / kKStep; ++ks) {
          bf16x8 b;
          for (int q = 0; q < 8; ++q)
            b[q] = layer == 0 ? W2t[j * 16 + r16][ks * kKStep + kq + q] : W3t[j * 16 + r16][ks * kKStep + kq + q];
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b, acc, 0, 0, 0);
        }
        const int c = j * 16 + r16;
        for (int q = 0; q < 4; ++q) {
          if (layer == 0) {
            H[w][rq + q][c] = (__bf16)silu_f(acc[q] + bias[kMlpHidden + c]);
          } else if (c < kMlpOut) {
            Ys[w][rq + q][c] = acc[q] + bias[2 * kMlpHidden + c];
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // head -> table: four lanes per row; lane part 0 also forms the thresholds
    const int r = lane >> 2, part = lane & 3;
    const int row = row0 + r;
    if (row < rows) {
      const float* h = Ys[w][r];
      if (part == 0) {
        double mx = -1e300;
        for (int k = 0; k < kMixK; ++k) mx = fmax(mx, (double)h[k]);
        double e[kMixK], se = 0.0;
        for (int k = 0; k < kMixK; ++k) { e[k] = exp((double)h[k] - mx); se += e[k]; }
        double cum = 0.0;
        for (int k = 0; k < kMixK; ++k) {
          const double lo = (double)alpha + (1.0 - (double)alpha) * cum;
          double tt = floor(lo * 4294967296.0);
          tt = tt > 4294967295.0 ? 4294967295.0 : tt;
          thr[(size_t)row * kMixK + k] = (uint32_t)tt;
          cum += e[k] / se;
        }
      }
      for (int k = part; k < kMixK; k += 4)
        for (int d = 0; d < kMixD; ++d) {
          mu[((size_t)row * kMixK + k) * kMixD + d] = h[kMixK + k * kMixD + d];
          const float lr = h[kMixK + kMixK * kMixD + k * kMixD + d];
          sigma[((size_t)row * kMixK + k) * kMixD + d] = expf(fminf(fmaxf(lr, kLsMin), kLsMax));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Per-species thermal mass squared averaged over the cells (one workgroup per
// species, fixed summation order).
__global__ void mass_mean_kernel(Grid G, const double* __restrict__ mass2, double* __restrict__ mean) {
  __shared__ double part[256];
  const int sp = blockIdx.x;
  double s = 0.0;
  for (int x = threadIdx.x; x < G.cells; x += blockDim.x) s += mass2[sp * G.cells + x];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[sp] = part[0] / G.cells;
}

// Conditioning inputs of every (channel, node) row; the masses are the
// per-species values in mass7 (cell averages), so one table serves all cells.
__global__ void features_kernel(Grid G, const Channel* __restrict__ chans, int nch, const double* __restrict__ mass7,
                                float* __restrict__ X) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nch * G.nodes) return;
  const int ci = r / G.nodes, node = r % G.nodes;
  const int iz = node % G.np[2], iy = (node / G.np[2]) % G.np[1], ix = node / (G.np[2] * G.np[1]);
  const double p[3] = {node_coord(G.ph[0], G.dp[0], ix), node_coord(G.ph[1], G.dp[1], iy),
                       node_coord(G.ph[2], G.dp[2], iz)};
  const double pn = sqrt(G.ph[0] * G.ph[0] + G.ph[1] * G.ph[1] + G.ph[2] * G.ph[2]);
  const int sp = chans[ci].sp[0];
  const double a = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  const double E1 = sqrt(a * a + mass7[sp]);
  float* x = X + (size_t)r * kMlpIn;
  x[0] = (float)(p[0] / G.ph[0]);
  x[1] = (float)(p[1] / G.ph[1]);
  x[2] = (float)(p[2] / G.ph[2]);
  x[3] = (float)(a / pn);
  x[4] = (float)(E1 / pn);
  x[5] = (float)(mass7[kGluon] / (pn * pn));
  x[6] = (float)(sp / 3.0 - 1.0);
  x[7] = nch > 1 ? (float)(2.0 * ci / (nch - 1) - 1.0) : 0.0f;
}

// Gather rows idx[i] of the recorded samples into a minibatch: X (FP32 and
// BF16) and the (y, w) block.
__global__ void gather_kernel(const float* __restrict__ rows, const int* __restrict__ idx, int n, float* __restrict__ X,
                              __bf16* __restrict__ Xb, float* __restrict__ yw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* src = rows + (size_t)idx[i] * kRecordWidth;
  for (int c = 0; c < kMlpIn; ++c) {
    X[(size_t)i * kMlpIn + c] = src[c];
    Xb[(size_t)i * kMlpIn + c] = (__bf16)src[c];
  }
  for (int c = 0; c < kMixD + 1; ++c) yw[(size_t)i * (kMixD + 1) + c] = src[kMlpIn + c];
}

unsigned blocks_for(size_t n, int t = 256) {
  size_t b = (n + t - 1) / t;
  return (unsigned)(b > 65535 ? 65535 : (b ? b : 1));
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.k_chunk < 0 || g.k_chunk % kKStep) return hipErrorInvalidValue;
  if (g.k_chunk > 0 && (!g.Cf || g.bias || g.silu || g.Cz || g.Cb)) return hipErrorInvalidValue;
  const int chunks = g.k_chunk > 0 ? (g.K + g.k_chunk - 1) / g.k_chunk : 1;
  dim3 grid((g.N + kTile - 1) / kTile, (g.M + kTile - 1) / kTile, chunks);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(kThreads), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* src, __bf16* dst, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_silu_backward(const float* dH, const float* Z, float* dZ, __bf16* dZb, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(silu_backward_kernel, dim3(blocks_for(n)), dim3(256), 0, st, dH, Z, dZ, dZb, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* M, int rows, int cols, float* out, hipStream_t st) {
  dim3 grid((cols + 63) / 64, (rows + kColsumRows - 1) / kColsumRows);
  hipLaunchKernelGGL(colsum_kernel, grid, dim3(256), 0, st, M, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_sum(const float* w, int stride, int rows, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_kernel, dim3(blocks_for(rows) > 256 ? 256 : blocks_for(rows)), dim3(256), 0, st, w, stride,
                     rows, out);
  return hipGetLastError();
}

hipError_t launch_nll(const float* Y, const float* yw, int yws, int rows, const double* wsum, float* dY, __bf16* dYb,
                      double* loss, hipStream_t st) {
  hipLaunchKernelGGL(nll_kernel, dim3((rows + 127) / 128), dim3(128), 0, st, Y, yw, yws, rows, wsum, dY, dYb, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, __bf16* pb, int n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, pb, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_features(const Grid& G, const Channel* chans, int nch, const double* mass2, double* mass7, float* X,
                           hipStream_t st) {
  hipLaunchKernelGGL(mass_mean_kernel, dim3(kSpecies), dim3(256), 0, st, G, mass2, mass7);
  const int rows = nch * G.nodes;
  if (rows > 0)
    hipLaunchKernelGGL(features_kernel, dim3((rows + 127) / 128), dim3(128), 0, st, G, chans, nch, mass7, X);
  return hipGetLastError();
}

hipError_t launch_mlp_table(const float* X, int rows, const __bf16* pb, const float* P, float alpha, uint32_t* thr,
                            float* mu, float* sigma, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int n_blocks = (rows + 15) / 16;
  int grid = (n_blocks + kInfWaves - 1) / kInfWaves;
  grid = grid > 512 ? 512 : grid;
  hipLaunchKernelGGL(mlp_table_kernel, dim3(grid), dim3(kInfWaves * 64), 0, st, X, rows, pb, P, alpha, thr, mu, sigma);
  return hipGetLastError();
}

hipError_t launch_gather(const float* rows, const int* idx, int n, float* X, __bf16* Xb, float* yw, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, dim3((n + 127) / 128), dim3(128), 0, st, rows, idx, n, X, Xb, yw);
  return hipGetLastError();
}

}  // namespace qgbe
