// Per-group opening angle chosen by a small network (12 -> 64 -> 64 -> 1).
//
// The paper uses one theta for every particle and studies how it trades
// accuracy for work (Sec. 3.5, Table "theta").  Here each group gets its own theta from 12
// features that describe how it sits in the surrounding mass (c members,
// c_g box centre, R box half-diagonal, x_g and m_g the members' centre of mass
// and mass, A1 the smallest cell with at least two sub-cells (not a bucket)
// that holds more than c particles, A2 the next such cell above it, A1 again
// at the root):
//   f0 = log2 c, f1 = log2(1 + R/eps), f2 = |x_g - c_g| / (R + eps),
//   f3 = log2(l(A1) / (R + eps)), f4 = log2(m(A1) / m_g),
//   f5 = |com(A1) - c_g| / l(A1), f11 = log2(m(A2) / m_g),
// and, from the group's interaction list at theta = 1 (the probe walk) with
// d = com - c_g over the entries outside the box (the probe walk, one wave per
// group, computes all twelve):
//   f6 = log2(|sum m d / (d^2 + eps^2)^1.5| + 2^-100),
//   f7 = log2(sum m / (d^2 + eps^2) + 2^-100),
//   f8 = log2(1 + single particles outside the box), f9 = log2(list length),
//   f10 = log2(mass of the entries inside the box / m_g); then
//   theta = 0.3 + 0.7 sigmoid(w3 . tanh(W2 tanh(W1 x' + b1) + b2) + b3 + shift),
// x' = (x - mu) / sigma.  Inference runs on the matrix cores in bfloat16
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation); training runs in FP32 with
// explicit forward, backward and Adam kernels, gradients summed over the
// batch in a fixed order.
//
// Parameters: one FP32 vector W1 [64][12], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3 [1].
#include <algorithm>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kIn = 12, kHid = 64;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kHid;
static_assert(oB3 + 1 == kMlpParams, "parameter layout");

// ---- inference (bfloat16 matrix cores) --------------------------------------

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ short to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float sigmoid_theta(float y) {
  return kThetaMin + kThetaSpan / (1.0f + expf(-y));
}

// One wave per tile of 16 rows.  Operand layout of the 16x16x16 product
// (wave64): lane l holds A[l % 16][4 (l / 16) + v] and B[4 (l / 16) + v][l % 16]
// for v = 0..3, and the result D[4 (l / 16) + v][l % 16].
__global__ __launch_bounds__(kWave) void k_mlp_infer(const float *__restrict__ P, const float *__restrict__ mu,
                                                     const float *__restrict__ sigma, const float *__restrict__ x,
                                                     int64_t rows_host, const DevInfo *__restrict__ info, float shift,
                                                     float *__restrict__ theta) {
  __shared__ short h1[16][kHid + 4];
  const int lane = lane_id();
  const int col = lane & 15, kb = lane >> 4;
  const int64_t rows = rows_host >= 0 ? rows_host : (int64_t)info->n_groups;
  const int64_t tiles = (rows + 15) / 16;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t row = t * 16 + col;
    bf16x4 ax;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 4 * kb + v;
      float xv = 0.0f;
      if (k < kIn && row < rows) xv = (x[row * kIn + k] - mu[k]) / sigma[k];
      ax[v] = (k < kIn) ? to_bf16(xv) : (short)0;
    }
    // layer 1: 4 column blocks of 16 hidden units
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int j = 16 * nb + col;
      bf16x4 bw;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 4 * kb + v;
        bw[v] = (k < kIn) ? to_bf16(P[oW1 + j * kIn + k]) : (short)0;
      }
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ax, bw, z, 0, 0, 0);
      const float b = P[oB1 + j];
#pragma unroll
      for (int v = 0; v < 4; ++v) h1[4 * kb + v][j] = to_bf16(tanhf(z[v] + b));
    }
    __syncthreads();
    // layer 2 and the output layer
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int j = 16 * nb + col;
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x4 ah, bw;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = 16 * ks + 4 * kb + v;
          ah[v] = h1[col][k];
          bw[v] = to_bf16(P[oW2 + j * kHid + k]);
        }
        z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bw, z, 0, 0, 0);
      }
      const float b = P[oB2 + j], w = P[oW3 + j];
#pragma unroll
      for (int v = 0; v < 4; ++v) part[v] += w * tanhf(z[v] + b);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) part[v] += __shfl_xor(part[v], d, kWave);
    }
    if (col == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = t * 16 + 4 * kb + v;
        if (r < rows) theta[r] = sigmoid_theta(part[v] + P[oB3] + shift);
      }
    }
    __syncthreads();
  }
}

// ---- training (FP32) ----------------------------------------------------------

// Sum of the sample weights (one block, fixed order).
__global__ void k_weight_sum(const float *__restrict__ w, int B, float *__restrict__ out) {
  __shared__ float s[256];
  float acc = 0.0f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) acc += w[b];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// Forward and backward through the activations, one thread per sample.
__global__ void k_mlp_fwd_bwd(const float *__restrict__ P, const float *__restrict__ mu,
                              const float *__restrict__ sigma, const float *__restrict__ x,
                              const float *__restrict__ target, const float *__restrict__ w,
                              const float *__restrict__ wsum, int B, MlpWork ws) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float xn[kIn], h1[kHid], h2[kHid];
#pragma unroll
  for (int k = 0; k < kIn; ++k) {
    xn[k] = (x[(int64_t)b * kIn + k] - mu[k]) / sigma[k];
    ws.xn[(int64_t)b * kIn + k] = xn[k];
  }
  for (int j = 0; j < kHid; ++j) {
    float z = P[oB1 + j];
#pragma unroll
    for (int k = 0; k < kIn; ++k) z += P[oW1 + j * kIn + k] * xn[k];
    h1[j] = tanhf(z);
    ws.h1[(int64_t)b * kHid + j] = h1[j];
  }
  float y = P[oB3];
  for (int j = 0; j < kHid; ++j) {
    float z = P[oB2 + j];
    for (int k = 0; k < kHid; ++k) z += P[oW2 + j * kHid + k] * h1[k];
    h2[j] = tanhf(z);
    ws.h2[(int64_t)b * kHid + j] = h2[j];
    y += P[oW3 + j] * h2[j];
  }
  const float sg = 1.0f / (1.0f + expf(-y));
  const float th = kThetaMin + kThetaSpan * sg;
  const float W = *wsum;
  const float r = th - target[b];
  ws.loss[b] = w[b] * r * r / W;
  const float dy = (2.0f * w[b] * r / W) * kThetaSpan * sg * (1.0f - sg);
  ws.dy[b] = dy;
  float dz2[kHid];
  for (int j = 0; j < kHid; ++j) {
    dz2[j] = dy * P[oW3 + j] * (1.0f - h2[j] * h2[j]);
    ws.dz2[(int64_t)b * kHid + j] = dz2[j];
  }
  for (int k = 0; k < kHid; ++k) {
    float s = 0.0f;
    for (int j = 0; j < kHid; ++j) s += dz2[j] * P[oW2 + j * kHid + k];
    ws.dz1[(int64_t)b * kHid + k] = s * (1.0f - h1[k] * h1[k]);
  }
}

// Gradient of one parameter per thread: a sum over the batch in sample order.
__global__ void k_mlp_grad(int B, MlpWork ws, float *__restrict__ grad, float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float s = 0.0f;
  if (p == kMlpParams) {
    for (int b = 0; b < B; ++b) s += ws.loss[b];
    if (loss) *loss = s;
    return;
  }
  if (p < oB1) {
    const int j = p / kIn, k = p % kIn;
    for (int b = 0; b < B; ++b) s += ws.dz1[(int64_t)b * kHid + j] * ws.xn[(int64_t)b * kIn + k];
  } else if (p < oW2) {
    const int j = p - oB1;
    for (int b = 0; b < B; ++b) s += ws.dz1[(int64_t)b * kHid + j];
  } else if (p < oB2) {
    const int j = (p - oW2) / kHid, k = (p - oW2) % kHid;
    for (int b = 0; b < B; ++b) s += ws.dz2[(int64_t)b * kHid + j] * ws.h1[(int64_t)b * kHid + k];
  } else if (p < oW3) {
    const int j = p - oB2;
    for (int b = 0; b < B; ++b) s += ws.dz2[(int64_t)b * kHid + j];
  } else if (p < oB3) {
    const int j = p - oW3;
    for (int b = 0; b < B; ++b) s += ws.dy[b] * ws.h2[(int64_t)b * kHid + j];
  } else {
    for (int b = 0; b < B; ++b) s += ws.dy[b];
  }
  grad[p] = s;
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace


void mlp_infer_device(const float *params, const float *mu, const float *sigma, const float *x, int64_t rows,
                      int64_t cap_rows, const DevInfo *info, float shift, float *theta, hipStream_t s) {
  const int64_t tiles = (cap_rows + 15) / 16;
  if (tiles <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(tiles, 4096);
  k_mlp_infer<<<grid, kWave, 0, s>>>(params, mu, sigma, x, rows, info, shift, theta);
}

void mlp_grad_device(const float *params, const float *mu, const float *sigma, int B, const float *x,
                     const float *target, const float *w, MlpWork ws, float *grad, float *loss, hipStream_t s) {
  k_weight_sum<<<1, 256, 0, s>>>(w, B, ws.wsum);
  k_mlp_fwd_bwd<<<(unsigned)((B + 63) / 64), 64, 0, s>>>(params, mu, sigma, x, target, w, ws.wsum, B, ws);
  k_mlp_grad<<<(unsigned)((kMlpParams + 1 + 255) / 256), 256, 0, s>>>(B, ws, grad, loss);
}

void adam_device(float *params, const float *grad, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(params, grad, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace bh
