// The (p, q) selector network on the GPU: forward pass, backward pass with
// the binary cross-entropy loss, and the Adam update, in FP32 with every sum
// taken in a fixed order (deterministic).
//
// Network 16 -> 64 (ReLU) -> 64 (ReLU) -> 40 logits, parameters in one flat
// vector: W1 (64 x 16 row-major), b1, W2 (64 x 64), b2, W3 (40 x 64), b3.
// Loss: mean over the entries with mask 1 of max(z,0) - z y + log(1 + e^-|z|).
// Adam: Kingma and Ba (ICLR 2015), bias-corrected.
#include "internal.hpp"

namespace rsvd {

constexpr int kIn = 16, kHid = 64, kOut = 40;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid, kNParam = oB3 + kOut;
static_assert(kNParam == 7848, "parameter count");

// One wave per item (4 items per 256-thread block); lane o computes unit o of each layer.
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* __restrict__ th, int B, const float* __restrict__ X,
                                                      float* __restrict__ H1, float* __restrict__ H2,
                                                      float* __restrict__ Z) {
  __shared__ float xs[4][kIn];
  __shared__ float h1s[4][kHid];
  __shared__ float h2s[4][kHid];
  const int w = threadIdx.x >> 6, o = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + w;
  const bool ok = b < B;
  if (ok && o < kIn) xs[w][o] = X[(int64_t)b * kIn + o];
  __syncthreads();
  float a = th[oB1 + o];
#pragma unroll
  for (int i = 0; i < kIn; ++i) a += th[oW1 + o * kIn + i] * xs[w][i];
  a = fmaxf(a, 0.f);
  h1s[w][o] = a;
  if (ok) H1[(int64_t)b * kHid + o] = a;
  __syncthreads();
  a = th[oB2 + o];
  for (int j = 0; j < kHid; ++j) a += th[oW2 + o * kHid + j] * h1s[w][j];
  a = fmaxf(a, 0.f);
  h2s[w][o] = a;
  if (ok) H2[(int64_t)b * kHid + o] = a;
  __syncthreads();
  if (o < kOut) {
    a = th[oB3 + o];
    for (int j = 0; j < kHid; ++j) a += th[oW3 + o * kHid + j] * h2s[w][j];
    if (ok) Z[(int64_t)b * kOut + o] = a;
  }
}

// loss[0] = masked mean BCE, loss[1] = number of entries with mask 1 (one block, fixed order).
__global__ __launch_bounds__(256) void mlp_loss_kernel(int B, const float* __restrict__ Z, const float* __restrict__ Y,
                                                       const float* __restrict__ M, float* __restrict__ loss) {
  __shared__ double red[2][4];
  double s = 0.0, c = 0.0;
  const int64_t tot = (int64_t)B * kOut;
  for (int64_t t = threadIdx.x; t < tot; t += 256) {
    const double z = Z[t], y = Y[t], m = M[t];
    s += m * (fmax(z, 0.0) - z * y + log1p(exp(-fabs(z))));
    c += m;
  }
  s = wave_sum(s);
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = s; red[1][threadIdx.x >> 6] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double S = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double C = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    loss[0] = (float)(S / fmax(C, 1.0));
    loss[1] = (float)C;
  }
}

// Per item: dZ = (sigmoid(z) - y) m / count, dH2 = (W3^T dZ) (h2 > 0), dH1 = (W2^T dH2) (h1 > 0).
__global__ __launch_bounds__(256) void mlp_bwd_item_kernel(const float* __restrict__ th, int B,
                                                           const float* __restrict__ H1, const float* __restrict__ H2,
                                                           const float* __restrict__ Z, const float* __restrict__ Y,
                                                           const float* __restrict__ M, const float* __restrict__ loss,
                                                           float* __restrict__ dZ, float* __restrict__ dH2,
                                                           float* __restrict__ dH1) {
  __shared__ float dzs[4][kOut];
  __shared__ float dh2s[4][kHid];
  const int w = threadIdx.x >> 6, o = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + w;
  const bool ok = b < B;
  const float inv = 1.f / fmaxf(loss[1], 1.f);
  if (o < kOut) {
    float g = 0.f;
    if (ok) {
      const int64_t t = (int64_t)b * kOut + o;
      g = (1.f / (1.f + expf(-Z[t])) - Y[t]) * M[t] * inv;
      dZ[t] = g;
    }
    dzs[w][o] = g;
  }
  __syncthreads();
  float a = 0.f;
  for (int j = 0; j < kOut; ++j) a += th[oW3 + j * kHid + o] * dzs[w][j];
  const float h2 = ok ? H2[(int64_t)b * kHid + o] : 0.f;
  a = h2 > 0.f ? a : 0.f;
  dh2s[w][o] = a;
  if (ok) dH2[(int64_t)b * kHid + o] = a;
  __syncthreads();
  a = 0.f;
  for (int j = 0; j < kHid; ++j) a += th[oW2 + j * kHid + o] * dh2s[w][j];
  const float h1 = ok ? H1[(int64_t)b * kHid + o] : 0.f;
  a = h1 > 0.f ? a : 0.f;
  if (ok) dH1[(int64_t)b * kHid + o] = a;
}

// One thread per parameter: the sum over the batch, item by item in order.
__global__ __launch_bounds__(256) void mlp_bwd_param_kernel(int B, const float* __restrict__ X,
                                                            const float* __restrict__ H1,
                                                            const float* __restrict__ H2,
                                                            const float* __restrict__ dZ,
                                                            const float* __restrict__ dH2,
                                                            const float* __restrict__ dH1, float* __restrict__ grad) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= kNParam) return;
  const float *D, *IN;
  int nd, ni, o, i;   // gradient (o, i) of a weight matrix; i < 0 for a bias
  if (t < oB1) { D = dH1; nd = kHid; IN = X; ni = kIn; o = t / kIn; i = t % kIn; }
  else if (t < oW2) { D = dH1; nd = kHid; IN = nullptr; ni = 0; o = t - oB1; i = -1; }
  else if (t < oB2) { D = dH2; nd = kHid; IN = H1; ni = kHid; o = (t - oW2) / kHid; i = (t - oW2) % kHid; }
  else if (t < oW3) { D = dH2; nd = kHid; IN = nullptr; ni = 0; o = t - oB2; i = -1; }
  else if (t < oB3) { D = dZ; nd = kOut; IN = H2; ni = kHid; o = (t - oW3) / kHid; i = (t - oW3) % kHid; }
  else { D = dZ; nd = kOut; IN = nullptr; ni = 0; o = t - oB3; i = -1; }
  float a = 0.f;
  if (i >= 0)
    for (int b = 0; b < B; ++b) a += D[(int64_t)b * nd + o] * IN[(int64_t)b * ni + i];
  else
    for (int b = 0; b < B; ++b) a += D[(int64_t)b * nd + o];
  grad[t] = a;
}

__global__ void adam_kernel(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.f - b1) * gi;
  const float vi = b2 * v[t] + (1.f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  th[t] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void sel_features_kernel(const double* __restrict__ sigma, int k, float* __restrict__ x) {
  const int i = threadIdx.x;
  if (i < 15) {
    const double s0 = sigma[0];
    const double r = s0 > 0.0 ? sigma[i + 1] / s0 : 0.0;
    x[i] = (float)(log10(fmax(r, 1e-12)) / 6.0);
  } else if (i == 15) {
    x[15] = (float)(log10((double)k) / 3.0);
  }
}

hipError_t launch_sel_features(const double* sigma, int k, float* x, hipStream_t s) {
  hipLaunchKernelGGL(sel_features_kernel, dim3(1), dim3(64), 0, s, sigma, k, x);
  return hipGetLastError();
}

int mlp_param_count() { return kNParam; }

hipError_t launch_mlp_forward(const float* th, int B, const float* X, float* H1, float* H2, float* Z, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, th, B, X, H1, H2, Z);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* th, int B, const float* X, const float* H1, const float* H2,
                               const float* Z, const float* Y, const float* M, float* grad, float* loss,
                               float* scratch, hipStream_t s) {
  float* dZ = scratch;
  float* dH2 = dZ + (size_t)B * kOut;
  float* dH1 = dH2 + (size_t)B * kHid;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, B, Z, Y, M, loss);
  hipLaunchKernelGGL(mlp_bwd_item_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, th, B, H1, H2, Z, Y, M,
                     loss, dZ, dH2, dH1);
  hipLaunchKernelGGL(mlp_bwd_param_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, s, B, X, H1, H2, dZ, dH2, dH1,
                     grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* th, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, step)));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, th, g, m, v, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace rsvd
