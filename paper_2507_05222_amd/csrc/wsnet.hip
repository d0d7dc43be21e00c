// Learned warm start of the pressure solve: a four-layer 3x3 convolutional
// network on the 64 x 64 coarse grid (rows: eta, zero padding; columns: xi,
// periodic padding), 3 -> 32 -> 32 -> 32 -> 1 channels, the taps of layer l spaced
// DIL[l] = 1, 2, 4, 8 apart (receptive field 31 x 31), tanh after the first
// three layers. Training in FP32 (forward, backward, Adam); the forward pass can
// round its operands to BF16 (FP32 accumulation) for inference.
//
// Parameter layout (floats): for each layer l = 0..3, weights w_l[co][ci][3][3]
// followed by the bias b_l[co].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/qtt.h"

namespace {

constexpr int H = 64, Wd = 64, HW = H * Wd;
constexpr int CIN[4] = {3, 32, 32, 32};
constexpr int COUT[4] = {32, 32, 32, 1};
constexpr int DIL[4] = {1, 2, 4, 8};

__host__ __device__ constexpr int wsize(int l) { return (l == 0 ? 3 : 32) * (l == 3 ? 1 : 32) * 9; }
__host__ __device__ constexpr int bsize(int l) { return l == 3 ? 1 : 32; }
__host__ __device__ constexpr int woff(int l) {
  return l == 0 ? 0 : woff(l - 1) + wsize(l - 1) + bsize(l - 1);
}
static_assert(woff(3) + wsize(3) + bsize(3) == QTT_WS_NPARAMS, "parameter count");

__device__ __forceinline__ float rbf16(float x) {   // round to nearest even BF16, back to FP32
  const uint32_t u = __float_as_uint(x);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(r & 0xFFFF0000u);
}

// out[b][co][i][j] = act(bias[co] + sum_{ci,di,dj} w[co][ci][di][dj] in[b][ci][i+d(di-1)][(j+d(dj-1)) mod 64])
// one thread per output pixel; grid (HW / 256, cout, B)
template <bool BF>
__global__ void __launch_bounds__(256) k_conv_fwd(const float* __restrict__ in, int cin, const float* __restrict__ w,
                                                   const float* __restrict__ bias, int cout, int act, int d,
                                                   float* __restrict__ out) {
  extern __shared__ float ws[];                       // weights of this output channel: cin * 9
  const int co = blockIdx.y, b = blockIdx.z;
  for (int t = threadIdx.x; t < cin * 9; t += blockDim.x) {
    const float v = w[(size_t)co * cin * 9 + t];
    ws[t] = BF ? rbf16(v) : v;
  }
  __syncthreads();
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= HW) return;
  const int i = pix / Wd, j = pix % Wd;
  float acc = bias[co];
  const float* ib = in + (size_t)b * cin * HW;
  for (int ci = 0; ci < cin; ++ci) {
    const float* ip = ib + (size_t)ci * HW;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = i + d * (di - 1);
      if (ii < 0 || ii >= H) continue;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        const int jj = (j + d * (dj - 1) + Wd) % Wd;
        const float x = ip[ii * Wd + jj];
        acc += ws[ci * 9 + di * 3 + dj] * (BF ? rbf16(x) : x);
      }
    }
  }
  out[((size_t)b * cout + co) * HW + pix] = act ? tanhf(acc) : acc;
}

// g_act = g_out * (1 - y^2) for tanh layers (in place on g)
__global__ void k_tanh_bwd(float* __restrict__ g, const float* __restrict__ y, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    g[e] *= 1.0f - y[e] * y[e];
}

// gradient of the weights and bias of one layer: one workgroup per (co, ci),
// the nine tap sums over (b, i, j) by a fixed-order block reduction
__global__ void __launch_bounds__(256) k_conv_bwd_w(const float* __restrict__ in, int cin, const float* __restrict__ g,
                                                     int cout, int B, int d, float* __restrict__ gw,
                                                     float* __restrict__ gb) {
  const int co = blockIdx.x, ci = blockIdx.y;
  float s[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) s[t] = 0.f;
  for (int e = threadIdx.x; e < B * HW; e += blockDim.x) {
    const int b = e / HW, pix = e % HW, i = pix / Wd, j = pix % Wd;
    const float gv = g[((size_t)b * cout + co) * HW + pix];
    const float* ip = in + ((size_t)b * cin + ci) * HW;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = i + d * (di - 1);
      const bool ok = ii >= 0 && ii < H;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        const int jj = (j + d * (dj - 1) + Wd) % Wd;
        s[di * 3 + dj] += ok ? gv * ip[ii * Wd + jj] : 0.f;
      }
    }
    s[9] += gv;
  }
  __shared__ float red[10][256];
#pragma unroll
  for (int t = 0; t < 10; ++t) red[t][threadIdx.x] = s[t];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int t = 0; t < 10; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 9) gw[((size_t)co * cin + ci) * 9 + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 9 && ci == 0) gb[co] = red[9][0];
}

// gradient of the input: gin[b][ci][i][j] = sum_{co,di,dj} w[co][ci][di][dj] g[b][co][i-d(di-1)][j-d(dj-1)]
// (the transposed stencil with the same padding rules); grid (HW / 256, cin, B)
__global__ void __launch_bounds__(256) k_conv_bwd_x(const float* __restrict__ g, int cout, const float* __restrict__ w,
                                                     int cin, int d, float* __restrict__ gin) {
  const int ci = blockIdx.y, b = blockIdx.z;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= HW) return;
  const int i = pix / Wd, j = pix % Wd;
  float acc = 0.f;
  for (int co = 0; co < cout; ++co) {
    const float* gp = g + ((size_t)b * cout + co) * HW;
    const float* wp = w + ((size_t)co * cin + ci) * 9;
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int oi = i - d * (di - 1);
      if (oi < 0 || oi >= H) continue;
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        const int oj = (j - d * (dj - 1) + Wd) % Wd;
        acc += wp[di * 3 + dj] * gp[oi * Wd + oj];
      }
    }
  }
  gin[((size_t)b * cin + ci) * HW + pix] = acc;
}

// Adam (Kingma & Ba 2015) with bias correction; t is the 1-based step count
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float gv = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gv;
    const float vv = b2 * v[e] + (1.f - b2) * gv * gv;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// d(mean squared error)/d(out) = 2 (out - target) / n, and the per-block partial
// sums of the squared error (fixed order)
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ out, const float* __restrict__ tgt, int n,
                                              float* __restrict__ gout, float* __restrict__ part) {
  __shared__ float red[256];
  float s = 0.f;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float d = out[e] - tgt[e];
    gout[e] = 2.f * d / (float)n;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

inline size_t act_floats(int B) { return (size_t)B * (32 + 32 + 32) * HW; }

}  // namespace

namespace qtt_solver_detail {
int set_error(qtt_ctx* ctx, int code, const char* msg);
}

extern "C" size_t qtt_ws_act_floats(int batch) { return batch > 0 ? act_floats(batch) : 0; }

extern "C" int qtt_ws_forward(qtt_ctx* ctx, const float* params, const float* in, int batch, float* acts, float* out,
                              int bf16, void* stream) {
  using qtt_solver_detail::set_error;
  if (!ctx) return QTT_EINVAL;
  if (!params || !in || !acts || !out || batch < 1 || batch > 4096) return set_error(ctx, QTT_EINVAL, "ws_forward: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const float* x = in;
  for (int l = 0; l < 4; ++l) {
    float* y = (l < 3) ? acts + (size_t)batch * 32 * HW * l : out;
    const float* w = params + woff(l);
    const float* b = w + wsize(l);
    dim3 grid(HW / 256, COUT[l], batch);
    const size_t lds = (size_t)CIN[l] * 9 * sizeof(float);
    if (bf16)
      hipLaunchKernelGGL(k_conv_fwd<true>, grid, dim3(256), lds, s, x, CIN[l], w, b, COUT[l], l < 3 ? 1 : 0, DIL[l], y);
    else
      hipLaunchKernelGGL(k_conv_fwd<false>, grid, dim3(256), lds, s, x, CIN[l], w, b, COUT[l], l < 3 ? 1 : 0, DIL[l], y);
    x = y;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  return QTT_OK;
}

extern "C" int qtt_ws_backward(qtt_ctx* ctx, const float* params, const float* in, int batch, float* acts,
                               float* gout, float* grads, float* scratch, void* stream) {
  using qtt_solver_detail::set_error;
  if (!ctx) return QTT_EINVAL;
  if (!params || !in || !acts || !gout || !grads || !scratch || batch < 1 || batch > 4096)
    return set_error(ctx, QTT_EINVAL, "ws_backward: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  // g holds dL/d(pre-activation output) of the current layer; scratch holds the
  // gradient propagated to its input (ping-pong between scratch halves)
  float* g = gout;
  float* bufs[2] = {scratch, scratch + (size_t)batch * 32 * HW};
  for (int l = 3; l >= 0; --l) {
    const float* xin = (l == 0) ? in : acts + (size_t)batch * 32 * HW * (l - 1);
    const float* w = params + woff(l);
    float* gw = grads + woff(l);
    float* gb = gw + wsize(l);
    hipLaunchKernelGGL(k_conv_bwd_w, dim3(COUT[l], CIN[l]), dim3(256), 0, s, xin, CIN[l], g, COUT[l], batch, DIL[l],
                       gw, gb);
    if (l > 0) {
      float* gin = bufs[l & 1];
      hipLaunchKernelGGL(k_conv_bwd_x, dim3(HW / 256, CIN[l], batch), dim3(256), 0, s, g, COUT[l], w, CIN[l], DIL[l],
                         gin);
      const size_t n = (size_t)batch * 32 * HW;
      hipLaunchKernelGGL(k_tanh_bwd, dim3(1024), dim3(256), 0, s, gin, acts + (size_t)batch * 32 * HW * (l - 1), n);
      g = gin;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  return QTT_OK;
}

extern "C" int qtt_ws_mse(qtt_ctx* ctx, const float* out, const float* target, int n, float* gout, float* partial,
                          void* stream) {
  using qtt_solver_detail::set_error;
  if (!ctx) return QTT_EINVAL;
  if (!out || !target || !gout || !partial || n < 1) return set_error(ctx, QTT_EINVAL, "ws_mse: bad arguments");
  hipLaunchKernelGGL(k_mse, dim3(QTT_WS_MSE_BLOCKS), dim3(256), 0, (hipStream_t)stream, out, target, n, gout, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  return QTT_OK;
}

extern "C" int qtt_ws_adam_step(qtt_ctx* ctx, float* params, const float* grads, float* m, float* v, int step, float lr,
                                void* stream) {
  using qtt_solver_detail::set_error;
  if (!ctx) return QTT_EINVAL;
  if (!params || !grads || !m || !v || step < 1 || !(lr > 0.f)) return set_error(ctx, QTT_EINVAL, "ws_adam: bad arguments");
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(80), dim3(256), 0, (hipStream_t)stream, params, grads, m, v, QTT_WS_NPARAMS, lr, b1,
                     b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  return QTT_OK;
}
