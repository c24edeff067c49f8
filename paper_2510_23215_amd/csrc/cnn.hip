// The spectral-window network: forward (FP32 or BF16 storage, FP32 accumulation), backward and
// Adam in FP32.  Four layers: conv 3x3 6->16 (stride 1) + ReLU, conv 3x3 16->32 (stride 2) +
// ReLU, dense 2048->64 + ReLU, dense 64->3; zero padding 1; parameters in one flat array
// W1[16,6,3,3] b1 W2[32,16,3,3] b2 W3[64,2048] b3 W4[3,64] b4.  Every reduction runs in a fixed
// order (no atomics), so results are reproducible.
#include "cnn.h"
#include "stencil.h"

namespace scsf {

// ---------------------------------------------------------------- storage conversions
__device__ inline float ldf(const float *p) { return *p; }
__device__ inline float ldf(const uint16_t *p) { return __uint_as_float((uint32_t)(*p) << 16); }
__device__ inline void stf(float *p, float v) { *p = v; }
__device__ inline void stf(uint16_t *p, float v) {            // round to nearest even
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  *p = (uint16_t)(u >> 16);
}

__device__ inline float block_sum_f(float v, float *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  float t = 0.f;
  for (int w = 0; w < nw; ++w) t += sh[w];
  return t;
}

// ---------------------------------------------------------------- forward
template <typename T>
__global__ void conv_fwd_kernel(const T *__restrict__ x, const T *__restrict__ W,
                                const T *__restrict__ bias, T *__restrict__ y, int n, int ci,
                                int H, int Wd, int co, int stride) {
  const int Ho = (H - 1) / stride + 1, Wo = (Wd - 1) / stride + 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * co * Ho * Wo) return;
  const int wo = (int)(idx % Wo), ho = (int)((idx / Wo) % Ho);
  const int o = (int)((idx / ((int64_t)Wo * Ho)) % co), s = (int)(idx / ((int64_t)Wo * Ho * co));
  float acc = ldf(bias + o);
  for (int c = 0; c < ci; ++c) {
    const T *xc = x + ((int64_t)s * ci + c) * H * Wd;
    const T *wc = W + ((int64_t)o * ci + c) * 9;
    for (int kh = 0; kh < 3; ++kh) {
      const int ih = ho * stride - 1 + kh;
      if (ih < 0 || ih >= H) continue;
      for (int kw = 0; kw < 3; ++kw) {
        const int iw = wo * stride - 1 + kw;
        if (iw < 0 || iw >= Wd) continue;
        acc += ldf(wc + kh * 3 + kw) * ldf(xc + ih * Wd + iw);
      }
    }
  }
  stf(y + idx, fmaxf(acc, 0.f));                      // both convolutions are followed by ReLU
}

// one wavefront per output y[s, o]: its lanes read the weight row and the input row with
// coalesced loads, and a fixed shuffle tree sums the 64 partial products
template <typename T>
__global__ void __launch_bounds__(256) fc_fwd_kernel(const T *__restrict__ x,
                                                     const T *__restrict__ W,
                                                     const T *__restrict__ bias,
                                                     T *__restrict__ y, int n, int I, int O,
                                                     int relu) {
  const int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (idx >= (int64_t)n * O) return;                  // uniform over the wavefront
  const int o = (int)(idx % O), s = (int)(idx / O);
  const T *xs = x + (int64_t)s * I;
  const T *wo = W + (int64_t)o * I;
  float acc = 0.f;
  for (int i = lane; i < I; i += 64) acc += ldf(wo + i) * ldf(xs + i);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    acc += ldf(bias + o);
    stf(y + idx, relu ? fmaxf(acc, 0.f) : acc);
  }
}

template <typename T>
static hipError_t forward_t(const T *params, const T *x, int n, T *a1, T *a2, T *a3, T *y,
                            hipStream_t st) {
  const int64_t e1 = (int64_t)n * 16 * 256, e2 = (int64_t)n * 32 * 64;
  conv_fwd_kernel<T><<<(unsigned)ceil_div(e1, 256), 256, 0, st>>>(
      x, params + kW1, params + kB1, a1, n, 6, 16, 16, 16, 1);
  conv_fwd_kernel<T><<<(unsigned)ceil_div(e2, 256), 256, 0, st>>>(
      a1, params + kW2, params + kB2, a2, n, 16, 16, 16, 32, 2);
  fc_fwd_kernel<T><<<(unsigned)ceil_div((int64_t)n * 64 * 64, 256), 256, 0, st>>>(
      a2, params + kW3, params + kB3, a3, n, 2048, 64, 1);
  fc_fwd_kernel<T><<<(unsigned)ceil_div((int64_t)n * 3 * 64, 256), 256, 0, st>>>(
      a3, params + kW4, params + kB4, y, n, 64, 3, 0);
  return hipGetLastError();
}

hipError_t cnn_forward(const float *params, const float *x, int n, float *a1, float *a2,
                       float *a3, float *y, hipStream_t st) {
  return forward_t<float>(params, x, n, a1, a2, a3, y, st);
}

__global__ void to_bf16_kernel(const float *__restrict__ a, uint16_t *__restrict__ b, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) stf(b + i, a[i]);
}

__global__ void from_bf16_kernel(const uint16_t *__restrict__ a, float *__restrict__ b,
                                 int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = ldf(a + i);
}

hipError_t cnn_forward_bf16(const float *params, const float *x, int n, uint16_t *pbf,
                            uint16_t *xbf, uint16_t *a1, uint16_t *a2, uint16_t *a3, uint16_t *ybf,
                            float *y, hipStream_t st) {
  to_bf16_kernel<<<(unsigned)ceil_div(kNetParams, 256), 256, 0, st>>>(params, pbf, kNetParams);
  const int64_t xe = (int64_t)n * 6 * 256;
  to_bf16_kernel<<<(unsigned)ceil_div(xe, 256), 256, 0, st>>>(x, xbf, xe);
  hipError_t e = forward_t<uint16_t>(pbf, xbf, n, a1, a2, a3, ybf, st);
  if (e != hipSuccess) return e;
  from_bf16_kernel<<<(unsigned)ceil_div((int64_t)n * 3, 256), 256, 0, st>>>(ybf, y, (int64_t)n * 3);
  return hipGetLastError();
}

// ---------------------------------------------------------------- loss and backward (FP32)
// d = (y - t) / (3 n); loss = sum (y - t)^2 / (6 n)
__global__ void __launch_bounds__(1024) loss_kernel(const float *__restrict__ y,
                                                    const float *__restrict__ t, int n,
                                                    float *__restrict__ d,
                                                    double *__restrict__ loss) {
  __shared__ float sh[16];
  const int cnt = 3 * n;
  float acc = 0.f;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const float r = y[i] - t[i];
    d[i] = r / (float)cnt;
    acc += r * r;
  }
  acc = block_sum_f(acc, sh);
  if (threadIdx.x == 0) *loss = 0.5 * (double)acc / (double)cnt;
}

// dW[o, i] = sum_s dy[s, o] x[s, i]; db[o] = sum_s dy[s, o]  (thread per weight)
__global__ void fc_bwd_w_kernel(const float *__restrict__ x, const float *__restrict__ dy, int n,
                                int I, int O, float *__restrict__ dW, float *__restrict__ db) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)O * I) {
    const int i = (int)(idx % I), o = (int)(idx / I);
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += dy[(int64_t)s * O + o] * x[(int64_t)s * I + i];
    dW[idx] = acc;
  }
  if (idx < O) {
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += dy[(int64_t)s * O + idx];
    db[idx] = acc;
  }
}

// dx[s, i] = (sum_o W[o, i] dy[s, o]) * (a[s, i] > 0)
__global__ void fc_bwd_x_kernel(const float *__restrict__ W, const float *__restrict__ dy,
                                const float *__restrict__ a, int n, int I, int O,
                                float *__restrict__ dx) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * I) return;
  const int i = (int)(idx % I), s = (int)(idx / I);
  float acc = 0.f;
  for (int o = 0; o < O; ++o) acc += W[(int64_t)o * I + i] * dy[(int64_t)s * O + o];
  dx[idx] = (a[idx] > 0.f) ? acc : 0.f;
}

// one workgroup per weight (o, c, kh, kw), plus one per bias (blocks past co*ci*9)
__global__ void __launch_bounds__(256) conv_bwd_w_kernel(
    const float *__restrict__ x, const float *__restrict__ dy, int n, int ci, int H, int Wd,
    int co, int stride, float *__restrict__ dW, float *__restrict__ db) {
  __shared__ float sh[4];
  const int Ho = (H - 1) / stride + 1, Wo = (Wd - 1) / stride + 1;
  const int wid = blockIdx.x;
  const int nw = co * ci * 9;
  float acc = 0.f;
  if (wid < nw) {
    const int kw = wid % 3, kh = (wid / 3) % 3, c = (wid / 9) % ci, o = wid / (9 * ci);
    const int64_t tot = (int64_t)n * Ho * Wo;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
      const int wo = (int)(e % Wo), ho = (int)((e / Wo) % Ho), s = (int)(e / ((int64_t)Wo * Ho));
      const int ih = ho * stride - 1 + kh, iw = wo * stride - 1 + kw;
      if (ih < 0 || ih >= H || iw < 0 || iw >= Wd) continue;
      acc += dy[(((int64_t)s * co + o) * Ho + ho) * Wo + wo] *
             x[(((int64_t)s * ci + c) * H + ih) * Wd + iw];
    }
    acc = block_sum_f(acc, sh);
    if (threadIdx.x == 0) dW[wid] = acc;
  } else {
    const int o = wid - nw;
    const int64_t tot = (int64_t)n * Ho * Wo;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
      const int64_t hw = e % ((int64_t)Ho * Wo), s = e / ((int64_t)Ho * Wo);
      acc += dy[((int64_t)s * co + o) * Ho * Wo + hw];
    }
    acc = block_sum_f(acc, sh);
    if (threadIdx.x == 0) db[o] = acc;
  }
}

// dx[s, c, h, w] = (sum_{o, kh, kw} W[o, c, kh, kw] dy[s, o, ho, wo]) * (a > 0),
// where h = ho*stride - 1 + kh, w = wo*stride - 1 + kw
__global__ void conv_bwd_x_kernel(const float *__restrict__ W, const float *__restrict__ dy,
                                  const float *__restrict__ a, int n, int ci, int H, int Wd,
                                  int co, int stride, float *__restrict__ dx) {
  const int Ho = (H - 1) / stride + 1, Wo = (Wd - 1) / stride + 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * ci * H * Wd) return;
  const int w = (int)(idx % Wd), hh = (int)((idx / Wd) % H);
  const int c = (int)((idx / ((int64_t)Wd * H)) % ci), s = (int)(idx / ((int64_t)Wd * H * ci));
  float acc = 0.f;
  for (int o = 0; o < co; ++o) {
    for (int kh = 0; kh < 3; ++kh) {
      const int t = hh + 1 - kh;
      if (t < 0 || t % stride) continue;
      const int ho = t / stride;
      if (ho >= Ho) continue;
      for (int kw = 0; kw < 3; ++kw) {
        const int u = w + 1 - kw;
        if (u < 0 || u % stride) continue;
        const int wo = u / stride;
        if (wo >= Wo) continue;
        acc += W[(((int64_t)o * ci + c) * 3 + kh) * 3 + kw] *
               dy[(((int64_t)s * co + o) * Ho + ho) * Wo + wo];
      }
    }
  }
  dx[idx] = (a[idx] > 0.f) ? acc : 0.f;
}

hipError_t cnn_loss_grad(const float *params, const float *x, const float *t, int n, float *a1,
                         float *a2, float *a3, float *y, float *d, float *da3, float *da2,
                         float *da1, float *grad, double *loss, hipStream_t st) {
  hipError_t e = cnn_forward(params, x, n, a1, a2, a3, y, st);
  if (e != hipSuccess) return e;
  loss_kernel<<<1, 1024, 0, st>>>(y, t, n, d, loss);
  // dense 64 -> 3
  fc_bwd_w_kernel<<<(unsigned)ceil_div(3 * 64, 256), 256, 0, st>>>(a3, d, n, 64, 3, grad + kW4,
                                                                  grad + kB4);
  fc_bwd_x_kernel<<<(unsigned)ceil_div((int64_t)n * 64, 256), 256, 0, st>>>(
      params + kW4, d, a3, n, 64, 3, da3);
  // dense 2048 -> 64
  fc_bwd_w_kernel<<<(unsigned)ceil_div((int64_t)64 * 2048, 256), 256, 0, st>>>(
      a2, da3, n, 2048, 64, grad + kW3, grad + kB3);
  fc_bwd_x_kernel<<<(unsigned)ceil_div((int64_t)n * 2048, 256), 256, 0, st>>>(
      params + kW3, da3, a2, n, 2048, 64, da2);
  // conv 16 -> 32, stride 2
  conv_bwd_w_kernel<<<32 * 16 * 9 + 32, 256, 0, st>>>(a1, da2, n, 16, 16, 16, 32, 2, grad + kW2,
                                                       grad + kB2);
  conv_bwd_x_kernel<<<(unsigned)ceil_div((int64_t)n * 16 * 256, 256), 256, 0, st>>>(
      params + kW2, da2, a1, n, 16, 16, 16, 32, 2, da1);
  // conv 6 -> 16, stride 1 (no input gradient needed)
  conv_bwd_w_kernel<<<16 * 6 * 9 + 16, 256, 0, st>>>(x, da1, n, 6, 16, 16, 16, 1, grad + kW1,
                                                     grad + kB1);
  return hipGetLastError();
}

// Adam (Kingma & Ba 2015), bias-corrected, step t >= 1
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, int64_t cnt, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t cnn_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                    hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  adam_kernel<<<(unsigned)ceil_div(kNetParams, 256), 256, 0, st>>>(params, grad, m, v, kNetParams,
                                                                   lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

// He-normal weights (Philox, keyed by the seed), zero biases
__global__ void init_kernel(float *__restrict__ p, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNetParams) return;
  float fan = 0.f;
  if (i < kB1) fan = 54.f;
  else if (i < kW2) fan = 0.f;
  else if (i < kB2) fan = 144.f;
  else if (i < kW3) fan = 0.f;
  else if (i < kB3) fan = 2048.f;
  else if (i < kW4) fan = 0.f;
  else if (i < kB4) fan = 64.f;
  if (fan == 0.f) { p[i] = 0.f; return; }
  const double2 gg = gauss2(seed, (uint64_t)i, 0x434E4E31u, 0x494E4954u);
  p[i] = (float)(gg.x * sqrt(2.0 / fan));
}

hipError_t cnn_init(float *params, uint64_t seed, hipStream_t st) {
  init_kernel<<<(unsigned)ceil_div(kNetParams, 256), 256, 0, st>>>(params, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------- glue to the solver
// network input: channel 2c = Re, 2c+1 = Im of the truncated-FFT channel c
__global__ void input_kernel(const double *__restrict__ feats, int n, int C, int p0,
                             float *__restrict__ x) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)2 * C * p0 * p0;
  if (idx >= (int64_t)n * per) return;
  const int64_t s = idx / per, r = idx % per;
  const int ch = (int)(r / (p0 * p0)), pos = (int)(r % (p0 * p0));
  const int c = ch >> 1, part = ch & 1;
  x[idx] = (float)feats[(((s * C + c) * p0 * p0) + pos) * 2 + part];
}

hipError_t cnn_input(const double *feats, int n, int C, int p0, float *x, hipStream_t st) {
  const int64_t cnt = (int64_t)n * 2 * C * p0 * p0;
  input_kernel<<<(unsigned)ceil_div(cnt, 256), 256, 0, st>>>(feats, n, C, p0, x);
  return hipGetLastError();
}

// targets (log lambda_1, log lambda_{L+1}, m* / 128) from the ascending Ritz values of a solve,
// m* = clamp(ceil(acosh(1e4) / acosh|t(lambda_L)|), 8, 128) over the damped [lambda_{L+1}, beta]
__global__ void labels_kernel(const double *__restrict__ ritz, int n, int k, int L,
                              const double *__restrict__ beta, float *__restrict__ t) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double *r = ritz + (int64_t)s * k;
  const double l1 = r[0], lL = r[L - 1], lL1 = r[L], bt = beta[s];
  const double c = 0.5 * (lL1 + bt), e = 0.5 * (bt - lL1);
  const double tt = fabs((lL - c) / e);
  double m = 128.0;
  if (tt > 1.0) m = fmin(128.0, fmax(8.0, ceil(acosh(1e4) / acosh(tt))));
  t[3 * s + 0] = (float)log(l1);
  t[3 * s + 1] = (float)log(lL1);
  t[3 * s + 2] = (float)(m / 128.0);
}

hipError_t cnn_labels(const double *ritz, int n, int k, int L, const double *beta, float *t,
                      hipStream_t st) {
  labels_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(ritz, n, k, L, beta, t);
  return hipGetLastError();
}

// hints (lambda_1, lambda_{L+1}, degree) from the network output; the degree is kept in the
// range of the training labels, [8, 128]
__global__ void hints_kernel(const float *__restrict__ y, int n, double *__restrict__ hints) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  hints[3 * s + 0] = exp((double)y[3 * s + 0]);
  hints[3 * s + 1] = exp((double)y[3 * s + 1]);
  hints[3 * s + 2] = fmin(128.0, fmax(8.0, rint(128.0 * (double)y[3 * s + 2])));  // label range
}

hipError_t cnn_hints(const float *y, int n, double *hints, hipStream_t st) {
  hints_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(y, n, hints);
  return hipGetLastError();
}

}  // namespace scsf
