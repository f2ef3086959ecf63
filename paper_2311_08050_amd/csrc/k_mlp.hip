// Learned warm start for the Newton mode: a small multilayer perceptron
//     h1 = GELU(W1 u + b1),  h2 = GELU(W2 h1 + b2),  x0 = W3 h2 + b3
// (u the normalised hyperparameters), trained on modes that the method itself
// produces, with hand-written FP32 forward, backward and Adam kernels.
// GELU is the exact erf form x * (1 + erf(x / sqrt 2)) / 2.
//
// Parameters are one flat FP32 array: W1 (H x I, row-major), b1 (H),
// W2 (H x H), b2 (H), W3 (O x H), b3 (O).
#include <cmath>
#include <cstdint>
#include <vector>

#include "device.hpp"
#include "host.hpp"

namespace inla {

// C(M x N) = A(M x K) * B(K x N) with A(i, k) = A[i*sar + k*sac],
// B(k, j) = B[k*sbr + j*sbc], C(i, j) = C[i*scr + j*scc]; 64 x 64 tiles, K in
// chunks of 16 through LDS, each thread 4 x 4 outputs, FP32 accumulate.
// Epilogue: + bias[j] (if bias), Z = pre-activation stored (if Z), C = GELU(.)
// (if gelu), or C = alpha * acc + beta * C.
struct GemmArgs {
  const float *A, *B;
  float *C, *Z;
  const float *bias;
  int M, N, K;
  int sar, sac, sbr, sbc, scr, scc;
  int gelu;
  float alpha, beta;
};

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs g) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int ti = (tid / 16) * 4, tj = (tid % 16) * 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e / 64, r = e % 64;
      const int i = i0 + r, k = k0 + kk, j = j0 + r;
      As[kk][r] = (i < g.M && k < g.K) ? g.A[(size_t)i * g.sar + (size_t)k * g.sac] : 0.0f;
      Bs[kk][r] = (k < g.K && j < g.N) ? g.B[(size_t)k * g.sbr + (size_t)j * g.sbc] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { a[u] = As[kk][ti + u]; b[u] = Bs[kk][tj + u]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ti + u, j = j0 + tj + v;
      if (i >= g.M || j >= g.N) continue;
      float val = acc[u][v];
      if (g.bias) val += g.bias[j];
      float *c = g.C + (size_t)i * g.scr + (size_t)j * g.scc;
      if (g.Z) g.Z[(size_t)i * g.N + j] = val;
      if (g.gelu) *c = gelu_f(val);
      else *c = g.alpha * val + (g.beta != 0.0f ? g.beta * *c : 0.0f);
    }
}

// dY <- dY * GELU'(Z) (elementwise).
__global__ void gelu_back_kernel(float *dY, const float *Z, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) dY[i] *= gelu_grad_f(Z[i]);
}

// Column sums of a (rows x cols) row-major matrix into out[cols] (bias
// gradients), fixed order.
__global__ void colsum_kernel(const float *X, int rows, int cols, float *out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + j];
  out[j] = s;
}

// dOut = 2 (out - target) / (B * O); per-block partial sums of the squared error.
__global__ void mse_grad_kernel(const float *out, const double *tgt, float *dout, int count, float scale, double *part) {
  __shared__ double sh[4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double se = 0.0;
  if (i < count) {
    const float d = out[i] - (float)tgt[i];
    dout[i] = scale * 2.0f * d;
    se = (double)d * d;
  }
  se = block_sum256(se, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = se;
}

// Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr mhat / (sqrt(vhat) + eps).
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int count, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Normalised inputs u = (theta - centre) / scale (FP32) and FP32 -> FP64 output
// scatter into per-theta vectors.
__global__ void theta_norm_kernel(const double *theta, int ld, int n_in, const double *centre, const double *scale,
                                  float *u, int B) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= B * n_in) return;
  const int b = i / n_in, c = i % n_in;
  u[i] = (float)((theta[(size_t)b * ld + c] - centre[c]) / scale[c]);
}
__global__ void scatter_modes_kernel(const float *y, int n_out, double *const *x) {
  const int b = blockIdx.y, i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_out) x[b][i] = (double)y[(size_t)b * n_out + i];
}

// Counter-based initialisation: splitmix64 of (seed, index) -> U(-a, a).
__global__ void init_uniform_kernel(float *p, int count, uint64_t seed, uint64_t offset, float a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (offset + (uint64_t)i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
  p[i] = (float)((2.0 * u - 1.0) * a);
}

}  // namespace inla

// ====================================================================== C-ABI
using namespace inla;

namespace inla {
hipStream_t handle_stream(inla_handle *h);   // host.hip
}

struct inla_mlp {
  inla_handle *h = nullptr;
  int I = 0, H = 0, O = 0;
  int64_t P = 0;
  float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  // activations for a batch of up to cap rows
  int cap = 0;
  float *u = nullptr, *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *out = nullptr, *dout = nullptr,
        *dh2 = nullptr, *dh1 = nullptr;
  double *part = nullptr;
  double *dtheta = nullptr, *dcentre = nullptr, *dscale = nullptr;
  double **dptrs = nullptr;
  int64_t step = 0;
  size_t off_W1() const { return 0; }
  size_t off_b1() const { return (size_t)H * I; }
  size_t off_W2() const { return off_b1() + H; }
  size_t off_b2() const { return off_W2() + (size_t)H * H; }
  size_t off_W3() const { return off_b2() + H; }
  size_t off_b3() const { return off_W3() + (size_t)O * H; }
};

namespace {

void free_acts(inla_mlp *m) {
  for (float **p : {&m->u, &m->z1, &m->h1, &m->z2, &m->h2, &m->out, &m->dout, &m->dh2, &m->dh1}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  if (m->part) (void)hipFree(m->part);
  if (m->dtheta) (void)hipFree(m->dtheta);
  if (m->dptrs) (void)hipFree(m->dptrs);
  m->part = nullptr;
  m->dtheta = nullptr;
  m->dptrs = nullptr;
  m->cap = 0;
}

int ensure_cap(inla_mlp *m, int B) {
  if (B <= m->cap) return 0;
  (void)hipDeviceSynchronize();
  free_acts(m);
  const int cap = std::max(B, 64);
  const size_t nb = (size_t)cap;
  bool ok = hipMalloc(&m->u, 4 * nb * m->I) == hipSuccess && hipMalloc(&m->z1, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->h1, 4 * nb * m->H) == hipSuccess && hipMalloc(&m->z2, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->h2, 4 * nb * m->H) == hipSuccess && hipMalloc(&m->out, 4 * nb * m->O) == hipSuccess &&
            hipMalloc(&m->dout, 4 * nb * m->O) == hipSuccess && hipMalloc(&m->dh2, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->dh1, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->part, 8 * ((nb * m->O + 255) / 256 + 1)) == hipSuccess &&
            hipMalloc(&m->dtheta, 8 * (nb * 8 + 16)) == hipSuccess && hipMalloc(&m->dptrs, 8 * nb) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_acts(m);
    return INLA_ERR_NOMEM;
  }
  m->cap = cap;
  return 0;
}

void gemm(hipStream_t s, const GemmArgs &g) {
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL(mlp_gemm_kernel, grid, dim3(256), 0, s, g);
}

GemmArgs ga(const float *A, int sar, int sac, const float *B, int sbr, int sbc, float *C, int scr, int scc, int M,
            int N, int K) {
  GemmArgs g{};
  g.A = A; g.B = B; g.C = C; g.M = M; g.N = N; g.K = K;
  g.sar = sar; g.sac = sac; g.sbr = sbr; g.sbc = sbc; g.scr = scr; g.scc = scc;
  g.alpha = 1.0f; g.beta = 0.0f;
  return g;
}

// Forward pass on m->u (B x I) into m->out (B x O), keeping pre-activations.
void forward(inla_mlp *m, hipStream_t s, int B) {
  const float *P = m->params;
  GemmArgs g = ga(m->u, m->I, 1, P + m->off_W1(), 1, m->I, m->h1, m->H, 1, B, m->H, m->I);
  g.bias = P + m->off_b1(); g.Z = m->z1; g.gelu = 1;
  gemm(s, g);
  g = ga(m->h1, m->H, 1, P + m->off_W2(), 1, m->H, m->h2, m->H, 1, B, m->H, m->H);
  g.bias = P + m->off_b2(); g.Z = m->z2; g.gelu = 1;
  gemm(s, g);
  g = ga(m->h2, m->H, 1, P + m->off_W3(), 1, m->H, m->out, m->O, 1, B, m->O, m->H);
  g.bias = P + m->off_b3();
  gemm(s, g);
}

// Backward pass from m->dout into m->grad (flat, same layout as params).
void backward(inla_mlp *m, hipStream_t s, int B) {
  const float *P = m->params;
  float *G = m->grad;
  const int I = m->I, H = m->H, O = m->O;
  // dW3 (O x H) = dout^T (O x B) * h2 (B x H)
  gemm(s, ga(m->dout, 1, O, m->h2, H, 1, G + m->off_W3(), H, 1, O, H, B));
  hipLaunchKernelGGL(colsum_kernel, dim3((O + 255) / 256), dim3(256), 0, s, m->dout, B, O, G + m->off_b3());
  // dh2 (B x H) = dout (B x O) * W3 (O x H), then * GELU'(z2)
  gemm(s, ga(m->dout, O, 1, P + m->off_W3(), H, 1, m->dh2, H, 1, B, H, O));
  hipLaunchKernelGGL(gelu_back_kernel, dim3((B * H + 255) / 256), dim3(256), 0, s, m->dh2, m->z2, B * H);
  gemm(s, ga(m->dh2, 1, H, m->h1, H, 1, G + m->off_W2(), H, 1, H, H, B));
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, m->dh2, B, H, G + m->off_b2());
  gemm(s, ga(m->dh2, H, 1, P + m->off_W2(), H, 1, m->dh1, H, 1, B, H, H));
  hipLaunchKernelGGL(gelu_back_kernel, dim3((B * H + 255) / 256), dim3(256), 0, s, m->dh1, m->z1, B * H);
  gemm(s, ga(m->dh1, 1, H, m->u, I, 1, G + m->off_W1(), I, 1, H, I, B));
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, m->dh1, B, H, G + m->off_b1());
}

int loss_and_grad(inla_mlp *m, int B, const float *x_in, const double *target, double *loss) {
  hipStream_t s = handle_stream(m->h);
  int rc = ensure_cap(m, B);
  if (rc) return rc;
  if (hipMemcpyAsync(m->u, x_in, 4 * (size_t)B * m->I, hipMemcpyDeviceToDevice, s) != hipSuccess) return INLA_ERR_HIP;
  forward(m, s, B);
  const int cnt = B * m->O, nblk = (cnt + 255) / 256;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nblk), dim3(256), 0, s, m->out, target, m->dout, cnt, 1.0f / (float)cnt,
                     m->part);
  backward(m, s, B);
  if (loss) {
    std::vector<double> h(nblk);
    if (hipMemcpyAsync(h.data(), m->part, 8 * nblk, hipMemcpyDeviceToHost, s) != hipSuccess) return INLA_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return INLA_ERR_HIP;
    double t = 0.0;
    for (double v : h) t += v;
    *loss = t / cnt;
  }
  return hipGetLastError() == hipSuccess ? 0 : INLA_ERR_HIP;
}

}  // namespace

extern "C" {

int inla_mlp_create(inla_handle *h, int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, inla_mlp **out) {
  if (!h) return -1;
  if (n_in < 1) return -2;
  if (n_hidden < 1) return -3;
  if (n_out < 1) return -4;
  if (!out) return -6;
  *out = nullptr;
  inla_mlp *m = new (std::nothrow) inla_mlp();
  if (!m) return INLA_ERR_NOMEM;
  m->h = h;
  m->I = n_in; m->H = n_hidden; m->O = n_out;
  m->P = (int64_t)n_hidden * n_in + n_hidden + (int64_t)n_hidden * n_hidden + n_hidden + (int64_t)n_out * n_hidden + n_out;
  const size_t pb = 4 * (size_t)m->P;
  if (hipMalloc(&m->params, pb) != hipSuccess || hipMalloc(&m->grad, pb) != hipSuccess ||
      hipMalloc(&m->m, pb) != hipSuccess || hipMalloc(&m->v, pb) != hipSuccess ||
      hipMalloc(&m->dcentre, 8 * 32) != hipSuccess || hipMalloc(&m->dscale, 8 * 32) != hipSuccess) {
    (void)hipGetLastError();
    inla_mlp_destroy(m);
    return INLA_ERR_NOMEM;
  }
  hipStream_t s = handle_stream(h);
  // uniform(-sqrt(6 / fan_in), +) weights (He-style for GELU), zero biases
  struct Seg { size_t off, cnt; float a; };
  const Seg segs[] = {{m->off_W1(), (size_t)m->H * m->I, sqrtf(6.0f / m->I)},
                      {m->off_b1(), (size_t)m->H, 0.0f},
                      {m->off_W2(), (size_t)m->H * m->H, sqrtf(6.0f / m->H)},
                      {m->off_b2(), (size_t)m->H, 0.0f},
                      {m->off_W3(), (size_t)m->O * m->H, sqrtf(3.0f / m->H)},
                      {m->off_b3(), (size_t)m->O, 0.0f}};
  for (const Seg &g : segs)
    hipLaunchKernelGGL(init_uniform_kernel, dim3((g.cnt + 255) / 256), dim3(256), 0, s, m->params + g.off, (int)g.cnt,
                       seed, (uint64_t)g.off, g.a);
  (void)hipMemsetAsync(m->m, 0, pb, s);
  (void)hipMemsetAsync(m->v, 0, pb, s);
  if (hipStreamSynchronize(s) != hipSuccess) { inla_mlp_destroy(m); return INLA_ERR_HIP; }
  *out = m;
  return INLA_OK;
}

int inla_mlp_destroy(inla_mlp *m) {
  if (!m) return INLA_OK;
  (void)hipDeviceSynchronize();
  free_acts(m);
  for (float *p : {m->params, m->grad, m->m, m->v}) if (p) (void)hipFree(p);
  if (m->dcentre) (void)hipFree(m->dcentre);
  if (m->dscale) (void)hipFree(m->dscale);
  delete m;
  return INLA_OK;
}

int inla_mlp_num_params(const inla_mlp *m, int64_t *count) {
  if (!m) return -1;
  if (!count) return -2;
  *count = m->P;
  return INLA_OK;
}

int inla_mlp_get_params(inla_mlp *m, float *dst) {
  if (!m) return -1;
  if (!dst) return -2;
  hipStream_t s = handle_stream(m->h);
  if (hipMemcpyAsync(dst, m->params, 4 * (size_t)m->P, hipMemcpyDeviceToDevice, s) != hipSuccess) return INLA_ERR_HIP;
  return hipStreamSynchronize(s) == hipSuccess ? INLA_OK : INLA_ERR_HIP;
}

int inla_mlp_set_params(inla_mlp *m, const float *src) {
  if (!m) return -1;
  if (!src) return -2;
  hipStream_t s = handle_stream(m->h);
  if (hipMemcpyAsync(m->params, src, 4 * (size_t)m->P, hipMemcpyDeviceToDevice, s) != hipSuccess) return INLA_ERR_HIP;
  (void)hipMemsetAsync(m->m, 0, 4 * (size_t)m->P, s);
  (void)hipMemsetAsync(m->v, 0, 4 * (size_t)m->P, s);
  m->step = 0;
  return hipStreamSynchronize(s) == hipSuccess ? INLA_OK : INLA_ERR_HIP;
}

int inla_mlp_forward(inla_mlp *m, int32_t B, const float *x_in, float *y_out) {
  if (!m) return -1;
  if (B < 0) return -2;
  if (B == 0) return INLA_OK;
  if (!x_in) return -3;
  if (!y_out) return -4;
  hipStream_t s = handle_stream(m->h);
  int rc = ensure_cap(m, B);
  if (rc) return rc;
  if (hipMemcpyAsync(m->u, x_in, 4 * (size_t)B * m->I, hipMemcpyDeviceToDevice, s) != hipSuccess) return INLA_ERR_HIP;
  forward(m, s, B);
  if (hipMemcpyAsync(y_out, m->out, 4 * (size_t)B * m->O, hipMemcpyDeviceToDevice, s) != hipSuccess) return INLA_ERR_HIP;
  return hipStreamSynchronize(s) == hipSuccess ? INLA_OK : INLA_ERR_HIP;
}

int inla_mlp_grad(inla_mlp *m, int32_t B, const float *x_in, const double *target, float *grad_out, double *loss) {
  if (!m) return -1;
  if (B < 1) return -2;
  if (!x_in) return -3;
  if (!target) return -4;
  int rc = loss_and_grad(m, B, x_in, target, loss);
  if (rc) return rc;
  hipStream_t s = handle_stream(m->h);
  if (grad_out && hipMemcpyAsync(grad_out, m->grad, 4 * (size_t)m->P, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return INLA_ERR_HIP;
  return hipStreamSynchronize(s) == hipSuccess ? INLA_OK : INLA_ERR_HIP;
}

int inla_mlp_train_step(inla_mlp *m, int32_t B, const float *x_in, const double *target, float lr, double *loss) {
  if (!m) return -1;
  if (B < 1) return -2;
  if (!x_in) return -3;
  if (!target) return -4;
  if (!(lr > 0.0f)) return -5;
  int rc = loss_and_grad(m, B, x_in, target, loss);
  if (rc) return rc;
  hipStream_t s = handle_stream(m->h);
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)m->step), c2 = 1.0f - powf(b2, (float)m->step);
  hipLaunchKernelGGL(adam_kernel, dim3((m->P + 255) / 256), dim3(256), 0, s, m->params, m->grad, m->m, m->v,
                     (int)m->P, lr, b1, b2, c1, c2, 1e-8f);
  return hipGetLastError() == hipSuccess ? INLA_OK : INLA_ERR_HIP;
}

int inla_mlp_predict_modes(inla_mlp *m, int32_t B, const double *theta, int32_t ldtheta, const double *centre,
                           const double *scale, double *const *x) {
  if (!m) return -1;
  if (B < 0) return -2;
  if (B == 0) return INLA_OK;
  if (!theta) return -3;
  if (ldtheta < m->I) return -4;
  if (!centre) return -5;
  if (!scale) return -6;
  if (!x) return -7;
  hipStream_t s = handle_stream(m->h);
  int rc = ensure_cap(m, B);
  if (rc) return rc;
  if (ldtheta > 8) return INLA_ERR_UNSUPPORTED;   // staging holds 8 doubles per theta
  if (hipMemcpyAsync(m->dtheta, theta, 8 * (size_t)B * ldtheta, hipMemcpyHostToDevice, s) != hipSuccess)
    return INLA_ERR_HIP;
  if (hipMemcpyAsync(m->dcentre, centre, 8 * m->I, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(m->dscale, scale, 8 * m->I, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(m->dptrs, x, 8 * (size_t)B, hipMemcpyHostToDevice, s) != hipSuccess)
    return INLA_ERR_HIP;
  hipLaunchKernelGGL(theta_norm_kernel, dim3((B * m->I + 255) / 256), dim3(256), 0, s, m->dtheta, ldtheta, m->I,
                     m->dcentre, m->dscale, m->u, B);
  forward(m, s, B);
  hipLaunchKernelGGL(scatter_modes_kernel, dim3((m->O + 255) / 256, B), dim3(256), 0, s, m->out, m->O, m->dptrs);
  return hipStreamSynchronize(s) == hipSuccess ? INLA_OK : INLA_ERR_HIP;
}

}  // extern "C"
