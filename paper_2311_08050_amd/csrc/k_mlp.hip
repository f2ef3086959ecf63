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
// B(k, j) = B[k*sbr + j*sbc], C(i, j) = C[i*scr + j*scc], on FP32 MFMA
// (v_mfma_f32_16x16x4f32, FP32 accumulate): 64 x 64 tiles per workgroup, 32 x 32
// per wave (2 x 2 blocks of 16 x 16), K in chunks of 16 through LDS.  Tile loads
// run along whichever index of an operand is contiguous, so every layout the
// network's forward and backward passes use is read coalesced.
// Epilogue: + bias[j] (if bias), Z = pre-activation stored (if Z), C = GELU(.)
// (if gelu), or C = alpha * acc + beta * C.  With `ksplit` > 1 the K range is
// split over blockIdx.z and each split writes its partial tile to `part`
// (ksplit x M x N); gemm_epilogue_kernel then sums the splits in a fixed order
// and applies the epilogue (the backward product through the output layer has
// K = n and only B x H outputs).
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

__device__ __forceinline__ void gemm_store(const GemmArgs &g, int i, int j, float val) {
  if (g.bias) val += g.bias[j];
  float *c = g.C + (size_t)i * g.scr + (size_t)j * g.scc;
  if (g.Z) g.Z[(size_t)i * g.N + j] = val;
  if (g.gelu) *c = gelu_f(val);
  else *c = g.alpha * val + (g.beta != 0.0f ? g.beta * *c : 0.0f);
}

typedef float f4m __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs g, float *part, int kper) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1, li = lane & 15, gq = lane >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kper, ke = min(g.K, kb + kper);
  const bool a_krow = g.sac == 1, b_kcol = g.sbc != 1;   // contiguous along k?
  f4m acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4m{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = q * 256 + tid;
      int r, kk;
      if (a_krow) { r = e >> 4; kk = e & 15; } else { kk = e >> 6; r = e & 63; }
      const int i = i0 + r, k = k0 + kk;
      As[kk][r] = (i < g.M && k < ke) ? g.A[(size_t)i * g.sar + (size_t)k * g.sac] : 0.0f;
      int c;
      if (b_kcol) { c = e >> 4; kk = e & 15; } else { kk = e >> 6; c = e & 63; }
      const int j = j0 + c, kb2 = k0 + kk;
      Bs[kk][c] = (j < g.N && kb2 < ke) ? g.B[(size_t)kb2 * g.sbr + (size_t)j * g.sbc] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int kk = 4 * gq + st;   // lane group gq supplies k = 4 gq + st at step st
      float av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk][wm * 32 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk][wn * 32 + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane l holds rows 4 (l / 16) + v, column l % 16 of each 16 x 16 block
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * 32 + a * 16 + 4 * gq + v, j = j0 + wn * 32 + b * 16 + li;
        if (i >= g.M || j >= g.N) continue;
        if (part) part[((size_t)blockIdx.z * g.M + i) * g.N + j] = acc[a][b][v];
        else gemm_store(g, i, j, acc[a][b][v]);
      }
}

// Sum of the K splits (fixed order) and the epilogue, one thread per output.
__global__ __launch_bounds__(256) void gemm_epilogue_kernel(GemmArgs g, const float *part, int ksplit) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)g.M * g.N) return;
  const int i = (int)(idx / g.N), j = (int)(idx % g.N);
  float s = 0.0f;
  for (int z = 0; z < ksplit; ++z) s += part[(size_t)z * g.M * g.N + idx];
  gemm_store(g, i, j, s);
}

// K splits of a product: enough workgroups for the chip (about 512) without
// splits shorter than 128.
static int gemm_ksplit(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int ks = std::max(1, 512 / std::max(1, tiles));
  ks = std::min(ks, std::max(1, K / 128));
  return ks;
}

// dY <- dY * GELU'(Z) (elementwise).
__global__ void gelu_back_kernel(float *dY, const float *Z, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) dY[i] *= gelu_grad_f(Z[i]);
}

// Column sums of a (rows x cols) row-major matrix into out[cols] (bias
// gradients), rows added in increasing order; eight rows' loads are issued
// ahead of their additions.
__global__ void colsum_kernel(const float *X, int rows, int cols, float *out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float s = 0.0f;
  for (int r0 = 0; r0 < rows; r0 += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = r0 + u < rows ? X[(size_t)(r0 + u) * cols + j] : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r0 + u < rows) s += v[u];
  }
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
  float *kpart = nullptr;   // partial products of split-K GEMMs
  size_t kpart_elems = 0;
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
  if (m->kpart) (void)hipFree(m->kpart);
  if (m->dtheta) (void)hipFree(m->dtheta);
  if (m->dptrs) (void)hipFree(m->dptrs);
  m->part = nullptr;
  m->kpart = nullptr;
  m->kpart_elems = 0;
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
  // split-K workspace: the largest ksplit x M x N over the products of a
  // forward and backward pass at batch `cap` (GEMMs of fewer rows need less)
  size_t kp = 0;
  const int I = m->I, H = m->H, O = m->O;
  const int shapes[][3] = {{cap, H, I}, {cap, H, H}, {cap, O, H}, {O, H, cap}, {cap, H, O}, {H, H, cap}, {H, I, cap}};
  for (const auto &sh : shapes) {
    const int ks = gemm_ksplit(sh[0], sh[1], sh[2]);
    if (ks > 1) kp = std::max(kp, (size_t)ks * sh[0] * sh[1]);
  }
  bool ok = hipMalloc(&m->u, 4 * nb * m->I) == hipSuccess && hipMalloc(&m->z1, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->h1, 4 * nb * m->H) == hipSuccess && hipMalloc(&m->z2, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->h2, 4 * nb * m->H) == hipSuccess && hipMalloc(&m->out, 4 * nb * m->O) == hipSuccess &&
            hipMalloc(&m->dout, 4 * nb * m->O) == hipSuccess && hipMalloc(&m->dh2, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->dh1, 4 * nb * m->H) == hipSuccess &&
            hipMalloc(&m->part, 8 * ((nb * m->O + 255) / 256 + 1)) == hipSuccess &&
            hipMalloc(&m->dtheta, 8 * (nb * 8 + 16)) == hipSuccess && hipMalloc(&m->dptrs, 8 * nb) == hipSuccess &&
            (kp == 0 || hipMalloc(&m->kpart, 4 * kp) == hipSuccess);
  if (!ok) {
    (void)hipGetLastError();
    free_acts(m);
    return INLA_ERR_NOMEM;
  }
  m->cap = cap;
  m->kpart_elems = kp;
  return 0;
}

void gemm(inla_mlp *m, hipStream_t s, const GemmArgs &g) {
  int ks = gemm_ksplit(g.M, g.N, g.K);
  if ((size_t)ks * g.M * g.N > m->kpart_elems) ks = 1;   // never past the workspace
  const int kper = ks > 1 ? ((g.K + ks - 1) / ks + 15) / 16 * 16 : g.K;
  ks = ks > 1 ? (g.K + kper - 1) / kper : 1;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, ks);
  hipLaunchKernelGGL(mlp_gemm_kernel, grid, dim3(256), 0, s, g, ks > 1 ? m->kpart : nullptr, kper);
  if (ks > 1) {
    const int64_t cnt = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(gemm_epilogue_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, g,
                       (const float *)m->kpart, ks);
  }
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
  gemm(m, s, g);
  g = ga(m->h1, m->H, 1, P + m->off_W2(), 1, m->H, m->h2, m->H, 1, B, m->H, m->H);
  g.bias = P + m->off_b2(); g.Z = m->z2; g.gelu = 1;
  gemm(m, s, g);
  g = ga(m->h2, m->H, 1, P + m->off_W3(), 1, m->H, m->out, m->O, 1, B, m->O, m->H);
  g.bias = P + m->off_b3();
  gemm(m, s, g);
}

// Backward pass from m->dout into m->grad (flat, same layout as params).
void backward(inla_mlp *m, hipStream_t s, int B) {
  const float *P = m->params;
  float *G = m->grad;
  const int I = m->I, H = m->H, O = m->O;
  // dW3 (O x H) = dout^T (O x B) * h2 (B x H)
  gemm(m, s, ga(m->dout, 1, O, m->h2, H, 1, G + m->off_W3(), H, 1, O, H, B));
  hipLaunchKernelGGL(colsum_kernel, dim3((O + 255) / 256), dim3(256), 0, s, m->dout, B, O, G + m->off_b3());
  // dh2 (B x H) = dout (B x O) * W3 (O x H), then * GELU'(z2)
  gemm(m, s, ga(m->dout, O, 1, P + m->off_W3(), H, 1, m->dh2, H, 1, B, H, O));
  hipLaunchKernelGGL(gelu_back_kernel, dim3((B * H + 255) / 256), dim3(256), 0, s, m->dh2, m->z2, B * H);
  gemm(m, s, ga(m->dh2, 1, H, m->h1, H, 1, G + m->off_W2(), H, 1, H, H, B));
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, m->dh2, B, H, G + m->off_b2());
  gemm(m, s, ga(m->dh2, H, 1, P + m->off_W2(), H, 1, m->dh1, H, 1, B, H, H));
  hipLaunchKernelGGL(gelu_back_kernel, dim3((B * H + 255) / 256), dim3(256), 0, s, m->dh1, m->z1, B * H);
  gemm(m, s, ga(m->dh1, 1, H, m->u, I, 1, G + m->off_W1(), I, 1, H, I, B));
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
