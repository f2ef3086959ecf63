// inla_logdet_noalloc: the log-determinants of inla_logdet (Eq. (41)'s Gaussian
// normalisers by blocked Cholesky) for callers that cannot allocate device
// memory: every scratch buffer of the factorisation (padded working matrices,
// diagonal-block inverses, result slots, status words, BF16 panel copies)
// lives in one file-scope device array of fixed size, `scratch`, instead of the
// handle's grow-only workspace.  Descriptors travel through the handle's
// upload ring (allocated by inla_create), launch chains are launched directly
// (no graph capture, which would allocate the graph's argument block), and no
// profiling events are recorded in the call.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <limits>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "host.hpp"
#include "model.hpp"

namespace inla {

// One copy per GPU, held until the process ends.
static __device__ __align__(256) char scratch[INLA_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each device, taken once per device with that
// device current (the array's name is only a host-side stand-in).
constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static bool scratch_done[MAX_DEVICES];
static char *scratch_ptr[MAX_DEVICES];

int noalloc_init_device(int device) {
  if (device < 0 || device >= MAX_DEVICES) return INLA_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_done[device]) return scratch_ptr[device] ? INLA_OK : INLA_ERR_HIP;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  scratch_done[device] = true;
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    scratch_ptr[device] = nullptr;
    return INLA_ERR_HIP;
  }
  scratch_ptr[device] = (char *)p;
  return INLA_OK;
}

static char *device_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_done[device] ? scratch_ptr[device] : nullptr;
}

// Status words start at zero: a fill kernel, not a memset, so that the call
// records no memset node if a caller captures its stream.
__global__ __launch_bounds__(256) void zero_ints_kernel(int *p, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0;
}

// Per matrix: log-determinant (2 sum log L_ii, from the finish kernel's slot)
// and the first failing pivot, gathered into two contiguous arrays.
__global__ __launch_bounds__(256) void gather_logdet_kernel(const ThetaDesc *__restrict__ td, const int *dinfo,
                                                            int info_slot, double *ld, int *info, int B) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= B) return;
  ld[i] = td[i].dres[DRES_LOGDET_L];
  info[i] = dinfo[4 * i + info_slot];
}

static size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// Restores the handle's settings that the call turns off.
struct NoAllocScope {
  Ctx &c;
  bool graphs, prof, look;
  char *pbf;
  size_t pbf_size;
  explicit NoAllocScope(Ctx &ctx)
      : c(ctx), graphs(ctx.graphs), prof(ctx.prof), look(ctx.lookahead), pbf(ctx.pbf), pbf_size(ctx.pbf_size) {
    c.graphs = false;     // a new graph allocates its argument block
    c.prof = false;       // timing events are created on demand
    c.lookahead = false;  // the side stream is created on first use
  }
  ~NoAllocScope() {
    c.graphs = graphs;
    c.prof = prof;
    c.lookahead = look;
    c.pbf = pbf;
    c.pbf_size = pbf_size;
  }
};

}  // namespace inla

using namespace inla;

extern "C" int inla_logdet_noalloc(inla_handle *h, int32_t B, const int32_t *n, double *const *Q, const int32_t *ldq,
                                   int32_t prec, double *logdet, int32_t *info) {
  if (!h) return -1;
  if (B < 0) return -2;
  if (B == 0) return INLA_OK;
  if (!n) return -3;
  if (!Q) return -4;
  if (!ldq) return -5;
  if (prec < 0 || prec >= INLA_PREC_COUNT) return INLA_ERR_UNSUPPORTED;
  if (!logdet) return -7;
  if (!info) return -8;
  for (int i = 0; i < B; ++i) {
    if (n[i] < 0) return -3;
    if (n[i] > 0 && !Q[i]) return -4;
    if (ldq[i] < std::max(1, n[i])) return -5;
  }
  Ctx &ctx = *handle_ctx(h);
  char *base = device_scratch(ctx.device);
  if (!base) return INLA_ERR_HIP;
  const size_t esz = prec == INLA_PREC_FP64 ? 8 : 4;
  // layout of the scratch array: per matrix [W | vectors | block inverses],
  // then status words, gathered results and (BF16) the panel copies
  std::vector<int> ids;
  std::vector<size_t> offs(B, 0);
  size_t total = 0;
  int nf_max = 0;
  for (int i = 0; i < B; ++i) {
    if (n[i] == 0) continue;
    const size_t np = (size_t)round_up(n[i], PADN);
    offs[i] = total;
    total += a256(esz * np * np) + a256(8 * (4 * np + 64 + DRES_COUNT)) + a256(esz * np * NBI);
    nf_max = std::max(nf_max, (int)np);
    ids.push_back(i);
  }
  const size_t off_info = total;
  total += a256(sizeof(int) * 4 * (size_t)B);
  const size_t off_ld = total;
  total += a256(sizeof(double) * (size_t)B);
  const size_t off_inf = total;
  total += a256(sizeof(int) * (size_t)B);
  const size_t off_pbf = total;
  if (prec == INLA_PREC_BF16 && !ids.empty()) {
    const int nb = tuned_config(ctx, prec, nf_max, (int)ids.size()).nb;
    for (int i : ids) total += 16 * 2 * (size_t)(nb / 8) * round_up(n[i], PADN);
  }
  if (total > (size_t)INLA_NOALLOC_SCRATCH_BYTES) return INLA_ERR_TOO_LARGE;

  NoAllocScope guard(ctx);
  PrecScope tag(ctx, prec);
  std::vector<ThetaDesc> td(ids.size());
  std::vector<HostFactor> fs;
  int *dinfo = (int *)(base + off_info);
  for (size_t q = 0; q < ids.size(); ++q) {
    const int i = ids[q];
    ThetaDesc &t = td[q];
    t = ThetaDesc{};
    t.n = n[i];
    t.n_pad = round_up(n[i], PADN);
    t.Quser = Q[i];
    t.ldquser = ldq[i];
    t.ldw = t.Nw = t.Ncw = t.n_pad;
    char *p = base + offs[i];
    t.W = p;
    p += a256(esz * (size_t)t.n_pad * t.n_pad);
    double *v = (double *)p;
    t.x = v; v += t.n_pad;
    t.r = v; v += t.n_pad;
    t.lam = v; v += 64;
    t.part = v; v += 2 * t.ldw;   // finish_kernel sums it; zero-filled below
    t.dres = v;
    p += a256(8 * (4 * (size_t)t.n_pad + 64 + DRES_COUNT));
    t.linv = p;
    HostFactor hf{};
    hf.d.A = t.W;
    hf.d.linv = t.linv;
    hf.d.info = dinfo + 4 * q + 1;
    hf.d.ld = t.ldw;
    hf.d.nf = hf.d.nrows = hf.d.ncols = t.n_pad;
    hf.d.id_row0 = INT_MAX;
    hf.n_real = t.n;
    fs.push_back(hf);
  }
  if (prec == INLA_PREC_BF16) {
    // the BF16 panel copies come from the scratch array too
    ctx.pbf = base + off_pbf;
    ctx.pbf_size = (size_t)INLA_NOALLOC_SCRATCH_BYTES - off_pbf;
  }
  const int Bq = (int)ids.size();
  if (Bq > 0) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3((4 * Bq + 255) / 256), dim3(256), 0, ctx.stream, dinfo, 4 * Bq);
    for (const ThetaDesc &t : td) {
      // part (2 ldw doubles) is summed by the finish kernel: start it at zero
      const int cnt = 2 * (int)(2 * t.ldw);
      hipLaunchKernelGGL(zero_ints_kernel, dim3((cnt + 255) / 256), dim3(256), 0, ctx.stream, (int *)t.part, cnt);
    }
    const ThetaDesc *d = (const ThetaDesc *)ctx.upload(td.data(), sizeof(ThetaDesc) * td.size());
    if (!d) return INLA_ERR_NOMEM;
    launch_copy_in(ctx, d, Bq, nf_max, prec);
    const int rc = factor_batch(ctx, fs, prec);
    if (rc) return rc;
    launch_finish(ctx, d, Bq, prec);
    int n_max = 0;
    for (int i : ids) n_max = std::max(n_max, n[i]);
    launch_copy_out(ctx, d, Bq, n_max, prec);
    hipLaunchKernelGGL(gather_logdet_kernel, dim3((Bq + 255) / 256), dim3(256), 0, ctx.stream, d, dinfo, 1,
                       (double *)(base + off_ld), (int *)(base + off_inf), Bq);
  }
  std::vector<double> hld(Bq);
  std::vector<int> hinf(Bq);
  if (Bq > 0 &&
      (hipMemcpyAsync(hld.data(), base + off_ld, sizeof(double) * Bq, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess ||
       hipMemcpyAsync(hinf.data(), base + off_inf, sizeof(int) * Bq, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess))
    return INLA_ERR_HIP;
  if (hipStreamSynchronize(ctx.stream) != hipSuccess) return INLA_ERR_HIP;
  const int rc = ctx.check();
  if (rc) return rc;
  for (int i = 0; i < B; ++i) { logdet[i] = 0.0; info[i] = 0; }
  for (int q = 0; q < Bq; ++q) {
    const int i = ids[q];
    info[i] = hinf[q];
    logdet[i] = hinf[q] ? std::numeric_limits<double>::quiet_NaN() : hld[q];
  }
  return INLA_OK;
}
