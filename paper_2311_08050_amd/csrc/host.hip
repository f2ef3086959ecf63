// C-ABI entry points and the host-side orchestration of the per-theta hot path:
// prior build, prior pass, Newton iteration with kriging, final pass at the mode
// and the Laplace objective of Eq. (41) (mode-approx).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>

#include "device.hpp"
#include "host.hpp"
#include "model.hpp"

namespace inla {

// ------------------------------------------------------------------ Ctx
static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// The optional streams (side: lookahead; aux: concurrent prior pass) are
// created on first use.  A failure leaves the feature off for the call and
// clears the runtime's error state, so that it is not reported by a later check.
int Ctx::side_ready() {
  if (side && ev_a && ev_b) return INLA_OK;
  if (!side && hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    side = nullptr;
    return INLA_ERR_HIP;
  }
  if ((!ev_a && hipEventCreateWithFlags(&ev_a, hipEventDisableTiming) != hipSuccess) ||
      (!ev_b && hipEventCreateWithFlags(&ev_b, hipEventDisableTiming) != hipSuccess)) {
    (void)hipGetLastError();
    return INLA_ERR_HIP;
  }
  return INLA_OK;
}

int Ctx::aux_ready() {
  if (aux && ev_c && ev_d) return INLA_OK;
  if (!aux && hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    aux = nullptr;
    return INLA_ERR_HIP;
  }
  if ((!ev_c && hipEventCreateWithFlags(&ev_c, hipEventDisableTiming) != hipSuccess) ||
      (!ev_d && hipEventCreateWithFlags(&ev_d, hipEventDisableTiming) != hipSuccess)) {
    (void)hipGetLastError();
    return INLA_ERR_HIP;
  }
  return INLA_OK;
}

int Ctx::sync_all() {
  // the caller's stream (NULL is the null stream), then the handle's own
  // streams if created; `stream` is always one of them
  if (hipStreamSynchronize(home) != hipSuccess) return INLA_ERR_HIP;
  for (hipStream_t s : {side, aux})
    if (s && hipStreamSynchronize(s) != hipSuccess) return INLA_ERR_HIP;
  return INLA_OK;
}

// The ring is reused once every earlier reader has finished: work on the
// caller's stream, the side stream and the aux stream.
static bool ring_wrap(Ctx &c) {
  if (c.sync_all() != INLA_OK) return false;
  c.ring_off = 0;
  return true;
}

void *Ctx::upload(const void *src, size_t bytes) {
  const size_t padded = align256(bytes);
  if (pg_mode != PG_OFF) {
    // a pass graph's argument block: the next slot, filled before the replay
    const size_t off = pg.host.size();
    if (off + padded > pg.cap) {
      pg.overflow = true;
      return nullptr;
    }
    pg.host.resize(off + padded, 0);
    std::memcpy(pg.host.data() + off, src, bytes);
    pg.sig.push_back(-(int64_t)bytes);
    return pg.dbase + off;
  }
  if (padded > ring_size) return nullptr;
  if (ring_off + padded > ring_size && !ring_wrap(*this)) return nullptr;
  std::memcpy(ring_host + ring_off, src, bytes);
  void *dst = ring + ring_off;
  if (hipMemcpyAsync(dst, ring_host + ring_off, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return nullptr;
  ring_off += padded;
  return dst;
}

int Ctx::upload_to(void *dst, const void *src, size_t bytes) {
  const size_t padded = align256(bytes);
  if (padded > ring_size) return INLA_ERR_NOMEM;
  if (ring_off + padded > ring_size && !ring_wrap(*this)) return INLA_ERR_HIP;
  std::memcpy(ring_host + ring_off, src, bytes);
  if (hipMemcpyAsync(dst, ring_host + ring_off, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return INLA_ERR_HIP;
  ring_off += padded;
  return INLA_OK;
}

static constexpr size_t GRAPH_CACHE_MAX = 1024;

int Ctx::sequence(int cls, const std::vector<int64_t> &key, const void *args, size_t nbytes,
                  const std::function<void(const void *)> &body) {
  const int rc = sequence_impl(cls, key, args, nbytes, body);
  if (rc && !sticky) sticky = rc;
  return rc;
}

int Ctx::sequence_impl(int cls, const std::vector<int64_t> &key0, const void *args, size_t nbytes,
                       const std::function<void(const void *)> &body) {
  if (pg_mode != PG_OFF) {
    // inside a pass graph: the arguments take a slot of its block and the
    // launches become part of the pass
    const void *d = upload(args, nbytes);
    if (!d) return INLA_ERR_NOMEM;
    pg.sig.insert(pg.sig.end(), key0.begin(), key0.end());
    body(d);
    return check();
  }
  if (capturing) return INLA_ERR_UNSUPPORTED;   // sequences do not nest
  if (!graphs) {
    const void *d = upload(args, nbytes);
    if (!d) return INLA_ERR_NOMEM;
    body(d);
    return check();
  }
  // one graph (and argument block) per stream lane
  std::vector<int64_t> key = key0;
  key.push_back(lane);
  auto it = graph_cache.find(key);
  if (it == graph_cache.end()) {
    if (!cap_stream && hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess) return INLA_ERR_HIP;
    if (graph_cache.size() >= GRAPH_CACHE_MAX) {
      auto lru = graph_cache.begin();
      for (auto q = graph_cache.begin(); q != graph_cache.end(); ++q)
        if (q->second.used < lru->second.used) lru = q;
      if (sync_all() != INLA_OK) return INLA_ERR_HIP;
      (void)hipGraphExecDestroy(lru->second.exec);
      (void)hipFree(lru->second.dargs);
      graph_cache.erase(lru);
    }
    Graph g;
    if (hipMalloc(&g.dargs, align256(nbytes)) != hipSuccess) {
      (void)hipGetLastError();
      return INLA_ERR_NOMEM;
    }
    // capture on the handle's private stream: nothing runs while capturing
    hipStream_t user = stream;
    stream = cap_stream;
    capturing = true;
    cap_flops = cap_bytes = 0;
    hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) body(g.dargs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cap_stream, &graph) : e;
    stream = user;
    capturing = false;
    if (e == hipSuccess && e2 == hipSuccess && graph) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    else e = e != hipSuccess ? e : (e2 != hipSuccess ? e2 : hipErrorUnknown);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      last = e;
      (void)hipGetLastError();
      (void)hipFree(g.dargs);
      return INLA_ERR_HIP;
    }
    g.flops = cap_flops;
    g.bytes = cap_bytes;
    ++graphs_captured;
    it = graph_cache.emplace(key, std::move(g)).first;
  }
  Graph &g = it->second;
  g.used = ++graph_clock;
  if (g.last.size() != nbytes || std::memcmp(g.last.data(), args, nbytes) != 0) {
    int rc = upload_to(g.dargs, args, nbytes);
    if (rc) return rc;
    g.last.assign((const char *)args, (const char *)args + nbytes);
  }
  hipGraphExec_t ex = g.exec;
  ++graphs_replayed;
  hipError_t le = hipSuccess;
  launch(cls, g.flops, g.bytes, [&] { le = hipGraphLaunch(ex, stream); });
  if (le != hipSuccess) {
    last = le;
    return INLA_ERR_HIP;
  }
  return check();
}

void Ctx::drop_graphs() {
  if (graph_cache.empty() && pass_cache.empty()) return;
  (void)sync_all();
  for (auto &kv : graph_cache) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipFree(kv.second.dargs);
  }
  graph_cache.clear();
  for (auto &kv : pass_cache) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.dargs) (void)hipFree(kv.second.dargs);
  }
  pass_cache.clear();
}

// Argument block of one pass graph, and the number of passes the handle keeps
// (graphs and keys seen once, least recently used dropped first).
static constexpr size_t PASS_ARGS_CAP = 4u << 20;
static constexpr size_t PASS_CACHE_MAX = 64;

int Ctx::pass_graph(int cls, const std::vector<int64_t> &key0, const std::function<int()> &body) {
  if (!graphs || !pass_graphs || prof || capturing || pg_mode != PG_OFF) return body();
  std::vector<int64_t> key = key0;
  key.push_back(lane);
  const int sticky0 = sticky;
  auto drop = [&](std::map<std::vector<int64_t>, PassGraph>::iterator q) {
    if (q->second.exec) {
      (void)sync_all();
      (void)hipGraphExecDestroy(q->second.exec);
    }
    if (q->second.dargs) (void)hipFree(q->second.dargs);
    pass_cache.erase(q);
  };
  auto replay = [&](PassGraph &g, std::vector<char> &args) -> int {
    g.used = ++graph_clock;
    if (args != g.last) {
      const int rc = upload_to(g.dargs, args.data(), args.size());
      if (rc) return rc;
      g.last.swap(args);
    }
    ++pass_replayed;
    hipError_t le = hipSuccess;
    launch(cls, g.flops, g.bytes, [&] { le = hipGraphLaunch(g.exec, stream); });
    if (le != hipSuccess) {
      last = le;
      return INLA_ERR_HIP;
    }
    return check();
  };
  auto it = pass_cache.find(key);
  if (it != pass_cache.end() && it->second.exec) {
    // the host side of the pass, enqueueing nothing: its arguments in upload
    // order, and its launch signature
    PassGraph &g = it->second;
    pg = PassRec{};
    pg.dbase = g.dargs;
    pg.cap = g.cap;
    pg_mode = PG_COLLECT;
    const int rc = body();
    pg_mode = PG_OFF;
    if (rc == INLA_OK && !pg.overflow && pg.sig == g.sig) return replay(g, pg.host);
    sticky = sticky0;
    if (rc == INLA_OK && !pg.overflow) drop(it);   // the key does not fix this pass: capture it anew next time
    return body();
  }
  if (it == pass_cache.end()) {
    // first sighting: remember the key, run directly
    if (pass_cache.size() >= PASS_CACHE_MAX) {
      auto lru = pass_cache.begin();
      for (auto q = pass_cache.begin(); q != pass_cache.end(); ++q)
        if (q->second.used < lru->second.used) lru = q;
      drop(lru);
    }
    PassGraph g;
    g.used = ++graph_clock;
    pass_cache.emplace(key, std::move(g));
    return body();
  }
  // second sighting: capture on the handle's private stream
  PassGraph &g = it->second;
  if (!cap_stream && hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    cap_stream = nullptr;
    return body();
  }
  if (!g.dargs) {
    if (hipMalloc(&g.dargs, PASS_ARGS_CAP) != hipSuccess) {
      (void)hipGetLastError();
      g.dargs = nullptr;
      return body();
    }
    g.cap = PASS_ARGS_CAP;
  }
  pg = PassRec{};
  pg.dbase = g.dargs;
  pg.cap = g.cap;
  hipStream_t user = stream;
  stream = cap_stream;
  pg_mode = PG_CAPTURE;
  hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed);
  const int rc = e == hipSuccess ? body() : INLA_ERR_HIP;
  hipGraph_t graph = nullptr;
  const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cap_stream, &graph) : e;
  stream = user;
  pg_mode = PG_OFF;
  hipGraphExec_t exec = nullptr;
  bool ok = rc == INLA_OK && !pg.overflow && e == hipSuccess && e2 == hipSuccess && graph;
  if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok) {
    // nothing of the pass has run: run it directly
    (void)hipGetLastError();
    sticky = sticky0;
    drop(it);
    return body();
  }
  g.exec = exec;
  g.sig.swap(pg.sig);
  g.flops = pg.flops;
  g.bytes = pg.bytes;
  ++pass_captured;
  return replay(g, pg.host);
}

char *Ctx::pbf_reserve(size_t bytes) {
  if (bytes <= pbf_size) return pbf;
  if (pbf) {
    if (sync_all() != INLA_OK) return nullptr;
    (void)hipFree(pbf);
    pbf = nullptr;
    pbf_size = 0;
  }
  if (hipMalloc(&pbf, bytes) != hipSuccess) {
    (void)hipGetLastError();
    pbf = nullptr;
    return nullptr;
  }
  pbf_size = bytes;
  return pbf;
}

bool Ctx::reserve(size_t bytes) {
  if (bytes <= ws_size) return true;
  if (ws) {
    if (sync_all() != INLA_OK) return false;
    (void)hipFree(ws);
    ws = nullptr;
    ws_size = 0;
  }
  if (hipMalloc(&ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ws = nullptr;
    return false;
  }
  ws_size = bytes;
  return true;
}

void Ctx::launch(int cls, double flops, double bytes, const std::function<void()> &f) {
  if (pg_mode != PG_OFF) {
    pg.sig.insert(pg.sig.end(), {cls, (int64_t)std::llround(flops), (int64_t)std::llround(bytes)});
    pg.flops += flops;
    pg.bytes += bytes;
    if (pg_mode == PG_CAPTURE) f();
    return;
  }
  if (capturing) {
    cap_flops += flops;
    cap_bytes += bytes;
    f();
    return;
  }
  if (!prof) {
    f();
    return;
  }
  hipEvent_t a, b;
  if (event_pool.size() >= 2) {
    a = event_pool.back(); event_pool.pop_back();
    b = event_pool.back(); event_pool.pop_back();
  } else {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  (void)hipEventRecord(a, stream);
  f();
  (void)hipEventRecord(b, stream);
  pending.push_back({a, b, cls, prec_tag, flops, bytes});
  if (pending.size() >= 8192) harvest();
}

void Ctx::harvest() {
  if (pending.empty()) return;
  (void)sync_all();
  for (auto &p : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      inla_kstats &s = stats[p.cls][p.prec];
      s.launches += 1;
      s.time_ms += ms;
      s.flops += p.flops;
      s.bytes += p.bytes;
    }
    event_pool.push_back(p.a);
    event_pool.push_back(p.b);
  }
  pending.clear();
}

int Ctx::check() {
  if (sticky) {
    const int r = sticky;
    sticky = 0;
    return r;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    last = e;
    return INLA_ERR_HIP;
  }
  return INLA_OK;
}

Ctx::~Ctx() {
  if (stream) (void)hipStreamSynchronize(stream);
  else (void)hipDeviceSynchronize();
  for (auto &p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : event_pool) (void)hipEventDestroy(e);
  for (auto &kv : graph_cache) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipFree(kv.second.dargs);
  }
  for (auto &kv : pass_cache) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.dargs) (void)hipFree(kv.second.dargs);
  }
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (hipStream_t *s : {&side, &aux})
    if (*s) {
      (void)hipStreamSynchronize(*s);
      (void)hipStreamDestroy(*s);
    }
  for (hipEvent_t e : {ev_a, ev_b, ev_c, ev_d})
    if (e) (void)hipEventDestroy(e);
  if (ws) (void)hipFree(ws);
  if (pbf) (void)hipFree(pbf);
  if (gh) (void)hipFree(gh);
  if (ring) (void)hipFree(ring);
  if (ring_host) (void)hipHostFree(ring_host);
}

// ------------------------------------------------------------------ planning
// Per-theta workspace plan.
struct Plan {
  ThetaDesc t{};
  size_t off_Qp = 0, off_W = 0, off_S = 0, off_vec = 0, off_linv = 0, off_linv_small = 0, off_obs = 0, off_symv = 0,
         bytes = 0;
  int ns_real = 0;
  bool needs_prior_build = false;
};

enum Mode { MODE_LAPLACE = 0, MODE_VAR = 1, MODE_LOGDET = 2 };

static int n_prior_params(int prior) { return prior == PRIOR_DENSE ? 0 : (prior == PRIOR_EXPCOV ? 2 : 3); }

// Validate one model; returns 0 or a negative argument index code.
static int check_model(const inla_model &m) {
  if (m.n < 1 || m.k < 0 || m.k >= m.n) return -1;
  if (m.m < 0 || (m.m > 0 && (m.nnz < 0 || !m.A_rowptr || (m.nnz > 0 && (!m.A_col || !m.A_val))))) return -1;
  if (m.lik != LIK_GAUSSIAN && m.lik != LIK_POISSON) return -1;
  if (!m.y) return -1;
  if (m.k > 0 && !m.C) return -1;
  if (m.prior == PRIOR_DENSE) {
    if (!m.Qprior || m.ldq < m.n) return -1;
  } else if (m.prior == PRIOR_EXPCOV) {
    if (!m.coords || m.n_s != m.n) return -1;
  } else if (m.prior == PRIOR_KRON) {
    if (!m.coords || m.n_s < 1 || m.n_t < 1 || (int64_t)m.n_s * m.n_t != m.n) return -1;
  } else {
    return -1;
  }
  return 0;
}

// aux: the plan of a prior pass run beside the Newton iteration; it reads the
// main plan's Q_prior (no slot of its own) and keeps no observation workspace.
static Plan make_plan(const inla_model &m, const double *th, Mode mode, bool aux = false) {
  Plan p;
  ThetaDesc &t = p.t;
  t.y = m.y; t.E = m.E; t.C = m.C; t.e = m.e; t.coords = m.coords; t.Quser = m.Qprior;
  t.n = m.n; t.k = m.k; t.lik = m.lik; t.prior = m.prior; t.n_s = m.n_s; t.n_t = m.n_t; t.ldquser = m.ldq;
  t.n_pad = round_up(m.n, PADN);
  const int npp = n_prior_params(m.prior);
  t.tau = npp ? std::exp(th[0]) : 1.0;
  t.rho = npp ? std::exp(th[1]) : 1.0;
  t.delta = npp == 3 ? std::exp(th[2]) : 0.0;
  const double lp = th[npp];
  t.lpar = m.lik == LIK_GAUSSIAN ? std::exp(lp) : lp;
  t.k_pad = round_up(m.k, PADN);
  t.ldqp = t.n_pad;
  if (mode == MODE_VAR) {
    t.Nw = t.n_pad + t.k_pad + t.n_pad;
    t.Ncw = t.n_pad + t.k_pad;
    t.Ns = t.k_pad + t.n_pad;
  } else {
    t.Nw = t.n_pad + round_up(m.k + 1, PADN);
    t.Ncw = t.Nw;
    t.Ns = t.k_pad + PADN;
  }
  t.ldw = t.Nw;
  t.lds = t.Ns;
  p.needs_prior_build = m.prior != PRIOR_DENSE;
  if (m.prior == PRIOR_EXPCOV) { t.ns_pad = t.n_pad; p.ns_real = m.n; }
  else if (m.prior == PRIOR_KRON) { t.ns_pad = round_up(m.n_s, PADN); p.ns_real = m.n_s; }
  t.Np = 2 * t.ns_pad;
  t.ldp = t.Np;
  // layout: [Qp][W/P alias][S][vectors][linv]
  size_t off = 0;
  p.off_Qp = off;
  if (!aux) off += align256(sizeof(double) * (size_t)t.n_pad * t.n_pad);
  p.off_W = off;
  const size_t wbytes = sizeof(double) * (size_t)t.ldw * t.Ncw;
  const size_t pbytes = sizeof(double) * (size_t)t.ldp * t.Np;
  off += align256(std::max(wbytes, pbytes));
  p.off_S = off; off += align256(sizeof(double) * (size_t)t.lds * std::max(t.k_pad, 1));
  p.off_vec = off;
  off += align256(sizeof(double) * (size_t)(5 * t.n_pad + 3 * std::max(t.k_pad, 64) + 2 * t.ldw + DRES_COUNT));
  // inverses of every 64 x 64 diagonal block: big factor (also used by the prior
  // build, whose order is at most n_pad) and kriging factor
  p.off_linv = off; off += align256(sizeof(double) * (size_t)t.n_pad * NBI);
  p.off_linv_small = off; off += align256(sizeof(double) * (size_t)std::max(t.k_pad, NBI) * NBI);
  // general design matrix: A x, g, W and log-likelihood per observation (the
  // prior pass reads none of it)
  t.m = aux ? 0 : m.m;
  t.A_rowptr = m.A_rowptr; t.A_col = m.A_col; t.A_val = m.A_val;
  p.off_obs = off; off += align256(sizeof(double) * 4 * (size_t)t.m);
  // Q_prior v partial sums (residuals and objective terms of the Newton passes)
  p.off_symv = off;
  if (!aux && mode == MODE_LAPLACE) off += align256(sizeof(double) * (size_t)(t.n_pad / 64 + 1) * t.n_pad);
  p.bytes = off;
  return p;
}

static void bind(Plan &p, char *base) {
  ThetaDesc &t = p.t;
  t.Qp = (double *)(base + p.off_Qp);
  t.W = (void *)(base + p.off_W);
  t.P = (double *)t.W;   // the prior build finishes before the working matrix is assembled
  t.S = (double *)(base + p.off_S);
  double *v = (double *)(base + p.off_vec);
  t.x = v; v += t.n_pad;
  t.r = v; v += t.n_pad;
  t.xn = v; v += t.n_pad;
  t.z = v; v += t.n_pad;
  t.u = v; v += t.n_pad;
  t.lam = v; v += std::max(t.k_pad, 64);
  t.dlam = v; v += std::max(t.k_pad, 64);
  t.rtwo = v; v += std::max(t.k_pad, 64);
  t.part = v; v += 2 * t.ldw;
  t.dres = v;
  t.linv = (void *)(base + p.off_linv);
  t.symv = (double *)(base + p.off_symv);
  if (t.m > 0) {
    double *o = (double *)(base + p.off_obs);
    t.obs_ax = o; t.obs_g = o + t.m; t.obs_W = o + 2 * (size_t)t.m; t.obs_ll = o + 3 * (size_t)t.m;
  }
}

// State shared by the passes of one call.
struct Batch {
  Ctx &ctx;
  std::vector<Plan> plans;
  std::vector<char *> bases;
  int *dinfo = nullptr;        // device [B * 4]: prior-build, big, small, spare
  double *ddres_all = nullptr; // device copy target list not needed: dres live in workspace
  std::vector<int> hinfo;
  std::vector<double> hdres;
  double *pin = nullptr;       // pinned staging for results
  std::vector<ThetaDesc> last_td;   // host copy of the last uploaded descriptor array
  char *design = nullptr;           // device: CSC and A^T A patterns of the general design matrices
  explicit Batch(Ctx &c) : ctx(c) {}
};

// HostFactor for one of the three matrices of a theta.
enum { F_PRIOR = 0, F_BIG = 1, F_SMALL = 2 };
static HostFactor factor_of(const Plan &p, int which, int *info, void *linv, Mode mode) {
  const ThetaDesc &t = p.t;
  HostFactor h{};
  h.d.info = info;
  h.d.linv = linv;
  h.d.id_row0 = std::numeric_limits<int>::max();
  if (which == F_PRIOR) {
    h.d.A = (void *)t.P; h.d.ld = t.ldp; h.d.nf = t.ns_pad; h.d.nrows = t.Np; h.d.ncols = t.Np; h.d.id_row0 = t.ns_pad;
    h.n_real = p.ns_real; h.kb_real = p.ns_real; h.ks_real = p.ns_real;
  } else if (which == F_BIG) {
    h.d.A = t.W; h.d.ld = t.ldw; h.d.nf = t.n_pad; h.d.nrows = t.Nw; h.d.ncols = t.Ncw;
    h.n_real = t.n;
    if (mode == MODE_VAR) {
      h.d.id_row0 = t.n_pad + t.k_pad;
      h.kb_real = t.k_pad + t.n;   // counts the identity rows as border rows
      h.ks_real = t.k;
    } else if (mode == MODE_LOGDET) {
      h.kb_real = 0; h.ks_real = 0;
    } else {
      h.kb_real = t.k + 1; h.ks_real = t.k + 1;
    }
  } else {
    h.d.A = t.S; h.d.ld = t.lds; h.d.nf = t.k_pad; h.d.nrows = t.Ns; h.d.ncols = t.k_pad;
    h.n_real = t.k;
    h.kb_real = mode == MODE_VAR ? t.n : 1;
    h.ks_real = 0;
  }
  return h;
}

// Upload the descriptors of a subset of thetas.
static ThetaDesc *upload_td(Batch &b, const std::vector<int> &ids) {
  std::vector<ThetaDesc> v;
  v.reserve(ids.size());
  for (int i : ids) v.push_back(b.plans[i].t);
  b.last_td = v;
  return (ThetaDesc *)b.ctx.upload(v.data(), sizeof(ThetaDesc) * v.size());
}

static int run_factor(Batch &b, const std::vector<int> &ids, int which, Mode mode, int prec = INLA_PREC_FP64) {
  std::vector<HostFactor> fs;
  for (int i : ids) {
    const Plan &p = b.plans[i];
    const size_t lo = which == F_SMALL ? p.off_linv_small : p.off_linv;
    HostFactor h = factor_of(p, which, b.dinfo + 4 * i + which, (void *)(b.bases[i] + lo), mode);
    if (h.d.nf > 0) fs.push_back(h);
  }
  return factor_batch(b.ctx, fs, prec);
}

// Read back dres and info of every theta (one synchronisation).
static int readback(Batch &b) {
  const int B = (int)b.plans.size();
  for (int i = 0; i < B; ++i) {
    if (hipMemcpyAsync(b.pin + DRES_COUNT * i, b.plans[i].t.dres, sizeof(double) * DRES_COUNT, hipMemcpyDeviceToHost,
                       b.ctx.stream) != hipSuccess)
      return INLA_ERR_HIP;
  }
  int *ipin = (int *)(b.pin + DRES_COUNT * B);
  if (hipMemcpyAsync(ipin, b.dinfo, sizeof(int) * 4 * B, hipMemcpyDeviceToHost, b.ctx.stream) != hipSuccess)
    return INLA_ERR_HIP;
  if (hipStreamSynchronize(b.ctx.stream) != hipSuccess) return INLA_ERR_HIP;
  b.hdres.assign(b.pin, b.pin + DRES_COUNT * B);
  b.hinfo.assign(ipin, ipin + 4 * B);
  return b.ctx.check();
}

static int max_over(const Batch &b, const std::vector<int> &ids, int ThetaDesc::*f) {
  int m = 0;
  for (int i : ids) m = std::max(m, b.plans[i].t.*f);
  return m;
}

// Prior build for every theta: Sigma^{-1} by the identity-bordered factorisation,
// then Q_prior.
static int prior_build(Batch &b, const std::vector<int> &ids) {
  std::vector<int> pb;
  for (int i : ids) if (b.plans[i].needs_prior_build) pb.push_back(i);
  int rc;
  if (!pb.empty()) {
    ThetaDesc *d = upload_td(b, pb);
    if (!d) return INLA_ERR_NOMEM;
    launch_expcov_bordered(b.ctx, d, (int)pb.size(), max_over(b, pb, &ThetaDesc::Np));
    if ((rc = run_factor(b, pb, F_PRIOR, MODE_LAPLACE))) return rc;
  }
  ThetaDesc *d = upload_td(b, ids);
  if (!d) return INLA_ERR_NOMEM;
  double bytes = 0;
  for (int i : ids) bytes += 8.0 * 0.5 * b.plans[i].t.n * (b.plans[i].t.n + 1.0);
  launch_prior_assemble(b.ctx, d, (int)ids.size(), max_over(b, ids, &ThetaDesc::n_pad), bytes);
  return b.ctx.check();
}

// One pass: assemble the bordered matrix at the current x, factor it, build and
// factor the kriging system, solve it; then (Newton) form the corrected
// right-hand side and back-substitute, or (prior / final) reduce the log-dets.
// PASS_STEP: a Newton step in correction form (factor and kriging system only;
// the correction itself is one refinement step from the current iterate).
enum Pass { PASS_PRIOR = 0, PASS_NEWTON = 1, PASS_FINAL = 2, PASS_STEP = 3 };

// Key of a pass graph: the pass, its precision, the tuning table's state and
// the sizes of every theta, in order (they fix every grid and scalar argument;
// the pass graph also checks the launch signature).
static std::vector<int64_t> pass_key(const Batch &b, const std::vector<int> &ids, int64_t tag, int prec) {
  std::vector<int64_t> k = {0x50415353, tag, prec, (int64_t)b.ctx.tune_epoch, (int64_t)ids.size()};
  for (int i : ids) {
    const ThetaDesc &t = b.plans[i].t;
    k.insert(k.end(), {t.n, t.k, t.n_pad, t.Nw, t.Ncw, t.k_pad, t.Ns, t.m, t.lik, t.prior});
  }
  return k;
}

static int run_pass_body(Batch &b, const std::vector<int> &ids, Pass pass, int prec);

// A pass of every theta in `ids`, enqueued as one hipGraph per pass shape where
// graphs allow (FP64 and FP32 passes; the BF16 trailing update's packed panel
// copies grow their buffer between launches).
static int run_pass(Batch &b, const std::vector<int> &ids, Pass pass, int prec) {
  PrecScope tag(b.ctx, prec);
  if (ids.empty()) return 0;
  if (prec == INLA_PREC_BF16) return run_pass_body(b, ids, pass, prec);
  return b.ctx.pass_graph(INLA_K_TRAIL, pass_key(b, ids, pass, prec),
                          [&]() -> int { return run_pass_body(b, ids, pass, prec); });
}

static int run_pass_body(Batch &b, const std::vector<int> &ids, Pass pass, int prec) {
  ThetaDesc *d = upload_td(b, ids);
  if (!d) return INLA_ERR_NOMEM;
  const int B = (int)ids.size();
  const double esz = prec != INLA_PREC_FP64 ? 4.0 : 8.0;
  double abytes = 0, tbytes = 0;
  for (int i : ids) {
    const ThetaDesc &t = b.plans[i].t;
    abytes += (8.0 + esz) * (0.5 * t.n * (t.n + 1.0)) + esz * (double)t.n * (t.k + 1);
    tbytes += esz * 0.5 * t.n * (t.n + 1.0);
  }
  launch_assemble(b.ctx, d, B, max_over(b, ids, &ThetaDesc::Ncw), pass != PASS_PRIOR, pass == PASS_FINAL, BORDER_CB,
                  abytes, prec, max_over(b, ids, &ThetaDesc::m));
  int rc;
  if ((rc = run_factor(b, ids, F_BIG, MODE_LAPLACE, prec))) return rc;
  launch_kriging_build(b.ctx, d, B, max_over(b, ids, &ThetaDesc::k_pad), prec);
  if ((rc = run_factor(b, ids, F_SMALL, MODE_LAPLACE))) return rc;
  launch_kriging_solve(b.ctx, d, B);
  if (pass == PASS_NEWTON) {
    const int npm = max_over(b, ids, &ThetaDesc::n_pad);
    launch_rhs(b.ctx, d, B, npm, 0, prec);
    launch_trsv_bwd(b.ctx, b.last_td, npm, V_R, V_XN, tbytes, prec);
    if (prec == INLA_PREC_FP64) launch_newton_accept(b.ctx, d, B);
  } else if (pass == PASS_STEP) {
    launch_restart(b.ctx, d, B, max_over(b, ids, &ThetaDesc::n_pad));
  } else {
    launch_finish(b.ctx, d, B, prec);
  }
  return b.ctx.check();
}

// Mixed precision: refine the constrained Newton solve of every theta in `ids`
// on the KKT system with FP64 residuals, using the low-precision factor.
// Returns the thetas whose refinement did not reach ||dx|| <= tol_ir * max(1, ||x||).
//
// With eta > 0 the refinement is the inner solve of an inexact Newton step taken
// in correction form: it also stops once the correction is below
// min(eta, d1 / X) times d1, where d1 is the first correction (the Newton step
// itself) and X the iterate's scale, which keeps Newton's quadratic reduction of
// the step without solving each linear system to FP64 accuracy.
static int refine(Batch &b, const std::vector<int> &ids, int prec, int max_ir, double tol_ir, std::vector<int> &failed,
                  std::vector<int> &steps, double eta = 0.0) {
  PrecScope tag(b.ctx, prec);
  std::vector<int> act = ids;
  std::vector<double> d1(b.plans.size(), 0.0);
  const double esz = prec != INLA_PREC_FP64 ? 4.0 : 8.0;
  for (int s = 1; s <= max_ir && !act.empty(); ++s) {
    // one refinement step of every theta in `act` (one hipGraph per shape)
    int rc = b.ctx.pass_graph(INLA_K_SOLVE, pass_key(b, act, 0x4952, prec), [&]() -> int {
      ThetaDesc *d = upload_td(b, act);
      if (!d) return INLA_ERR_NOMEM;
      const int B = (int)act.size();
      double rb = 0, tb = 0;
      for (int i : act) {
        const ThetaDesc &t = b.plans[i].t;
        rb += 8.0 * 0.5 * (double)t.n * (t.n + 1.0);   // the lower triangle of Q_prior
        tb += esz * (double)t.n * t.n;
      }
      const int npm = max_over(b, act, &ThetaDesc::n_pad), kpm = max_over(b, act, &ThetaDesc::k_pad);
      launch_kkt_residual(b.ctx, d, B, npm, kpm, rb);
      launch_trsv_fwd(b.ctx, b.last_td, npm, V_Z, V_U, 0.5 * tb, prec);
      launch_ir_correct(b.ctx, d, B, kpm, prec);
      launch_rhs(b.ctx, d, B, npm, 1, prec);
      launch_trsv_bwd(b.ctx, b.last_td, npm, V_R, V_U, 0.5 * tb, prec);
      launch_ir_update(b.ctx, d, B);
      return b.ctx.check();
    });
    if (rc) return rc;
    for (int i : act) steps[i] += 1;
    {
      if ((rc = readback(b))) return rc;
      std::vector<int> next;
      for (int i : act) {
        const double *dr = &b.hdres[DRES_COUNT * i];
        const double dx = dr[DRES_IR_DX], X = dr[DRES_IR_X];
        if (s == 1) d1[i] = dx;
        const bool inner = eta > 0.0 && s > 1 && dx <= std::min(eta, d1[i] / X) * d1[i];
        if (!(dx <= tol_ir * X) && !inner) next.push_back(i);
      }
      act.swap(next);
    }
  }
  failed = act;
  return b.ctx.check();
}

static int setup_design(Batch &b, const inla_model *models, int B);

// Allocate and bind the workspace of a batch; zero the per-theta scratch.  With
// `aux`, the same allocation also holds the workspace of a prior pass run on
// the aux stream (the aux batch shares the main batch's Q_prior).
static int setup(Batch &b, int B, const inla_model *models, const double *theta, int ldtheta, Mode mode,
                 Batch *aux = nullptr) {
  const int nb = aux ? 2 : 1;
  Batch *bs[2] = {&b, aux};
  size_t total = 0;
  std::vector<size_t> offs[2];
  for (int q = 0; q < nb; ++q) {
    bs[q]->plans.resize(B);
    offs[q].resize(B);
    for (int i = 0; i < B; ++i) {
      bs[q]->plans[i] = make_plan(models[i], theta ? theta + (size_t)i * ldtheta : nullptr, mode, q == 1);
      offs[q][i] = total;
      total += bs[q]->plans[i].bytes;
    }
  }
  const size_t info_off = total;
  total += nb * align256(sizeof(int) * 4 * B);
  if (!b.ctx.reserve(total)) return INLA_ERR_NOMEM;
  for (int q = 0; q < nb; ++q) {
    Batch &x = *bs[q];
    x.bases.resize(B);
    for (int i = 0; i < B; ++i) {
      x.bases[i] = b.ctx.ws + offs[q][i];
      bind(x.plans[i], x.bases[i]);
      if (q == 1) x.plans[i].t.Qp = b.plans[i].t.Qp;
    }
    x.dinfo = (int *)(b.ctx.ws + info_off + q * align256(sizeof(int) * 4 * B));
    if (hipMemsetAsync(x.dinfo, 0, sizeof(int) * 4 * B, b.ctx.stream) != hipSuccess) return INLA_ERR_HIP;
    for (int i = 0; i < B; ++i) {
      const ThetaDesc &t = x.plans[i].t;
      if (hipMemsetAsync(t.dres, 0, sizeof(double) * DRES_COUNT, b.ctx.stream) != hipSuccess) return INLA_ERR_HIP;
      // the prior pass never reads its iterate; zero it all the same
      if (q == 1 && hipMemsetAsync(t.x, 0, sizeof(double) * t.n_pad, b.ctx.stream) != hipSuccess) return INLA_ERR_HIP;
    }
    if (hipHostMalloc(&x.pin, sizeof(double) * DRES_COUNT * B + sizeof(int) * 4 * B + 64) != hipSuccess)
      return INLA_ERR_NOMEM;
  }
  return setup_design(b, models, B);
}

static void teardown(Batch &b) {
  if (b.pin) (void)hipHostFree(b.pin);
  b.pin = nullptr;
  if (b.design) {
    (void)hipStreamSynchronize(b.ctx.stream);
    (void)hipFree(b.design);
    b.design = nullptr;
  }
}

// Host-side structures of a general design matrix A (m x n, CSR): its CSC and
// the lower pattern of A^T A, each entry (r, c) with the observations i that
// contribute A_{i r} A_{i c} to (A^T W A)_{r c}.
struct DesignHost {
  std::vector<int> cscp, csci, patp, patr, patt, tobs;
  std::vector<double> cscv, tcoef;
};

static int build_design(const inla_model &m, hipStream_t s, DesignHost &dh) {
  const int M = m.m, n = m.n;
  std::vector<int> rp(M + 1), ci;
  std::vector<double> v;
  if (hipMemcpyAsync(rp.data(), m.A_rowptr, sizeof(int) * (M + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return INLA_ERR_HIP;
  const int nnz = rp[M];
  if (rp[0] != 0 || nnz != m.nnz) return -3;
  for (int i = 0; i < M; ++i)
    if (rp[i + 1] < rp[i]) return -3;
  ci.resize(nnz);
  v.resize(nnz);
  if (nnz > 0 && (hipMemcpyAsync(ci.data(), m.A_col, sizeof(int) * nnz, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipMemcpyAsync(v.data(), m.A_val, sizeof(double) * nnz, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipStreamSynchronize(s) != hipSuccess))
    return INLA_ERR_HIP;
  for (int c : ci)
    if (c < 0 || c >= n) return -3;
  // CSC
  dh.cscp.assign(n + 1, 0);
  for (int c : ci) dh.cscp[c + 1]++;
  for (int c = 0; c < n; ++c) dh.cscp[c + 1] += dh.cscp[c];
  dh.csci.resize(nnz);
  dh.cscv.resize(nnz);
  std::vector<int> fill(dh.cscp.begin(), dh.cscp.end() - 1);
  for (int i = 0; i < M; ++i)
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      const int q = fill[ci[p]]++;
      dh.csci[q] = i;
      dh.cscv[q] = v[p];
    }
  // lower pattern of A^T A: per column c, rows r >= c in increasing order
  std::vector<std::map<int, std::vector<std::pair<int, double>>>> cols(n);
  for (int i = 0; i < M; ++i)
    for (int a = rp[i]; a < rp[i + 1]; ++a)
      for (int b = rp[i]; b < rp[i + 1]; ++b) {
        const int r = ci[a], c = ci[b];
        if (r < c) continue;
        if (r == c && a != b) continue;   // a repeated column index: its diagonal term comes from (a, a)
        cols[c][r].push_back({i, v[a] * v[b]});
      }
  dh.patp.assign(n + 1, 0);
  dh.patt.assign(1, 0);
  for (int c = 0; c < n; ++c) {
    for (auto &kv : cols[c]) {
      dh.patr.push_back(kv.first);
      for (auto &tr : kv.second) {
        dh.tobs.push_back(tr.first);
        dh.tcoef.push_back(tr.second);
      }
      dh.patt.push_back((int)dh.tobs.size());
    }
    dh.patp[c + 1] = (int)dh.patr.size();
  }
  return INLA_OK;
}

// Upload the design structures of every model with a general A (one copy per
// distinct A) and bind them into the descriptors.
static int setup_design(Batch &b, const inla_model *models, int B) {
  std::map<const int32_t *, int> seen;
  std::vector<DesignHost> hs;
  std::vector<int> which(B, -1);
  for (int i = 0; i < B; ++i) {
    if (models[i].m == 0) continue;
    auto it = seen.find(models[i].A_rowptr);
    if (it == seen.end()) {
      DesignHost dh;
      const int rc = build_design(models[i], b.ctx.stream, dh);
      if (rc) return rc;
      it = seen.emplace(models[i].A_rowptr, (int)hs.size()).first;
      hs.push_back(std::move(dh));
    }
    which[i] = it->second;
  }
  if (hs.empty()) return INLA_OK;
  // one allocation: per design [cscp csci patp patr patt tobs | cscv tcoef]
  std::vector<size_t> off(hs.size());
  size_t total = 0;
  auto a8 = [](size_t v) { return (v + 255) & ~size_t(255); };
  for (size_t d = 0; d < hs.size(); ++d) {
    const DesignHost &h = hs[d];
    off[d] = total;
    total += a8(4 * (h.cscp.size() + h.csci.size() + h.patp.size() + h.patr.size() + h.patt.size() + h.tobs.size())) +
             a8(8 * (h.cscv.size() + h.tcoef.size())) + 256;
  }
  if (hipMalloc(&b.design, total) != hipSuccess) {
    (void)hipGetLastError();
    b.design = nullptr;
    return INLA_ERR_NOMEM;
  }
  std::vector<char> host(total, 0);
  struct Ptrs { const int *cscp, *csci, *patp, *patr, *patt, *tobs; const double *cscv, *tcoef; };
  std::vector<Ptrs> ptrs(hs.size());
  for (size_t d = 0; d < hs.size(); ++d) {
    const DesignHost &h = hs[d];
    size_t o = off[d];
    auto put_i = [&](const std::vector<int> &vec) {
      std::memcpy(host.data() + o, vec.data(), 4 * vec.size());
      const int *p = (const int *)(b.design + o);
      o += 4 * vec.size();
      return p;
    };
    Ptrs &P = ptrs[d];
    P.cscp = put_i(h.cscp); P.csci = put_i(h.csci); P.patp = put_i(h.patp);
    P.patr = put_i(h.patr); P.patt = put_i(h.patt); P.tobs = put_i(h.tobs);
    o = off[d] + a8(4 * (h.cscp.size() + h.csci.size() + h.patp.size() + h.patr.size() + h.patt.size() + h.tobs.size()));
    std::memcpy(host.data() + o, h.cscv.data(), 8 * h.cscv.size());
    P.cscv = (const double *)(b.design + o);
    o += 8 * h.cscv.size();
    std::memcpy(host.data() + o, h.tcoef.data(), 8 * h.tcoef.size());
    P.tcoef = (const double *)(b.design + o);
  }
  if (hipMemcpy(b.design, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) return INLA_ERR_HIP;
  for (int i = 0; i < B; ++i) {
    if (which[i] < 0) continue;
    const Ptrs &P = ptrs[which[i]];
    ThetaDesc &t = b.plans[i].t;
    t.cscp = P.cscp; t.csci = P.csci; t.cscv = P.cscv;
    t.patp = P.patp; t.patr = P.patr; t.patt = P.patt; t.tobs = P.tobs; t.tcoef = P.tcoef;
  }
  return INLA_OK;
}

// Memory budget for one chunk of thetas: 85% of the device's free memory.
static size_t budget(Ctx &ctx) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (size_t)64 << 30;
  return (size_t)((fr + ctx.ws_size) * 0.85);
}

static int validate_common(inla_handle *h, int B, const inla_model *models, const double *theta, int ldtheta,
                           inla_result *res_or_null, bool need_res) {
  if (!h) return -1;
  if (B < 0) return -2;
  if (B > 0 && !models) return -3;
  if (B > 0 && !theta) return -4;
  int maxp = 0;
  for (int i = 0; i < B; ++i) {
    if (check_model(models[i])) return -3;
    maxp = std::max(maxp, n_prior_params(models[i].prior) + 1);
  }
  if (B > 0 && ldtheta < maxp) return -5;
  if (need_res && B > 0 && !res_or_null) return -8;
  return 0;
}

// Split [0, B) into chunks whose workspace fits the budget.
static std::vector<std::pair<int, int>> chunks(Ctx &ctx, int B, const inla_model *models, const double *theta,
                                               int ldtheta, Mode mode, bool aux = false) {
  std::vector<std::pair<int, int>> out;
  const size_t cap = budget(ctx);
  int s = 0;
  while (s < B) {
    size_t tot = 0;
    int e = s;
    while (e < B) {
      const double *th = theta + (size_t)e * ldtheta;
      const size_t need = make_plan(models[e], th, mode).bytes + (aux ? make_plan(models[e], th, mode, true).bytes : 0) +
                          8192;
      if (e > s && tot + need > cap) break;
      tot += need;
      ++e;
    }
    out.push_back({s, e});
    s = e;
  }
  return out;
}

// The whole per-theta evaluation for one chunk.  `prec` selects the precision
// of the Newton and final-pass factorisations (the prior pass is always FP64).
// A theta whose mixed-precision refinement does not converge is re-evaluated
// in FP64 and flagged.
static int eval_chunk(Ctx &ctx, int B, const inla_model *models, const double *theta, int ldtheta, double *const *x,
                      const inla_opts *opts, inla_result *res, bool laplace) {
  // The prior pass depends on theta alone, and the Newton passes never read
  // its factor (they assemble Q_prior + W from the built prior), so with
  // overlap on it runs on the aux stream, in its own workspace, while the
  // caller's stream runs the Newton iteration; its results are read after the
  // iteration.  Every kernel computes what it would in order, so the results
  // are identical either way.
  const bool overlap = ctx.overlap && ctx.aux_ready() == INLA_OK;
  Batch b(ctx), pb(ctx);
  int rc = setup(b, B, models, theta, ldtheta, MODE_LAPLACE, overlap ? &pb : nullptr);
  if (rc) { (void)ctx.sync_all(); teardown(pb); teardown(b); return rc; }
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 50;
  const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-11;
  const bool warm = opts && opts->start == 1;
  const int prec = opts ? opts->prec : INLA_PREC_FP64;
  const bool mixed = prec != INLA_PREC_FP64;
  const int ref_prec = prec == INLA_PREC_BF16 ? INLA_PREC_FP32 : prec;   // refined steps and the final pass
  const int max_ir = 10;
  const double tol_ir = 1e-13;
  std::vector<int> all, ok;
  for (int i = 0; i < B; ++i) {
    res[i] = inla_result{};
    const ThetaDesc &t = b.plans[i].t;
    bool finite = true;
    for (int j = 0; j < ldtheta && j <= n_prior_params(t.prior); ++j) finite = finite && std::isfinite(theta[(size_t)i * ldtheta + j]);
    if (!finite) { res[i].info = INLA_INFO_NONFINITE; continue; }
    all.push_back(i);
    if (warm) {
      if (hipMemcpyAsync(t.x, x[i], sizeof(double) * t.n, hipMemcpyDeviceToDevice, ctx.stream) != hipSuccess) { teardown(pb); teardown(b); return INLA_ERR_HIP; }
      if (t.n_pad > t.n && hipMemsetAsync(t.x + t.n, 0, sizeof(double) * (t.n_pad - t.n), ctx.stream) != hipSuccess) { teardown(pb); teardown(b); return INLA_ERR_HIP; }
    } else if (hipMemsetAsync(t.x, 0, sizeof(double) * t.n_pad, ctx.stream) != hipSuccess) {
      teardown(pb); teardown(b); return INLA_ERR_HIP;
    }
    if (mixed && (hipMemsetAsync(t.lam, 0, sizeof(double) * std::max(t.k_pad, 64), ctx.stream) != hipSuccess ||
                  hipMemsetAsync(t.xn, 0, sizeof(double) * t.n_pad, ctx.stream) != hipSuccess)) {
      teardown(pb); teardown(b); return INLA_ERR_HIP;
    }
  }
  auto fail = [&](int r) { (void)ctx.sync_all(); teardown(pb); teardown(b); return r; };
  // prior-pass status and results of theta i (from the host copy read back
  // from `pp`); returns whether theta i passed
  auto prior_ok = [&](Batch &pp, int i) {
    const int *inf = &pp.hinfo[4 * i];
    const double *dr = &pp.hdres[DRES_COUNT * i];
    if (inf[F_PRIOR]) { res[i].info = inf[F_PRIOR]; return false; }
    if (inf[F_BIG]) { res[i].info = inf[F_BIG]; return false; }
    if (inf[F_SMALL] || dr[DRES_RANK] != 0.0) { res[i].info = INLA_INFO_CONSTRAINT_RANK; return false; }
    res[i].logdet_qprior = dr[DRES_LOGDET_L];
    res[i].logdet_sprior = dr[DRES_LOGDET_S];
    res[i].ese = dr[DRES_WNORM2];
    return true;
  };
  if ((rc = prior_build(b, all))) return fail(rc);
  if (overlap) {
    if (!all.empty()) {
      // the prior build's status travels with the prior pass's (the Newton
      // iteration clears the main batch's status slots)
      if (hipMemcpyAsync(pb.dinfo, b.dinfo, sizeof(int) * 4 * B, hipMemcpyDeviceToDevice, ctx.stream) != hipSuccess ||
          hipEventRecord(ctx.ev_c, ctx.stream) != hipSuccess || hipStreamWaitEvent(ctx.aux, ctx.ev_c, 0) != hipSuccess)
        return fail(INLA_ERR_HIP);
      {
        AuxScope lane(ctx);
        rc = run_pass(pb, all, PASS_PRIOR, INLA_PREC_FP64);
      }
      if (rc) return fail(rc);
      if (hipEventRecord(ctx.ev_d, ctx.aux) != hipSuccess) return fail(INLA_ERR_HIP);
    }
    ok = all;   // prior failures are sorted out after the Newton iteration
  } else {
    if ((rc = run_pass(b, all, PASS_PRIOR, INLA_PREC_FP64))) return fail(rc);
    if ((rc = readback(b))) return fail(rc);
    for (int i : all)
      if (prior_ok(b, i)) ok.push_back(i);
  }
  // Newton iteration (warm-start vectors were checked for finiteness by the
  // first assembly: a non-finite W or b sets the flag).
  std::vector<int> active = ok, done, redo;
  std::vector<char> failed(B, 0);
  std::vector<int> irsteps(B, 0), last_ir(B, 0), far_ir(B, 0);
  std::vector<double> prev_step(B, INFINITY), prev_scale(B, 1.0);
  for (int it = 1; it <= max_iter && !active.empty(); ++it) {
    if (hipMemsetAsync(b.dinfo, 0, sizeof(int) * 4 * B, ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    if (!mixed) {
      if ((rc = run_pass(b, active, PASS_NEWTON, prec))) return fail(rc);
    } else {
      // Every Newton step with a low-precision factor is taken in correction
      // form: x + the solution of the KKT system whose right-hand side is the
      // FP64 residual at x.  Solved for the whole next iterate instead, the
      // step would carry an error of order kappa u |x| that never shrinks (and
      // larger through the constraint block C Q^{-1} C^T, which the factor
      // forms by cancellation); in correction form the error is of order
      // kappa u times the step.  Far from the mode (previous step above 1e-3
      // of the iterate's scale) one refinement step is taken, with BF16
      // trailing operands in BF16 mode.  Near the mode the factor is FP32 and
      // the step is refined until the correction falls below min(1e-3, step)
      // times the step, which keeps Newton's quadratic convergence; such a
      // step counts as refined: its size bounds the distance to the exact
      // Newton iterate.  A Gaussian likelihood's single Newton step is exact,
      // so it is solved once and refined to FP64 accuracy.
      std::vector<int> gauss, near, far, nconv;
      for (int i : active) {
        if (b.plans[i].t.lik == LIK_GAUSSIAN) gauss.push_back(i);
        else if (prev_step[i] <= 1e-3 * prev_scale[i]) near.push_back(i);
        else far.push_back(i);
      }
      std::vector<int> unconv;
      if (!far.empty()) {
        if ((rc = run_pass(b, far, PASS_STEP, prec))) return fail(rc);
        if ((rc = refine(b, far, prec, 1, 0.0, unconv, far_ir))) return fail(rc);
      }
      if (!near.empty()) {
        if ((rc = run_pass(b, near, PASS_STEP, ref_prec))) return fail(rc);
        if ((rc = refine(b, near, ref_prec, max_ir, tol_ir, nconv, irsteps, 1e-3))) return fail(rc);
      }
      if (!gauss.empty()) {
        if ((rc = run_pass(b, gauss, PASS_NEWTON, ref_prec))) return fail(rc);
        if ((rc = refine(b, gauss, ref_prec, max_ir, tol_ir, nconv, irsteps))) return fail(rc);
      }
      for (int i : nconv) { failed[i] = 1; redo.push_back(i); }
      std::vector<int> keep;
      for (int i : active) if (!failed[i]) keep.push_back(i);
      active.swap(keep);
      ThetaDesc *d = upload_td(b, active);
      if (!active.empty() && !d) return fail(INLA_ERR_NOMEM);
      launch_newton_accept(ctx, d, (int)active.size());
    }
    if ((rc = readback(b))) return fail(rc);
    std::vector<int> next;
    for (int i : active) {
      const int *inf = &b.hinfo[4 * i];
      const double *dr = &b.hdres[DRES_COUNT * i];
      res[i].iters = it;
      // A low-precision factor that meets a non-positive pivot, or whose kriging
      // system comes out numerically singular, says nothing about Q* itself:
      // the prior pass (FP64) has already checked C's rank, and Q* may be
      // positive definite in FP64 while its FP32 factorisation breaks down
      // (condition number beyond 1 / u_32).  Such a theta is re-evaluated in
      // FP64.  The failed factor's NaNs also reach the iterate, so this test
      // comes before the non-finite one.
      if (mixed && (inf[F_BIG] || inf[F_SMALL] || dr[DRES_RANK] != 0.0)) { failed[i] = 1; redo.push_back(i); continue; }
      if (dr[DRES_NONFINITE] != 0.0) { res[i].info = INLA_INFO_NONFINITE; failed[i] = 1; continue; }
      if (inf[F_BIG]) { res[i].info = inf[F_BIG]; failed[i] = 1; continue; }
      if (inf[F_SMALL] || dr[DRES_RANK] != 0.0) { res[i].info = INLA_INFO_CONSTRAINT_RANK; failed[i] = 1; continue; }
      res[i].step = dr[DRES_STEP];
      const double before = prev_step[i];
      prev_step[i] = dr[DRES_STEP];
      prev_scale[i] = dr[DRES_SCALE];
      const bool refined = !mixed || irsteps[i] > last_ir[i];
      last_ir[i] = irsteps[i];
      // a mixed-precision step only counts once it was refined to FP64 accuracy
      bool conv = refined && (b.plans[i].t.lik == LIK_GAUSSIAN || dr[DRES_STEP] <= tol * dr[DRES_SCALE]);
      // Mixed precision also stops on the predicted error of the new iterate:
      // with quadratic convergence it is about C s^2, C estimated from the last
      // two steps as s / s_prev^2; a refined step s <= 1e-7 of the scale whose
      // prediction is below a tenth of the tolerance ends the iteration one
      // step before the step itself would.  The reused factor then sits within
      // s of the mode, which moves log|Q*| by at most about n s (relative
      // ~1e-8 at the configurations here, below the FP32 factor's own error).
      if (!conv && mixed && refined && it >= 2 && before > 0.0 && std::isfinite(before)) {
        const double sk = dr[DRES_STEP], sc = dr[DRES_SCALE];
        if (sk <= 1e-7 * sc && (sk / (before * before)) * sk * sk <= 0.1 * tol * sc) conv = true;
      }
      if (conv) done.push_back(i);
      else if (it == max_iter && mixed && !warm) { failed[i] = 1; redo.push_back(i); }   // FP64 re-evaluation
      else if (it == max_iter) { res[i].info = INLA_INFO_NEWTON_MAXIT; done.push_back(i); }
      else next.push_back(i);
    }
    active.swap(next);
  }
  if (overlap && !all.empty()) {
    // the prior pass: its status and log-determinants
    if (hipStreamWaitEvent(ctx.stream, ctx.ev_d, 0) != hipSuccess) return fail(INLA_ERR_HIP);
    if ((rc = readback(pb))) return fail(rc);
    std::vector<char> bad(B, 0);
    for (int i : all)
      if (!prior_ok(pb, i)) {
        // reported as without overlap: the status alone, no Newton work
        const int code = res[i].info;
        res[i] = inla_result{};
        res[i].info = code;
        irsteps[i] = far_ir[i] = 0;
        failed[i] = 1;
        bad[i] = 1;
      }
    std::vector<int> keep;
    for (int i : redo) if (!bad[i]) keep.push_back(i);
    redo.swap(keep);
  }
  // copy the modes out
  for (int i : ok) {
    if (failed[i]) continue;
    const ThetaDesc &t = b.plans[i].t;
    if (hipMemcpyAsync(x[i], t.x, sizeof(double) * t.n, hipMemcpyDeviceToDevice, ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
  }
  if (laplace) {
    std::vector<int> fin;
    for (int i : done) if (!failed[i]) fin.push_back(i);
    if (hipMemsetAsync(b.dinfo, 0, sizeof(int) * 4 * B, ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    if (mixed) {
      // The last Newton factorisation was taken at an iterate within the Newton
      // tolerance (1e-11) of the mode; its log-dets differ from a refactorisation
      // at the mode by far less than the FP32 factor's own error, so it is reused.
      PrecScope tag(ctx, ref_prec);
      ThetaDesc *d = upload_td(b, fin);
      if (!fin.empty() && !d) return fail(INLA_ERR_NOMEM);
      double by = 0;
      for (int i : fin) by += 8.0 * 0.5 * b.plans[i].t.n * (b.plans[i].t.n + 1.0);
      launch_objective_terms(ctx, d, (int)fin.size(), max_over(b, fin, &ThetaDesc::n_pad), by);
      launch_finish(ctx, d, (int)fin.size(), ref_prec);
    } else if ((rc = run_pass(b, fin, PASS_FINAL, prec))) {
      return fail(rc);
    }
    if ((rc = readback(b))) return fail(rc);
    for (int i : fin) {
      const int *inf = &b.hinfo[4 * i];
      const double *dr = &b.hdres[DRES_COUNT * i];
      if (inf[F_BIG]) { res[i].info = inf[F_BIG]; continue; }
      if (inf[F_SMALL] || dr[DRES_RANK] != 0.0) { res[i].info = INLA_INFO_CONSTRAINT_RANK; continue; }
      inla_result &r = res[i];
      r.logdet_qstar = dr[DRES_LOGDET_L];
      r.logdet_s = dr[DRES_LOGDET_S];
      r.xqx = dr[DRES_XQX];
      r.loglik = dr[DRES_LOGLIK];
      r.objective = 0.5 * r.logdet_qprior + 0.5 * r.logdet_sprior + 0.5 * r.ese - 0.5 * r.xqx + r.loglik -
                    0.5 * r.logdet_qstar - 0.5 * r.logdet_s;
    }
  } else {
    if (hipStreamSynchronize(ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
  }
  for (int i = 0; i < B; ++i) res[i].ir_steps = irsteps[i] + far_ir[i];
  ctx.harvest();
  teardown(pb);
  teardown(b);
  if ((rc = ctx.check())) return rc;
  // FP64 re-evaluation of thetas whose refinement did not converge
  if (!redo.empty()) {
    std::vector<inla_model> m2;
    std::vector<double> th2;
    std::vector<double *> x2;
    for (int i : redo) {
      m2.push_back(models[i]);
      th2.insert(th2.end(), theta + (size_t)i * ldtheta, theta + (size_t)(i + 1) * ldtheta);
      x2.push_back(x[i]);
    }
    inla_opts o2 = opts ? *opts : inla_opts{};
    o2.prec = INLA_PREC_FP64;
    std::vector<inla_result> r2(redo.size());
    rc = eval_chunk(ctx, (int)redo.size(), m2.data(), th2.data(), ldtheta, x2.data(), &o2, r2.data(), laplace);
    if (rc) return rc;
    for (size_t q = 0; q < redo.size(); ++q) {
      const int st = res[redo[q]].ir_steps;
      res[redo[q]] = r2[q];
      res[redo[q]].fallback = 1;
      res[redo[q]].ir_steps = st;
    }
  }
  return INLA_OK;
}

static int var_chunk(Ctx &ctx, int B, const inla_model *models, const double *theta, int ldtheta,
                     const double *const *xm, double *const *var, int32_t *info) {
  Batch b(ctx);
  int rc = setup(b, B, models, theta, ldtheta, MODE_VAR);
  if (rc) { teardown(b); return rc; }
  auto fail = [&](int r) { teardown(b); return r; };
  std::vector<int> all;
  for (int i = 0; i < B; ++i) {
    info[i] = 0;
    ThetaDesc &t = b.plans[i].t;
    t.out = var[i];
    if (hipMemcpyAsync(t.x, xm[i], sizeof(double) * t.n, hipMemcpyDeviceToDevice, ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    if (t.n_pad > t.n && hipMemsetAsync(t.x + t.n, 0, sizeof(double) * (t.n_pad - t.n), ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    all.push_back(i);
  }
  if ((rc = prior_build(b, all))) return fail(rc);
  ThetaDesc *d = upload_td(b, all);
  if (!d) return fail(INLA_ERR_NOMEM);
  launch_assemble(ctx, d, B, max_over(b, all, &ThetaDesc::Ncw), 1, 0, BORDER_CI, 0.0, INLA_PREC_FP64,
                  max_over(b, all, &ThetaDesc::m));
  if ((rc = run_factor(b, all, F_BIG, MODE_VAR))) return fail(rc);
  launch_var_small_build(ctx, d, B, max_over(b, all, &ThetaDesc::k_pad));
  if ((rc = run_factor(b, all, F_SMALL, MODE_VAR))) return fail(rc);
  launch_var_norms(ctx, d, B, max_over(b, all, &ThetaDesc::n_pad));
  if ((rc = readback(b))) return fail(rc);
  for (int i = 0; i < B; ++i) {
    const int *inf = &b.hinfo[4 * i];
    if (inf[F_PRIOR]) info[i] = inf[F_PRIOR];
    else if (inf[F_BIG]) info[i] = inf[F_BIG];
    else if (inf[F_SMALL]) info[i] = INLA_INFO_CONSTRAINT_RANK;
    else if (b.hdres[DRES_COUNT * i + DRES_NONFINITE] != 0.0) info[i] = INLA_INFO_NONFINITE;
  }
  ctx.harvest();
  teardown(b);
  return ctx.check();
}

// Variational-Bayes correction of the posterior mean for one chunk: from the
// Laplace mode in x, repeated constrained Newton-form passes whose likelihood
// terms are Gauss-Hermite expectations over the fixed marginal variances.
static int vb_chunk(Ctx &ctx, int B, const inla_model *models, const double *theta, int ldtheta,
                    const double *const *var, double *const *x, int ngh, int max_iter, double tol, int32_t *iters,
                    int32_t *info) {
  Batch b(ctx);
  int rc = setup(b, B, models, theta, ldtheta, MODE_LAPLACE);
  if (rc) { teardown(b); return rc; }
  auto fail = [&](int r) { teardown(b); return r; };
  std::vector<int> all;
  for (int i = 0; i < B; ++i) {
    iters[i] = 0;
    info[i] = 0;
    ThetaDesc &t = b.plans[i].t;
    t.vb_var = var[i];
    t.gh = ctx.gh;
    t.ngh = ngh;
    if (hipMemcpyAsync(t.x, x[i], sizeof(double) * t.n, hipMemcpyDeviceToDevice, ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    if (t.n_pad > t.n && hipMemsetAsync(t.x + t.n, 0, sizeof(double) * (t.n_pad - t.n), ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    all.push_back(i);
  }
  if ((rc = prior_build(b, all))) return fail(rc);
  std::vector<int> active = all;
  for (int it = 1; it <= max_iter && !active.empty(); ++it) {
    if (hipMemsetAsync(b.dinfo, 0, sizeof(int) * 4 * B, ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
    if ((rc = run_pass(b, active, PASS_NEWTON, INLA_PREC_FP64))) return fail(rc);
    if ((rc = readback(b))) return fail(rc);
    std::vector<int> next;
    for (int i : active) {
      const int *inf = &b.hinfo[4 * i];
      const double *dr = &b.hdres[DRES_COUNT * i];
      iters[i] = it;
      if (inf[F_PRIOR]) info[i] = inf[F_PRIOR];
      else if (dr[DRES_NONFINITE] != 0.0) info[i] = INLA_INFO_NONFINITE;
      else if (inf[F_BIG]) info[i] = inf[F_BIG];
      else if (inf[F_SMALL] || dr[DRES_RANK] != 0.0) info[i] = INLA_INFO_CONSTRAINT_RANK;
      else if (dr[DRES_STEP] <= tol * dr[DRES_SCALE]) continue;
      else if (it == max_iter) info[i] = INLA_INFO_NEWTON_MAXIT;
      else next.push_back(i);
    }
    active.swap(next);
  }
  for (int i = 0; i < B; ++i)
    if (info[i] == 0 &&
        hipMemcpyAsync(x[i], b.plans[i].t.x, sizeof(double) * b.plans[i].t.n, hipMemcpyDeviceToDevice, ctx.stream) != hipSuccess)
      return fail(INLA_ERR_HIP);
  if (hipStreamSynchronize(ctx.stream) != hipSuccess) return fail(INLA_ERR_HIP);
  ctx.harvest();
  teardown(b);
  return ctx.check();
}

}  // namespace inla

// ====================================================================== C-ABI
using namespace inla;

struct inla_handle {
  Ctx ctx;
};

namespace inla {
hipStream_t handle_stream(inla_handle *h) { return h->ctx.stream; }
Ctx *handle_ctx(inla_handle *h) { return &h->ctx; }
}  // namespace inla

extern "C" {

const char *inla_version(void) { return "inla_dense 0.1 (gfx950, fp64 mfma)"; }

int inla_create(inla_handle **h, void *stream) {
  if (!h) return -1;
  *h = nullptr;
  inla_handle *p = new (std::nothrow) inla_handle();
  if (!p) return INLA_ERR_NOMEM;
  p->ctx.stream = p->ctx.home = (hipStream_t)stream;
  if (hipGetDevice(&p->ctx.device) != hipSuccess) { delete p; return INLA_ERR_HIP; }
  // the no-allocation entry point's scratch on this device (its failure is
  // reported by that entry point, not here)
  (void)noalloc_init_device(p->ctx.device);
  p->ctx.ring_size = (size_t)16 << 20;
  if (hipMalloc(&p->ctx.ring, p->ctx.ring_size) != hipSuccess ||
      hipHostMalloc(&p->ctx.ring_host, p->ctx.ring_size) != hipSuccess) {
    delete p;
    return INLA_ERR_NOMEM;
  }
  *h = p;
  return INLA_OK;
}

int inla_destroy(inla_handle *h) {
  delete h;
  return INLA_OK;
}

int inla_set_stream(inla_handle *h, void *stream) {
  if (!h) return -1;
  if (h->ctx.sync_all() != INLA_OK) return INLA_ERR_HIP;
  h->ctx.stream = h->ctx.home = (hipStream_t)stream;
  return INLA_OK;
}

int inla_logdet(inla_handle *h, int32_t B, const int32_t *n, double *const *Q, const int32_t *ldq, int32_t prec,
                double *logdet, int32_t *info) {
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
  Ctx &ctx = h->ctx;
  PrecScope tag(ctx, prec);
  const size_t esz = prec == INLA_PREC_FP64 ? 8 : 4;
  // one chunk per memory budget
  const size_t cap = budget(ctx);
  int s = 0;
  while (s < B) {
    std::vector<int> ids;
    size_t tot = 0;
    int e = s;
    for (; e < B; ++e) {
      const int np = round_up(std::max(n[e], 1), PADN);
      const size_t need = align256(esz * np * np) + align256(8ull * (2 * np + 64 + 2 * np + DRES_COUNT)) + align256(esz * np * NBI);
      if (e > s && tot + need > cap) break;
      tot += need;
    }
    Batch b(ctx);
    const int Bc = e - s;
    b.plans.resize(Bc);
    size_t total = 0;
    std::vector<size_t> offs(Bc);
    for (int i = 0; i < Bc; ++i) {
      Plan &p = b.plans[i];
      ThetaDesc &t = p.t;
      t.n = n[s + i]; t.n_pad = round_up(std::max(t.n, 1), PADN);
      t.Quser = Q[s + i]; t.ldquser = ldq[s + i];
      t.ldw = t.Nw = t.Ncw = t.n_pad;
      size_t off = 0;
      p.off_W = off; off += align256(esz * t.n_pad * t.n_pad);
      p.off_vec = off; off += align256(8ull * (2 * t.n_pad + 64 + 2 * t.ldw + DRES_COUNT));
      p.off_linv = off; off += align256(esz * t.n_pad * NBI);
      p.bytes = off;
      offs[i] = total; total += off;
    }
    const size_t info_off = total;
    total += align256(sizeof(int) * 4 * Bc);
    if (!ctx.reserve(total)) return INLA_ERR_NOMEM;
    b.bases.resize(Bc);
    for (int i = 0; i < Bc; ++i) {
      Plan &p = b.plans[i];
      b.bases[i] = ctx.ws + offs[i];
      ThetaDesc &t = p.t;
      t.W = (void *)(b.bases[i] + p.off_W);
      double *v = (double *)(b.bases[i] + p.off_vec);
      t.x = v; v += t.n_pad; t.r = v; v += t.n_pad; t.lam = v; v += 64; t.part = v; v += 2 * t.ldw; t.dres = v;
      t.Qp = nullptr; t.S = nullptr; t.P = nullptr;
    }
    b.dinfo = (int *)(ctx.ws + info_off);
    if (hipMemsetAsync(b.dinfo, 0, sizeof(int) * 4 * Bc, ctx.stream) != hipSuccess) return INLA_ERR_HIP;
    if (hipHostMalloc(&b.pin, sizeof(double) * DRES_COUNT * Bc + sizeof(int) * 4 * Bc + 64) != hipSuccess)
      return INLA_ERR_NOMEM;
    std::vector<int> ids2;
    for (int i = 0; i < Bc; ++i) if (b.plans[i].t.n > 0) ids2.push_back(i);
    int rc = 0;
    if (!ids2.empty()) {
      ThetaDesc *d = upload_td(b, ids2);
      if (!d) { teardown(b); return INLA_ERR_NOMEM; }
      launch_copy_in(ctx, d, (int)ids2.size(), max_over(b, ids2, &ThetaDesc::n_pad), prec);
      if ((rc = run_factor(b, ids2, F_BIG, MODE_LOGDET, prec))) { teardown(b); return rc; }
      launch_finish(ctx, d, (int)ids2.size(), prec);
      launch_copy_out(ctx, d, (int)ids2.size(), max_over(b, ids2, &ThetaDesc::n), prec);
    }
    if ((rc = readback(b))) { teardown(b); return rc; }
    for (int i = 0; i < Bc; ++i) {
      const int f = b.hinfo[4 * i + F_BIG];
      info[s + i] = f;
      logdet[s + i] = b.plans[i].t.n == 0 ? 0.0 : (f ? std::numeric_limits<double>::quiet_NaN() : b.hdres[DRES_COUNT * i + DRES_LOGDET_L]);
    }
    ctx.harvest();
    teardown(b);
    s = e;
  }
  return ctx.check();
}

static int mode_or_eval(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                        double *const *x, const inla_opts *opts, inla_result *res, bool laplace) {
  int rc = validate_common(h, B, models, theta, ldtheta, res, true);
  if (rc) return rc;
  if (B == 0) return INLA_OK;
  if (!x) return -6;
  for (int i = 0; i < B; ++i) if (!x[i]) return -6;
  if (opts && (opts->prec < 0 || opts->prec >= INLA_PREC_COUNT)) return INLA_ERR_UNSUPPORTED;
  if (opts && opts->prec != INLA_PREC_FP64)
    for (int i = 0; i < B; ++i)
      if (models[i].m > 0) return INLA_ERR_UNSUPPORTED;   // general design matrices are evaluated in FP64
  for (auto c : chunks(h->ctx, B, models, theta, ldtheta, MODE_LAPLACE, h->ctx.overlap)) {
    rc = eval_chunk(h->ctx, c.second - c.first, models + c.first, theta + (size_t)c.first * ldtheta, ldtheta,
                    x + c.first, opts, res + c.first, laplace);
    if (rc) return rc;
  }
  // A warm start (start == 1) that fails (non-finite, no convergence within
  // opts->max_iter, or a failed pivot) is retried from x = 0 with the default
  // iteration budget.
  if (opts && opts->start == 1) {
    std::vector<int> redo;
    for (int i = 0; i < B; ++i) {
      const int inf = res[i].info;
      if (inf == INLA_INFO_NEWTON_MAXIT || inf == INLA_INFO_NONFINITE || inf > 0) redo.push_back(i);
    }
    if (!redo.empty()) {
      std::vector<inla_model> m2;
      std::vector<double> th2;
      std::vector<double *> x2;
      for (int i : redo) {
        m2.push_back(models[i]);
        th2.insert(th2.end(), theta + (size_t)i * ldtheta, theta + (size_t)(i + 1) * ldtheta);
        x2.push_back(x[i]);
      }
      inla_opts o2 = *opts;
      o2.start = 0;
      o2.max_iter = 0;
      std::vector<inla_result> r2(redo.size());
      rc = mode_or_eval(h, (int)redo.size(), m2.data(), th2.data(), ldtheta, x2.data(), &o2, r2.data(), laplace);
      if (rc) return rc;
      for (size_t q = 0; q < redo.size(); ++q) {
        res[redo[q]] = r2[q];
        res[redo[q]].fallback |= 2;
      }
    }
  }
  return INLA_OK;
}

int inla_constrained_mode(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                          double *const *x, const inla_opts *opts, inla_result *res) {
  return mode_or_eval(h, B, models, theta, ldtheta, x, opts, res, false);
}

int inla_laplace_eval(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                      double *const *x, const inla_opts *opts, inla_result *res) {
  return mode_or_eval(h, B, models, theta, ldtheta, x, opts, res, true);
}

int inla_marginal_var(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                      const double *const *x_mode, double *const *var, int32_t *info) {
  int rc = validate_common(h, B, models, theta, ldtheta, nullptr, false);
  if (rc) return rc;
  if (B == 0) return INLA_OK;
  if (!x_mode) return -6;
  if (!var) return -7;
  if (!info) return -8;
  for (int i = 0; i < B; ++i) if (!x_mode[i] || !var[i]) return -6;
  for (auto c : chunks(h->ctx, B, models, theta, ldtheta, MODE_VAR)) {
    rc = var_chunk(h->ctx, c.second - c.first, models + c.first, theta + (size_t)c.first * ldtheta, ldtheta,
                   x_mode + c.first, var + c.first, info + c.first);
    if (rc) return rc;
  }
  return INLA_OK;
}

int inla_set_graphs(inla_handle *h, int32_t enable) {
  if (!h) return -1;
  h->ctx.graphs = enable != 0;
  if (!enable) h->ctx.drop_graphs();
  return INLA_OK;
}

int inla_set_lookahead(inla_handle *h, int32_t enable) {
  if (!h) return -1;
  h->ctx.lookahead = enable != 0;
  return INLA_OK;
}

int inla_set_overlap(inla_handle *h, int32_t enable) {
  if (!h) return -1;
  h->ctx.overlap = enable != 0;
  return INLA_OK;
}

int inla_graph_stats(inla_handle *h, int64_t *captured, int64_t *replays) {
  if (!h) return -1;
  if (captured) *captured = h->ctx.graphs_captured;
  if (replays) *replays = h->ctx.graphs_replayed;
  return INLA_OK;
}

int inla_set_pass_graphs(inla_handle *h, int32_t enable) {
  if (!h) return -1;
  h->ctx.pass_graphs = enable != 0;
  if (!enable) h->ctx.drop_graphs();
  return INLA_OK;
}

int inla_pass_graph_stats(inla_handle *h, int64_t *captured, int64_t *replays) {
  if (!h) return -1;
  if (captured) *captured = h->ctx.pass_captured;
  if (replays) *replays = h->ctx.pass_replayed;
  return INLA_OK;
}

int inla_autotune(inla_handle *h, int32_t B, const int32_t *n, const int32_t *kb, int32_t prec, int32_t reps,
                  int32_t *config, double *ms, int32_t *n_cand) {
  if (!h) return -1;
  if (B < 1) return -2;
  if (!n) return -3;
  if (!kb) return -4;
  for (int i = 0; i < B; ++i) {
    if (n[i] < 1) return -3;
    if (kb[i] < 0) return -4;
  }
  if (prec < 0 || prec >= INLA_PREC_COUNT) return INLA_ERR_UNSUPPORTED;
  if (reps < 1) return -6;
  TuneCfg best;
  const int rc = autotune(h->ctx, B, n, kb, prec, reps, &best, ms, n_cand);
  if (rc) return rc;
  if (config) { config[0] = best.nb; config[1] = best.tm; config[2] = best.look; }
  return INLA_OK;
}

int inla_tune_set(inla_handle *h, int32_t prec, int32_t n_max, int32_t B, const int32_t *config) {
  if (!h) return -1;
  if (prec < 0 || prec >= INLA_PREC_COUNT) return INLA_ERR_UNSUPPORTED;
  if (n_max < 1) return -3;
  if (B < 1) return -4;
  const std::vector<int64_t> key = tune_key(prec, round_up(n_max, PADN), B);
  if (!config) {
    h->ctx.tune.erase(key);
    ++h->ctx.tune_epoch;
    return INLA_OK;
  }
  const TuneCfg c{config[0], config[1], config[2]};
  if (!tune_valid(prec, c)) return -5;
  h->ctx.tune[key] = c;
  ++h->ctx.tune_epoch;
  return INLA_OK;
}

int inla_tune_get(inla_handle *h, int32_t prec, int32_t n_max, int32_t B, int32_t *config) {
  if (!h) return -1;
  if (prec < 0 || prec >= INLA_PREC_COUNT) return INLA_ERR_UNSUPPORTED;
  if (n_max < 1) return -3;
  if (B < 1) return -4;
  if (!config) return -5;
  const TuneCfg c = tuned_config(h->ctx, prec, round_up(n_max, PADN), B);
  config[0] = c.nb; config[1] = c.tm; config[2] = c.look;
  return INLA_OK;
}

int inla_vb_mean(inla_handle *h, int32_t B, const inla_model *models, const double *theta, int32_t ldtheta,
                 const double *const *var, double *const *x, int32_t n_gh, const inla_opts *opts, int32_t *iters,
                 int32_t *info) {
  int rc = validate_common(h, B, models, theta, ldtheta, nullptr, false);
  if (rc) return rc;
  if (B == 0) return INLA_OK;
  if (!var) return -6;
  if (!x) return -7;
  for (int i = 0; i < B; ++i) {
    if (!var[i]) return -6;
    if (!x[i]) return -7;
  }
  if (n_gh <= 0) n_gh = 20;
  if (n_gh > 64) return -8;
  if (opts && opts->prec != INLA_PREC_FP64) return INLA_ERR_UNSUPPORTED;
  for (int i = 0; i < B; ++i)
    if (models[i].m > 0) return INLA_ERR_UNSUPPORTED;   // written for A = I
  if (!iters) return -10;
  if (!info) return -11;
  Ctx &ctx = h->ctx;
  if (!ctx.gh && hipMalloc(&ctx.gh, sizeof(double) * 128) != hipSuccess) {
    (void)hipGetLastError();
    ctx.gh = nullptr;
    return INLA_ERR_NOMEM;
  }
  const std::vector<double> rule = gauss_hermite(n_gh);
  if ((rc = ctx.upload_to(ctx.gh, rule.data(), sizeof(double) * rule.size()))) return rc;
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 50;
  const double tol = (opts && opts->tol > 0) ? opts->tol : 1e-11;
  for (auto c : chunks(ctx, B, models, theta, ldtheta, MODE_LAPLACE)) {
    rc = vb_chunk(ctx, c.second - c.first, models + c.first, theta + (size_t)c.first * ldtheta, ldtheta,
                  var + c.first, x + c.first, n_gh, max_iter, tol, iters + c.first, info + c.first);
    if (rc) return rc;
  }
  return INLA_OK;
}

int inla_profile(inla_handle *h, int32_t enable) {
  if (!h) return -1;
  h->ctx.harvest();
  h->ctx.prof = enable != 0;
  if (enable)
    for (auto &row : h->ctx.stats)
      for (auto &s : row) s = inla_kstats{};
  return INLA_OK;
}

int inla_profile_get(inla_handle *h, int32_t kclass, int32_t prec, inla_kstats *out) {
  if (!h) return -1;
  if (kclass < 0 || kclass >= INLA_K_COUNT) return -2;
  if (prec < 0 || prec >= INLA_PREC_COUNT) return -3;
  if (!out) return -4;
  h->ctx.harvest();
  *out = h->ctx.stats[kclass][prec];
  return INLA_OK;
}

}  // extern "C"
