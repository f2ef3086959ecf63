// Host-side context shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#include "../../include/inla_dense.h"
#include "device.hpp"

namespace inla {

// A matrix to factor plus the real (unpadded) sizes used to count algorithmic work.
struct HostFactor {
  FactorDesc d;
  int n_real;    // real factor columns (< nf means identity padding)
  int kb_real;   // real border rows starting at row nf
  int ks_real;   // real Schur columns starting at column nf
};

// Blocked-Cholesky configuration: panel width, trailing tile, lookahead.
struct TuneCfg {
  int nb = 512, tm = 128, look = 0;
};

struct Ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  // workspace: one grow-only device allocation
  char *ws = nullptr;
  size_t ws_size = 0;
  // descriptor upload ring (device) and pinned staging (host)
  char *ring = nullptr;
  char *ring_host = nullptr;
  size_t ring_size = 0, ring_off = 0;
  // profiling
  bool prof = false;
  int prec_tag = INLA_PREC_FP64;  // precision of the pass being enqueued
  inla_kstats stats[INLA_K_COUNT][INLA_PREC_COUNT] = {};
  struct Pending { hipEvent_t a, b; int cls, prec; double flops, bytes; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  hipError_t last = hipSuccess;
  // hipGraph capture of launch-bound kernel sequences (see sequence())
  bool graphs = true;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  double cap_flops = 0, cap_bytes = 0;
  struct Graph {
    hipGraphExec_t exec = nullptr;
    void *dargs = nullptr;           // device copy of the argument block the graph's kernels read
    std::vector<char> last;          // argument bytes last copied into dargs
    double flops = 0, bytes = 0;     // algorithmic work of one replay
    uint64_t used = 0;
  };
  std::map<std::vector<int64_t>, Graph> graph_cache;
  uint64_t graph_clock = 0;
  int64_t graphs_captured = 0, graphs_replayed = 0;
  int sticky = 0;   // first failure of a sequence() whose caller has no return path; reported by check()
  // Whole-pass graphs (see pass_graph()).  While a pass is collected or
  // captured, upload() hands out consecutive slots of the pass graph's device
  // argument block and appends the bytes to `pg.host`; sequence() does the
  // same with its argument block and runs its body in place; launch() records
  // the launch in `pg.sig` and, when collecting, enqueues nothing.
  bool pass_graphs = true;
  enum { PG_OFF = 0, PG_COLLECT = 1, PG_CAPTURE = 2 };
  int pg_mode = PG_OFF;
  struct PassRec {
    char *dbase = nullptr;        // the pass graph's device argument block
    size_t cap = 0;               // its capacity
    bool overflow = false;        // an upload did not fit
    std::vector<char> host;       // argument bytes in upload order
    std::vector<int64_t> sig;     // launch classes and work, upload sizes, sequence keys
    double flops = 0, bytes = 0;
  } pg;
  struct PassGraph {
    hipGraphExec_t exec = nullptr;
    char *dargs = nullptr;
    size_t cap = 0;
    std::vector<char> last;       // argument bytes last copied into dargs
    std::vector<int64_t> sig;
    double flops = 0, bytes = 0;
    uint64_t used = 0;
  };
  std::map<std::vector<int64_t>, PassGraph> pass_cache;
  int64_t pass_captured = 0, pass_replayed = 0;
  // Enqueue `body` (which enqueues one pass's launches and uploads, and
  // reads nothing back) as one hipGraph per distinct `key` (plus the stream
  // lane).  Graphs on, profiling off and no capture in progress; otherwise, or
  // when the pass's launch signature differs from the captured one, or its
  // arguments outgrow the block, `body` runs directly.  Profiling times a
  // replay as one launch of class `cls`.
  int pass_graph(int cls, const std::vector<int64_t> &key, const std::function<int()> &body);
  // lookahead in the blocked Cholesky: a second stream of the handle (default
  // priority) runs the bulk of each trailing update while the caller's stream
  // factors the next panel (used where the tuned configuration asks for it and
  // `lookahead` allows it)
  bool lookahead = true;
  hipStream_t side = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  int side_ready();   // creates the side stream and its events on first use
  // Concurrent prior pass: a third stream of the handle (default priority)
  // runs the FP64 factorisation of the prior while the caller's stream runs
  // the Newton iteration; ev_c / ev_d order the two.  `lane` is 1 while work
  // is enqueued for that stream: it keys the hipGraphs apart (each graph owns
  // one argument block, which two streams must not share) and keeps lookahead
  // (which uses `side`) to lane 0.
  bool overlap = false;
  hipStream_t aux = nullptr;
  hipEvent_t ev_c = nullptr, ev_d = nullptr;
  int lane = 0;
  hipStream_t home = nullptr;   // the caller's stream (`stream` is swapped to side or aux at times)
  int aux_ready();    // creates the aux stream and its events on first use
  int sync_all();     // waits for the caller's, side and aux streams
  // Gauss-Hermite rule of the variational-Bayes correction (device, 2 x 64 doubles)
  double *gh = nullptr;
  // scratch of the BF16 panel copies (grow-only, reallocated after a stream sync)
  char *pbf = nullptr;
  size_t pbf_size = 0;
  char *pbf_reserve(size_t bytes);
  // autotuned (panel width, trailing tile) per (precision, padded order, batch bucket)
  std::map<std::vector<int64_t>, TuneCfg> tune;
  uint64_t tune_epoch = 0;   // counts changes of `tune` (pass graph keys carry it)

  // Copy a small host array to device memory through the ring; returns the device
  // pointer (valid for work enqueued after this call on `stream`).
  void *upload(const void *src, size_t bytes);
  // Copy a small host array into device memory `dst` through the pinned ring
  // (stream-ordered on `stream`).
  int upload_to(void *dst, const void *src, size_t bytes);
  // Enqueue a launch-bound kernel sequence.  `body` launches the kernels and
  // reads its argument block (`args`, `nbytes`) through the device pointer it
  // is given.  With graphs enabled the sequence is captured once per distinct
  // `key` (which must determine every launch's grid and scalar arguments) into
  // a hipGraph that owns a device copy of the argument block; later calls with
  // the same key copy the current arguments into that block (skipped when they
  // are unchanged) and replay the graph.  Without graphs the kernels are
  // launched directly.  Profiling times a replay as one launch of class `cls`.
  int sequence(int cls, const std::vector<int64_t> &key, const void *args, size_t nbytes,
               const std::function<void(const void *dargs)> &body);
  int sequence_impl(int cls, const std::vector<int64_t> &key, const void *args, size_t nbytes,
                    const std::function<void(const void *dargs)> &body);
  void drop_graphs();   // also drops the pass graphs
  // Grow the workspace to at least `bytes`.  Returns false on allocation failure.
  bool reserve(size_t bytes);
  // Launch through a wrapper that records events when profiling.
  void launch(int cls, double flops, double bytes, const std::function<void()> &f);
  // Collect profiling events (synchronises the stream).
  void harvest();
  int check();
  ~Ctx();
};

// Enqueues the work of its scope on the handle's aux stream (lane 1).
struct AuxScope {
  Ctx &c;
  hipStream_t old;
  int old_lane;
  explicit AuxScope(Ctx &ctx) : c(ctx), old(ctx.stream), old_lane(ctx.lane) {
    c.stream = c.aux;
    c.lane = 1;
  }
  ~AuxScope() {
    c.stream = old;
    c.lane = old_lane;
  }
};

// Tags the launches enqueued in its scope with a precision for the profiling counters.
struct PrecScope {
  Ctx &c;
  int old;
  PrecScope(Ctx &ctx, int prec) : c(ctx), old(ctx.prec_tag) { c.prec_tag = prec; }
  ~PrecScope() { c.prec_tag = old; }
};

// Library entry points implemented in other translation units.
// cfg == nullptr: the tuned (or default) configuration for this batch.
int factor_batch(Ctx &ctx, const std::vector<HostFactor> &fs, int prec, const TuneCfg *cfg = nullptr);
// The configuration used without a tuning table entry.
TuneCfg default_config(int prec, int nf_max);
// The configuration factor_batch uses for a batch of `B` factorisations whose
// largest padded order is `nf_max`.
TuneCfg tuned_config(const Ctx &ctx, int prec, int nf_max, int B);
std::vector<int64_t> tune_key(int prec, int nf_max, int B);
bool tune_valid(int prec, const TuneCfg &c);
constexpr int TUNE_MAX_CAND = 9;
// Time every candidate configuration on a synthetic batch and record the fastest.
int autotune(Ctx &ctx, int B, const int *n, const int *kb, int prec, int reps, TuneCfg *best_out, double *ms_out,
             int *n_cand);

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// The handle's context (C-ABI handles wrap one Ctx).
Ctx *handle_ctx(inla_handle *h);
// Takes the device address of inla_logdet_noalloc's scratch array on `device`
// (the current device) once per device; INLA_OK or INLA_ERR_HIP.
int noalloc_init_device(int device);
// Block-structured pseudo-inverse priors (woodbury.hip): validation for order n
// and theta dimension t (t < 0: unchecked), 0 or -3; and Q_prior(theta_b)^+ for B
// points into the device arrays out[b] (n x n, ld n).
int pinv_prior_check(const inla_pinv_prior *pp, int n, int t);
int pinv_prior_assemble(Ctx &ctx, const inla_pinv_prior &pp, int n, int B, const double *theta, int ldtheta,
                        double *const *out);

// Small dense symmetric eigen-decomposition (host) and the Gauss-Hermite rule
// built on it (nodes, then weights / sqrt(pi)).
void sym_eigen(int t, std::vector<double> A, std::vector<double> &w, std::vector<double> &V);
std::vector<double> gauss_hermite(int d);

}  // namespace inla
