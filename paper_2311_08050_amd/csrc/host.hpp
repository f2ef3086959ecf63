// Host-side context shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
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

  // Copy a small host array to device memory through the ring; returns the device
  // pointer (valid for work enqueued after this call on `stream`).
  void *upload(const void *src, size_t bytes);
  // Grow the workspace to at least `bytes`.  Returns false on allocation failure.
  bool reserve(size_t bytes);
  // Launch through a wrapper that records events when profiling.
  void launch(int cls, double flops, double bytes, const std::function<void()> &f);
  // Collect profiling events (synchronises the stream).
  void harvest();
  int check();
  ~Ctx();
};

// Tags the launches enqueued in its scope with a precision for the profiling counters.
struct PrecScope {
  Ctx &c;
  int old;
  PrecScope(Ctx &ctx, int prec) : c(ctx), old(ctx.prec_tag) { c.prec_tag = prec; }
  ~PrecScope() { c.prec_tag = old; }
};

// Library entry points implemented in other translation units.
int factor_batch(Ctx &ctx, const std::vector<HostFactor> &fs, int nb, int prec);

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace inla
