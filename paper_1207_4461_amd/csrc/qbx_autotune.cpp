// Autotuner of the launch shapes (qbx_autotune, qbx_autotune_batched): times
// candidate tunings of the library's own entry points on the caller's problem
// with hipEvents and installs the fastest.  Host code only; it allocates its
// own device buffers, which no other entry point does.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <set>
#include <vector>

#include "../../include/qbx.h"
#include "qbx_internal.h"

namespace qbx {
namespace {

// device buffers owned by one autotuner call
struct DeviceBuffers {
  std::vector<void*> ptrs;
  ~DeviceBuffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  hipError_t get(size_t bytes, void** p) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// minimum time in ms of `passes` runs of fn after one warm-up; < 0 on failure
// (rc holds the failing status)
double time_min(const std::function<int()>& fn, int passes, hipStream_t s, Events& ev, int* rc) {
  *rc = fn();
  if (*rc) return -1.0;
  double best = 1e300;
  for (int i = 0; i < passes; ++i) {
    if (hipEventRecord(ev.a, s) != hipSuccess) {
      *rc = fail(QBX_EDEVICE, "autotuner: event record failed");
      return -1.0;
    }
    *rc = fn();
    if (*rc) return -1.0;
    float ms = 0.f;
    if (hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
        hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) {
      *rc = fail(QBX_EDEVICE, "autotuner: event timing failed");
      return -1.0;
    }
    best = std::min(best, (double)ms);
  }
  return best;
}

const int kWaveCandidates[] = {2048, 4096, 8192, 16384, 32768, 65536, 131072};
const int kTileCandidates[] = {2048, 4096, 8192, 16384, 32768};

}  // namespace
}  // namespace qbx

using namespace qbx;

extern "C" {

int qbx_autotune(const qbx_geometry* g, const double* density, double k, int p, double r,
                 int oversample, int side, int kind, int passes, int fields, qbx_tuning* best,
                 hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (passes < 1 || passes > 20) return fail(QBX_EINVAL, "passes = %d outside [1, 20]", passes);
  if (fields <= 0 || (fields & ~QBX_TUNE_ALL))
    return fail(QBX_EINVAL, "fields = %d: a nonzero combination of the QBX_TUNE_ bits", fields);
  qbx_tuning saved;
  qbx_get_tuning(&saved);
  // a workspace large enough for every candidate
  size_t ws_bytes = 0;
  for (int c : kWaveCandidates) {
    for (int f : kTileCandidates) {
      set_contour_tuning(c, c, c, f);
      ws_bytes = std::max(ws_bytes, qbx_workspace_bytes(d.P, kQ, p, oversample, side, kind));
    }
  }
  qbx_set_tuning(&saved);
  const size_t out_bytes = sizeof(double) * 2 * (size_t)d.n_sides * d.nk * d.T;
  DeviceBuffers mem;
  void *ws, *out, *tape, *gd, *gn;
  hipError_t e = mem.get(ws_bytes, &ws);
  if (e == hipSuccess) e = mem.get(out_bytes, &out);
  if (e == hipSuccess) e = mem.get(qbx_tape_bytes(d.P, kQ, p, side, kind), &tape);
  if (e == hipSuccess) e = mem.get(sizeof(double) * 2 * (size_t)d.nk * d.T, &gd);
  if (e == hipSuccess) e = mem.get(sizeof(double) * 2 * (size_t)d.T, &gn);
  if (e != hipSuccess) return device_fail(e, "autotuner buffers");
  Events ev;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return device_fail(e, "autotuner events");
  double* o = static_cast<double*>(out);
  double* tp = static_cast<double*>(tape);
  auto fwd = [&] {
    return qbx_layer_potential(g, density, k, p, r, oversample, side, kind, o, nullptr, ws,
                               ws_bytes, stream);
  };
  auto fwd_tape = [&] {
    return qbx_layer_potential(g, density, k, p, r, oversample, side, kind, o, tp, ws, ws_bytes,
                               stream);
  };
  // the forward output serves as the cotangent: any values give the same cost
  auto adj = [&] {
    return qbx_layer_potential_adjoint(g, density, k, p, r, oversample, side, kind, o, tp,
                                       static_cast<double*>(gd), static_cast<double*>(gn), ws,
                                       ws_bytes, stream);
  };
  // the adjoint without a tape: the fused pass
  auto adj_fused = [&] {
    return qbx_layer_potential_adjoint(g, density, k, p, r, oversample, side, kind, o, nullptr,
                                       static_cast<double*>(gd), static_cast<double*>(gn), ws,
                                       ws_bytes, stream);
  };
  qbx_tuning cur = saved;
  // which = 0 forward, 1 tape, 2 adjoint with the tape, 3 fused adjoint
  for (int which = 0; which < 4; ++which) {
    if (!(fields & (1 << which))) continue;
    if (which == 2 && !(fields & QBX_TUNE_TAPE)) {
      // the adjoint with the tape reads one: write it once
      if ((rc = fwd_tape()) != QBX_OK) {
        qbx_set_tuning(&saved);
        return rc;
      }
    }
    std::set<long long> shapes;
    double t_best = 1e300;
    int* field = which == 0 ? &cur.forward_waves : which == 1 ? &cur.tape_waves
                 : which == 2 ? &cur.adjoint_waves : &cur.fused_tiles;
    int v_best = *field;
    const int* cands = which == 3 ? kTileCandidates : kWaveCandidates;
    const int n_cands = which == 3 ? (int)(sizeof(kTileCandidates) / sizeof(int))
                                   : (int)(sizeof(kWaveCandidates) / sizeof(int));
    for (int ic = 0; ic < n_cands; ++ic) {
      const int c = cands[ic];
      qbx_tuning t = cur;
      (which == 0 ? t.forward_waves : which == 1 ? t.tape_waves
       : which == 2 ? t.adjoint_waves : t.fused_tiles) = c;
      qbx_set_tuning(&t);
      Dims dc;
      make_dims(d.P, kQ, p, oversample, side, kind, k, r, &dc);
      const long long shape = which == 0 ? dc.n_split : which == 1 ? dc.n_tsplit
                              : which == 2 ? dc.n_csplit : (long long)dc.chunks_per_sb;
      if (!shapes.insert(shape).second) continue;
      const double ms = time_min(which == 0 ? std::function<int()>(fwd)
                                 : which == 1 ? std::function<int()>(fwd_tape)
                                 : which == 2 ? std::function<int()>(adj)
                                              : std::function<int()>(adj_fused),
                                 passes, stream, ev, &rc);
      if (ms < 0.0) {
        qbx_set_tuning(&saved);
        return rc ? rc : fail(QBX_EDEVICE, "autotuner timing failed");
      }
      if (ms < t_best) {
        t_best = ms;
        v_best = c;
      }
    }
    *field = v_best;
    qbx_set_tuning(&cur);
  }
  if (best) *best = cur;
  return QBX_OK;
}

int qbx_autotune_batched(const qbx_batch_item* items, int n_items, const double* nodes,
                         const double* density, int oversample, int passes, int fields,
                         qbx_tuning* best, hipStream_t stream) {
  if (!items || n_items < 1 || !nodes || !density)
    return fail(QBX_EINVAL, "NULL or empty batch arguments");
  if (passes < 1 || passes > 20) return fail(QBX_EINVAL, "passes = %d outside [1, 20]", passes);
  if (fields <= 0 || (fields & ~QBX_TUNE_ALL))
    return fail(QBX_EINVAL, "fields = %d: a nonzero combination of the QBX_TUNE_ bits", fields);
  if (qbx_batched_workspace_bytes(items, n_items, oversample) == 0)
    return fail(QBX_EINVAL, "invalid batch (an item's parameters, offsets or oversample)");
  qbx_tuning saved;
  qbx_get_tuning(&saved);
  static const int kTaskCandidates[] = {2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144};
  static const double kScaleCandidates[] = {0.5, 1.0, 2.0, 4.0};
  static const int kChunkCandidates[] = {4, 8, 16, 32};
  size_t ws_bytes = 0;
  for (int c : kTaskCandidates) {
    for (int f : kChunkCandidates) {
      qbx_tuning t = saved;
      t.batch_adjoint_tasks = c;
      t.batch_fused_chunks = f;
      qbx_set_tuning(&t);
      ws_bytes = std::max(ws_bytes, qbx_batched_workspace_bytes(items, n_items, oversample));
    }
  }
  qbx_set_tuning(&saved);
  // extents of the caller's packed arrays, from the items
  long long n_out = 0, n_dens = 0, n_panels = 0;
  for (int i = 0; i < n_items; ++i) {
    const qbx_batch_item& it = items[i];
    const long long T = 16LL * it.n_panels;
    const int nk = it.kind == 3 ? 2 : 1, ns = it.side == 0 ? 2 : 1;
    n_out = std::max(n_out, it.out_offset + (long long)ns * nk * T);
    n_dens = std::max(n_dens, it.density_offset + (long long)nk * T);
    n_panels = std::max(n_panels, it.node_offset + (long long)it.n_panels);
  }
  DeviceBuffers mem;
  void *ws, *out, *tape, *gd, *gn;
  hipError_t e = mem.get(ws_bytes, &ws);
  if (e == hipSuccess) e = mem.get(sizeof(double) * 2 * (size_t)n_out, &out);
  if (e == hipSuccess) e = mem.get(qbx_batched_tape_bytes(items, n_items), &tape);
  if (e == hipSuccess) e = mem.get(sizeof(double) * 2 * (size_t)n_dens, &gd);
  if (e == hipSuccess) e = mem.get(sizeof(double) * 32 * (size_t)n_panels, &gn);
  if (e == hipSuccess) e = hipMemsetAsync(out, 0, sizeof(double) * 2 * (size_t)n_out, stream);
  if (e != hipSuccess) return device_fail(e, "autotuner buffers");
  Events ev;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return device_fail(e, "autotuner events");
  double* o = static_cast<double*>(out);
  double* tp = static_cast<double*>(tape);
  auto fwd = [&] {
    return qbx_layer_potential_batched(items, n_items, nodes, density, o, nullptr, oversample, ws,
                                       ws_bytes, stream);
  };
  auto fwd_tape = [&] {
    return qbx_layer_potential_batched(items, n_items, nodes, density, o, tp, oversample, ws,
                                       ws_bytes, stream);
  };
  auto adj = [&] {
    return qbx_layer_potential_batched_adjoint(items, n_items, nodes, density, o, tp,
                                               static_cast<double*>(gd), static_cast<double*>(gn),
                                               oversample, ws, ws_bytes, stream);
  };
  auto adj_fused = [&] {
    return qbx_layer_potential_batched_adjoint(items, n_items, nodes, density, o, nullptr,
                                               static_cast<double*>(gd), static_cast<double*>(gn),
                                               oversample, ws, ws_bytes, stream);
  };
  qbx_tuning cur = saved;
  int rc = QBX_OK;
  // times fn at each candidate written by set(t, i) into the current tuning and
  // keeps the fastest in cur
  auto sweep = [&](int n, const std::function<void(qbx_tuning&, int)>& set,
                   const std::function<int()>& fn) -> int {
    double t_best = 1e300;
    int i_best = -1;
    for (int i = 0; i < n; ++i) {
      qbx_tuning t = cur;
      set(t, i);
      qbx_set_tuning(&t);
      const double ms = time_min(fn, passes, stream, ev, &rc);
      if (ms < 0.0) return rc ? rc : fail(QBX_EDEVICE, "autotuner timing failed");
      if (ms < t_best) {
        t_best = ms;
        i_best = i;
      }
    }
    set(cur, i_best);
    qbx_set_tuning(&cur);
    return QBX_OK;
  };
  if (fields & QBX_TUNE_FORWARD)
    rc = sweep(4, [&](qbx_tuning& t, int i) { t.batch_grid_scale = kScaleCandidates[i]; }, fwd);
  if (!rc && (fields & QBX_TUNE_ADJOINT)) {
    rc = fwd_tape();   // the adjoint with the tape reads one
    if (!rc)
      rc = sweep(8, [&](qbx_tuning& t, int i) { t.batch_adjoint_tasks = kTaskCandidates[i]; }, adj);
  }
  if (!rc && (fields & QBX_TUNE_FUSED))
    rc = sweep(4, [&](qbx_tuning& t, int i) { t.batch_fused_chunks = kChunkCandidates[i]; },
               adj_fused);
  if (rc) {
    qbx_set_tuning(&saved);
    return rc;
  }
  if (best) *best = cur;
  return QBX_OK;
}

}  // extern "C"
