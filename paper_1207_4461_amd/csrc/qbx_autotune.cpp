// Autotuner of the launch shapes (qbx_autotune, qbx_autotune_batched): times
// candidate tunings of the library's own entry points on the caller's problem
// with hipEvents and installs the fastest.  Host code only.  Device memory comes
// from the caller's workspace (qbx_autotune_workspace_bytes,
// qbx_autotune_batched_workspace_bytes); an optional cache file keeps the
// results per device and problem so that later runs install them untimed.
#include <hip/hip_runtime.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/qbx.h"
#include "qbx_internal.h"

namespace qbx {
namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// consecutive 256-byte aligned pieces of a caller workspace
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* ws) : base(static_cast<char*>(ws)) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off = align_up(off + std::max<size_t>(bytes, 256));
    return p;
  }
};

// ---------------------------------------------------------------------------
// cache file: one line per result, "<key> => <value>"; '#' starts a comment.
// The key names the device (architecture and compute units) and the problem.
// ---------------------------------------------------------------------------
int device_tag(std::string* tag) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return device_fail(e, "autotuner: device properties for the cache key");
  char buf[160];
  std::snprintf(buf, sizeof(buf), "arch=%s cus=%d", prop.gcnArchName, prop.multiProcessorCount);
  *tag = buf;
  return QBX_OK;
}

// 1: found (value set), 0: no such line or no file, QBX_EIO: unreadable file
int cache_lookup(const char* path, const std::string& key, std::string* value) {
  struct stat st;
  if (stat(path, &st) == 0 && !S_ISREG(st.st_mode))
    return fail(QBX_EIO, "%s is not a regular file", path);
  std::ifstream f(path);
  if (!f.is_open()) return access(path, F_OK) == 0 ? fail(QBX_EIO, "cannot read %s", path) : 0;
  std::string line;
  const std::string lead = key + " => ";
  int found = 0;
  while (std::getline(f, line)) {
    if (line.compare(0, lead.size(), lead) == 0) {
      *value = line.substr(lead.size());
      found = 1;   // the last line of a key wins
    }
  }
  if (f.bad()) return fail(QBX_EIO, "error reading %s", path);
  return found;
}

// replaces (or adds) the key's line: the whole file is rewritten to a temporary
// file beside it and renamed over it
int cache_store(const char* path, const std::string& key, const std::string& value) {
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    const std::string lead = key + " => ";
    while (f.is_open() && std::getline(f, line))
      if (line.compare(0, lead.size(), lead) != 0) lines.push_back(line);
  }
  if (lines.empty()) lines.push_back("# libqbx autotuner cache: <device and problem> => <tuning>");
  lines.push_back(key + " => " + value);
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o.is_open()) return fail(QBX_EIO, "cannot write %s", tmp.c_str());
    for (const std::string& l : lines) o << l << '\n';
    o.flush();
    if (!o.good()) {
      std::remove(tmp.c_str());
      return fail(QBX_EIO, "error writing %s", tmp.c_str());
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(QBX_EIO, "cannot rename %s to %s", tmp.c_str(), path);
  }
  return QBX_OK;
}

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
const int kTaskCandidates[] = {2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144};
const double kScaleCandidates[] = {0.5, 1.0, 2.0, 4.0};
const int kChunkCandidates[] = {4, 8, 16, 32};

// the per-contour pieces: a workspace for every candidate, out, tape, gradients
struct ContourSizes {
  size_t ws, out, tape, gd, gn, total;
};

ContourSizes contour_sizes(const Dims& d, int p, int oversample, int side, int kind) {
  qbx_tuning saved;
  qbx_get_tuning(&saved);
  ContourSizes z{};
  for (int c : kWaveCandidates) {
    for (int f : kTileCandidates) {
      set_contour_tuning(c, c, c, f);
      z.ws = std::max(z.ws, qbx_workspace_bytes(d.P, kQ, p, oversample, side, kind));
    }
  }
  qbx_set_tuning(&saved);
  z.out = sizeof(double) * 2 * (size_t)d.n_sides * d.nk * d.T;
  z.tape = qbx_tape_bytes(d.P, kQ, p, side, kind);
  z.gd = sizeof(double) * 2 * (size_t)d.nk * d.T;
  z.gn = sizeof(double) * 2 * (size_t)d.T;
  Carve c(nullptr);
  for (size_t b : {z.ws, z.out, z.tape, z.gd, z.gn}) c.take(b);
  z.total = c.off;
  return z;
}

// the batched pieces, and the extents of the packed arrays the items address
struct BatchSizes {
  size_t ws, out, tape, gd, gn, total;
};

BatchSizes batch_sizes(const qbx_batch_item* items, int n_items, int oversample) {
  qbx_tuning saved;
  qbx_get_tuning(&saved);
  BatchSizes z{};
  for (int c : kTaskCandidates) {
    for (int f : kChunkCandidates) {
      qbx_tuning t = saved;
      t.batch_adjoint_tasks = c;
      t.batch_fused_chunks = f;
      qbx_set_tuning(&t);
      z.ws = std::max(z.ws, qbx_batched_workspace_bytes(items, n_items, oversample));
    }
  }
  qbx_set_tuning(&saved);
  long long n_out = 0, n_dens = 0, n_panels = 0;
  for (int i = 0; i < n_items; ++i) {
    const qbx_batch_item& it = items[i];
    const long long T = 16LL * it.n_panels;
    const int nk = it.kind == 3 ? 2 : 1, ns = it.side == 0 ? 2 : 1;
    n_out = std::max(n_out, it.out_offset + (long long)ns * nk * T);
    n_dens = std::max(n_dens, it.density_offset + (long long)nk * T);
    n_panels = std::max(n_panels, it.node_offset + (long long)it.n_panels);
  }
  z.out = sizeof(double) * 2 * (size_t)n_out;
  z.tape = qbx_batched_tape_bytes(items, n_items);
  z.gd = sizeof(double) * 2 * (size_t)n_dens;
  z.gn = sizeof(double) * 32 * (size_t)n_panels;
  Carve c(nullptr);
  for (size_t b : {z.ws, z.out, z.tape, z.gd, z.gn}) c.take(b);
  z.total = c.off;
  return z;
}

// FNV-1a over the bytes of the fields that shape a batch's launches
uint64_t batch_signature(const qbx_batch_item* items, int n_items, int oversample) {
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ULL;
    }
  };
  mix(&n_items, sizeof(n_items));
  mix(&oversample, sizeof(oversample));
  for (int i = 0; i < n_items; ++i) {
    const qbx_batch_item& it = items[i];
    mix(&it.n_panels, sizeof(it.n_panels));
    mix(&it.p, sizeof(it.p));
    mix(&it.kind, sizeof(it.kind));
    mix(&it.side, sizeof(it.side));
  }
  return h;
}

int valid_passes_fields(int passes, int fields) {
  if (passes < 1 || passes > 20) return fail(QBX_EINVAL, "passes = %d outside [1, 20]", passes);
  if (fields <= 0 || (fields & ~QBX_TUNE_ALL))
    return fail(QBX_EINVAL, "fields = %d: a nonzero combination of the QBX_TUNE_ bits", fields);
  return QBX_OK;
}

}  // namespace
}  // namespace qbx

using namespace qbx;

extern "C" {

size_t qbx_autotune_workspace_bytes(int n_panels, int q, int p, int oversample, int side,
                                    int kind) {
  Dims d;
  if (!make_dims(n_panels, q, p, oversample, side, kind, 1.0, 0.5, &d)) return 0;
  return contour_sizes(d, p, oversample, side, kind).total;
}

size_t qbx_autotune_batched_workspace_bytes(const qbx_batch_item* items, int n_items,
                                            int oversample) {
  if (!items || n_items < 1 || qbx_batched_workspace_bytes(items, n_items, oversample) == 0)
    return 0;
  return batch_sizes(items, n_items, oversample).total;
}

int qbx_autotune(const qbx_geometry* g, const double* density, double k, int p, double r,
                 int oversample, int side, int kind, int passes, int fields,
                 const char* cache_path, qbx_tuning* best, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if ((rc = valid_passes_fields(passes, fields))) return rc;
  qbx_tuning saved;
  qbx_get_tuning(&saved);
  std::string key;
  if (cache_path) {
    std::string tag;
    if ((rc = device_tag(&tag))) return rc;
    char buf[200];
    std::snprintf(buf, sizeof(buf), "contour %s P=%d p=%d os=%d side=%d kind=%d fields=%d",
                  tag.c_str(), d.P, p, oversample, side, kind, fields);
    key = buf;
    std::string val;
    rc = cache_lookup(cache_path, key, &val);
    if (rc < 0) return rc;
    if (rc == 1) {
      int fw, tw, aw, ft;
      if (std::sscanf(val.c_str(), "forward_waves=%d tape_waves=%d adjoint_waves=%d fused_tiles=%d",
                      &fw, &tw, &aw, &ft) != 4)
        return fail(QBX_EIO, "malformed cache entry in %s: %s", cache_path, val.c_str());
      qbx_tuning t = saved;
      if (fields & QBX_TUNE_FORWARD) t.forward_waves = fw;
      if (fields & QBX_TUNE_TAPE) t.tape_waves = tw;
      if (fields & QBX_TUNE_ADJOINT) t.adjoint_waves = aw;
      if (fields & QBX_TUNE_FUSED) t.fused_tiles = ft;
      if (qbx_set_tuning(&t) != QBX_OK)
        return fail(QBX_EIO, "cache entry out of range in %s: %s", cache_path, val.c_str());
      if (best) *best = t;
      return QBX_OK;
    }
  }
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const ContourSizes z = contour_sizes(d, p, oversample, side, kind);
  if (ws_bytes < z.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, z.total);
  Carve c(ws);
  void* wsc = c.take(z.ws);
  double* o = static_cast<double*>(c.take(z.out));
  double* tp = static_cast<double*>(c.take(z.tape));
  double* gd = static_cast<double*>(c.take(z.gd));
  double* gn = static_cast<double*>(c.take(z.gn));
  Events ev;
  hipError_t e;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return device_fail(e, "autotuner events");
  auto fwd = [&] {
    return qbx_layer_potential(g, density, k, p, r, oversample, side, kind, o, nullptr, wsc, z.ws,
                               stream);
  };
  auto fwd_tape = [&] {
    return qbx_layer_potential(g, density, k, p, r, oversample, side, kind, o, tp, wsc, z.ws,
                               stream);
  };
  // the forward output serves as the cotangent: any values give the same cost
  auto adj = [&] {
    return qbx_layer_potential_adjoint(g, density, k, p, r, oversample, side, kind, o, tp, gd, gn,
                                       wsc, z.ws, stream);
  };
  // the adjoint without a tape: the fused pass
  auto adj_fused = [&] {
    return qbx_layer_potential_adjoint(g, density, k, p, r, oversample, side, kind, o, nullptr,
                                       gd, gn, wsc, z.ws, stream);
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
      const int cv = cands[ic];
      qbx_tuning t = cur;
      (which == 0 ? t.forward_waves : which == 1 ? t.tape_waves
       : which == 2 ? t.adjoint_waves : t.fused_tiles) = cv;
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
        v_best = cv;
      }
    }
    *field = v_best;
    qbx_set_tuning(&cur);
  }
  if (best) *best = cur;
  if (cache_path) {
    char val[160];
    std::snprintf(val, sizeof(val),
                  "forward_waves=%d tape_waves=%d adjoint_waves=%d fused_tiles=%d",
                  cur.forward_waves, cur.tape_waves, cur.adjoint_waves, cur.fused_tiles);
    if ((rc = cache_store(cache_path, key, val))) return rc;
  }
  return QBX_OK;
}

int qbx_autotune_batched(const qbx_batch_item* items, int n_items, const double* nodes,
                         const double* density, int oversample, int passes, int fields,
                         const char* cache_path, qbx_tuning* best, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  if (!items || n_items < 1 || !nodes || !density)
    return fail(QBX_EINVAL, "NULL or empty batch arguments");
  int rc = valid_passes_fields(passes, fields);
  if (rc) return rc;
  if (qbx_batched_workspace_bytes(items, n_items, oversample) == 0)
    return fail(QBX_EINVAL, "invalid batch (an item's parameters, offsets or oversample)");
  qbx_tuning saved;
  qbx_get_tuning(&saved);
  std::string key;
  if (cache_path) {
    std::string tag;
    if ((rc = device_tag(&tag))) return rc;
    char buf[200];
    std::snprintf(buf, sizeof(buf), "batch %s items=%d os=%d sig=%016" PRIx64 " fields=%d",
                  tag.c_str(), n_items, oversample, batch_signature(items, n_items, oversample),
                  fields);
    key = buf;
    std::string val;
    rc = cache_lookup(cache_path, key, &val);
    if (rc < 0) return rc;
    if (rc == 1) {
      double gs;
      int at, fc;
      if (std::sscanf(val.c_str(), "batch_grid_scale=%lf batch_adjoint_tasks=%d batch_fused_chunks=%d",
                      &gs, &at, &fc) != 3)
        return fail(QBX_EIO, "malformed cache entry in %s: %s", cache_path, val.c_str());
      qbx_tuning t = saved;
      if (fields & QBX_TUNE_FORWARD) t.batch_grid_scale = gs;
      if (fields & QBX_TUNE_ADJOINT) t.batch_adjoint_tasks = at;
      if (fields & QBX_TUNE_FUSED) t.batch_fused_chunks = fc;
      if (qbx_set_tuning(&t) != QBX_OK)
        return fail(QBX_EIO, "cache entry out of range in %s: %s", cache_path, val.c_str());
      if (best) *best = t;
      return QBX_OK;
    }
  }
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const BatchSizes z = batch_sizes(items, n_items, oversample);
  if (ws_bytes < z.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, z.total);
  Carve c(ws);
  void* wsc = c.take(z.ws);
  double* o = static_cast<double*>(c.take(z.out));
  double* tp = static_cast<double*>(c.take(z.tape));
  double* gd = static_cast<double*>(c.take(z.gd));
  double* gn = static_cast<double*>(c.take(z.gn));
  // the output serves as the adjoint's cotangent: give it defined values
  hipError_t e = hipMemsetAsync(o, 0, z.out, stream);
  if (e != hipSuccess) return device_fail(e, "autotuner buffers");
  Events ev;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return device_fail(e, "autotuner events");
  auto fwd = [&] {
    return qbx_layer_potential_batched(items, n_items, nodes, density, o, nullptr, oversample, wsc,
                                       z.ws, stream);
  };
  auto fwd_tape = [&] {
    return qbx_layer_potential_batched(items, n_items, nodes, density, o, tp, oversample, wsc,
                                       z.ws, stream);
  };
  auto adj = [&] {
    return qbx_layer_potential_batched_adjoint(items, n_items, nodes, density, o, tp, gd, gn,
                                               oversample, wsc, z.ws, stream);
  };
  auto adj_fused = [&] {
    return qbx_layer_potential_batched_adjoint(items, n_items, nodes, density, o, nullptr, gd, gn,
                                               oversample, wsc, z.ws, stream);
  };
  qbx_tuning cur = saved;
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
  if (cache_path) {
    char val[160];
    std::snprintf(val, sizeof(val),
                  "batch_grid_scale=%.17g batch_adjoint_tasks=%d batch_fused_chunks=%d",
                  cur.batch_grid_scale, cur.batch_adjoint_tasks, cur.batch_fused_chunks);
    if ((rc = cache_store(cache_path, key, val))) return rc;
  }
  return QBX_OK;
}

}  // extern "C"
