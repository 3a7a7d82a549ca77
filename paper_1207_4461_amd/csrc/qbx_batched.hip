// Batched QBX: many contours of different panel counts, wavenumbers, orders
// and kinds, with the pair work of all contours of one (kind, p) class in one
// persistent launch.
//
// The host builds a plan: per-contour dimensions and offsets into packed
// workspace arrays, and, per (kind, p) class present in the batch, two task
// lists ordered by decreasing cost per task (forward: one task per center,
// cost ~ sources; adjoint: one task per 64-source chunk, cost ~ centers),
// stored as prefix sums over the class's contours in that order.  Each class
// runs a persistent kernel compiled for its (kind, p) -- the register budget of
// the per-contour kernel of that class, not of the largest case -- on a grid of
// resident workgroups; every wavefront takes the next task index from the
// class's device counter, finds its contour by binary search in the prefix
// array and runs the pair-loop body of the per-contour kernels (qbx_pair.h).
// Every wavefront leaves once the counter passes the task count.  Geometry,
// per-center and per-source steps run as ordinary grids over all contours'
// panels, centers or sources.
#include <algorithm>
#include <mutex>
#include <cmath>
#include <numeric>
#include <vector>

#include "../../include/qbx.h"
#include "qbx_batched.h"

namespace qbx {

// the contours of one (kind, p) class: their slice of the order and prefix
// arrays (order at ord_at, n entries; prefix sums at pre_at, n + 1 entries)
struct BatchClass {
  int kind, p, n;
  int ord_at, pre_at;
  long long tasks_f, tasks_a, tasks_x;   // forward, adjoint source pass, fused adjoint tiles
};

struct BatchPlan {
  int n;
  int qs;
  std::vector<BatchItemDev> items;
  std::vector<BatchClass> cls;                    // heaviest class first
  std::vector<int> order_f, order_a, order_x;     // per class: contours by decreasing task cost
  std::vector<long long> pre_f, pre_a, pre_x;     // per class: task prefix sums in that order
  std::vector<long long> pre_panel, pre_ctr, pre_src, pre_G;  // prefix sums in item order
  long long n_panels = 0, n_ctr = 0, n_src = 0, n_G = 0, n_densw = 0, n_jtab = 0, n_tape = 0,
            n_spart = 0, n_cpart = 0;
  // workspace offsets
  size_t o_items, o_ord_f, o_ord_a, o_ord_x, o_pre_f, o_pre_a, o_pre_x, o_pre_panel, o_pre_ctr, o_pre_src, o_pre_G,
      o_counter, o_tables, o_geo, o_densw, o_wgt, o_h, o_ctr, o_jtab, o_tape, o_G, o_cg, o_spart, o_cpart,
      o_sg, total;
};

// launch tunables (qbx_set_tuning)
static double g_batch_grid_scale = 1.0;       // persistent grid = resident blocks x this
static double g_batch_adjoint_tasks = 16384;  // adjoint tasks per (kind, p) class
static int g_batch_fused_chunks = 4;          // 64-source chunks per fused adjoint tile

static bool build_plan(const qbx_batch_item* items, int n, int oversample, BatchPlan* P) {
  if (!items || n < 1 || oversample < 1 || oversample > QBX_OVERSAMPLE_MAX) return false;
  P->n = n;
  P->qs = kQ * oversample;
  P->items.resize(n);
  P->pre_panel.assign(n + 1, 0);
  P->pre_ctr.assign(n + 1, 0);
  P->pre_src.assign(n + 1, 0);
  P->pre_G.assign(n + 1, 0);
  std::vector<double> cost_f(n), cost_a(n), cost_x(n);
  for (int i = 0; i < n; ++i) {
    const qbx_batch_item& it = items[i];
    BatchItemDev& B = P->items[i];
    if (!(it.k > 0.0) || !std::isfinite(it.k) || !(it.r > 0.0) || !std::isfinite(it.r)) return false;
    if (it.node_offset < 0 || it.density_offset < 0 || it.out_offset < 0) return false;
    if (!make_dims(it.n_panels, kQ, it.p, oversample, it.side, it.kind, it.k, it.r, &B.d))
      return false;
    const Dims& d = B.d;
    B.node_off = it.node_offset * 2 * kQ;
    B.din_off = it.density_offset * 2;
    B.out_off = it.out_offset * 2;
    B.panel_off = P->n_panels;
    B.src_off = P->n_src;
    B.ctr_off = P->n_ctr;
    B.densw_off = P->n_densw;
    B.jtab_off = P->n_jtab;
    B.tape_off = P->n_tape;
    B.G_off = P->n_G;
    P->n_panels += d.P;
    P->n_src += d.N;
    P->n_ctr += d.Mc;
    P->n_densw += (long long)d.nk * d.N;
    P->n_jtab += (long long)d.Mc * d.NJ;
    P->n_tape += (long long)d.Mc * d.nk * 4;
    P->n_G += (long long)d.nk * d.Mc;
    P->pre_panel[i + 1] = P->n_panels;
    P->pre_ctr[i + 1] = P->n_ctr;
    P->pre_src[i + 1] = P->n_src;
    P->pre_G[i + 1] = P->n_G;
    const double per_pair = (double)(d.p + 8) * d.nk;
    cost_f[i] = (double)d.N * per_pair;    // one center against all sources
    cost_a[i] = (double)d.Mc * per_pair;   // 64 sources against all centers
  }
  if (P->n_src > (1LL << 31) - 1 || P->n_ctr > (1LL << 31) - 1) return false;
  // classes, heaviest (total forward cost) first
  std::vector<double> cls_cost;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < n; ++i) {
    const Dims& d = P->items[i].d;
    size_t c = 0;
    while (c < P->cls.size() && !(P->cls[c].kind == d.kind && P->cls[c].p == d.p)) ++c;
    if (c == P->cls.size()) {
      P->cls.push_back(BatchClass{d.kind, d.p, 0, 0, 0, 0, 0, 0});
      cls_cost.push_back(0.0);
      members.emplace_back();
    }
    members[c].push_back(i);
    cls_cost[c] += cost_f[i] * d.Mc;
  }
  std::vector<int> rank(P->cls.size());
  std::iota(rank.begin(), rank.end(), 0);
  std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return cls_cost[a] > cls_cost[b]; });
  std::vector<BatchClass> sorted;
  std::vector<std::vector<int>> sorted_members;
  for (int r : rank) {
    sorted.push_back(P->cls[r]);
    sorted_members.push_back(members[r]);
  }
  P->cls = sorted;
  P->order_f.clear();
  P->order_a.clear();
  P->order_x.clear();
  P->pre_x.clear();
  P->pre_f.clear();
  P->pre_a.clear();
  for (size_t c = 0; c < P->cls.size(); ++c) {
    BatchClass& C = P->cls[c];
    const std::vector<int>& mem = sorted_members[c];
    C.n = (int)mem.size();
    C.ord_at = (int)P->order_f.size();
    C.pre_at = (int)P->pre_f.size();
    auto append = [&](const std::vector<double>& cost, std::vector<int>& ord,
                      std::vector<long long>& pre, bool centers) {
      std::vector<int> o = mem;
      std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return cost[a] > cost[b]; });
      long long acc = 0;
      pre.push_back(0);
      for (int i : o) {
        const Dims& d = P->items[i].d;
        acc += centers ? d.Mc : (long long)d.chunks * d.n_csplit;
        ord.push_back(i);
        pre.push_back(acc);
      }
      return acc;
    };
    // adjoint tasks: (center split, 64-source chunk); the class's work is cut
    // into about g_batch_adjoint_tasks tasks of at least 16 centers each
    double work = 0.0;
    for (int i : mem) work += (double)P->items[i].d.chunks * P->items[i].d.Mc;
    const long long g = std::max<long long>(16, (long long)std::ceil(work / g_batch_adjoint_tasks));
    for (int i : mem) {
      Dims& d = P->items[i].d;
      d.centers_per_split = (int)std::min<long long>(d.Mc, g);
      d.n_csplit = (d.Mc + d.centers_per_split - 1) / d.centers_per_split;
    }
    C.tasks_f = append(cost_f, P->order_f, P->pre_f, true);
    C.tasks_a = append(cost_a, P->order_a, P->pre_a, false);
    // fused adjoint tiles: fused_tile_height centers x g_batch_fused_chunks
    // 64-source chunks; tile cost ~ centers of the tile
    for (int i : mem) {
      Dims& d = P->items[i].d;
      d.fused_cblock = fused_tile_height(d.Mc, d.N, d.kind);
      d.n_cb = (d.Mc + d.fused_cblock - 1) / d.fused_cblock;
      d.chunks_per_sb = d.chunks < g_batch_fused_chunks ? d.chunks : g_batch_fused_chunks;
      d.n_sb = (d.chunks + d.chunks_per_sb - 1) / d.chunks_per_sb;
      cost_x[i] = (double)d.fused_cblock;
    }
    {
      std::vector<int> o = mem;
      std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return cost_x[a] > cost_x[b]; });
      long long acc = 0;
      P->pre_x.push_back(0);
      for (int i : o) {
        const Dims& d = P->items[i].d;
        acc += (long long)d.n_cb * d.n_sb;
        P->order_x.push_back(i);
        P->pre_x.push_back(acc);
      }
      C.tasks_x = acc;
    }
  }
  for (int i = 0; i < n; ++i) {
    BatchItemDev& B = P->items[i];
    B.spart_off = P->n_spart;
    P->n_spart += (long long)std::max(B.d.n_csplit, B.d.n_cb) * src_slots(B.d.kind) * B.d.N;
    B.cpart_off = P->n_cpart;
    P->n_cpart += (long long)B.d.n_sb * B.d.Mc * 4;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  P->o_items = take(sizeof(BatchItemDev) * n);
  P->o_ord_f = take(sizeof(int) * n);
  P->o_ord_a = take(sizeof(int) * n);
  P->o_ord_x = take(sizeof(int) * n);
  P->o_pre_f = take(sizeof(long long) * P->pre_f.size());
  P->o_pre_a = take(sizeof(long long) * P->pre_a.size());
  P->o_pre_x = take(sizeof(long long) * P->pre_x.size());
  P->o_pre_panel = take(sizeof(long long) * (n + 1));
  P->o_pre_ctr = take(sizeof(long long) * (n + 1));
  P->o_pre_src = take(sizeof(long long) * (n + 1));
  P->o_pre_G = take(sizeof(long long) * (n + 1));
  P->o_counter = take(sizeof(int) * 3 * P->cls.size());
  P->o_tables = take(sizeof(double) * table_layout(P->qs).total);
  P->o_geo = take(sizeof(double4) * P->n_src);
  P->o_densw = take(sizeof(double2) * P->n_densw);
  P->o_wgt = take(sizeof(double) * P->n_src);
  P->o_h = take(sizeof(double) * P->n_panels);
  P->o_ctr = take(sizeof(CenterRec) * P->n_ctr);
  P->o_jtab = take(sizeof(double) * P->n_jtab);
  P->o_tape = take(sizeof(double2) * P->n_tape);
  P->o_G = take(sizeof(double2) * P->n_G);
  P->o_cg = take(sizeof(double) * 8 * P->n_ctr);
  P->o_spart = take(sizeof(double2) * P->n_spart);
  P->o_cpart = take(sizeof(double) * P->n_cpart);
  P->o_sg = take(sizeof(double) * 8 * P->n_src);
  P->total = o;
  return true;
}

template <typename T>
static T* wsp(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

__global__ void k_zero_ints(int* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

// ---------------------------------------------------------------------------
// geometry of every contour: one block per panel of the batch
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_upsample_batched(
    const BatchItemDev* __restrict__ items, const long long* __restrict__ pre_panel, int n,
    const double* __restrict__ nodes, const double* __restrict__ density,
    const double* __restrict__ tab, double4* __restrict__ geo, double2* __restrict__ densw,
    double* __restrict__ wgt, double* __restrict__ hpan, CenterRec* __restrict__ ctr,
    double* __restrict__ jtab) {
  const int it = find_slot(pre_panel, n, blockIdx.x);
  const BatchItemDev& B = items[it];
  const Dims d = B.d;
  const int m = (int)(blockIdx.x - pre_panel[it]);
  upsample_panel(d, m, nodes + B.node_off, density + B.din_off, tab, geo + B.src_off,
                 densw + B.densw_off, wgt + B.src_off, hpan + B.panel_off, ctr + B.ctr_off,
                 jtab + B.jtab_off);
}

// ---------------------------------------------------------------------------
// per-element and per-panel steps over the whole batch
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_make_G_batched(const BatchItemDev* __restrict__ items,
                                                        const long long* __restrict__ pre_G, int n,
                                                        long long total,
                                                        const double* __restrict__ cot,
                                                        double2* __restrict__ G) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int it = find_slot(pre_G, n, e);
  const BatchItemDev& B = items[it];
  make_G_elem((int)(e - pre_G[it]), B.d.Mc, B.d.T, B.d.nk, cot + B.out_off, G + B.G_off);
}

__global__ __launch_bounds__(256) void k_center_grads_batched(
    const BatchItemDev* __restrict__ items, const long long* __restrict__ pre_ctr, int n,
    long long total, const CenterRec* __restrict__ ctr, const double2* __restrict__ tape,
    const double2* __restrict__ G, double* __restrict__ cg) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int it = find_slot(pre_ctr, n, e);
  const BatchItemDev& B = items[it];
  center_grad_elem((int)(e - pre_ctr[it]), B.d.Mc, B.d.nk, B.d.side, B.d.T, ctr + B.ctr_off,
                   tape + B.tape_off, G + B.G_off, cg + B.ctr_off * 8);
}

// per center of the batch: the fused center-side sums over the contour's source
// blocks, then the gradient assembly
__global__ __launch_bounds__(256) void k_fused_center_grads_batched(
    const BatchItemDev* __restrict__ items, const long long* __restrict__ pre_ctr, int n,
    long long total, const CenterRec* __restrict__ ctr, const double* __restrict__ cpart,
    double* __restrict__ cg) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int it = find_slot(pre_ctr, n, e);
  const BatchItemDev& B = items[it];
  const Dims& d = B.d;
  const int ci = (int)(e - pre_ctr[it]);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sb = 0; sb < d.n_sb; ++sb) {
    const double* q = cpart + B.cpart_off + ((size_t)sb * d.Mc + ci) * 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) s[b] += q[b];
  }
  center_grad_from_sums(ci, d.side, d.T, ctr + B.ctr_off, s[0], s[1], s[2], s[3],
                        cg + B.ctr_off * 8);
}

__global__ __launch_bounds__(256) void k_source_finalize_batched(
    const BatchItemDev* __restrict__ items, const long long* __restrict__ pre_src, int n,
    long long total, int fused, const double4* __restrict__ geo,
    const double2* __restrict__ spart, double* __restrict__ sg) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int it = find_slot(pre_src, n, e);
  const BatchItemDev& B = items[it];
  // the source sums come in n_cb parts from the fused pass, n_csplit otherwise
  source_finalize_elem((int)(e - pre_src[it]), B.d.N, B.d.kind,
                       fused ? B.d.n_cb : B.d.n_csplit, geo + B.src_off, spart + B.spart_off,
                       sg + B.src_off * 8);
}

__global__ __launch_bounds__(128) void k_chain_batched(
    const BatchItemDev* __restrict__ items, const long long* __restrict__ pre_panel, int n,
    const double* __restrict__ nodes, const double* __restrict__ density,
    const double* __restrict__ tab, const double* __restrict__ sg, const double* __restrict__ cg,
    double* __restrict__ grad_density, double* __restrict__ grad_nodes) {
  const int it = find_slot(pre_panel, n, blockIdx.x);
  const BatchItemDev& B = items[it];
  const Dims d = B.d;
  const int m = (int)(blockIdx.x - pre_panel[it]);
  chain_panel(d, m, nodes + B.node_off, density + B.din_off, tab, sg + B.src_off * 8,
              cg + B.ctr_off * 8, nullptr, nullptr,
              grad_density ? grad_density + B.din_off : nullptr,
              grad_nodes ? grad_nodes + B.node_off : nullptr);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int upload_plan(const BatchPlan& P, void* ws, hipStream_t s) {
  struct Up {
    size_t off;
    const void* src;
    size_t bytes;
  } ups[] = {
      {P.o_items, P.items.data(), sizeof(BatchItemDev) * P.n},
      {P.o_ord_f, P.order_f.data(), sizeof(int) * P.n},
      {P.o_ord_a, P.order_a.data(), sizeof(int) * P.n},
      {P.o_ord_x, P.order_x.data(), sizeof(int) * P.n},
      {P.o_pre_f, P.pre_f.data(), sizeof(long long) * P.pre_f.size()},
      {P.o_pre_a, P.pre_a.data(), sizeof(long long) * P.pre_a.size()},
      {P.o_pre_x, P.pre_x.data(), sizeof(long long) * P.pre_x.size()},
      {P.o_pre_panel, P.pre_panel.data(), sizeof(long long) * (P.n + 1)},
      {P.o_pre_ctr, P.pre_ctr.data(), sizeof(long long) * (P.n + 1)},
      {P.o_pre_src, P.pre_src.data(), sizeof(long long) * (P.n + 1)},
      {P.o_pre_G, P.pre_G.data(), sizeof(long long) * (P.n + 1)},
  };
  for (const Up& u : ups) {
    hipError_t e = hipMemcpyAsync(static_cast<char*>(ws) + u.off, u.src, u.bytes,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_fail(e, "upload of the batch plan");
  }
  return QBX_OK;
}

static int batch_prepare(const BatchPlan& P, const double* nodes, const double* density, void* ws,
                         hipStream_t s) {
  int rc = upload_plan(P, ws, s);
  if (rc) return rc;
  Dims d0 = P.items[0].d;
  hipError_t e = launch_tables(d0, wsp<double>(ws, P.o_tables), s);
  if (e != hipSuccess) return device_fail(e, "tables kernel");
  hipLaunchKernelGGL(k_upsample_batched, dim3((unsigned)P.n_panels), dim3(128), 0, s,
                     wsp<BatchItemDev>(ws, P.o_items), wsp<long long>(ws, P.o_pre_panel), P.n,
                     nodes, density, wsp<double>(ws, P.o_tables), wsp<double4>(ws, P.o_geo),
                     wsp<double2>(ws, P.o_densw), wsp<double>(ws, P.o_wgt),
                     wsp<double>(ws, P.o_h), wsp<CenterRec>(ws, P.o_ctr),
                     wsp<double>(ws, P.o_jtab));
  e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "batched upsample kernel");
}

// which = 0 forward, 1 adjoint source pass, 2 fused adjoint tiles
static BatchTasks class_tasks(const BatchPlan& P, void* ws, size_t c, int which) {
  const BatchClass& C = P.cls[c];
  BatchTasks t;
  t.items = wsp<BatchItemDev>(ws, P.o_items);
  t.order = wsp<int>(ws, which == 0 ? P.o_ord_f : which == 1 ? P.o_ord_a : P.o_ord_x) + C.ord_at;
  t.pre = wsp<long long>(ws, which == 0 ? P.o_pre_f : which == 1 ? P.o_pre_a : P.o_pre_x) +
          C.pre_at;
  t.n = C.n;
  t.n_tasks = which == 0 ? C.tasks_f : which == 1 ? C.tasks_a : C.tasks_x;
  t.counter = wsp<int>(ws, P.o_counter) + (size_t)which * P.cls.size() + c;
  return t;
}

static int zero_counters(const BatchPlan& P, void* ws, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(256), 0, s, wsp<int>(ws, P.o_counter),
                     (int)(3 * P.cls.size()));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "counter reset kernel");
}

// Concurrent classes.  The (kind, p) classes of one pass are independent (disjoint
// contours, their own task counters and output ranges), so they are spread over
// the caller's stream and up to kAuxStreams library streams of the current device
// (default priority), forked from the caller's stream and joined back to it with
// events.  Each class's persistent kernel fills the GPU on its own; the next
// class's workgroups take compute units as its tail frees them, instead of every
// class's tail leaving the GPU idle in turn.  Results do not depend on it: every
// sum keeps its fixed order.  The streams and events are created on a device's
// first batched call and kept until the process ends; the enqueueing is
// serialised by a lock, so calls from several host threads stay well formed.
namespace {
constexpr int kAuxStreams = 3;
constexpr int kMaxDevices = 64;
struct ClassStreams {
  hipStream_t aux[kAuxStreams];
  hipEvent_t fork, join[kAuxStreams];
  bool ready = false;
};
ClassStreams g_class_streams[kMaxDevices];
std::mutex g_class_streams_mu;

// classes are launched on lane c % (1 + kAuxStreams): lane 0 is the caller's stream
struct ClassFork {
  ClassStreams* cs = nullptr;
  hipStream_t caller;
  int lanes = 1;
  std::unique_lock<std::mutex> lock;
  hipStream_t stream(size_t c) const {
    const int l = (int)(c % (size_t)lanes);
    return l == 0 ? caller : cs->aux[l - 1];
  }
};

// fork n_classes over the caller's stream and the library streams
int class_fork(size_t n_classes, hipStream_t caller, ClassFork* f) {
  f->caller = caller;
  f->lanes = 1;
  if (n_classes < 2) return QBX_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return QBX_OK;   // serial on the caller's stream
  f->lock = std::unique_lock<std::mutex>(g_class_streams_mu);
  ClassStreams& cs = g_class_streams[dev];
  if (!cs.ready) {
    for (int i = 0; i < kAuxStreams; ++i) {
      if ((e = hipStreamCreateWithFlags(&cs.aux[i], hipStreamNonBlocking)) != hipSuccess)
        return device_fail(e, "class stream creation");
      if ((e = hipEventCreateWithFlags(&cs.join[i], hipEventDisableTiming)) != hipSuccess)
        return device_fail(e, "class event creation");
    }
    if ((e = hipEventCreateWithFlags(&cs.fork, hipEventDisableTiming)) != hipSuccess)
      return device_fail(e, "class event creation");
    cs.ready = true;
  }
  f->cs = &cs;
  f->lanes = 1 + (int)std::min<size_t>(kAuxStreams, n_classes - 1);
  if ((e = hipEventRecord(cs.fork, caller)) != hipSuccess)
    return device_fail(e, "class fork event");
  for (int i = 0; i + 1 < f->lanes; ++i)
    if ((e = hipStreamWaitEvent(cs.aux[i], cs.fork, 0)) != hipSuccess)
      return device_fail(e, "class fork wait");
  return QBX_OK;
}

// the caller's stream waits for every library stream used
int class_join(ClassFork* f) {
  for (int i = 0; i + 1 < f->lanes; ++i) {
    hipError_t e = hipEventRecord(f->cs->join[i], f->cs->aux[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(f->caller, f->cs->join[i], 0);
    if (e != hipSuccess) return device_fail(e, "class join");
  }
  return QBX_OK;
}
}  // namespace

static int batch_forward(const BatchPlan& P, double* out, double2* tape, void* ws, hipStream_t s) {
  int rc = zero_counters(P, ws, s);
  if (rc) return rc;
  timer_begin(2, s);
  ClassFork f;
  rc = class_fork(P.cls.size(), s, &f);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  for (size_t c = 0; c < P.cls.size() && e == hipSuccess; ++c) {
    const BatchTasks t = class_tasks(P, ws, c, 0);
    e = launch_forward_batched(tape ? 1 : 0, P.cls[c].kind, P.cls[c].p, t,
                               wsp<double4>(ws, P.o_geo), wsp<double2>(ws, P.o_densw),
                               wsp<CenterRec>(ws, P.o_ctr), wsp<double>(ws, P.o_jtab), out, tape,
                               g_batch_grid_scale, f.stream(c));
  }
  rc = class_join(&f);
  timer_end(2, s);
  if (e != hipSuccess) return device_fail(e, "batched forward kernel");
  return rc;
}

hipError_t launch_forward_batched_0(int, int, const BatchTasks&, const double4*, const double2*,
                                    const CenterRec*, const double*, double*, double2*, double,
                                    hipStream_t);
hipError_t launch_forward_batched_1(int, int, const BatchTasks&, const double4*, const double2*,
                                    const CenterRec*, const double*, double*, double2*, double,
                                    hipStream_t);

hipError_t launch_forward_batched(int mode, int kind, int p, const BatchTasks& t,
                                  const double4* geo, const double2* densw, const CenterRec* ctr,
                                  const double* jtab, double* out, double2* tape, double grid_scale,
                                  hipStream_t s) {
  return mode ? launch_forward_batched_1(kind, p, t, geo, densw, ctr, jtab, out, tape, grid_scale, s)
              : launch_forward_batched_0(kind, p, t, geo, densw, ctr, jtab, out, tape, grid_scale, s);
}

void set_batch_tuning(double grid_scale, double adjoint_tasks, int fused_chunks) {
  g_batch_grid_scale = std::min(8.0, std::max(0.125, grid_scale));
  g_batch_adjoint_tasks = std::min(4194304.0, std::max(256.0, adjoint_tasks));
  g_batch_fused_chunks = std::min(64, std::max(1, fused_chunks));
}
void get_batch_tuning(double* grid_scale, double* adjoint_tasks, int* fused_chunks) {
  *grid_scale = g_batch_grid_scale;
  *adjoint_tasks = g_batch_adjoint_tasks;
  *fused_chunks = g_batch_fused_chunks;
}

}  // namespace qbx

using namespace qbx;

extern "C" {

size_t qbx_batched_workspace_bytes(const qbx_batch_item* items, int n_items, int oversample) {
  BatchPlan P;
  if (!build_plan(items, n_items, oversample, &P)) return 0;
  return P.total;
}

size_t qbx_batched_tape_bytes(const qbx_batch_item* items, int n_items) {
  BatchPlan P;
  if (!build_plan(items, n_items, 1, &P)) return 0;
  return sizeof(double2) * (size_t)P.n_tape;
}

int qbx_layer_potential_batched(const qbx_batch_item* items, int n_items, const double* nodes,
                                const double* density, double* out, double* tape, int oversample,
                                void* ws, size_t ws_bytes, hipStream_t stream) {
  BatchPlan P;
  if (!build_plan(items, n_items, oversample, &P))
    return fail(QBX_EINVAL, "invalid batch (an item's parameters, offsets or oversample)");
  if (!nodes || !density || !out || !ws) return fail(QBX_EINVAL, "NULL array argument");
  if (ws_bytes < P.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, P.total);
  int rc = batch_prepare(P, nodes, density, ws, stream);
  if (rc) return rc;
  return batch_forward(P, out, reinterpret_cast<double2*>(tape), ws, stream);
}

int qbx_layer_potential_batched_adjoint(const qbx_batch_item* items, int n_items,
                                        const double* nodes, const double* density,
                                        const double* cotangent, const double* tape,
                                        double* grad_density, double* grad_nodes, int oversample,
                                        void* ws, size_t ws_bytes, hipStream_t stream) {
  BatchPlan P;
  if (!build_plan(items, n_items, oversample, &P))
    return fail(QBX_EINVAL, "invalid batch (an item's parameters, offsets or oversample)");
  if (!nodes || !density || !cotangent || !ws) return fail(QBX_EINVAL, "NULL array argument");
  if (ws_bytes < P.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, P.total);
  if (!grad_density && !grad_nodes) return QBX_OK;
  int rc = batch_prepare(P, nodes, density, ws, stream);
  if (rc) return rc;
  const double2* tp = reinterpret_cast<const double2*>(tape);
  const bool fused = !tp && grad_nodes;   // no tape: one fused pass for both sides
  const long long nG = P.n_G, nC = P.n_ctr, nS = P.n_src;
  auto blocks = [](long long n, int b) { return dim3((unsigned)((n + b - 1) / b)); };
  BatchItemDev* it = wsp<BatchItemDev>(ws, P.o_items);
  hipLaunchKernelGGL(k_make_G_batched, blocks(nG, 256), dim3(256), 0, stream, it,
                     wsp<long long>(ws, P.o_pre_G), P.n, nG, cotangent, wsp<double2>(ws, P.o_G));
  // with a tape, its center sums; without one and only the density gradient
  // wanted, no center side at all (the chain step then reads no center data)
  if (tp)
    hipLaunchKernelGGL(k_center_grads_batched, blocks(nC, 256), dim3(256), 0, stream, it,
                       wsp<long long>(ws, P.o_pre_ctr), P.n, nC, wsp<CenterRec>(ws, P.o_ctr), tp,
                       wsp<double2>(ws, P.o_G), wsp<double>(ws, P.o_cg));
  rc = zero_counters(P, ws, stream);
  if (rc) return rc;
  timer_begin(2, stream);
  ClassFork f;
  rc = class_fork(P.cls.size(), stream, &f);
  if (rc) return rc;
  hipError_t ea = hipSuccess;
  for (size_t c = 0; c < P.cls.size() && ea == hipSuccess; ++c) {
    const BatchTasks t = class_tasks(P, ws, c, fused ? 2 : 1);
    const hipStream_t sc = f.stream(c);
    ea = fused ? launch_adjoint_fused_batched(P.cls[c].kind, P.cls[c].p, t,
                                              wsp<double4>(ws, P.o_geo),
                                              wsp<double2>(ws, P.o_densw),
                                              wsp<CenterRec>(ws, P.o_ctr),
                                              wsp<double>(ws, P.o_jtab), wsp<double2>(ws, P.o_G),
                                              wsp<double2>(ws, P.o_spart),
                                              wsp<double>(ws, P.o_cpart), g_batch_grid_scale, sc)
               : launch_adjoint_batched(P.cls[c].kind, P.cls[c].p, t, wsp<double4>(ws, P.o_geo),
                                        wsp<double2>(ws, P.o_densw),
                                        wsp<CenterRec>(ws, P.o_ctr), wsp<double>(ws, P.o_jtab),
                                        wsp<double2>(ws, P.o_G), wsp<double2>(ws, P.o_spart),
                                        g_batch_grid_scale, sc);
  }
  rc = class_join(&f);
  timer_end(2, stream);
  if (ea != hipSuccess) return device_fail(ea, "batched adjoint kernel");
  if (rc) return rc;
  if (fused)
    hipLaunchKernelGGL(k_fused_center_grads_batched, blocks(nC, 256), dim3(256), 0, stream, it,
                       wsp<long long>(ws, P.o_pre_ctr), P.n, nC, wsp<CenterRec>(ws, P.o_ctr),
                       wsp<double>(ws, P.o_cpart), wsp<double>(ws, P.o_cg));
  hipLaunchKernelGGL(k_source_finalize_batched, blocks(nS, 256), dim3(256), 0, stream, it,
                     wsp<long long>(ws, P.o_pre_src), P.n, nS, fused ? 1 : 0,
                     wsp<double4>(ws, P.o_geo), wsp<double2>(ws, P.o_spart),
                     wsp<double>(ws, P.o_sg));
  hipLaunchKernelGGL(k_chain_batched, dim3((unsigned)P.n_panels), dim3(128), 0, stream, it,
                     wsp<long long>(ws, P.o_pre_panel), P.n, nodes, density,
                     wsp<double>(ws, P.o_tables), wsp<double>(ws, P.o_sg), wsp<double>(ws, P.o_cg),
                     grad_density, grad_nodes);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? QBX_OK : device_fail(e, "batched adjoint kernels");
}

}  // extern "C"
