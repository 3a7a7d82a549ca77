// Host side of libqbx: argument validation, workspace layout, launch order and
// error reporting behind the C ABI of include/qbx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qbx.h"
#include "qbx_internal.h"
#include "qbx_special.h"

namespace qbx {

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int device_fail(hipError_t e, const char* where) {
  return fail(QBX_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// launch tunables of the per-contour path (qbx_set_tuning): wavefronts aimed
// for per launch of the plain forward, the forward-with-tape and the adjoint
// source pass
static int g_forward_waves = 16384;
static int g_tape_waves = 16384;
static int g_adjoint_waves = 16384;
static int g_fused_tiles = 16384;  // fused adjoint workgroups aimed for
static const int kSplitFarWaves = 65536;  // far-pass wavefronts aimed for
static const int kFusedMinTile = 32;      // fewest centers a fused adjoint tile takes
static double g_fused_part_bytes = 2147483648.0;  // fused adjoint partial-sum bound

double fused_part_budget() { return g_fused_part_bytes; }

void set_contour_tuning(int forward_waves, int tape_waves, int adjoint_waves, int fused_tiles) {
  g_forward_waves = forward_waves;
  g_tape_waves = tape_waves;
  g_adjoint_waves = adjoint_waves;
  g_fused_tiles = fused_tiles;
}

void get_contour_tuning(int* forward_waves, int* tape_waves, int* adjoint_waves,
                        int* fused_tiles) {
  *forward_waves = g_forward_waves;
  *tape_waves = g_tape_waves;
  *adjoint_waves = g_adjoint_waves;
  *fused_tiles = g_fused_tiles;
}

// source splits of the forward kernels and center splits of the adjoint source
// pass, from the tuning targets (see qbx_set_tuning)
void set_launch_shape(Dims* d) {
  d->chunks = (int)(((long)d->N + kWave - 1) / kWave);
  // forward: enough wavefronts to fill 256 CUs several times over, but at
  // least four 64-source chunks per wavefront
  const long want_waves = g_forward_waves;
  long split = (want_waves + d->Mc - 1) / d->Mc;
  long max_split = d->chunks / 4;
  if (max_split < 1) max_split = 1;
  if (split > max_split) split = max_split;
  if (split < 1) split = 1;
  d->chunks_per_split = (int)((d->chunks + split - 1) / split);
  d->n_split = (d->chunks + d->chunks_per_split - 1) / d->chunks_per_split;
  // forward-with-tape: the same rule with its own target
  long tsplit = (g_tape_waves + d->Mc - 1) / d->Mc;
  if (tsplit > max_split) tsplit = max_split;
  if (tsplit < 1) tsplit = 1;
  d->tape_chunks_per_split = (int)((d->chunks + tsplit - 1) / tsplit);
  d->n_tsplit = (d->chunks + d->tape_chunks_per_split - 1) / d->tape_chunks_per_split;
  // adjoint: one wave per 64 sources and center split, >= 16 centers per split
  long cs = ((long)g_adjoint_waves + d->chunks - 1) / d->chunks;
  long max_cs = d->Mc / 16;
  if (max_cs < 1) max_cs = 1;
  if (cs > max_cs) cs = max_cs;
  if (cs < 1) cs = 1;
  d->centers_per_split = (int)(((long)d->Mc + cs - 1) / cs);
  d->n_csplit = (int)(((long)d->Mc + d->centers_per_split - 1) / d->centers_per_split);
  // fused adjoint: tiles of fused_tile_height centers; enough source blocks for
  // about g_fused_tiles tiles, each of at least four chunks (one per wave)
  d->fused_cblock = fused_tile_height(d->Mc, d->N, d->kind);
  d->n_cb = (d->Mc + d->fused_cblock - 1) / d->fused_cblock;
  long max_sb = (d->chunks + 3) / 4;
  // small contours: when even the finest source blocks leave fewer tiles than
  // aimed for, shorter tiles (down to kFusedMinTile centers) make up the rest,
  // within the partial-sum bound
  if ((long)d->n_cb * max_sb < g_fused_tiles && d->fused_cblock > kFusedMinTile) {
    const long want_cb = ((long)g_fused_tiles + max_sb - 1) / max_sb;
    const long h = std::max((long)kFusedMinTile, ((long)d->Mc + want_cb - 1) / want_cb);
    const long n_cb = ((long)d->Mc + h - 1) / h;
    if (h < d->fused_cblock &&
        (double)n_cb * src_slots(d->kind) * (double)d->N * 16.0 <= fused_part_budget()) {
      d->fused_cblock = (int)h;
      d->n_cb = (int)n_cb;
    }
  }
  long sbs = ((long)g_fused_tiles + d->n_cb - 1) / d->n_cb;
  if (sbs > max_sb) sbs = max_sb;
  if (sbs < 1) sbs = 1;
  d->chunks_per_sb = (int)((d->chunks + sbs - 1) / sbs);
  d->n_sb = (d->chunks + d->chunks_per_sb - 1) / d->chunks_per_sb;
  // split forward, far pass: 64 targets a wave; enough source splits (split sp
  // takes panels sp, sp + n_fsplit, ...) for about kSplitFarWaves waves
  const long n_tb = ((long)d->T + kWave - 1) / kWave;
  long fs = (kSplitFarWaves + n_tb - 1) / n_tb;
  if (fs > d->P) fs = d->P;
  if (fs < 1) fs = 1;
  d->panels_per_fsplit = (int)((d->P + fs - 1) / fs);
  d->n_fsplit = (d->P + d->panels_per_fsplit - 1) / d->panels_per_fsplit;
  // its adjoint, far part: 64 far sources a wave, target splits alike
  long as = (kSplitFarWaves + n_tb - 1) / n_tb;
  if (as > d->P) as = d->P;
  if (as < 1) as = 1;
  d->panels_per_asplit = (int)((d->P + as - 1) / as);
  d->n_asplit = (d->P + d->panels_per_asplit - 1) / d->panels_per_asplit;
}

bool make_dims(int n_panels, int q, int p, int oversample, int side, int kind, double k, double r,
               Dims* d) {
  if (n_panels < 3 || q != kQ || p < 0 || p > kPMax || oversample < 1 ||
      oversample > QBX_OVERSAMPLE_MAX)
    return false;
  if (side != QBX_INTERIOR && side != QBX_EXTERIOR && side != QBX_BOTH) return false;
  if (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D)) return false;
  const long T = (long)n_panels * kQ;
  const long N = T * oversample;
  const long Mc = T * (side == QBX_BOTH ? 2 : 1);
  if (N > (1L << 30) || Mc > (1L << 28)) return false;
  d->P = n_panels;
  d->qs = kQ * oversample;
  d->T = (int)T;
  d->N = (int)N;
  d->n_sides = side == QBX_BOTH ? 2 : 1;
  d->nk = (kind == 3) ? 2 : 1;
  d->p = p;
  d->Mc = (int)Mc;
  d->NJ = 2 * (p + 4);   // J_0..J_{p+3}, then J'_0..J'_{p+3}
  d->side = side;
  d->kind = kind;
  d->dipole = 0;
  d->center_rule = 0;
  d->k = k;
  d->r = r;
  set_launch_shape(d);
  return true;
}

Layout make_layout(const Dims& d) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.tables = take(sizeof(double) * table_layout(d.qs).total);
  L.geo = take(sizeof(double4) * (size_t)d.N);
  L.dens = take(sizeof(double2) * (size_t)d.nk * d.N);
  L.wgt = take(sizeof(double) * (size_t)d.N);
  L.h = take(sizeof(double) * (size_t)d.P);
  L.ctr = take(sizeof(CenterRec) * (size_t)d.Mc);
  L.jtab = take(sizeof(double) * (size_t)d.Mc * (d.NJ + d.NJ / 2));
  // forward partials [n_split][nk][Mc], tape partials [n_tsplit][nk][Mc][5]
  const size_t n_part = std::max((size_t)d.n_split, (size_t)d.n_tsplit * 5);
  L.partial = take(sizeof(double2) * n_part * d.nk * d.Mc);
  L.tape = take(sizeof(double2) * (size_t)d.Mc * d.nk * 4);
  L.G = take(sizeof(double2) * (size_t)d.nk * d.Mc);
  L.cg = take(sizeof(double) * (size_t)d.Mc * 8);
  L.spart = take(sizeof(double2) * (size_t)std::max(d.n_csplit, d.n_cb) * src_slots(d.kind) * d.N);
  L.cpart = take(sizeof(double) * (size_t)d.n_sb * d.Mc * 4);
  L.sg = take(sizeof(double) * (size_t)d.N * 8);
  L.scratch = take(sizeof(double) * (16 + (size_t)d.Mc));
  L.bnd = take(sizeof(double4) * (size_t)d.P);
  L.ncount = take(sizeof(int) * (size_t)d.P);
  L.nlist = take(sizeof(int) * (size_t)d.P * kNearCap);
  L.fpart = take(sizeof(double2) * (size_t)d.n_fsplit * d.nk * d.T * 2);
  L.gfar = take(sizeof(double2) * (size_t)d.nk * d.T);
  L.aacc = take(sizeof(double2) * (size_t)d.nk * d.N);
  L.ngeo = take(sizeof(double4) * (size_t)d.T);
  L.ndens = take(sizeof(double2) * (size_t)d.nk * d.T);
  L.nw = take(sizeof(double) * (size_t)d.T);
  L.apart = take(sizeof(double2) * (size_t)d.n_asplit * (d.nk + 2) * d.T);
  L.gtw = take(sizeof(double) * (size_t)d.T * 2);
  L.gde = take(sizeof(double2) * (size_t)d.nk * d.T);
  L.total = o;
  return L;
}

// The arrays the plain forward alone uses (tables, source grid, centers, J
// tables without the order-weighted block, forward partial sums), packed; the
// other offsets are left at 0 and must not be used.
Layout make_forward_layout(const Dims& d) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.tables = take(sizeof(double) * table_layout(d.qs).total);
  L.geo = take(sizeof(double4) * (size_t)d.N);
  L.dens = take(sizeof(double2) * (size_t)d.nk * d.N);
  L.wgt = take(sizeof(double) * (size_t)d.N);
  L.h = take(sizeof(double) * (size_t)d.P);
  L.ctr = take(sizeof(CenterRec) * (size_t)d.Mc);
  L.jtab = take(sizeof(double) * (size_t)d.Mc * d.NJ);
  L.partial = take(sizeof(double2) * (size_t)d.n_split * d.nk * d.Mc);
  L.total = o;
  return L;
}

template <typename T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

int validate(const qbx_geometry* g, int p, double k, double r, int oversample, int side,
             int kind, Dims* d) {
  if (!g) return fail(QBX_EINVAL, "geometry is NULL");
  if (!g->nodes) return fail(QBX_EINVAL, "geometry nodes pointer is NULL");
  if (g->q != kQ) return fail(QBX_EINVAL, "q = %d, only %d nodes per panel are supported", g->q, kQ);
  if (g->n_panels < 3) return fail(QBX_EINVAL, "n_panels = %d < 3", g->n_panels);
  if (p < 0 || p > kPMax) return fail(QBX_EINVAL, "order p = %d outside [0, %d]", p, kPMax);
  if (!(k > 0.0) || !std::isfinite(k)) return fail(QBX_EINVAL, "wavenumber k = %g must be > 0", k);
  if (!(r > 0.0) || !std::isfinite(r)) return fail(QBX_EINVAL, "center distance r = %g must be > 0", r);
  if (oversample < 1 || oversample > QBX_OVERSAMPLE_MAX)
    return fail(QBX_EINVAL, "oversample = %d outside [1, %d]", oversample, QBX_OVERSAMPLE_MAX);
  if (side != QBX_INTERIOR && side != QBX_EXTERIOR && side != QBX_BOTH)
    return fail(QBX_EINVAL, "side = %d is not -1, 0 or 1", side);
  if (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D))
    return fail(QBX_EINVAL, "kind = %d is not 1 (S), 2 (D) or 3 (S|D)", kind);
  if (!make_dims(g->n_panels, g->q, p, oversample, side, kind, k, r, d))
    return fail(QBX_EINVAL, "problem too large");
  return QBX_OK;
}

// ---- kernel timer ----
struct TimerRec {
  int cls;
  hipEvent_t a, b;
};
static bool g_timer_on = false;
static std::vector<TimerRec> g_timer;
static hipEvent_t g_pending[QBX_TIMER_CLASSES];

// an event recorded on s, or nullptr when either call fails (the launch is then
// simply not timed)
static hipEvent_t timer_event(hipStream_t s) {
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return nullptr;
  }
  return e;
}

void timer_begin(int cls, hipStream_t s) {
  if (!g_timer_on) return;
  g_pending[cls] = timer_event(s);
}

void timer_end(int cls, hipStream_t s) {
  if (!g_timer_on || !g_pending[cls]) return;
  hipEvent_t e = timer_event(s);
  if (e) {
    g_timer.push_back({cls, g_pending[cls], e});
  } else {
    (void)hipEventDestroy(g_pending[cls]);
  }
  g_pending[cls] = nullptr;
}

static void timer_clear() {
  for (auto& r : g_timer) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_timer.clear();
  for (auto& e : g_pending) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
}

// tables + source grid + centers into the workspace
static int prepare(const Dims& d, const Layout& L, const double* nodes, const double* density,
                   void* ws, hipStream_t stream) {
  hipError_t e = launch_tables(d, at<double>(ws, L.tables), stream);
  if (e != hipSuccess) return device_fail(e, "tables kernel");
  e = launch_upsample(d, nodes, density, at<double>(ws, L.tables), at<double4>(ws, L.geo),
                      at<double2>(ws, L.dens), at<double>(ws, L.wgt), at<double>(ws, L.h),
                      at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab), stream);
  if (e != hipSuccess) return device_fail(e, "upsample kernel");
  return QBX_OK;
}

// the 16-node differentiation matrix by the barycentric formula, built once
const NodeDiff& node_diff() {
  static const NodeDiff D = [] {
    NodeDiff r;
    double t16[kQ], w16[kQ], bw[kQ];
    for (int a = 0; a < kQ; ++a) gauss_legendre_node(kQ, a, &t16[a], &w16[a]);
    for (int a = 0; a < kQ; ++a) {
      double pr = 1.0;
      for (int c = 0; c < kQ; ++c)
        if (c != a) pr *= (t16[a] - t16[c]);
      bw[a] = 1.0 / pr;
    }
    for (int b = 0; b < kQ; ++b)
      for (int a = 0; a < kQ; ++a) {
        if (a != b) {
          r.d[b][a] = (bw[a] / bw[b]) / (t16[b] - t16[a]);
        } else {
          double v = 0.0;
          for (int c = 0; c < kQ; ++c)
            if (c != b) v += 1.0 / (t16[b] - t16[c]);
          r.d[b][a] = v;
        }
      }
    return r;
  }();
  return D;
}

int run_forward(const Dims& d, const Layout& L, const double* nodes, const double* density,
                double* out, void* ws, hipStream_t stream, bool timed) {
  int rc = prepare(d, L, nodes, density, ws, stream);
  if (rc) return rc;
  if (timed) timer_begin(0, stream);
  hipError_t e = launch_forward(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                                at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                                at<double2>(ws, L.partial), stream);
  if (timed) timer_end(0, stream);
  if (e != hipSuccess) return device_fail(e, "forward kernel");
  e = launch_finalize(d, at<double2>(ws, L.partial), out, stream);
  if (e != hipSuccess) return device_fail(e, "finalize kernel");
  return QBX_OK;
}

}  // namespace qbx

using namespace qbx;

extern "C" {

size_t qbx_workspace_bytes(int n_panels, int q, int p, int oversample, int side, int kind) {
  Dims d;
  if (!make_dims(n_panels, q, p, oversample, side, kind, 1.0, 0.5, &d)) return 0;
  return make_layout(d).total;
}

size_t qbx_tape_bytes(int n_panels, int q, int p, int side, int kind) {
  Dims d;
  if (!make_dims(n_panels, q, p, 1, side, kind, 1.0, 0.5, &d)) return 0;
  // per center and kind: sum_j w sigma dK/dR, dK/dtheta and grad_v K (x, y)
  return sizeof(double2) * (size_t)d.Mc * d.nk * 4;
}

int qbx_layer_potential(const qbx_geometry* g, const double* density, double k, int p, double r,
                        int oversample, int side, int kind, double* out, double* tape, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!out) return fail(QBX_EINVAL, "out is NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  if (!tape) return run_forward(d, L, g->nodes, density, out, ws, stream);
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  hipError_t e;
  {
    timer_begin(3, stream);
    e = launch_forward_tape(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                            at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                            at<double2>(ws, L.partial), stream);
    timer_end(3, stream);
    if (e != hipSuccess) return device_fail(e, "forward (tape) kernel");
    e = launch_finalize_tape(d, at<double2>(ws, L.partial), out, reinterpret_cast<double2*>(tape),
                             stream);
    if (e != hipSuccess) return device_fail(e, "finalize (tape) kernel");
    return QBX_OK;
  }
}

int qbx_layer_potential_ext(const qbx_geometry* g, const double* density, double k, int p,
                            double r, int oversample, int side, int kind,
                            const qbx_forward_options* opt, double* out, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (opt) {
    if (opt->dipole != 0 && opt->dipole != 1)
      return fail(QBX_EINVAL, "dipole = %d is not 0 or 1", opt->dipole);
    if (opt->center_rule != 0 && opt->center_rule != 1)
      return fail(QBX_EINVAL, "center_rule = %d is not 0 or 1", opt->center_rule);
    d.dipole = opt->dipole;
    d.center_rule = opt->center_rule;
  }
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!out) return fail(QBX_EINVAL, "out is NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  timer_begin(0, stream);
  hipError_t e = launch_forward(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                                at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                                at<double2>(ws, L.partial), stream);
  timer_end(0, stream);
  if (e != hipSuccess) return device_fail(e, "forward kernel");
  e = launch_finalize(d, at<double2>(ws, L.partial), out, stream);
  if (e != hipSuccess) return device_fail(e, "finalize kernel");
  return QBX_OK;
}

}  // extern "C"

// the split's panel records, near lists and far sources (every split entry
// point, after prepare)
static int split_geometry(const Dims& d, const Layout& L, const qbx_geometry* g,
                          const double* density, double g2, void* ws, hipStream_t stream,
                          NearLists* nl, NystromSources* ns) {
  hipError_t e = launch_panel_bounds(d, g->nodes, at<double4>(ws, L.bnd), stream);
  if (e != hipSuccess) return device_fail(e, "panel bounds kernel");
  ns->geo = at<double4>(ws, L.ngeo);
  ns->dens = at<double2>(ws, L.ndens);
  ns->w = at<double>(ws, L.nw);
  e = launch_nystrom_sources(d, g->nodes, density, at<double>(ws, L.tables), *ns, stream);
  if (e != hipSuccess) return device_fail(e, "far source kernel");
  e = launch_near_lists(d, at<double4>(ws, L.bnd), g2, at<int>(ws, L.ncount), at<int>(ws, L.nlist),
                        stream);
  if (e != hipSuccess) return device_fail(e, "near list kernel");
  nl->count = at<int>(ws, L.ncount);
  nl->list = at<int>(ws, L.nlist);
  return QBX_OK;
}

extern "C" {

int qbx_layer_potential_split(const qbx_geometry* g, const double* density, double k, int p,
                              double r, int oversample, int side, int kind, double gamma,
                              double* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!(gamma > 0.0)) return fail(QBX_EINVAL, "near-panel factor gamma = %g must be > 0", gamma);
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!out) return fail(QBX_EINVAL, "out is NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  const double g2 = gamma * gamma;
  NearLists nl;
  NystromSources ns;
  if ((rc = split_geometry(d, L, g, density, g2, ws, stream, &nl, &ns))) return rc;
  timer_begin(6, stream);
  hipError_t e = launch_split_near(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                                   at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                                   at<double4>(ws, L.bnd), g2, nl, at<double2>(ws, L.partial),
                                   stream);
  timer_end(6, stream);
  if (e != hipSuccess) return device_fail(e, "split near kernel");
  timer_begin(7, stream);
  e = launch_split_far(d, ns, g->nodes, at<double4>(ws, L.bnd), g2, at<double2>(ws, L.fpart),
                       stream);
  timer_end(7, stream);
  if (e != hipSuccess) return device_fail(e, "split far kernel");
  e = launch_split_finalize(d, at<double2>(ws, L.partial), at<double2>(ws, L.fpart), out, stream);
  if (e != hipSuccess) return device_fail(e, "split finalize kernel");
  return QBX_OK;
}

int qbx_layer_potential_split_gradient(const qbx_geometry* g, const double* density, double k,
                                       int p, double r, int oversample, int side, int kind,
                                       double gamma, double* grad, double* dn, void* ws,
                                       size_t ws_bytes, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!(gamma > 0.0)) return fail(QBX_EINVAL, "near-panel factor gamma = %g must be > 0", gamma);
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!grad && !dn) return fail(QBX_EINVAL, "grad and dn are both NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  NearLists nl;
  NystromSources ns;
  if ((rc = split_geometry(d, L, g, density, gamma * gamma, ws, stream, &nl, &ns))) return rc;
  hipError_t e = launch_order_weighted(d, at<double>(ws, L.jtab), stream);
  if (e != hipSuccess) return device_fail(e, "order-weighted table kernel");
  e = launch_split_gradient(d, g->nodes, at<double4>(ws, L.geo), at<double2>(ws, L.dens), ns,
                            at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                            at<double4>(ws, L.bnd), gamma * gamma, nl,
                            at<double2>(ws, L.partial), at<double2>(ws, L.fpart), grad, dn,
                            stream);
  if (e != hipSuccess) return device_fail(e, "split gradient kernels");
  return QBX_OK;
}

int qbx_layer_potential_split_adjoint(const qbx_geometry* g, const double* density, double k,
                                      int p, double r, int oversample, int side, int kind,
                                      double gamma, const double* cotangent,
                                      double* grad_density, double* grad_nodes, void* ws,
                                      size_t ws_bytes, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!(gamma > 0.0)) return fail(QBX_EINVAL, "near-panel factor gamma = %g must be > 0", gamma);
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!cotangent) return fail(QBX_EINVAL, "cotangent is NULL");
  if (!grad_density && !grad_nodes)
    return fail(QBX_EINVAL, "grad_density and grad_nodes are both NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  NearLists nl;
  NystromSources ns;
  if ((rc = split_geometry(d, L, g, density, gamma * gamma, ws, stream, &nl, &ns))) return rc;
  hipError_t e = launch_make_G(d, cotangent, at<double2>(ws, L.G), stream);
  if (e != hipSuccess) return device_fail(e, "cotangent kernel");
  if (grad_nodes) {
    SplitNodeScratch w;
    w.Gf = at<double2>(ws, L.gfar);
    w.cg = at<double>(ws, L.cg);
    w.spart = at<double2>(ws, L.spart);
    w.fpart = at<double2>(ws, L.fpart);
    w.apart = at<double2>(ws, L.apart);
    w.sg = at<double>(ws, L.sg);
    w.gtw = at<double>(ws, L.gtw);
    w.gde = at<double2>(ws, L.gde);
    e = launch_split_adjoint_nodes(d, g->nodes, density, at<double>(ws, L.tables),
                                   at<double4>(ws, L.geo), at<double2>(ws, L.dens), ns,
                                   at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                                   at<double4>(ws, L.bnd), gamma * gamma, nl,
                                   at<double2>(ws, L.G), w, grad_density, grad_nodes, stream);
  } else {
    e = launch_split_adjoint_density(d, g->nodes, at<double>(ws, L.tables), at<double4>(ws, L.geo),
                                     at<double>(ws, L.wgt), ns, at<CenterRec>(ws, L.ctr),
                                     at<double>(ws, L.jtab), at<double4>(ws, L.bnd), gamma * gamma,
                                     nl, at<double2>(ws, L.G), at<double2>(ws, L.gfar),
                                     at<double2>(ws, L.aacc), at<double2>(ws, L.apart),
                                     grad_density, stream);
  }
  if (e != hipSuccess) return device_fail(e, "split adjoint kernels");
  return QBX_OK;
}

int qbx_layer_potential_gradient(const qbx_geometry* g, const double* density, double k, int p,
                                 double r, int oversample, int side, int kind, double* grad,
                                 double* dn, void* ws, size_t ws_bytes, hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!grad && !dn) return fail(QBX_EINVAL, "grad and dn are both NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  hipError_t e = launch_order_weighted(d, at<double>(ws, L.jtab), stream);
  if (e != hipSuccess) return device_fail(e, "order-weighted table kernel");
  timer_begin(5, stream);
  e = launch_forward_grad(d, at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                                    at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab),
                                    at<double2>(ws, L.partial), stream);
  timer_end(5, stream);
  if (e != hipSuccess) return device_fail(e, "target-derivative kernel");
  e = launch_finalize_gradient(d, at<CenterRec>(ws, L.ctr), at<double2>(ws, L.partial), grad, dn,
                               stream);
  if (e != hipSuccess) return device_fail(e, "gradient finalize kernel");
  return QBX_OK;
}

int qbx_layer_potential_adjoint(const qbx_geometry* g, const double* density, double k, int p,
                                double r, int oversample, int side, int kind,
                                const double* cotangent, const double* tape, double* grad_density,
                                double* grad_nodes, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, k, r, oversample, side, kind, &d);
  if (rc) return rc;
  if (!density) return fail(QBX_EINVAL, "density is NULL");
  if (!cotangent) return fail(QBX_EINVAL, "cotangent is NULL");
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  if (!grad_density && !grad_nodes) return QBX_OK;
  rc = prepare(d, L, g->nodes, density, ws, stream);
  if (rc) return rc;
  hipError_t e;
  const double2* tp = reinterpret_cast<const double2*>(tape);
  if (!tp && grad_nodes) {
    // no tape: one fused pass evaluates each pair once for both gradient sides
    e = launch_adjoint_fused(d, g->nodes, density, at<double>(ws, L.tables),
                             at<double4>(ws, L.geo), at<double2>(ws, L.dens),
                             at<CenterRec>(ws, L.ctr), at<double>(ws, L.jtab), cotangent,
                             at<double2>(ws, L.G), at<double>(ws, L.cpart), at<double>(ws, L.cg),
                             at<double2>(ws, L.spart), at<double>(ws, L.sg), grad_density,
                             grad_nodes, stream);
    return e == hipSuccess ? QBX_OK : device_fail(e, "fused adjoint kernels");
  }
  e = launch_adjoint_rest(d, g->nodes, density, at<double>(ws, L.tables), at<double4>(ws, L.geo),
                          at<double2>(ws, L.dens), at<CenterRec>(ws, L.ctr),
                          at<double>(ws, L.jtab), cotangent, tp, at<double2>(ws, L.G),
                          at<double>(ws, L.cg), at<double2>(ws, L.spart), at<double>(ws, L.sg),
                          grad_density, grad_nodes, stream);
  if (e != hipSuccess) return device_fail(e, "adjoint kernels");
  return QBX_OK;
}

int qbx_principal_value(const double* out, const double* density, int n_panels, int side,
                        int kind, double* pv, hipStream_t stream) {
  if (!out || !pv) return fail(QBX_EINVAL, "out or pv is NULL");
  if (n_panels < 3) return fail(QBX_EINVAL, "n_panels = %d < 3", n_panels);
  if (side != QBX_INTERIOR && side != QBX_EXTERIOR && side != QBX_BOTH)
    return fail(QBX_EINVAL, "side = %d is not -1, 0 or 1", side);
  if (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D))
    return fail(QBX_EINVAL, "kind = %d is not 1 (S), 2 (D) or 3 (S|D)", kind);
  if (side != QBX_BOTH && (kind & QBX_D) && !density)
    return fail(QBX_EINVAL, "density is needed for the one-sided D jump");
  const long T = (long)n_panels * kQ;
  if (T > (1L << 28)) return fail(QBX_EINVAL, "problem too large");
  const int nk = kind == 3 ? 2 : 1;
  hipError_t e = launch_principal_value((int)T, nk, side, kind, out, density, pv, stream);
  return e == hipSuccess ? QBX_OK : device_fail(e, "principal value kernel");
}

int qbx_gradient_principal_value(const qbx_geometry* g, const double* density, int side,
                                 int kind, const double* grad, const double* dn, double* grad_pv,
                                 double* dn_pv, hipStream_t stream) {
  if (!g || !g->nodes) return fail(QBX_EINVAL, "geometry or its nodes is NULL");
  if (g->q != kQ) return fail(QBX_EINVAL, "q = %d, only %d nodes per panel are supported", g->q, kQ);
  if (g->n_panels < 3) return fail(QBX_EINVAL, "n_panels = %d < 3", g->n_panels);
  if (side != QBX_INTERIOR && side != QBX_EXTERIOR && side != QBX_BOTH)
    return fail(QBX_EINVAL, "side = %d is not -1, 0 or 1", side);
  if (kind != QBX_S && kind != QBX_D && kind != (QBX_S | QBX_D))
    return fail(QBX_EINVAL, "kind = %d is not 1 (S), 2 (D) or 3 (S|D)", kind);
  if (!grad != !grad_pv || !dn != !dn_pv)
    return fail(QBX_EINVAL, "grad and grad_pv (dn and dn_pv) must be given together");
  if (!grad && !dn) return fail(QBX_EINVAL, "grad and dn are both NULL");
  if (side != QBX_BOTH && !density)
    return fail(QBX_EINVAL, "density is needed for the one-sided jumps");
  const long T = (long)g->n_panels * kQ;
  if (T > (1L << 28)) return fail(QBX_EINVAL, "problem too large");
  const int nk = kind == 3 ? 2 : 1;
  hipError_t e = launch_gradient_principal_value((int)T, nk, side, kind, node_diff(), g->nodes,
                                                 density, grad, dn, grad_pv, dn_pv, stream);
  return e == hipSuccess ? QBX_OK : device_fail(e, "gradient principal value kernel");
}

int qbx_check_geometry(const qbx_geometry* g, int p, double r, int oversample, int side,
                       double* area, double* min_ratio, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
  Dims d;
  int rc = validate(g, p, 1.0, r, oversample, side, QBX_S, &d);
  if (rc) return rc;
  if (!ws) return fail(QBX_EINVAL, "workspace is NULL");
  const Layout L = make_layout(d);
  if (ws_bytes < L.total)
    return fail(QBX_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  // any density works for the geometry; use the nodes array itself as a
  // harmless real input (only its values are read)
  Dims dg = d;
  rc = prepare(dg, L, g->nodes, g->nodes, ws, stream);
  if (rc) return rc;
  hipError_t e = launch_check(d, at<double4>(ws, L.geo), at<double>(ws, L.wgt),
                              at<CenterRec>(ws, L.ctr), at<double>(ws, L.scratch), stream);
  if (e != hipSuccess) return device_fail(e, "check kernels");
  double res[2];
  e = hipMemcpyAsync(res, at<double>(ws, L.scratch), sizeof(res), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return device_fail(e, "copy of check results");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return device_fail(e, "stream synchronize");
  if (area) *area = res[0];
  if (min_ratio) *min_ratio = res[1];
  if (res[0] < 0.0) return fail(QBX_EORIENT, "signed area %g < 0: contour is clockwise", res[0]);
  if (res[1] < 1.0 - 1e-12)
    return fail(QBX_EGRAF, "a source lies inside a center's disk (min |x'-c|/R = %.15g)", res[1]);
  return QBX_OK;
}

int qbx_signed_area_host(const double* nodes, int n_panels, double* area) {
  if (!nodes) return fail(QBX_EINVAL, "nodes is NULL");
  if (n_panels < 3) return fail(QBX_EINVAL, "n_panels = %d < 3", n_panels);
  // 16-point rule on each panel: area = 1/2 sum_a omega_a (x y' - y x')(tau_a)
  double t16[kQ], w16[kQ];
  for (int a = 0; a < kQ; ++a) gauss_legendre_node(kQ, a, &t16[a], &w16[a]);
  const auto& D = node_diff().d;
  double A = 0.0;
  for (int m = 0; m < n_panels; ++m) {
    const double* X = nodes + (size_t)m * 2 * kQ;
    for (int b = 0; b < kQ; ++b) {
      double dx = 0.0, dy = 0.0;
      for (int a = 0; a < kQ; ++a) {
        dx += D[b][a] * X[2 * a];
        dy += D[b][a] * X[2 * a + 1];
      }
      A += 0.5 * w16[b] * (X[2 * b] * dy - X[2 * b + 1] * dx);
    }
  }
  if (area) *area = A;
  if (!std::isfinite(A)) return fail(QBX_EINVAL, "non-finite node coordinates");
  if (A < 0.0) return fail(QBX_EORIENT, "signed area %g < 0: contour is clockwise", A);
  return QBX_OK;
}

int qbx_set_tuning(const qbx_tuning* t) {
  if (!t) return fail(QBX_EINVAL, "tuning is NULL");
  const int lo = 256, hi = 1 << 22;
  auto in = [&](int v) { return v >= lo && v <= hi; };
  if (!in(t->forward_waves) || !in(t->tape_waves) || !in(t->adjoint_waves) ||
      !in(t->batch_adjoint_tasks) || !in(t->fused_tiles))
    return fail(QBX_EINVAL, "tuning wave / task / tile targets must lie in [%d, %d]", lo, hi);
  if (!(t->batch_grid_scale >= 0.125 && t->batch_grid_scale <= 8.0))
    return fail(QBX_EINVAL, "batch_grid_scale = %g outside [0.125, 8]", t->batch_grid_scale);
  if (t->batch_fused_chunks < 1 || t->batch_fused_chunks > 64)
    return fail(QBX_EINVAL, "batch_fused_chunks = %d outside [1, 64]", t->batch_fused_chunks);
  if (!(t->fused_part_bytes >= 4096.0 && t->fused_part_bytes <= 1099511627776.0))
    return fail(QBX_EINVAL, "fused_part_bytes = %g outside [4096, 2^40]", t->fused_part_bytes);
  set_contour_tuning(t->forward_waves, t->tape_waves, t->adjoint_waves, t->fused_tiles);
  g_fused_part_bytes = t->fused_part_bytes;
  set_batch_tuning(t->batch_grid_scale, (double)t->batch_adjoint_tasks, t->batch_fused_chunks);
  return QBX_OK;
}

int qbx_get_tuning(qbx_tuning* t) {
  if (!t) return fail(QBX_EINVAL, "tuning is NULL");
  int fw, tw, aw, ft, fc;
  get_contour_tuning(&fw, &tw, &aw, &ft);
  double gs, at;
  get_batch_tuning(&gs, &at, &fc);
  t->forward_waves = fw;
  t->tape_waves = tw;
  t->adjoint_waves = aw;
  t->batch_adjoint_tasks = (int32_t)at;
  t->batch_grid_scale = gs;
  t->fused_tiles = ft;
  t->batch_fused_chunks = fc;
  t->fused_part_bytes = g_fused_part_bytes;
  return QBX_OK;
}

int qbx_kernel_timer(int enable) {
  timer_clear();
  g_timer_on = enable != 0;
  return QBX_OK;
}

int qbx_kernel_timer_read(double* ms, int* launches) {
  if (!ms || !launches) return fail(QBX_EINVAL, "NULL output array");
  for (int c = 0; c < QBX_TIMER_CLASSES; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (auto& r : g_timer) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return device_fail(e, "event synchronize");
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) return device_fail(e, "event elapsed time");
    ms[r.cls] += t;
    launches[r.cls] += 1;
  }
  return QBX_OK;
}

const char* qbx_strerror(int code) {
  switch (code) {
    case QBX_OK: return "success";
    case QBX_EINVAL: return "invalid argument";
    case QBX_EWORKSPACE: return "workspace too small";
    case QBX_EORIENT: return "contour is clockwise";
    case QBX_EGRAF: return "Graf condition violated (source inside an expansion disk)";
    case QBX_EDEVICE: return "HIP device error";
    case QBX_EIO: return "autotuner cache file error";
    default: return "unknown error";
  }
}

const char* qbx_last_error(void) { return g_last_error.c_str(); }

int qbx_debug_hankel01(const double* z, int n, double* h0, double* h1, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!z || !h0 || !h1))) return fail(QBX_EINVAL, "bad debug_hankel01 args");
  hipError_t e = launch_debug_hankel01(z, n, h0, h1, stream);
  return e == hipSuccess ? QBX_OK : device_fail(e, "debug_hankel01");
}

int qbx_debug_besselj(const double* x, int n, int L, double* out, hipStream_t stream) {
  if (n < 0 || L < 0 || L > QBX_PMAX + 3 || (n > 0 && (!x || !out)))
    return fail(QBX_EINVAL, "bad debug_besselj args");
  hipError_t e = launch_debug_besselj(x, n, L, out, stream);
  return e == hipSuccess ? QBX_OK : device_fail(e, "debug_besselj");
}

}  // extern "C"
