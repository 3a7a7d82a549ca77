// Internal declarations shared by the host C-ABI and the HIP kernels of libqbx.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/qbx.h"

namespace qbx {

constexpr int kQ = 16;      // nodes per panel
constexpr int kWave = 64;   // CDNA wavefront
// near/far split: capacity of a panel's near list; a panel with more near panels
// is served by the scan of all panels instead
constexpr int kNearCap = 64;

// per-panel near lists of the split: count[m] and, when count[m] <= kNearCap,
// list[m * kNearCap + i], i < count[m], the panels near m in ascending order
struct NearLists {
  const int* count;
  const int* list;
};

// the split's far sources, the Nystrom grid: per node {x, y, n_x, n_y}, the weighted
// densities [nk][T] and the 16-point weights w = omega |X'|
struct NystromSources {
  double4* geo;
  double2* dens;
  double* w;
};
constexpr int kPMax = 24;

// One expansion center: position, radius and the direction of its target,
// e^{i theta} = (ct, st) with theta = arg(x - c).  64 bytes so that a wave reads
// a record with one scalar load.
struct CenterRec {
  double cx, cy, R, ct, st, x, y, pad;
};

// Problem dimensions derived from the call arguments.
struct Dims {
  int P;        // panels
  int qs;       // source nodes per panel (16 * oversample)
  int T;        // targets (16 * P)
  int N;        // sources (qs * P)
  int n_sides;  // 1 or 2
  int nk;       // kinds (1 or 2)
  int p;        // expansion order
  int Mc;       // centers (T * n_sides)
  int NJ;       // J table length per center: J_0..J_{p+3}, J'_0..J'_{p+3}
  int side;     // QBX_INTERIOR / QBX_BOTH / QBX_EXTERIOR
  int kind;     // bit mask S=1, D=2
  int dipole;       // 0: the D slot differentiates along the source normal; 1: along
                    // the tangent (the operator R)
  int center_rule;  // 0: center distance r h_m; 1: r sqrt(h_m)
  double k, r;
  // forward launch shape
  int chunks;            // ceil(N / 64)
  int n_split;           // source splits per center
  int chunks_per_split;  // 64-source chunks per split
  // forward-with-tape launch shape (source splits)
  int n_tsplit;
  int tape_chunks_per_split;
  // adjoint source-major launch shape
  int n_csplit;           // center splits per 64-source chunk
  int centers_per_split;  // centers per split
  // fused adjoint launch shape: workgroup tiles of fused_cblock centers x
  // chunks_per_sb 64-source chunks, n_cb x n_sb tiles
  int fused_cblock, n_cb, n_sb, chunks_per_sb;
  // split forward, far pass: waves of 64 targets x about panels_per_fsplit
  // source panels (16 far sources each: the Nystrom grid), n_fsplit source
  // splits, split sp taking panels sp, sp + n_fsplit, ...
  int n_fsplit, panels_per_fsplit;
  // its adjoint, far part: waves of 64 far sources x about panels_per_asplit
  // target panels, n_asplit target splits taken alike
  int n_asplit, panels_per_asplit;
};

// Byte offsets of the workspace arrays (all 256-byte aligned).
struct Layout {
  size_t tables;   // double[table_doubles(qs)]
  size_t geo;      // double4[N]  {x, y, nx, ny}
  size_t dens;     // double2[nk][N]  w * density on the source grid
  size_t wgt;      // double[N] source quadrature weights w
  size_t h;        // double[P] panel lengths
  size_t ctr;      // CenterRec[Mc]
  size_t jtab;     // double[Mc][NJ], then double[Mc][NJ / 2] l J_l (target derivatives)
  size_t partial;  // forward: double2[n_split][nk][Mc]; forward-with-tape: double2[n_tsplit][nk][Mc][5]
  size_t tape;     // double2[Mc][nk][4] tape recomputed by the adjoint when none is given
  size_t G;        // double2[nk][Mc] conj(cotangent) i/4
  size_t cg;       // double[Mc][8] per-center gradients
  size_t spart;    // double2[max(n_csplit, n_cb)][src_slots(kind)][N] source-side partial sums
  size_t cpart;    // double[n_sb][Mc][4] fused adjoint: center-side partial sums
  size_t sg;       // double[N][8] per-source gradients
  size_t scratch;  // double[16 + Mc] small reductions
  size_t bnd;      // double4[P] split forward: panel mean and squared radius
  size_t ncount;   // int[P] split: near-panel counts
  size_t nlist;    // int[P][kNearCap] split: near-panel lists
  size_t fpart;    // double2[n_fsplit][nk][T][2] split: far sums (forward: first half)
  size_t gfar;     // double2[nk][T] split adjoint: cotangent weights of both sides
  size_t aacc;     // double2[nk][N] split adjoint: near sums per source
  size_t ngeo;     // double4[T] split: the far sources (Nystrom grid) {x, y, nx, ny}
  size_t ndens;    // double2[nk][T] split: their weighted densities
  size_t nw;       // double[T] split: their 16-point weights
  size_t apart;    // double2[n_asplit][nk + 2][T] split adjoint: far sums per far source
                   // (density; with the node gradient also position and normal)
  size_t gtw;      // double[T][2] split node adjoint: far weights' tangent gradients
  size_t gde;      // double2[nk][T] split node adjoint: far node density gradients
  size_t total;
};

// Offsets (in doubles) of the Gauss-Legendre / interpolation tables.
struct TableLayout {
  int tau16, w16, taus, ws, V, Vd, Dn, total;
};

__host__ __device__ inline TableLayout table_layout(int qs) {
  TableLayout t;
  t.tau16 = 0;
  t.w16 = 16;
  t.taus = 32;
  t.ws = t.taus + qs;
  t.V = t.ws + qs;            // [qs][16] value map 16 nodes -> source node
  t.Vd = t.V + qs * kQ;       // [qs][16] d/dtau map
  t.Dn = t.Vd + qs * kQ;      // [16][16] d/dtau at the nodes
  t.total = t.Dn + kQ * kQ;
  return t;
}

// side index -> sign (+1 exterior, -1 interior)
__host__ __device__ inline double side_sign(int side, int si) {
  if (side == 0) return si == 0 ? 1.0 : -1.0;
  return side > 0 ? 1.0 : -1.0;
}

bool make_dims(int n_panels, int q, int p, int oversample, int side, int kind, double k, double r,
               Dims* d);
void set_launch_shape(Dims* d);
// error reporting shared by the C entry points (qbx_last_error)
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int device_fail(hipError_t e, const char* where);
size_t align256(size_t x);
Layout make_layout(const Dims& d);
// the plain forward's arrays only (tables ... partial), packed from offset 0
Layout make_forward_layout(const Dims& d);
// tables, source grid and centers, then the plain forward and its finalize
// into out, with the arrays of L (make_layout or make_forward_layout) in ws;
// timed: bracket the pair kernel with the kernel timer's events when it is on
int run_forward(const Dims& d, const Layout& L, const double* nodes, const double* density,
                double* out, void* ws, hipStream_t stream, bool timed = true);

// ---- launchers (qbx_geometry.hip / qbx_forward.hip) ----
hipError_t launch_tables(const Dims& d, double* tables, hipStream_t s);
hipError_t launch_upsample(const Dims& d, const double* nodes, const double* density,
                           const double* tables, double4* geo, double2* dens, double* wgt,
                           double* h, CenterRec* ctr, double* jtab, hipStream_t s);
hipError_t launch_forward(const Dims& d, const double4* geo, const double2* dens,
                          const CenterRec* ctr, const double* jtab, double2* partial,
                          hipStream_t s);
hipError_t launch_finalize(const Dims& d, const double2* partial, double* out, hipStream_t s);
hipError_t launch_principal_value(int T, int nk, int side, int kind, const double* out,
                                  const double* density, double* pv, hipStream_t s);
// d[b][a]: derivative in the panel parameter, at node b, of the degree-15
// Lagrange basis polynomial of node a (16-point Gauss-Legendre nodes)
struct NodeDiff {
  double d[kQ][kQ];
};
const NodeDiff& node_diff();
// on-surface target derivatives from one-sided limits (Section 3.2 jumps):
// grad [n_sides][nk][T][2] -> grad_pv [nk][T][2], dn [n_sides][nk][T] -> dn_pv
// [nk][T] (either pair may be NULL)
hipError_t launch_gradient_principal_value(int T, int nk, int side, int kind, const NodeDiff& D,
                                           const double* nodes, const double* density,
                                           const double* grad, const double* dn,
                                           double* grad_pv, double* dn_pv, hipStream_t s);
// ---- split forward (qbx_split.hip) ----
// per panel {b_x, b_y, rad2, sqrt(rad2)}: the near relation's mean and squared
// node radius, and the node radius
hipError_t launch_panel_bounds(const Dims& d, const double* nodes, double4* bnd, hipStream_t s);
// the Nystrom grid's far sources from the nodes, node densities and tables
hipError_t launch_nystrom_sources(const Dims& d, const double* nodes, const double* density,
                                  const double* tables, NystromSources ns, hipStream_t s);
// partial [nk][Mc]: QBX sums over the sources of near panels
hipError_t launch_split_near(const Dims& d, const double4* geo, const double2* dens,
                             const CenterRec* ctr, const double* jtab, const double4* bnd,
                             double g2, NearLists nl, double2* partial, hipStream_t s);
// the near lists of every panel (count, list: NearLists' arrays)
hipError_t launch_near_lists(const Dims& d, const double4* bnd, double g2, int* count, int* list,
                             hipStream_t s);
// partial [n_fsplit][nk][T]: direct sums over the far sources (ns) of far panels
hipError_t launch_split_far(const Dims& d, NystromSources ns, const double* nodes,
                            const double4* bnd, double g2, double2* partial, hipStream_t s);
hipError_t launch_split_finalize(const Dims& d, const double2* nearp, const double2* farp,
                                 double* out, hipStream_t s);
// the split's target derivatives: near sums [nk][Mc][2], far sums
// [n_fsplit][nk][T][2], then grad and n . grad (either may be NULL)
hipError_t launch_split_gradient(const Dims& d, const double* nodes, const double4* geo,
                                 const double2* dens, NystromSources ns, const CenterRec* ctr,
                                 const double* jtab, const double4* bnd, double g2, NearLists nl,
                                 double2* nearp, double2* farp, double* grad, double* dn,
                                 hipStream_t s);
// the split's adjoint with respect to the density (G from launch_make_G)
hipError_t launch_split_adjoint_density(const Dims& d, const double* nodes, const double* tables,
                                        const double4* geo, const double* wgt, NystromSources ns,
                                        const CenterRec* ctr, const double* jtab,
                                        const double4* bnd, double g2, NearLists nl,
                                        const double2* G, double2* Gf, double2* acc,
                                        double2* partial, double* grad_density, hipStream_t s);
// the split's adjoint with respect to the nodes (and the density, through the
// chain rule; either output may be NULL): cg [Mc][8], spart [src_slots][N], fpart
// [n_fsplit][nk][T][2], apart [n_asplit][nk + 2][T], sg [N][8], gtw [T][2],
// gde [nk][T]
struct SplitNodeScratch {
  double2* Gf;
  double* cg;
  double2* spart;
  double2* fpart;
  double2* apart;
  double* sg;
  double* gtw;
  double2* gde;
};
hipError_t launch_split_adjoint_nodes(const Dims& d, const double* nodes, const double* density,
                                      const double* tables, const double4* geo,
                                      const double2* dens, NystromSources ns,
                                      const CenterRec* ctr, const double* jtab,
                                      const double4* bnd, double g2, NearLists nl,
                                      const double2* G, SplitNodeScratch w,
                                      double* grad_density, double* grad_nodes, hipStream_t s);
// ---- adjoint (qbx_adjoint.hip) ----
// the chain rule to the nodes and node densities from the per-source (sg) and
// per-center (cg) gradients; one block per panel
// (gtw, gde: the optional node terms of chain_panel, or NULL)
hipError_t launch_chain(const Dims& d, const double* nodes, const double* density,
                        const double* tables, const double* sg, const double* cg,
                        const double* gtw, const double* gde, double* grad_density,
                        double* grad_nodes, hipStream_t s);
hipError_t launch_forward_tape(const Dims& d, const double4* geo, const double2* dens,
                               const CenterRec* ctr, const double* jtab, double2* partial,
                               hipStream_t s);
hipError_t launch_finalize_tape(const Dims& d, const double2* partial, double* out, double2* tape,
                                hipStream_t s);
// target derivatives: the pair pass (partial [n_tsplit][nk][Mc][2]), then the
// gradient and normal derivative from its sums
// jtab[Mc NJ + ci nj + l] = l J_l(k R_ci), nj = NJ / 2: the order-weighted Bessel values
// the target-derivative sums take, scaled once per center instead of once per pair
hipError_t launch_order_weighted(const Dims& d, double* jtab, hipStream_t s);
hipError_t launch_forward_grad(const Dims& d, const double4* geo, const double2* dens,
                               const CenterRec* ctr, const double* jtab, double2* partial,
                               hipStream_t s);
hipError_t launch_finalize_gradient(const Dims& d, const CenterRec* ctr, const double2* partial,
                                    double* grad, double* dn, hipStream_t s);
hipError_t launch_adjoint_src(const Dims& d, const double4* geo, const double2* dens,
                              const CenterRec* ctr, const double* jtab, const double2* G,
                              double2* partial, hipStream_t s);
hipError_t launch_make_G(const Dims& d, const double* cot, double2* G, hipStream_t s);
// adjoint without a tape: one pass over the pairs for both gradient sides
hipError_t launch_adjoint_fused(const Dims& d, const double* nodes, const double* density,
                                const double* tables, const double4* geo, const double2* dens,
                                const CenterRec* ctr, const double* jtab, const double* cot,
                                double2* G, double* cpart, double* cg, double2* spartial,
                                double* sg, double* grad_density, double* grad_nodes,
                                hipStream_t s);
// double2 slots per source of the adjoint's source-side partial sums:
//   0 .. nk-1    sum_i conj(G_i K_ij), one per kind (the density gradients)
//   nk           sum_i Re(G_i q_j grad_v K_ij), both components, over the kinds
//   nk + 1 (D)   (sum_i Re(G_i q_j dK_ij/dpsi), 0)
__host__ __device__ constexpr int src_slots(int kind) {
  return (kind == 3 ? 2 : 1) + 1 + ((kind & 2) ? 1 : 0);
}
// centers per fused tile: each of the four waves keeps its own LDS sums of
// the tile's centers (4 x 32 B a center), small enough that as many workgroups
// share a CU (160 KB of LDS) as the kernel's registers allow
#ifndef QBX_FUSED_CENTERS
#define QBX_FUSED_CENTERS 256
#endif
__host__ __device__ constexpr int fused_centers(int) { return QBX_FUSED_CENTERS; }
// bound in bytes on the fused adjoint's source-side partial sums (the tuning's
// fused_part_bytes)
double fused_part_budget();
// centers per fused tile (taken in sub-blocks of fused_centers()): the
// source-side partial sums are one row of sources per tile of centers, so they
// take sources x centers / height x 16 B a slot.  The height starts at one
// sub-block (fine-grained tiles) and doubles while those sums would pass
// fused_part_budget() bytes.
inline int fused_tile_height(int Mc, int N, int kind) {
  const double budget = fused_part_budget();
  long long h = fused_centers(kind);
  while (h < Mc && (double)((Mc + h - 1) / h) * src_slots(kind) * (double)N * 16.0 > budget)
    h *= 2;
  return h < Mc ? (int)h : Mc;
}
hipError_t launch_adjoint_rest(const Dims& d, const double* nodes, const double* density,
                               const double* tables, const double4* geo, const double2* dens,
                               const CenterRec* ctr, const double* jtab, const double* cot,
                               const double2* tape, double2* G, double* cg, double2* spartial,
                               double* sg, double* grad_density, double* grad_nodes,
                               hipStream_t s);
// scratch[0] = signed area, scratch[1] = min_ij |x'_j - c_i| / R_i
hipError_t launch_check(const Dims& d, const double4* geo, const double* wgt,
                        const CenterRec* ctr, double* scratch, hipStream_t s);
hipError_t launch_debug_hankel01(const double* z, int n, double* h0, double* h1, hipStream_t s);
hipError_t launch_debug_besselj(const double* x, int n, int L, double* out, hipStream_t s);

}  // namespace qbx

namespace qbx {
// tunables of the per-contour (qbx_api.cpp) and batched (qbx_batched.hip) paths
void set_contour_tuning(int forward_waves, int tape_waves, int adjoint_waves, int fused_tiles);
void get_contour_tuning(int* forward_waves, int* tape_waves, int* adjoint_waves,
                        int* fused_tiles);
void set_batch_tuning(double grid_scale, double adjoint_tasks, int fused_chunks);
void get_batch_tuning(double* grid_scale, double* adjoint_tasks, int* fused_chunks);
int validate(const qbx_geometry* g, int p, double k, double r, int oversample, int side,
             int kind, Dims* d);
}  // namespace qbx

// return FN<p>(args...) for the runtime order PV in [0, 24]
#define QBX_P_SWITCH(PV, FN, ...)                                                            \
  switch (PV) {                                                                             \
    case 0: return FN<0>(__VA_ARGS__);   case 1: return FN<1>(__VA_ARGS__);                \
    case 2: return FN<2>(__VA_ARGS__);   case 3: return FN<3>(__VA_ARGS__);                \
    case 4: return FN<4>(__VA_ARGS__);   case 5: return FN<5>(__VA_ARGS__);                \
    case 6: return FN<6>(__VA_ARGS__);   case 7: return FN<7>(__VA_ARGS__);                \
    case 8: return FN<8>(__VA_ARGS__);   case 9: return FN<9>(__VA_ARGS__);                \
    case 10: return FN<10>(__VA_ARGS__); case 11: return FN<11>(__VA_ARGS__);              \
    case 12: return FN<12>(__VA_ARGS__); case 13: return FN<13>(__VA_ARGS__);              \
    case 14: return FN<14>(__VA_ARGS__); case 15: return FN<15>(__VA_ARGS__);              \
    case 16: return FN<16>(__VA_ARGS__); case 17: return FN<17>(__VA_ARGS__);              \
    case 18: return FN<18>(__VA_ARGS__); case 19: return FN<19>(__VA_ARGS__);              \
    case 20: return FN<20>(__VA_ARGS__); case 21: return FN<21>(__VA_ARGS__);              \
    case 22: return FN<22>(__VA_ARGS__); case 23: return FN<23>(__VA_ARGS__);              \
    case 24: return FN<24>(__VA_ARGS__);                                                   \
    default: return hipErrorInvalidValue;                                                  \
  }

namespace qbx {
// kernel timer (qbx_kernel_timer): records an event pair around a launch of
// kernel class `cls` when enabled; no-op otherwise
void timer_begin(int cls, hipStream_t s);
void timer_end(int cls, hipStream_t s);
}  // namespace qbx
